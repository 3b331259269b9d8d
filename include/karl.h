/*
 * karl.h -- C ABI of libkarl, the MI355X (gfx950) implementation of the particle-history
 * transport of the KARL Monte Carlo method (Sendlinger, Kellerer, Spanier, arXiv 2503.10263).
 *
 * A job is the paper's problem statement: a cylindrical gas column (Sec. 2.2, "Scalar
 * field"), a uniform axial magnetic field or none (Sec. 3.1), the tracked species and their
 * interactions with cross sections given as 1-D functions (Sec. 3.3), an injector (Sec. 3.5)
 * and the diagnostics -- density fields, current collectors, deletion logger (Sec. 2.2, 2.3,
 * 3.2, 3.4).  karl_transport() runs the main simulation cycle of Sec. 2.1 for a range of
 * primary events on the GPU: every history is followed through free flights with
 * d = -lambda ln(eta) (eqs. 1-2), segment stops, interactions and secondaries until all its
 * particles terminate.
 *
 * Conventions
 *   - SI units, energies in eV.  All pointers in karl_job_desc are HOST memory owned by the
 *     caller and deep-copied by karl_create_job (the caller may free them on return), except
 *     `workspace`, which is DEVICE memory owned by the caller; it must stay allocated until
 *     karl_destroy_job and must not be used by anything else meanwhile.
 *   - Every entry point returns a karl_status; nothing throws across the ABI.  On failure
 *     karl_last_error() returns a message for the calling thread.
 *   - Results depend only on (descriptor, set of primary ids): random numbers are
 *     Philox4x32-10 keyed by (seed, primary id) and counted by (step, slot, lineage), so
 *     launch partitioning, chunking, batching and queue sizes do not change any integer
 *     tally; floating-point tallies differ only in the order of their additions.
 */
#ifndef KARL_H
#define KARL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t karl_status;
#define KARL_OK         0
#define KARL_EINVAL    (-1)  /* invalid descriptor, argument or buffer size          */
#define KARL_ENOMEM    (-2)  /* workspace smaller than karl_workspace_bytes()        */
#define KARL_EDEVICE   (-3)  /* a HIP call failed                                     */
#define KARL_EOVERFLOW (-4)  /* a single primary's secondaries exceed the queue       */
#define KARL_ESTATE    (-5)  /* call on a destroyed or failed job                     */
#define KARL_ENUMERIC  (-6)  /* NaN/Inf met in the particle state                     */

#define KARL_MAX_PROC 16
#define KARL_MAX_SPECIES 4

/* interaction classes (Sec. 3.3): elastic scattering, excitation, ionization (the ion made is
   the process's `product` species: the molecular ion, or the atomic ion of dissociative
   ionization), recombination, charge exchange (the projectile continues with the velocity of a
   target particle) and clustering (the projectile is replaced by a particle of the `product`
   species moving along a target particle's velocity with that particle's momentum) */
enum { KARL_ELASTIC = 0, KARL_EXCITATION = 1, KARL_IONIZATION = 2, KARL_RECOMBINATION = 3,
       KARL_CHARGE_EXCHANGE = 4, KARL_CLUSTERING = 5 };
/* target of a process: the gas, or the density field of the process's `partner` species
   (Sec. 2.2 "Density fields"); TARGET_ION_FIELD is the older name of the electrons' case */
enum { KARL_TARGET_GAS = 0, KARL_TARGET_FIELD = 1, KARL_TARGET_ION_FIELD = 1 };
/* KARL_SOURCE_PAIR: both species from the beam position and direction, even primary ids
   electrons at beam_energy, odd ids ions at beam_energy_1 */
enum { KARL_SOURCE_BETA = 0, KARL_SOURCE_BEAM = 1, KARL_SOURCE_PAIR = 2 };
enum { KARL_FP64 = 0, KARL_FP32 = 1 };
/* how karl_transport maps flights onto the device (job descriptor field `mapping`):
   KARL_MAP_LANE  one particle per lane, one flight segment per step;
   KARL_MAP_WAVE  one particle per lane, but a particle whose last segment ended on a z-face
                  (guiding-centre mode) has its flight advanced by the whole wave: lane k takes
                  segment k with its own free-path draw, up to 64 segments at once;
   KARL_MAP_AUTO  run the job's first chunk with LANE, measure its flight segments per
                  interaction, and use WAVE from the next chunk on if that is at least 32 (the
                  crossover measured on MI355X).
   The free path is redrawn at every face (Sec. 3.1) from a draw keyed by the step, so segment k
   needs nothing from segments before it: results do not depend on the mapping.  Straight-line
   jobs and batched launches use LANE. */
enum { KARL_MAP_AUTO = 0, KARL_MAP_LANE = 1, KARL_MAP_WAVE = 2 };
/* movers (Sec. 3.1): KARL_MOVER_DRIFT moves along the exact helix about the guiding centre in
   the uniform axial field bz (straight lines when bz = 0) and stops at every segment face;
   KARL_MOVER_BORIS advances each particle by Boris pushes of a fixed time step per species with
   the electric and magnetic fields of its field bin (one push per transport step), and stops a
   movement when the particle leaves the domain, its segment or its energy bin (no interaction,
   a new distance is drawn) or when the moved distance exceeds the drawn one (interaction at the
   current position).  The time of a movement goes to the segment and energy bin it started in. */
enum { KARL_MOVER_DRIFT = 0, KARL_MOVER_BORIS = 1 };

/* job flags */
#define KARL_FLAG_DIGESTS 1u   /* per-primary 64-bit digest of the event sequence          */
#define KARL_FLAG_HISTORY 2u   /* per-primary ledger: E_in, E_accounted, n_born, n_deleted  */

/* deletion reasons (Sec. 3.2, deletion logger); KARL_CONVERTED: the projectile of a clustering
   reaction, replaced by its product */
enum { KARL_EXIT_LOW = 0, KARL_EXIT_HIGH, KARL_WALL, KARL_CUTOFF, KARL_RECOMBINED, KARL_CAP,
       KARL_LIFETIME, KARL_UNTRACKED, KARL_CONVERTED, KARL_NREASON };

/* layout of the counters array (int64); per-species entries have KARL_MAX_SPECIES slots */
#define KARL_C_BIRTH          0  /* [4] particles born per species                      */
#define KARL_C_STEP           4  /* [4] flight segments per species                     */
#define KARL_C_COLL           8  /* [4] interactions per species                        */
#define KARL_C_ZCROSS        12  /* [4] z-face crossings per species                    */
#define KARL_C_RCROSS        16  /* [4] r-face crossings per species (wall included)    */
#define KARL_C_TARGET_REDRAW 20  /* ionization target-velocity redraws                  */
#define KARL_C_BEB_TRIES     21  /* secondary-energy proposals                          */
#define KARL_C_BETA_TRIES    22  /* beta-energy proposals                               */
#define KARL_C_PROC          24  /* [16] interactions per process                       */
#define KARL_C_DEATH         40  /* [4][9] deletions per species and reason             */
#define KARL_NCOUNTERS       80

/* layout of the ledger array (double) */
#define KARL_L_E_PRIMARY      0  /* summed birth energy of primaries (eV)               */
#define KARL_L_E_DEATH        1  /* [4][9] energy at deletion per species and reason    */
#define KARL_L_E_EXC         37  /* excitation energy losses                            */
#define KARL_L_E_BIND        38  /* ionization binding energies                         */
#define KARL_L_E_GAS         39  /* energy exchanged with the gas: elastic recoil, the
                                    ionization frame, charge exchange, and minus the energy of
                                    ionization and clustering products (a target particle's
                                    velocity)                                           */
#define KARL_L_T_ALIVE       40  /* [4] summed particle lifetimes (s)                   */
#define KARL_L_E_FIELD       44  /* work of the electric field on the particles (eV)    */
#define KARL_NLEDGER         48

#define KARL_NHIST            4  /* per-primary ledger entries                          */

typedef struct {
    double mass;            /* kg */
    double charge;          /* C, signed; sets the gyration sense */
    double e_cut;           /* eV; a particle with E < e_cut is deleted (strict) */
    double lifetime;        /* s; deletion once the summed flight time reaches it (INFINITY: none) */
    int64_t cap;            /* maximum number of interactions (Sec. 3.2) */
    int32_t tracked;        /* 0: counted at birth and deleted, never transported */
    int32_t reserved0;
    double xs_emin;         /* eV; energy of the first cross-section node */
    double xs_emax;         /* eV; energy of the last node; nodes are log-spaced */
    const double* edges;    /* [n_bins+1] increasing spectrum bin edges (eV) */
    const double* dens_edges;  /* [n_dens_bins+1] increasing energy-bin edges of the
                                  energy-resolved density field (eV); NULL without it */
} karl_species_desc;

typedef struct {
    int32_t kind;           /* KARL_ELASTIC ... KARL_CLUSTERING */
    int32_t species;        /* projectile slot 0..n_species-1 (slot 0: electrons) */
    int32_t target;         /* KARL_TARGET_GAS or KARL_TARGET_FIELD */
    int32_t product;        /* ionization: the ion species made (1..n_species-1); clustering:
                               the species the projectile becomes; ignored otherwise */
    int32_t partner;        /* KARL_TARGET_FIELD: the species whose density field is the
                               target (all field processes of one species share one partner);
                               recombination: the species whose field logs the deletion */
    int32_t density_power;  /* gas targets: the rate goes as n_gas^density_power, 1 or 2
                               (three-body clustering: xs holds k/v in m^5); 0 means 1 */
    double e_th;            /* eV: excitation energy or ionization binding energy; 0 else */
    const double* xs;       /* [n_e] cross section (m^2) at the projectile species' nodes */
    /* elastic scattering angle (Sec. 3.3 "Elastic scattering"): isotropic in the centre-of-mass
       frame when ang_bins == 0 or the centre-of-mass impact energy is below e_iso (a composite
       distribution); otherwise drawn from the piecewise linear density over the polar angle of
       the impact-energy bin (below the first edge: the first bin, from the last edge on: the
       last).  Elastic processes only. */
    int32_t ang_bins;       /* energy bins, 0..1024 */
    int32_t ang_nodes;      /* angle nodes per bin, 2..4096 */
    double e_iso;           /* eV */
    const double* ang_edges;  /* [ang_bins+1] increasing centre-of-mass energies (eV) */
    const double* ang_theta;  /* [ang_nodes] increasing polar angles in [0, pi] (rad) */
    const double* ang_pdf;    /* [ang_bins][ang_nodes] densities >= 0, positive area per bin */
} karl_process_desc;

typedef struct {
    double radius, length;        /* cylinder r <= radius, 0 <= z <= length (m) */
    int32_t n_r, n_z;             /* segments of the density/current grid (>= 1) */
    const double* n_gas;          /* [n_z] gas density per z-segment (m^-3) */
    /* [n_r*n_z] density field of each species (m^-3), seen by field-target processes that
       name it as partner; NULL: 0 */
    const double* n_field[KARL_MAX_SPECIES];
    double t_gas;                 /* gas temperature (K); 0: target at rest */
    double m_gas;                 /* gas molecule mass (kg) */
    double bz;                    /* axial field (T); 0 selects straight-line transport */
    karl_species_desc species[KARL_MAX_SPECIES]; /* slot 0 electrons, 1.. ions */
    int32_t n_species;            /* 2..KARL_MAX_SPECIES; 0 means 2 */
    int32_t n_proc;               /* <= KARL_MAX_PROC */
    int32_t n_e;                  /* cross-section nodes per table, 2..1024 */
    karl_process_desc proc[KARL_MAX_PROC];
    int32_t source;               /* KARL_SOURCE_BETA, KARL_SOURCE_BEAM or KARL_SOURCE_PAIR */
    int32_t beam_species;
    double beta_e0, beta_z, beta_fmax;  /* endpoint (eV), daughter charge, shape bound */
    double beam_energy, beam_pos[3], beam_dir[3];
    double beam_energy_1;         /* ion energy of KARL_SOURCE_PAIR (eV) */
    uint32_t seed;
    int32_t n_bins;               /* spectrum bins per species (edges hold n_bins+1) */
    int32_t n_planes;             /* spectrum planes, each a z-face index 0..n_z */
    int32_t reserved0;
    const int32_t* planes;
    int64_t n_primaries;          /* primary ids are 0 .. n_primaries-1 */
    int32_t precision;            /* KARL_FP64 or KARL_FP32 transport state */
    uint32_t flags;               /* KARL_FLAG_* */
    int64_t queue_capacity;       /* secondary-queue entries per buffer; 0: 1<<22 */
    int64_t chunk;                /* initial primaries per launch; 0: 65536 */
    void* workspace;              /* device memory, >= karl_workspace_bytes() */
    uint64_t workspace_bytes;
    int32_t mapping;              /* KARL_MAP_AUTO, KARL_MAP_LANE or KARL_MAP_WAVE */
    int32_t n_dens_bins;          /* energy bins of the energy-resolved density field (Sec. 3.4:
                                     times per segment with an energy axis), 0..4096; 0: none */
    int32_t mover;                /* KARL_MOVER_DRIFT or KARL_MOVER_BORIS */
    int32_t reserved1;
    /* Boris mover: time step per species (s; every species of the job needs one, and a finite
       lifetime of at most 2^31 steps so that every particle ends).  Fields as arrays over a
       cylindrical binning of field_radius x field_length in field_nr x field_nz bins, each bin a
       vector of (r, phi, z) components, zero outside the binning (Sec. 3.8 "Vector field",
       from arrays); e_field NULL: no electric field, b_field NULL: the uniform axial field bz.
       The drift mover takes no field arrays. */
    double boris_dt[KARL_MAX_SPECIES];
    int32_t field_nr, field_nz;
    double field_radius, field_length;
    const double* e_field;        /* [field_nr][field_nz][3] V/m */
    const double* b_field;        /* [field_nr][field_nz][3] T */
    /* Deferred-queue launch in slices.  A scheduling option: the order in which particles run
       is free (Sec. 3.9 takes the next particle at random from the list; Sec. 3.6 evens out
       uneven loads over long cycles), and results do not depend on it, up to the summation
       order of floating-point tallies.  The species that make no products run after the other
       generations, in one launch over all their particles.  With slice_steps > 0, a particle
       of that launch goes back to the end of the launch's work every slice_steps of its steps
       (where its slices end is staggered from particle to particle): into a ring of
       slice_ring entries in the workspace, with its whole state, and its lane takes the next
       item.  So the long histories of the launch advance in turn and end together, instead of
       the last ones started running on alone while the other lanes idle.  A particle whose
       ring slot has not been read yet keeps its lane for another slice.  slice_steps: 0 (no
       slices, no ring) or a power of two up to 2^30.  slice_ring: ring entries, 0:
       queue_capacity + 2^20 (the launch's particles plus its lanes fit without full slots). */
    int64_t slice_steps;
    int64_t slice_ring;
} karl_job_desc;

/* Host buffers for karl_read_tallies; any NULL pointer is skipped.  Sizes in elements, with
   S = n_species: counters KARL_NCOUNTERS; ledger KARL_NLEDGER; density_time S*n_r*n_z;
   recomb S*n_r*n_z; jz S*n_r*(n_z+1)*2; jr S*(n_r+1)*n_z*2; spectra S*n_planes*2*(n_bins+2);
   digests n_primaries (needs KARL_FLAG_DIGESTS); hist n_primaries*KARL_NHIST
   (needs KARL_FLAG_HISTORY).  Index order is row-major in the order written. */
typedef struct {
    int64_t* counters;
    double* ledger;
    double* density_time;   /* [species][r][z] seconds spent per segment (eq. 3 numerator) */
    int64_t* recomb;        /* [species][r][z] recombinations logged in that species' field:
                               N_gamma of eq. 3 (made by its partners) */
    int64_t* jz;            /* [species][r][z-face][dir] crossings, dir 1 = +z (Sec. 2.3) */
    int64_t* jr;            /* [species][r-face][z][dir] crossings, dir 1 = outward */
    int64_t* spectra;       /* [species][plane][dir][bin] with under/overflow bins 0, n_bins+1 */
    uint64_t* digests;
    double* hist;
    double* density_time_e; /* [species][r][z][n_dens_bins+2] seconds per energy bin: each
                               flight segment's time in the bin of the particle's energy (bin 0
                               below the first edge, n_dens_bins+1 at or above the last) */
} karl_tallies;

/* Device bytes a job needs (tables, tallies and their snapshot, two secondary queues). */
karl_status karl_workspace_bytes(const karl_job_desc* desc, uint64_t* bytes);

/* Validate, deep-copy and upload a job; tallies start at zero.  The device is the current
   HIP device of the calling thread.  On success *out owns host resources until
   karl_destroy_job. */
karl_status karl_create_job(const karl_job_desc* desc, void** out);

/* Transport primaries pid_begin .. pid_end-1 (0 <= begin <= end <= n_primaries) and add
   their contributions to the job's tallies.  Work is enqueued on `hip_stream` (NULL: the
   null stream); the call returns after the last launch has completed, because the number of
   secondary generations is only known on the device.  Disjoint ranges accumulate;
   overlapping ranges count twice. */
karl_status karl_transport(void* job, int64_t pid_begin, int64_t pid_end, void* hip_stream);

/* Transport without allocation, for callers that cannot allocate memory at transport time:
   code under stream or graph capture, tight serving loops, harnesses that forbid hipMalloc.
   Same arguments, results and errors as karl_transport (the same kernels; digests and integer
   tallies identical, FP64 tallies up to the order of additions), but the call allocates
   nothing -- no device or pinned memory, no events: the generation and deferred queues, the
   control words and the tally snapshot used to undo a chunk whose queue overflowed live in a
   static device array of KARL_NOALLOC_SCRATCH_BYTES (64 MiB) that the library holds on every
   device it runs on until the process ends.  The job's tallies (its workspace) must leave
   room in that array for queues of 4096 entries (else KARL_EINVAL); the queue capacity is
   whatever the array leaves, and chunks halve on overflow as in karl_transport.  The deferred
   launch runs whole histories (no slices, whatever the job's slice_steps), and the launches
   are not timed (karl_job_stats does not count them).  Every call on a device shares that
   device's array and finds the previous call's contents in it (the control words are cleared
   at each call): calls that overlap on one device would race, so the library serializes them
   with a lock per device.  Synchronous like karl_transport. */
#define KARL_NOALLOC_SCRATCH_BYTES ((uint64_t)64 << 20)
karl_status karl_transport_noalloc(void* job, int64_t pid_begin, int64_t pid_end, void* hip_stream);

/* Copy the tallies into caller-owned host buffers (synchronizes `hip_stream`). Returns the
   job's sticky device status (KARL_EOVERFLOW, KARL_ENUMERIC) if one was raised. */
karl_status karl_read_tallies(void* job, karl_tallies* out, void* hip_stream);

/* Normalised fields (S12 readout) from the tallies of all primaries transported since creation
   or the last reset, N_prim: the simulated time is t_sim = N_prim / activity (eq. 4, activity
   in decays per second); density[species][r][z] = (time spent in the segment)/(t_sim V) minus,
   the recombinations logged in that species' field in the segment per volume (eq. 3); jz_current
   [species][r][z-face] and jr_current[species][r-face][z] = (N+ - N-)/(A t_sim) through the
   face (current collection, Sec. 2.3), in particles per m^2 per s; A of r-face 0 is zero and
   its current is reported as 0.  Sizes S*n_r*n_z, S*n_r*(n_z+1), S*(n_r+1)*n_z doubles (S =
   n_species); NULL pointers are skipped.  KARL_ESTATE if nothing was transported. */
karl_status karl_read_fields(void* job, double activity, double* density, double* jz_current,
                             double* jr_current, void* hip_stream);

/* Self-consistent target fields (Sec. 2.2 "Density fields", Sec. 3.6 cycles): set the density
   field of each species that a KARL_TARGET_FIELD process names as partner to that species'
   density from the tallies of all primaries transported so far, eq. (3) with
   t_sim = N_prim / activity (eq. 4), negative values set to zero.  Calling it after every
   cycle of primaries makes the later cycles interact with the particles of the earlier ones.
   No effect on a job without field targets; KARL_ESTATE if nothing was transported. */
karl_status karl_update_target_fields(void* job, double activity, void* hip_stream);

/* Zero the tallies and the count of transported primaries. */
karl_status karl_reset_tallies(void* job, void* hip_stream);

/* Timing of the transport kernels since creation or the last reset, measured with HIP
   events on the launch stream: *kernel_ms total, *n_launches launches, *generations
   secondary generations processed, *max_queue the largest generation. */
karl_status karl_job_stats(void* job, double* kernel_ms, int64_t* n_launches,
                           int64_t* generations, int64_t* max_queue);

/* Of karl_job_stats: the deferred launches alone (the launch over the deferred queue of
   species that make no secondaries, run after the generations of every chunk), *kernel_ms and
   *n_launches since creation or the last reset. */
karl_status karl_job_drain_stats(void* job, double* kernel_ms, int64_t* n_launches);

/* Particles that the job's deferred launches put into the ring at the end of a slice
   (karl_job_desc.slice_steps), since creation or the last karl_reset_tallies; 0 without
   slices.  Both pointers must be valid. */
karl_status karl_job_slices(void* job, int64_t* ring_entries);

/* The mapping karl_transport uses for this job (KARL_MAP_LANE or KARL_MAP_WAVE; KARL_MAP_AUTO
   while not yet tuned), the segments per interaction that chose it (0 if not tuned), the kernel
   time per flight segment of the last chunk run with each mapping (0 if none), and the segments
   advanced by wave-cooperative flights so far.  Any pointer may be NULL. */
karl_status karl_job_mapping(void* job, int32_t* mapping, double* segments_per_interaction,
                             double* ms_per_segment_lane, double* ms_per_segment_wave,
                             int64_t* wave_segments);

/* Release host resources of the job (the caller still owns the workspace). */
karl_status karl_destroy_job(void* job);

/* ---- batches: many jobs in one launch (scheduler, continuous batching) ----
   A batch owns the secondary queues and the job table of a launch over up to max_jobs jobs.
   Every lane carries the index of its job; each job keeps its own tables and tallies.
   Results of a job are the same alone and in any batch (integer tallies exactly). */

/* Device bytes of a batch with room for max_jobs jobs and queue_capacity entries per queue
   (0: 1<<22). */
karl_status karl_batch_workspace_bytes(int32_t max_jobs, int64_t queue_capacity, uint64_t* bytes);

/* Create a batch on the current HIP device; `workspace` is caller-owned device memory of at
   least karl_batch_workspace_bytes() bytes that must outlive the batch. */
karl_status karl_create_batch(int32_t max_jobs, int64_t queue_capacity, void* workspace,
                              uint64_t workspace_bytes, void** out);

/* Transport, in one sequence of launches shared by all of them, the primaries
   ranges[2i] .. ranges[2i+1]-1 of jobs[i] for i < n_jobs (all jobs of one precision, on the
   batch's device; 0 <= n_jobs <= max_jobs).  Tallies accumulate in each job.  Returns after the
   last launch has completed. */
karl_status karl_transport_batch(void* batch, void* const* jobs, const int64_t* ranges,
                                 int32_t n_jobs, void* hip_stream);

/* Kernel time, launches, secondary generations and largest generation of the batch. */
karl_status karl_batch_stats(void* batch, double* kernel_ms, int64_t* n_launches,
                             int64_t* generations, int64_t* max_queue);

/* Flight segments advanced by wave-cooperative flights in the batch's launches since its
   creation: a batched launch gives the flights of jobs whose mapping is (or was tuned to)
   KARL_MAP_WAVE to the whole wave, the others one lane per particle.  A job on KARL_MAP_AUTO
   chooses after the chunk in which its flight segments since creation reach 1e5: the wave
   mapping if it made at least 32 segments per interaction.  Results do not depend on it. */
karl_status karl_batch_wave_segments(void* batch, int64_t* wave_segments);

/* Release host resources of the batch (the caller still owns its workspace). */
karl_status karl_destroy_batch(void* batch);

/* ---- serving: continuous batching of transport requests ----
   A server takes job descriptors as they arrive, admits them while the HBM they need for
   tables, tallies and queues fits into its arena (device memory it sub-allocates, first fit),
   and transports them in rounds of one karl_transport_batch each: every round gives each of a
   worker's jobs up to a quantum of its next primaries; the quantum starts at max_quantum and
   follows a target round time (the larger of round_ms and twice the shortest recent round,
   since no round is shorter than its longest chain of histories).  Each admitted job belongs to one of n_workers workers (the least loaded); a worker
   owns a batch and a stream.  Rounds run either in the calling thread (karl_server_step) or,
   after karl_server_start, in one thread per worker, so that the rounds of different workers
   run concurrently and one round's tail (its longest histories) overlaps another's work.  Jobs
   admitted while others run join their worker's next round; a job leaves when its last
   primary is done and keeps its arena space, with its tallies, until it is released.  Because a history depends
   only on (seed, primary id), a job's tallies are the same served in any mix as transported
   alone (integer tallies exactly, FP64 sums up to the order of addition).  The paper's
   parallel runs balance uneven work over processes (Sec. 3.6); this is the single-device
   counterpart for many independent jobs.  A server is driven by one host thread. */
typedef struct {
    int32_t max_jobs;        /* jobs transported together (admission slots), >= 1 */
    int32_t precision;       /* KARL_FP64 or KARL_FP32: every submitted job must match */
    int64_t queue_capacity;  /* entries per secondary queue of the shared batch (0: 1<<22) */
    uint64_t arena_bytes;    /* device bytes for job workspaces: the admission budget */
    double round_ms;         /* target wall time of one round (<= 0: 50 ms) */
    int64_t min_quantum;     /* bounds of the primaries per job per round (0: 64 and 1<<22) */
    int64_t max_quantum;
    int32_t n_workers;       /* concurrent rounds, one batch and stream each (0: 2; max 4) */
    void* workspace;         /* caller-owned device memory of karl_server_workspace_bytes() */
    uint64_t workspace_bytes;
} karl_server_desc;

typedef struct {
    int64_t submitted, admitted, completed, released, rounds;
    int64_t primaries;       /* primaries transported by all rounds */
    double kernel_ms;        /* transport kernel time of all rounds (HIP events) */
    double busy_ms;          /* host wall time spent inside rounds */
    uint64_t arena_used, arena_peak;   /* bytes held by admitted, unreleased jobs */
    int64_t quantum;         /* current primaries per job per round */
} karl_server_stats;

/* Device bytes of a server (n_workers batch regions plus arena_bytes). */
karl_status karl_server_workspace_bytes(const karl_server_desc* desc, uint64_t* bytes);

/* Create a server on the current HIP device. */
karl_status karl_create_server(const karl_server_desc* desc, void** out);

/* Queue a job (deep-copied; its workspace fields are ignored: the arena provides them).
   *ticket identifies it from now on.  KARL_EINVAL for an invalid descriptor, a precision other
   than the server's, or a job larger than the whole arena. */
karl_status karl_server_submit(void* server, const karl_job_desc* desc, int64_t* ticket);

/* Without worker threads: admit queued jobs in arrival order while they fit, then run one
   round of every worker, one after the other on `hip_stream` (returns at once if no job is
   active).  *n_active and *n_pending (either may be NULL) are the counts afterwards.
   KARL_ESTATE while worker threads run. */
karl_status karl_server_step(void* server, void* hip_stream, int32_t* n_active, int32_t* n_pending);

/* Start one thread per worker; from now on admission and rounds run in the background on
   non-blocking streams of the server's own (default priority).  Submit, poll, job, release
   and stats may be called from the host thread meanwhile. */
karl_status karl_server_start(void* server);

/* Block until a completed job is waiting to be polled, a worker failed, or timeout_ms passed.
   Returns a worker's failure status (with its message) once one occurred. */
karl_status karl_server_wait(void* server, double timeout_ms, int32_t* n_active, int32_t* n_pending);

/* Let every worker finish its current round and join the threads (jobs not yet done stay
   active and can be continued by karl_server_step or another start). */
karl_status karl_server_stop(void* server);

/* Tickets of jobs completed since the last poll, oldest first, up to `capacity`. */
karl_status karl_server_poll(void* server, int64_t* tickets, int32_t capacity, int32_t* n);

/* The job handle of a ticket (valid until the ticket is released) for karl_read_tallies,
   karl_read_fields and karl_job_stats.  KARL_ESTATE while the job is not yet admitted. */
karl_status karl_server_job(void* server, int64_t ticket, void** job);

/* Return a completed job's arena space (its handle becomes invalid).  KARL_ESTATE if the job
   has not completed. */
karl_status karl_server_release(void* server, int64_t ticket);

karl_status karl_server_stats_get(void* server, karl_server_stats* out);

/* Stop the workers if they run, then destroy the server and every job it still holds (the
   caller still owns the workspace). */
karl_status karl_destroy_server(void* server);

/* Message of the last failure on this thread ("" if none). */
const char* karl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KARL_H */

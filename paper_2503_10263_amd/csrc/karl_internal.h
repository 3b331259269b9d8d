// Internal interface between the C-ABI host code (karl_api.hip) and the device code
// (karl_kernels.hip) of libkarl.  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "karl.h"

namespace karl {

// Secondary queue in structure-of-arrays layout: one coalesced array per field.
struct QueueSoA {
    double* x;
    double* y;
    double* z;
    double* u;
    double* v;
    double* w;
    double* e;
    unsigned long long* lin;   // lineage
    uint32_t* pid;             // primary id
    uint32_t* meta;            // species (0..3) | r-cell << 2 | z-cell << 13
    uint32_t* job;             // index into the launch's job table
};

// Target codes of the device process table: the gas (rate n sigma), a density field (rate
// n_field sigma) and the gas squared (three-body: rate n (n sigma)).
enum : int32_t { TGT_GAS = 0, TGT_FIELD = 1, TGT_GAS2 = 2 };

constexpr int kS = KARL_MAX_SPECIES;

// Per-species constants of a job, indexed by species slot.  Single-job launches stage them in
// LDS (one indexed read per use, whatever the species mix of a wave); batched launches read
// them from HBM with a wave-uniform species.
struct SpeciesConst {
    int32_t nps[kS];
    int32_t field_of[kS];        // species whose density field this species' field processes see, or -1
    int32_t defer[kS];           // particles of this species make no products: queued for the drain
    int32_t tracked[kS];
    int64_t cap[kS];
    double mass[kS], charge[kS], e_cut[kS], lifetime[kS];
    double msum[kS];       // mass + m_gas
    double xs_emin[kS], inv_dlog[kS];
    double omega[kS];      // charge * bz / mass
    double mfrac[kS];      // mass / (mass + m_gas)
    double gfrac[kS];      // m_gas / (mass + m_gas), also E_xs / E
    double inv_emin[kS];   // 1 / xs_emin
    double inv_om[kS];     // 1 / omega (0 without field)
    double e_from_v2[kS];  // E(eV) = v^2 * e_from_v2
    double v2_from_e[kS];  // v^2 = E(eV) * v2_from_e
    double boris_dt[kS];   // Boris time step (s)
    double boris_h[kS];    // q dt / (2 m) of the Boris push
    double* field[kS];     // [n_r*n_z] density field of each species (m^-3), or NULL
};

// Everything the transport kernel needs about one job, passed by value.
struct DevJob {
    double radius, length;
    int32_t n_r, n_z, n_e, n_proc, n_bins, n_planes;
    int32_t gc, source, beam_species, flags;
    uint32_t seed;
    int32_t beam_ir, beam_iz, n_species;
    int32_t boris;               // Boris mover (KARL_MOVER_BORIS)
    int32_t field_nr, field_nz;  // field binning of e_fld / b_fld
    double field_radius, field_length;
    double bz;                   // uniform axial field when b_fld is NULL
    const double* e_fld;         // [field_nr][field_nz][3] (r, phi, z) components, or NULL
    const double* b_fld;
    SpeciesConst sc;
    double sigma_v;        // sqrt(k T / m_gas)
    double m_gas;
    double p2scale;        // TGT_GAS2 tables are stored divided by this (FP32 range), rate times it
    double beta_e0, beta_z, beta_fmax;
    double beam_e, beam_e1, beam_pos[3], beam_dir[3];
    int32_t pidx[kS][KARL_MAX_PROC];  // global process index of the j-th process of a species
    int32_t kind[KARL_MAX_PROC];
    int32_t target[KARL_MAX_PROC];    // TGT_*
    int32_t product[KARL_MAX_PROC];   // ionization / clustering product species
    int32_t partner[KARL_MAX_PROC];   // field targets: species of the field
    double conv[KARL_MAX_PROC];       // clustering: m_gas / m_product
    double e_th[KARL_MAX_PROC];
    float e_th_f[KARL_MAX_PROC];
    // elastic angle tables: per process edges [nb+1], theta [n], cdf [nb][n], pdf [nb][n]
    const double* ang[KARL_MAX_PROC];
    int32_t ang_nb[KARL_MAX_PROC], ang_n[KARL_MAX_PROC];
    double e_iso[KARL_MAX_PROC];
    // device tables (Real = double or float according to the precision)
    const void* xs;        // [n_proc][n_e]
    const void* n_gas;     // [n_z]
    const void* zf;        // [n_z+1] z faces
    const void* rf;        // [n_r+1] r faces
    const void* zcdf;      // [n_z+1] cumulative gas weights
    const double* edges;   // [n_species][n_bins+1]
    const int32_t* plane_of;   // [n_z+1] plane index or -1
    const double* dens_edges;  // [n_species][n_dens_bins+1] or NULL
    int32_t n_dens_bins;
    int32_t wave;          // batched launches: flights of this job's particles by the whole wave
    // tallies
    unsigned long long* counters;
    double* ledger;
    double* dens;
    unsigned long long* recomb;
    unsigned long long* jz;
    unsigned long long* jr;
    unsigned long long* spectra;
    unsigned long long* digests;
    double* hist;
    double* dense;         // [n_species][n_r][n_z][n_dens_bins+2] or NULL
    unsigned int* status;
};

// One generation of a launch over a table of jobs: primaries (mode 0; item i belongs to the job
// j with item_offs[j] <= i < item_offs[j+1] and has id pid_begin[j] + i - item_offs[j]) or
// queued particles (mode 1).  Products go to the next generation's queue, or -- for species
// that never produce secondaries -- to the deferred queue, which is processed in one launch
// once the other generations are done.
struct GenArgs {
    int32_t mode;
    int32_t n_jobs;
    int64_t n_items;
    int64_t pid_begin0;            // single-job launches: id of item 0
    // batched launches: the items of job j are job_count[j] consecutive items starting at
    // job_first[j] -- the first primary id (mode 0) or the first entry of the job-sorted queue
    // (mode 1); each wave fetches from one job at a time through job_fetch[j]
    const int64_t* job_first;
    const int64_t* job_count;
    // job_cum[j]: number of items of jobs 0..j-1 (waves start on jobs in proportion to their
    // items); job_waves[j]: waves currently fetching from job j
    const int64_t* job_cum;
    unsigned long long* job_fetch;
    unsigned long long* job_waves;
    unsigned long long* fetch;
    QueueSoA qin;
    QueueSoA qout;
    unsigned long long* qout_count;
    QueueSoA qdef;
    unsigned long long* qdef_count;
    int64_t capacity;
    unsigned int* status;          // launch status (queue overflow)
    unsigned long long* wave_segments;   // segments advanced by wave-cooperative flights (or NULL)
    // deferred launch in slices (single job): a particle whose step count reaches a multiple of
    // slice_mask + 1 goes to the ring when its slot is free; claim indices past n_items are ring
    // entries.  ring_flag[k] of the entry with index i in slot k = i mod ring_cap: 2i+1 written,
    // 2i+2 read (0: never used in this launch).  slice_mask 0: no slices.
    uint32_t slice_mask;
    int64_t ring_cap;
    struct RingEntry* ring;
    unsigned long long* ring_flag;
    unsigned long long* ring_tail;  // ring indices reserved so far
};

// The whole state of a particle between two slices of the deferred launch.
struct RingEntry {
    double x, y, z, u, v, w, e, vel, s_path, t_alive, t_cell, e_exc, e_bind, e_gas;
    unsigned long long lin, dg;
    uint32_t pid, s;
    int32_t sp, ir, iz, fly;
    int64_t n_int;
};
static_assert(sizeof(RingEntry) == 160, "ring entries are 160 bytes");

enum : unsigned int { STATUS_OVERFLOW = 1u, STATUS_NUMERIC = 2u };

size_t lds_bytes(const DevJob& j, int precision);
hipError_t launch_transport(const DevJob* jobs_dev, bool batched, bool coop, bool drain, bool dense,
                            bool boris, const GenArgs& g, int precision, int grid, int block, size_t lds,
                            hipStream_t s);
hipError_t launch_target_fields(const DevJob& j, double t_sim, hipStream_t s);
// the deferred-launch kernels (their own compilation unit): launch and blocks per CU
hipError_t launch_transport_drain(const DevJob* jobs_dev, bool dense, const GenArgs& g, int precision,
                                  int grid, int block, size_t lds, hipStream_t s);
hipError_t transport_occupancy_drain(int precision, int block, size_t lds, int* blocks_per_cu);
// the batched kernels (their own compilation unit): launch and blocks per CU
hipError_t launch_transport_batched(const DevJob* jobs_dev, bool boris, bool coop, const GenArgs& g, int precision,
                                    int grid, int block, size_t lds, hipStream_t s);
hipError_t transport_occupancy_batched(int precision, bool boris, bool coop, int block, size_t lds, int* blocks_per_cu);
hipError_t launch_fields(const DevJob& j, double t_sim, double* density, double* jz, double* jr,
                         hipStream_t s);
// Regroup n queue entries by job: count per job, exclusive scan into first/count, scatter.
hipError_t launch_sort_by_job(const QueueSoA& in, const QueueSoA& out, int64_t n, int32_t n_jobs,
                              unsigned long long* counts, int64_t* first, int64_t* count,
                              unsigned long long* cursor, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, size_t n, unsigned long long value,
                           hipStream_t s);
hipError_t transport_occupancy(int precision, bool batched, bool coop, bool drain, bool boris, int block,
                               size_t lds, int* blocks_per_cu);
size_t batched_lds_bytes();

}  // namespace karl

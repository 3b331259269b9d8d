/*
 * karl_oracle.h -- plain, slow, sequential FP64 CPU oracle of the particle-history
 * transport of the KARL Monte Carlo method (arXiv 2503.10263).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or call
 * this code: only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code, header, table or constant with the HIP
 * library; it is written from the paper, and where the paper leaves a choice open
 * (the draw schedule of the random numbers, geometry conventions, kinematic details)
 * each function states the reading it takes.
 *
 * All arrays are host memory owned by the caller.  Functions return 0 on success
 * and a negative value on invalid input; they never abort.
 */
#ifndef KARL_ORACLE_H
#define KARL_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KO_MAX_PROC 16
#define KO_MAX_SPECIES 4

/* interaction classes of Sec. 3.3: elastic scattering, excitation, ionization (with or without
   dissociation of the target: the ion species made is the process's `product`), recombination,
   charge exchange (the projectile takes the velocity of a target particle) and clustering (the
   projectile becomes the `product` species) */
enum { KO_ELASTIC = 0, KO_EXCITATION = 1, KO_IONIZATION = 2, KO_RECOMBINATION = 3,
       KO_CHARGE_EXCHANGE = 4, KO_CLUSTERING = 5 };
/* KO_TARGET_FIELD: the density field of the process's `partner` species, Sec. 2.2 "Density
   fields" */
enum { KO_TARGET_GAS = 0, KO_TARGET_FIELD = 1 };
/* KO_SOURCE_PAIR: both species from the beam position and direction, even primary ids electrons
   at beam_energy, odd ids ions at beam_energy_1 */
enum { KO_SOURCE_BETA = 0, KO_SOURCE_BEAM = 1, KO_SOURCE_PAIR = 2 };
/* movers (Sec. 3.1): drift (exact helix in a uniform axial field, straight lines without one)
   or Boris pushes with electric and magnetic fields from arrays */
enum { KO_MOVER_DRIFT = 0, KO_MOVER_BORIS = 1 };
/* KO_CONVERTED: the projectile of a clustering reaction, replaced by its product */
enum { KO_EXIT_LOW = 0, KO_EXIT_HIGH, KO_WALL, KO_CUTOFF, KO_RECOMBINED, KO_CAP,
       KO_LIFETIME, KO_UNTRACKED, KO_CONVERTED, KO_NREASON };

/* counters (int64) */
#define KO_C_BIRTH         0   /* [4] particles born per species                  */
#define KO_C_STEP          4   /* [4] flight segments per species                 */
#define KO_C_COLL          8   /* [4] collisions per species                      */
#define KO_C_ZCROSS        12  /* [4] z-face crossings per species                */
#define KO_C_RCROSS        16  /* [4] r-face crossings per species (incl. wall)   */
#define KO_C_TARGET_REDRAW 20  /* ionization target-velocity redraws              */
#define KO_C_BEB_TRIES     21  /* secondary-energy proposals                      */
#define KO_C_BETA_TRIES    22  /* beta-energy proposals                           */
#define KO_C_PROC          24  /* [16] collisions per process                     */
#define KO_C_DEATH         40  /* [4][9] deletions per species and reason         */
#define KO_NCOUNTERS       80

/* energy / time ledger (double) */
#define KO_L_E_PRIMARY     0   /* birth energy of primaries (eV)                  */
#define KO_L_E_DEATH       1   /* [4][9] energy at deletion per species/reason    */
#define KO_L_E_EXC         37  /* excitation losses                               */
#define KO_L_E_BIND        38  /* ionization binding energies                     */
#define KO_L_E_GAS         39  /* energy exchanged with the gas: elastic recoil, the ionization
                                  frame, charge exchange, and minus the energy of clustering and
                                  ionization products, whose velocity is a target particle's */
#define KO_L_T_ALIVE       40  /* [4] summed particle lifetimes (s)               */
#define KO_L_E_FIELD       44  /* work of the electric field (Boris mover)        */
#define KO_NLEDGER         48

#define KO_NHIST           4   /* per history: E_in, E_accounted, n_born, n_dead  */

typedef struct {
    double mass;          /* kg */
    double charge;        /* C, signed */
    double e_cut;         /* eV: E < e_cut terminates */
    double lifetime;      /* s */
    int64_t cap;          /* maximum interactions */
    int32_t tracked;      /* 0: counted at birth, never transported */
    int32_t pad;
    double xs_emin;       /* eV: first table node */
    double xs_emax;       /* eV: last table node */
    const double* edges;  /* [n_bins+1] spectrum bin edges (eV), increasing */
    const double* dens_edges;  /* [n_dens_bins+1] energy bins of the density field (eV) or NULL */
} ko_species;

typedef struct {
    int32_t kind;         /* KO_ELASTIC ... KO_CLUSTERING */
    int32_t species;      /* projectile slot 0..n_species-1 (slot 0: electrons) */
    int32_t target;       /* KO_TARGET_GAS or KO_TARGET_FIELD */
    int32_t product;      /* ionization: the ion species made (1..n_species-1); clustering: the
                             species the projectile becomes; ignored otherwise */
    int32_t partner;      /* KO_TARGET_FIELD: the species whose density field is the target;
                             recombination: the species whose field logs the deletion */
    int32_t density_power;/* gas targets: the collision rate goes as n_gas^density_power (1, or 2
                             for three-body clustering, whose "cross section" is k/v in m^5);
                             0 means 1 */
    double e_th;          /* excitation energy or binding energy (eV); 0 otherwise */
    const double* xs;     /* [n_e] cross section (m^2) at the species' nodes */
    /* elastic scattering angle (Sec. 3.3 "Elastic scattering"): isotropic in the centre-of-mass
       frame when ang_bins == 0 or the impact energy in that frame is below e_iso; otherwise a
       piecewise linear density over the polar angle, one per impact-energy bin */
    int32_t ang_bins;     /* energy bins of the table (0: isotropic) */
    int32_t ang_nodes;    /* angle nodes per bin (>= 2) */
    double e_iso;         /* eV: isotropic below this centre-of-mass energy */
    const double* ang_edges;  /* [ang_bins+1] bin edges in centre-of-mass energy (eV) */
    const double* ang_theta;  /* [ang_nodes] increasing polar angles (rad) within [0, pi] */
    const double* ang_pdf;    /* [ang_bins][ang_nodes] density values >= 0 at the nodes */
} ko_process;

typedef struct {
    double radius, length;       /* m */
    int32_t n_r, n_z;            /* grid (>= 1 each) */
    const double* n_gas;         /* [n_z] gas density per z-cell (m^-3) */
    /* [n_r*n_z] density field of each species (m^-3), the target of processes with that
       partner; NULL = 0 */
    const double* n_field[KO_MAX_SPECIES];
    double t_gas;                /* K */
    double m_gas;                /* kg */
    double bz;                   /* T; 0: straight lines */
    ko_species sp[KO_MAX_SPECIES];
    int32_t n_species;           /* 2..4; 0 means 2 */
    int32_t n_proc, n_e;
    ko_process proc[KO_MAX_PROC];
    int32_t source, beam_species;
    double beta_e0, beta_z, beta_fmax;
    double beam_energy, beam_pos[3], beam_dir[3];
    double beam_energy_1;        /* ion energy of KO_SOURCE_PAIR (eV) */
    uint32_t seed;
    int32_t n_bins;
    int32_t n_planes, pad2;
    const int32_t* planes;       /* [n_planes] z-face indices */
    int64_t n_primaries;
    int32_t n_dens_bins;         /* energy bins of the density field (Sec. 3.4); 0: none */
    int32_t mover;               /* KO_MOVER_DRIFT or KO_MOVER_BORIS */
    /* Boris mover: time step per species (s), and the fields as arrays over a cylindrical
       binning of field_radius x field_length in field_nr x field_nz bins, each bin a vector of
       (r, phi, z) components; zero outside the binning (VectorFieldFromArray, Sec. 3.8).
       e_field NULL: no electric field; b_field NULL: the uniform axial field bz */
    double boris_dt[KO_MAX_SPECIES];
    int32_t field_nr, field_nz;
    double field_radius, field_length;
    const double* e_field;       /* [field_nr][field_nz][3] V/m */
    const double* b_field;       /* [field_nr][field_nz][3] T */
} ko_desc;

typedef struct {
    int64_t* counters;     /* [KO_NCOUNTERS] */
    double* ledger;        /* [KO_NLEDGER] */
    /* leading index: species 0..n_species-1 */
    double* density_time;  /* [S][n_r][n_z] seconds */
    int64_t* recomb;       /* [S][n_r][n_z] recombinations logged in the field of each species */
    int64_t* jz;           /* [S][n_r][n_z+1][2] */
    int64_t* jr;           /* [S][n_r+1][n_z][2] */
    int64_t* spectra;      /* [S][n_planes][2][n_bins+2] */
    uint64_t* digests;     /* [n_primaries] or NULL */
    double* hist;          /* [n_primaries][KO_NHIST] or NULL */
    /* [S][n_r][n_z][n_dens_bins+2] time per segment and energy bin (bin 0 below the first
       edge, n_dens_bins+1 at or above the last), or NULL */
    double* density_time_e;
} ko_tallies;

/* Transport primaries pid_begin..pid_end-1 and add their contributions to t. */
int ko_run(const ko_desc* d, int64_t pid_begin, int64_t pid_end, ko_tallies* t);

/* Densities per species and segment, eq. (3) with t_sim = n_prim/activity, eq. (4), minus the
   recombinations logged in that species' field per volume; currents (N+ - N-)/(A t_sim) through the
   z-faces of each ring ([S][n_r][n_z+1]) and the r-faces of each z-segment ([S][n_r+1][n_z]). */
int ko_fields(const ko_desc* d, const ko_tallies* t, double n_prim, double activity,
              double* density, double* jz_cur, double* jr_cur);

/* ---- single-step entry points used by the oracle's own pin tests ---- */
void ko_philox(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
               uint32_t out[4]);
double ko_u53(uint32_t a, uint32_t b);
/* QE (J/eV), k_B, m_e c^2 (eV), alpha, pi, 2 pi as used by the oracle */
void ko_constants(double out[6]);
uint64_t ko_mix64(uint64_t z);
/* natural logarithm and sine/cosine from IEEE basic operations (see karl_oracle.c) */
double ko_log(double x);
void ko_sincos(double x, double* s, double* c);
double ko_beta_shape(double e, double e0, double z);
/* polar scattering angle (rad) of elastic process `proc` at centre-of-mass energy e_cm for the
   uniform number u in [0,1) (the table path; isotropic processes return acos(2u-1)) */
double ko_debug_angle(const ko_desc* d, int proc, double e_cm, double u);
/* birth state of primary pid: x,y,z,u,v,w,E,tries */
int ko_birth(const ko_desc* d, int64_t pid, double out[8]);
/* kinematics of process `proc` for one particle at the origin:
   out[0]=E', out[1..3]=dir', out[4]=alive, out[5]=n_products,
   out[6]=E_slow, out[7..9]=dir_slow, out[10]=E_ion, out[11..13]=dir_ion (ionization; the
   clustering product is reported as the ion), out[14]=energy to gas, out[15]=w (ionization) */
int ko_debug_collide(const ko_desc* d, int proc, int64_t pid, uint64_t lineage, uint32_t s,
                     double e, const double dir[3], double out[16]);
/* n Boris pushes of a particle of species sp from position x[3] with velocity v[3] (m/s),
   without segments or interactions: out[0..2] position, out[3..5] velocity */
int ko_debug_boris(const ko_desc* d, int sp, const double x[3], const double v[3], int n,
                   double out[6]);
/* helix: position and direction after path length `path` (guiding-centre formulas) */
void ko_debug_helix(double charge, double mass, double bz, const double pos[3],
                    const double dir[3], double speed, double path, double out[6]);

#ifdef __cplusplus
}
#endif
#endif

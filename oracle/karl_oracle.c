/*
 * karl_oracle.c -- plain sequential FP64 oracle of the KARL particle-history transport.
 *
 * TEST INFRASTRUCTURE ONLY (see karl_oracle.h).  Built with -O2 -ffp-contract=off so
 * that every operation rounds once, in source order.
 *
 * What it follows, by section of the paper:
 *   - main cycle: a primary is injected, the particle list is processed until empty,
 *     each particle is moved and interacted with until it terminates (Sec. 2.1
 *     "General diagram").  Here the list is a LIFO stack; identity-keyed random
 *     streams make the processing order irrelevant.
 *   - mean free path, eq. (1), and free path d = -lambda ln(eta), eq. (2), eta in (0,1].
 *   - interaction choice weighted by sigma_i n_i, products (not the incident particle)
 *     added to the list (Sec. 2.1).
 *   - movement stops at segment faces without interaction and a new distance is drawn
 *     (Sec. 3.1 "Movement"); the time spent in a segment is added to the density
 *     field when the particle leaves it (Sec. 3.1, eq. (3) numerator).
 *   - drift mover for a uniform axial field without electric field: exact helix about
 *     the guiding centre (Sec. 3.1 "Drift mover" and "Comparison").
 *   - Boris mover (Sec. 3.1 "Boris mover"): pushes of a fixed time step per species with the
 *     electric and magnetic fields of the particle's cylindrical field bin; the movement ends
 *     when the particle leaves the domain, its segment or its energy bin (no interaction, a
 *     new distance is drawn) or when the moved distance exceeds the drawn one (interaction
 *     at the current position); the time counter of the movement goes to its segment.
 *   - terminator: geometry, interaction cap, lifetime; deletion logger (Sec. 3.2).
 *   - interactions (Sec. 3.3): elastic scattering with a thermal target and a CM-frame
 *     rotation; excitation E' = E - E_x without deflection; ionization with target
 *     redraw, secondary energy from the Kim-Rudd BEB distribution, E_e = E_i - E_ion -
 *     E_i^new, phi_e = phi_i - pi, ion (of the process's product species: the molecular
 *     ion, or the atomic ion of dissociative ionization) given the target velocity;
 *     recombination logs one deletion in the partner's field and removes the particle;
 *     charge exchange gives the projectile the velocity of a target particle; clustering
 *     replaces the projectile by a particle of the product species that moves along the
 *     target particle's velocity with that particle's momentum.  Three-body clustering
 *     goes with the square of the gas density.
 *   - current collection N+ / N- through faces (Sec. 2.3), spectra at planes.
 *   - injector with the allowed beta spectrum drawn by rejection (Sec. 3.5; Sec. 3.8 "Velocity distribution").
 */
#include "karl_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* constants (CODATA 2018; QE and KB exact) */
#define QE      1.602176634e-19
#define KB      1.380649e-23
#define MEC2    510998.95
#define ALPHA   7.2973525693e-3
#define PI      3.14159265358979323846
#define TWO_PI  6.28318530717958647692
#define TWO_M53 1.1102230246251565404e-16   /* 2^-53 */
#define PHI64   0x9E3779B97F4A7C15ULL
#define DIGEST0 0x5851F42D4C957F2DULL
#define BIRTH_STEP 0xFFFFFFFFu

/* ------------------------------------------------------------------ */
/* random numbers: Philox4x32-10 (Salmon et al., SC'11)               */
/* ------------------------------------------------------------------ */
void ko_philox(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
               uint32_t out[4]) {
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53-bit uniform in [0,1) from two words: 27 high bits of a, 26 high bits of b */
double ko_u53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * TWO_M53;
}

void ko_constants(double out[6]) {
    out[0] = QE; out[1] = KB; out[2] = MEC2; out[3] = ALPHA; out[4] = PI; out[5] = TWO_PI;
}

/* SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA 2014) */
uint64_t ko_mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return z;
}


/* ------------------------------------------------------------------ */
/* elementary functions written out with IEEE basic operations only     */
/* (fused multiply-add, rounded once, among them: every series step is   */
/* one fma), so that an independent implementation of the same steps     */
/* reproduces them bit for bit (the guiding-centre phase amplifies any   */
/* 1-ulp difference)                                                     */
/* ------------------------------------------------------------------ */
#define SQRT_HALF 0.70710678118654757
#define LN2_HI 0.6931471805601177        /* ln 2 rounded to 40 bits: e*LN2_HI is exact */
#define LN2_LO (-1.7239444525614835e-13) /* ln 2 - LN2_HI */
#define PIO4 0.78539816339744828
#define TWO_OVER_PI 0.6366197723675814
#define PIO2_1 1.5707963407039642        /* pi/2 in four 26-bit pieces */
#define PIO2_2 (-1.3909067675399456e-08)
#define PIO2_3 6.123233932053594e-17
#define PIO2_4 6.368317178484799e-25

/* ln x: x = m 2^e with m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s), s = (m-1)/(m+1),
   atanh(s)/s = sum z^n/(2n+1), z = s^2 <= 0.0295, summed to n = 12 (truncation < 2^-62) */
double ko_log(double x) {
    if (!(x > 0.0)) return (x == 0.0) ? -INFINITY : NAN;
    if (isinf(x)) return x;
    int e;
    double m = frexp(x, &e);
    if (m < SQRT_HALF) {
        m = m * 2.0;
        e = e - 1;
    }
    double f = m - 1.0;
    double s = f / (m + 1.0);
    double z = s * s;
    double p = 0.04;                             /* 1/25 */
    p = fma(z, p, 0.043478260869565216);         /* 1/23 */
    p = fma(z, p, 0.047619047619047616);         /* 1/21 */
    p = fma(z, p, 0.05263157894736842);          /* 1/19 */
    p = fma(z, p, 0.058823529411764705);         /* 1/17 */
    p = fma(z, p, 0.06666666666666667);          /* 1/15 */
    p = fma(z, p, 0.07692307692307693);          /* 1/13 */
    p = fma(z, p, 0.09090909090909091);          /* 1/11 */
    p = fma(z, p, 0.1111111111111111);           /* 1/9  */
    p = fma(z, p, 0.14285714285714285);          /* 1/7  */
    p = fma(z, p, 0.2);                          /* 1/5  */
    p = fma(z, p, 0.3333333333333333);           /* 1/3  */
    double t = 2.0 * s;
    double lm = fma(t, z * p, t);
    double de = (double)e;
    return fma(de, LN2_HI, fma(de, LN2_LO, lm));
}

/* sin and cos: r = x - k pi/2 (Cody-Waite with four 26-bit pieces of pi/2, exact products
   for |k| < 2^27), Taylor series on |r| <= pi/4 to r^19 and r^20, quadrant from k mod 4 */
void ko_sincos(double x, double* sn, double* cs) {
    if (!isfinite(x)) {
        *sn = NAN;
        *cs = NAN;
        return;
    }
    double r = x;
    long long q = 0;
    if (fabs(x) > PIO4) {
        double xx = x;
        if (fabs(xx) >= 2.0e8) xx = xx - trunc(xx / TWO_PI) * TWO_PI;
        double k = floor(fma(xx, TWO_OVER_PI, 0.5));
        r = fma(-k, PIO2_1, xx);
        r = fma(-k, PIO2_2, r);
        r = fma(-k, PIO2_3, r);
        r = fma(-k, PIO2_4, r);
        q = (long long)k;
    }
    double z = r * r;
    double ps = -8.22063524662433e-18;           /* -1/19! */
    ps = fma(z, ps, 2.8114572543455206e-15);     /*  1/17! */
    ps = fma(z, ps, -7.647163731819816e-13);     /* -1/15! */
    ps = fma(z, ps, 1.6059043836821613e-10);     /*  1/13! */
    ps = fma(z, ps, -2.505210838544172e-08);     /* -1/11! */
    ps = fma(z, ps, 2.7557319223985893e-06);     /*  1/9!  */
    ps = fma(z, ps, -0.0001984126984126984);     /* -1/7!  */
    ps = fma(z, ps, 0.008333333333333333);       /*  1/5!  */
    ps = fma(z, ps, -0.16666666666666666);       /* -1/3!  */
    double sv = fma(r, z * ps, r);
    double pc = 4.110317623312165e-19;           /*  1/20! */
    pc = fma(z, pc, -1.5619206968586225e-16);    /* -1/18! */
    pc = fma(z, pc, 4.779477332387385e-14);      /*  1/16! */
    pc = fma(z, pc, -1.1470745597729725e-11);    /* -1/14! */
    pc = fma(z, pc, 2.08767569878681e-09);       /*  1/12! */
    pc = fma(z, pc, -2.755731922398589e-07);     /* -1/10! */
    pc = fma(z, pc, 2.48015873015873e-05);       /*  1/8!  */
    pc = fma(z, pc, -0.001388888888888889);      /* -1/6!  */
    pc = fma(z, pc, 0.041666666666666664);       /*  1/4!  */
    double cv = fma(z * z, pc, fma(-0.5, z, 1.0));
    switch (q & 3) {
        case 0: *sn = sv; *cs = cv; break;
        case 1: *sn = cv; *cs = -sv; break;
        case 2: *sn = -sv; *cs = -cv; break;
        default: *sn = -cv; *cs = sv; break;
    }
}


typedef struct { double d0, d1; } pair_t;

/* one slot of the draw schedule: key (seed, pid), counter (step, slot, lineage) */
static pair_t draw(uint32_t seed, uint32_t pid, uint64_t lineage, uint32_t s, uint32_t slot) {
    uint32_t w[4];
    ko_philox(seed, pid, s, slot, (uint32_t)lineage, (uint32_t)(lineage >> 32), w);
    pair_t p;
    p.d0 = ko_u53(w[0], w[1]);
    p.d1 = ko_u53(w[2], w[3]);
    return p;
}

static uint64_t child_lineage(uint64_t parent, uint32_t s, uint32_t j) {
    return ko_mix64(parent ^ (PHI64 * ((((uint64_t)s) << 3) | (uint64_t)(j + 1))));
}

static uint64_t digest_event(uint64_t d, uint32_t s, uint32_t kind, uint32_t a, uint32_t b) {
    uint64_t w = ((uint64_t)s << 32) | ((uint64_t)(kind & 0xFu) << 28) |
                 ((uint64_t)(a & 0xFFu) << 20) | (uint64_t)(b & 0xFFFFFu);
    return ko_mix64(d ^ w);
}

/* ------------------------------------------------------------------ */
/* allowed beta spectrum (Sec. 3.8, TritiumBetaDecay)               */
/* ------------------------------------------------------------------ */
double ko_beta_shape(double e, double e0, double z) {
    if (!(e > 0.0) || !(e < e0)) return 0.0;
    double wt = e + MEC2;                      /* total energy */
    double p = sqrt(e * (e + 2.0 * MEC2));     /* momentum (eV/c) */
    double y = TWO_PI * ALPHA * z * wt / p;    /* 2 pi times the Sommerfeld parameter */
    double q = e0 - e;
    return (TWO_PI * ALPHA * z * wt / (1.0 - exp(-y))) * wt * q * q;
}

/* ------------------------------------------------------------------ */
/* compensated (Neumaier) accumulation                                 */
/* ------------------------------------------------------------------ */
static void nadd(double* s, double* c, double x) {
    double t = *s + x;
    if (fabs(*s) >= fabs(x)) *c += (*s - t) + x;
    else *c += (x - t) + *s;
    *s = t;
}

/* ------------------------------------------------------------------ */
/* job context                                                         */
/* ------------------------------------------------------------------ */
typedef struct {
    double x, y, z, u, v, w, e;
    uint64_t lineage;
    int32_t sp, ir, iz;
} seed_t;

typedef struct {
    const ko_desc* d;
    ko_tallies* t;
    double* zf;          /* [n_z+1] z faces */
    double* rf;          /* [n_r+1] r faces */
    double* zcdf;        /* [n_z+1] cumulative gas weights */
    int32_t* plane_of;   /* [n_z+1] plane index or -1 */
    int n_species;
    double inv_dlog[KO_MAX_SPECIES];
    double omega[KO_MAX_SPECIES];     /* q B / m */
    /* per-species constants of the kinematics, evaluated once */
    double mfrac[KO_MAX_SPECIES];     /* m / (m + M) */
    double gfrac[KO_MAX_SPECIES];     /* M / (m + M): also E_xs / E (centre-of-mass energy factor) */
    double inv_emin[KO_MAX_SPECIES];  /* 1 / first table energy */
    double inv_om[KO_MAX_SPECIES];    /* 1 / omega (0 without field) */
    double e_from_v2[KO_MAX_SPECIES]; /* E(eV) = v^2 * e_from_v2 = v^2 m / (2 e) */
    double v2_from_e[KO_MAX_SPECIES]; /* v^2 = E(eV) * v2_from_e = E 2 e / m */
    double sigma_v;      /* thermal target speed scale sqrt(kT/M) */
    double conv[KO_MAX_PROC];         /* clustering: M / m_product (momentum of the target) */
    int boris;                        /* Boris mover */
    double boris_h[KO_MAX_SPECIES];   /* q dt / (2 m) of the Boris push */
    int32_t nps[KO_MAX_SPECIES];
    int32_t pidx[KO_MAX_SPECIES][KO_MAX_PROC];
    /* compensated accumulators */
    double* dens_s; double* dens_c;
    double* dense_s; double* dense_c;   /* energy-resolved times (or NULL) */
    double led_s[KO_NLEDGER], led_c[KO_NLEDGER];
    /* particle stack */
    seed_t* stack; int64_t n_stack, cap_stack;
    int gc;              /* guiding-centre mode (bz != 0) */
} ctx_t;

typedef struct {
    int32_t sp, ir, iz, alive;
    uint32_t pid, s;
    uint64_t lineage, dg;
    double x, y, z, u, v, w, e, vel;
    double s_path, t_alive, t_cell;
    double e_exc, e_bind, e_gas;  /* per-particle losses, added to the ledgers at deletion */
    int64_t n_int;
    double e_rates;          /* energy at which sig[] was evaluated */
    double sig[KO_MAX_PROC]; /* per-species process cross sections */
} part_t;

static void push(ctx_t* c, const seed_t* s) {
    if (c->n_stack == c->cap_stack) {
        c->cap_stack = c->cap_stack ? 2 * c->cap_stack : 256;
        c->stack = (seed_t*)realloc(c->stack, (size_t)c->cap_stack * sizeof(seed_t));
    }
    c->stack[c->n_stack++] = *s;
}

static int ctx_init(ctx_t* c, const ko_desc* d, ko_tallies* t) {
    memset(c, 0, sizeof(*c));
    c->d = d;
    c->t = t;
    if (d->n_r < 1 || d->n_z < 1 || d->n_e < 2 || d->n_proc < 0 || d->n_proc > KO_MAX_PROC)
        return -1;
    if (!(d->radius > 0.0) || !(d->length > 0.0) || d->n_bins < 1) return -1;
    c->n_species = d->n_species ? d->n_species : 2;
    if (c->n_species < 2 || c->n_species > KO_MAX_SPECIES) return -1;
    c->zf = (double*)malloc(sizeof(double) * (size_t)(d->n_z + 1));
    c->rf = (double*)malloc(sizeof(double) * (size_t)(d->n_r + 1));
    c->zcdf = (double*)malloc(sizeof(double) * (size_t)(d->n_z + 1));
    c->plane_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)(d->n_z + 1));
    size_t nd = (size_t)c->n_species * d->n_r * d->n_z;
    c->dens_s = (double*)calloc(nd, sizeof(double));
    c->dens_c = (double*)calloc(nd, sizeof(double));
    if (t && t->density_time_e && d->n_dens_bins > 0) {
        size_t ne = nd * (size_t)(d->n_dens_bins + 2);
        c->dense_s = (double*)calloc(ne, sizeof(double));
        c->dense_c = (double*)calloc(ne, sizeof(double));
    }
    for (int k = 0; k <= d->n_z; ++k) c->zf[k] = d->length * (double)k / (double)d->n_z;
    for (int k = 0; k <= d->n_r; ++k) c->rf[k] = d->radius * (double)k / (double)d->n_r;
    c->zcdf[0] = 0.0;
    for (int k = 0; k < d->n_z; ++k) c->zcdf[k + 1] = c->zcdf[k] + d->n_gas[k];
    for (int k = 0; k <= d->n_z; ++k) c->plane_of[k] = -1;
    for (int p = 0; p < d->n_planes; ++p) {
        int f = d->planes[p];
        if (f < 0 || f > d->n_z) return -1;
        if (c->plane_of[f] < 0) c->plane_of[f] = p;
    }
    for (int s = 0; s < c->n_species; ++s) {
        c->inv_dlog[s] = (double)(d->n_e - 1) / log(d->sp[s].xs_emax / d->sp[s].xs_emin);
        c->omega[s] = d->sp[s].charge * d->bz / d->sp[s].mass;
        double mt = d->sp[s].mass + d->m_gas;
        c->mfrac[s] = d->sp[s].mass / mt;
        c->gfrac[s] = d->m_gas / mt;
        c->inv_emin[s] = 1.0 / d->sp[s].xs_emin;
        c->inv_om[s] = (c->omega[s] != 0.0) ? 1.0 / c->omega[s] : 0.0;
        c->e_from_v2[s] = 0.5 * d->sp[s].mass / QE;
        c->v2_from_e[s] = 2.0 * QE / d->sp[s].mass;
    }
    c->sigma_v = sqrt(KB * d->t_gas / d->m_gas);
    for (int i = 0; i < d->n_proc; ++i) {
        const ko_process* pr = &d->proc[i];
        int s = pr->species;
        if (s < 0 || s >= c->n_species) return -1;
        if (pr->kind < KO_ELASTIC || pr->kind > KO_CLUSTERING) return -1;
        if (pr->kind == KO_IONIZATION && (pr->product < 1 || pr->product >= c->n_species)) return -1;
        if (pr->kind == KO_CLUSTERING &&
            (pr->product < 0 || pr->product >= c->n_species || pr->product == s)) return -1;
        if ((pr->target == KO_TARGET_FIELD || pr->kind == KO_RECOMBINATION) &&
            (pr->partner < 0 || pr->partner >= c->n_species))
            return -1;
        if (pr->target != KO_TARGET_GAS && pr->target != KO_TARGET_FIELD) return -1;
        if (pr->density_power < 0 || pr->density_power > 2) return -1;
        if (pr->density_power == 2 && pr->target != KO_TARGET_GAS) return -1;
        if (pr->kind == KO_CLUSTERING) c->conv[i] = d->m_gas / d->sp[pr->product].mass;
        c->pidx[s][c->nps[s]++] = i;
    }
    if (d->source == KO_SOURCE_BEAM && (d->beam_species < 0 || d->beam_species >= c->n_species))
        return -1;
    c->boris = (d->mover == KO_MOVER_BORIS);
    if (d->mover != KO_MOVER_DRIFT && d->mover != KO_MOVER_BORIS) return -1;
    if (!c->boris && (d->e_field || d->b_field)) return -1;   /* the drift mover: uniform B only */
    if ((d->e_field || d->b_field) &&
        (d->field_nr < 1 || d->field_nz < 1 || !(d->field_radius > 0.0) || !(d->field_length > 0.0)))
        return -1;
    if (c->boris)
        for (int s = 0; s < c->n_species; ++s) {
            const double dt = d->boris_dt[s];
            if (!(dt > 0.0) || !(d->sp[s].lifetime < INFINITY) || !(d->sp[s].lifetime / dt <= 2147483648.0))
                return -1;
            c->boris_h[s] = 0.5 * dt * d->sp[s].charge / d->sp[s].mass;
        }
    c->gc = (d->bz != 0.0) && !c->boris;
    return 0;
}

static void ctx_free(ctx_t* c) {
    free(c->zf); free(c->rf); free(c->zcdf); free(c->plane_of);
    free(c->dens_s); free(c->dens_c); free(c->stack);
    free(c->dense_s); free(c->dense_c);
}

static void ledger_add(ctx_t* c, int i, double x) { nadd(&c->led_s[i], &c->led_c[i], x); }

static int count_faces_le(const double* faces, int n, double r) {
    /* number of faces k = 1..n-1 with faces[k] <= r */
    int k = 0;
    for (int j = 1; j < n; ++j)
        if (faces[j] <= r) k = j;
    return k;
}

static int find_bin(const double* edges, int n_bins, double e) {
    if (e < edges[0]) return 0;
    if (!(e < edges[n_bins])) return n_bins + 1;
    int lo = 0, hi = n_bins;   /* edges[lo] <= e < edges[hi] */
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (edges[mid] <= e) lo = mid;
        else hi = mid;
    }
    return lo + 1;
}

/* ------------------------------------------------------------------ */
/* cross sections: linear in sigma over ln E, zero below threshold     */
/* ------------------------------------------------------------------ */
static double xs_lookup(const ctx_t* c, int i, double exs) {
    const ko_desc* d = c->d;
    const ko_process* pr = &d->proc[i];
    if (exs < pr->e_th) return 0.0;
    int s = pr->species;
    double x = ko_log(exs * c->inv_emin[s]) * c->inv_dlog[s];
    int k;
    double f;
    if (!(x > 0.0)) {
        k = 0;
        f = 0.0;
    } else if (x >= (double)(d->n_e - 1)) {
        k = d->n_e - 2;
        f = 1.0;
    } else {
        k = (int)x;
        f = x - (double)k;
    }
    const double* tb = pr->xs;
    return tb[k] + f * (tb[k + 1] - tb[k]);
}

static void eval_sigmas(const ctx_t* c, part_t* p) {
    double exs = p->e * c->gfrac[p->sp];
    for (int j = 0; j < c->nps[p->sp]; ++j) p->sig[j] = xs_lookup(c, c->pidx[p->sp][j], exs);
    p->e_rates = p->e;
}

/* ------------------------------------------------------------------ */
/* tallies                                                              */
/* ------------------------------------------------------------------ */
static void flush_time(ctx_t* c, part_t* p) {
    if (p->t_cell != 0.0) {
        size_t k = ((size_t)p->sp * c->d->n_r + (size_t)p->ir) * c->d->n_z + (size_t)p->iz;
        nadd(&c->dens_s[k], &c->dens_c[k], p->t_cell);
        p->t_cell = 0.0;
    }
}

static void ev(part_t* p, uint32_t kind, uint32_t a, uint32_t b) {
    p->dg = digest_event(p->dg, p->s, kind, a, b);
}

static void hist_add(ctx_t* c, const part_t* p, int slot, double x) {
    if (c->t->hist) c->t->hist[(size_t)p->pid * KO_NHIST + (size_t)slot] += x;
}

static void kill(ctx_t* c, part_t* p, int reason) {
    flush_time(c, p);
    c->t->counters[KO_C_DEATH + p->sp * KO_NREASON + reason] += 1;
    ledger_add(c, KO_L_E_DEATH + p->sp * KO_NREASON + reason, p->e);
    ledger_add(c, KO_L_T_ALIVE + p->sp, p->t_alive);
    ledger_add(c, KO_L_E_EXC, p->e_exc);
    ledger_add(c, KO_L_E_BIND, p->e_bind);
    ledger_add(c, KO_L_E_GAS, p->e_gas);
    ev(p, 6, (uint32_t)reason, 0);
    if (c->t->digests) c->t->digests[p->pid] += p->dg;
    hist_add(c, p, 1, ((p->e + p->e_exc) + p->e_bind) + p->e_gas);
    hist_add(c, p, 3, 1.0);
    p->alive = 0;
}

/* r-face crossing (dir 1 outward); the wall is face n_r */
static void cross_r(ctx_t* c, part_t* p, int f, int dir) {
    const ko_desc* d = c->d;
    c->t->counters[KO_C_RCROSS + p->sp] += 1;
    c->t->jr[(((size_t)p->sp * (d->n_r + 1) + (size_t)f) * d->n_z + (size_t)p->iz) * 2 + (size_t)dir] += 1;
    ev(p, 4, (uint32_t)dir, (uint32_t)(f * d->n_z + p->iz));
}

/* guiding centre from position and velocity; returns 1 if the orbit touches the wall.
   At birth the r-cell is set from the guiding-centre radius; after a collision every
   r-face between the old and the new guiding-centre radius is counted as crossed. */
static int gc_set(ctx_t* c, part_t* p, double xp, double yp, int at_birth) {
    const ko_desc* d = c->d;
    double iom = c->inv_om[p->sp];
    double gx = xp + (p->vel * p->v) * iom;
    double gy = yp - (p->vel * p->u) * iom;
    double rho = sqrt(gx * gx + gy * gy);
    double rl = (p->vel * sqrt(p->u * p->u + p->v * p->v)) * fabs(iom);
    p->x = gx;
    p->y = gy;
    p->s_path = 0.0;
    int nir = count_faces_le(c->rf, d->n_r, rho);
    if (at_birth) {
        p->ir = nir;
    } else if (nir != p->ir) {
        flush_time(c, p);
        if (nir > p->ir) {
            for (int f = p->ir + 1; f <= nir; ++f) cross_r(c, p, f, 1);
        } else {
            for (int f = p->ir; f > nir; --f) cross_r(c, p, f, 0);
        }
        p->ir = nir;
    }
    return rho + rl >= d->radius;
}

/* ------------------------------------------------------------------ */
/* kinematics                                                           */
/* ------------------------------------------------------------------ */
static void rotate(double u, double v, double w, double mu, double phi, double out[3]) {
    double s = sqrt(fmax(0.0, 1.0 - mu * mu));
    double sp, cp;
    ko_sincos(phi, &sp, &cp);
    double a, b, cc;
    if (fabs(w) < 1.0 - 1e-10) {
        double t = sqrt(1.0 - w * w);
        double it = 1.0 / t;
        a = mu * u + s * (u * w * cp - v * sp) * it;
        b = mu * v + s * (v * w * cp + u * sp) * it;
        cc = mu * w - s * t * cp;
    } else {
        a = s * cp;
        b = s * sp;
        cc = (w > 0.0) ? mu : -mu;
    }
    double in = 1.0 / sqrt(a * a + b * b + cc * cc);
    out[0] = a * in;
    out[1] = b * in;
    out[2] = cc * in;
}

/* thermal target velocity from two Box-Muller slots */
static void thermal(const ctx_t* c, const part_t* p, uint32_t sa, uint32_t sb, double V[3]) {
    if (!(c->sigma_v > 0.0)) {
        V[0] = V[1] = V[2] = 0.0;
        return;
    }
    pair_t a = draw(c->d->seed, p->pid, p->lineage, p->s, sa);
    pair_t b = draw(c->d->seed, p->pid, p->lineage, p->s, sb);
    double r1 = sqrt(-2.0 * ko_log(a.d0 + TWO_M53));
    double r2 = sqrt(-2.0 * ko_log(b.d0 + TWO_M53));
    double a1 = TWO_PI * a.d1;
    double a2 = TWO_PI * b.d1;
    double s1, c1, s2, c2;
    ko_sincos(a1, &s1, &c1);
    ko_sincos(a2, &s2, &c2);
    V[0] = c->sigma_v * (r1 * c1);
    V[1] = c->sigma_v * (r1 * s1);
    V[2] = c->sigma_v * (r2 * c2);
}

static void set_velocity(part_t* p, double e_from_v2, const double vv[3]) {
    double v2 = vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2];
    p->e = v2 * e_from_v2;
    p->vel = sqrt(v2);
    if (p->vel > 0.0) {
        double iv = 1.0 / p->vel;
        p->u = vv[0] * iv;
        p->v = vv[1] * iv;
        p->w = vv[2] * iv;
    }
}

/* Polar angle from the piecewise linear density of one energy bin (Sec. 3.3): the interval is the
   one where the running area (trapezoids, left to right) first exceeds u times the total, and
   inside it the linear density is integrated exactly: f0 x + (s/2) x^2 = r, solved as
   x = 2 r / (f0 + sqrt(f0^2 + 2 s r)). */
static double table_angle(const ko_process* pr, int b, double u) {
    const int n = pr->ang_nodes;
    const double* th = pr->ang_theta;
    const double* f = pr->ang_pdf + (size_t)b * n;
    double total = 0.0;
    for (int k = 0; k + 1 < n; ++k) total += 0.5 * (f[k] + f[k + 1]) * (th[k + 1] - th[k]);
    double a = u * total;
    double run = 0.0;
    int k = 0;
    for (; k + 1 < n - 1; ++k) {
        double next = run + 0.5 * (f[k] + f[k + 1]) * (th[k + 1] - th[k]);
        if (a < next) break;
        run = next;
    }
    double h = th[k + 1] - th[k];
    double r = a - run;
    double s = (f[k + 1] - f[k]) / h;
    double den = f[k] + sqrt(f[k] * f[k] + 2.0 * s * r);
    double x = (r > 0.0 && den > 0.0) ? 2.0 * r / den : 0.0;
    if (x > h) x = h;
    return th[k] + x;
}

/* cosine of the centre-of-mass scattering angle for impact energy ecm and uniform u */
static double scatter_mu(const ko_process* pr, double ecm, double u) {
    if (pr->ang_bins <= 0 || ecm < pr->e_iso) return 2.0 * u - 1.0;
    int b = 0;
    while (b < pr->ang_bins - 1 && ecm >= pr->ang_edges[b + 1]) ++b;
    double sn, cs;
    ko_sincos(table_angle(pr, b, u), &sn, &cs);
    return cs;
}

static void k_elastic(ctx_t* c, part_t* p, int pi, double* gas_out) {
    const ko_desc* d = c->d;
    const int s = p->sp;
    double v[3] = {p->vel * p->u, p->vel * p->v, p->vel * p->w};
    double V[3];
    thermal(c, p, 2, 3, V);
    double g[3] = {v[0] - V[0], v[1] - V[1], v[2] - V[2]};
    double gm = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    double gh[3] = {0.0, 0.0, 1.0};
    if (gm > 0.0) {
        double ig = 1.0 / gm;
        gh[0] = g[0] * ig;
        gh[1] = g[1] * ig;
        gh[2] = g[2] * ig;
    }
    /* centre-of-mass velocity (m v + M V)/(m + M) */
    double mf = c->mfrac[s], gf = c->gfrac[s];
    double cm[3] = {mf * v[0] + gf * V[0], mf * v[1] + gf * V[1], mf * v[2] + gf * V[2]};
    pair_t q = draw(d->seed, p->pid, p->lineage, p->s, 1);
    /* impact energy in the centre-of-mass frame selects the angle distribution */
    double ecm = (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) * c->e_from_v2[s] * gf;
    double mu = scatter_mu(&d->proc[pi], ecm, q.d0);
    double phi = TWO_PI * q.d1;
    double gn[3];
    rotate(gh[0], gh[1], gh[2], mu, phi, gn);
    double a = gf * gm;
    double vn[3] = {cm[0] + a * gn[0], cm[1] + a * gn[1], cm[2] + a * gn[2]};
    double e0 = p->e;
    set_velocity(p, c->e_from_v2[s], vn);
    *gas_out = e0 - p->e;
}

/* Kim-Rudd BEB secondary-energy distribution (Q = 1), w = W/B on [0,(t-1)/2],
   exact rejection from a four-term envelope with closed-form inverse CDFs */
static double beb_sample(const ctx_t* c, const part_t* p, double t, int64_t* tries) {
    if (!(t > 1.0)) return 0.0;
    double tp1 = t + 1.0;
    double lt = ko_log(t);
    double a4 = 4.0 / (tp1 * tp1);
    double it2 = 1.0 / (t * t);
    double i1 = (t - 1.0) / tp1;
    double i2 = (t - 1.0) / (t * tp1);
    double i3 = 0.5 * lt * (1.0 - a4);
    double i4 = 0.5 * lt * (a4 - it2);
    double c1 = i1, c2 = c1 + i2, c3 = c2 + i3, tot = c3 + i4;
    double wmax = 0.5 * (t - 1.0);
    double w = 0.0;
    for (uint32_t k = 0; k < 64; ++k) {
        pair_t a = draw(c->d->seed, p->pid, p->lineage, p->s, 8u + 2u * k);
        pair_t b = draw(c->d->seed, p->pid, p->lineage, p->s, 9u + 2u * k);
        double pick = a.d0 * tot;
        double u = a.d1;
        if (pick < c1) w = 1.0 / (1.0 - u * (1.0 - 2.0 / tp1)) - 1.0;
        else if (pick < c2) w = t - 1.0 / (1.0 / t + u * (2.0 / tp1 - 1.0 / t));
        else if (pick < c3) w = 1.0 / sqrt(1.0 - u * (1.0 - a4)) - 1.0;
        else w = t - 1.0 / sqrt(it2 + u * (a4 - it2));
        if (w < 0.0) w = 0.0;
        if (w > wmax) w = wmax;
        double x1 = 1.0 / (w + 1.0), x2 = 1.0 / (t - w);
        double env = x1 * x1 + x2 * x2 + lt * (x1 * x1 * x1 + x2 * x2 * x2);
        double g = env - (x1 + x2) / tp1;
        *tries += 1;
        if (b.d0 * env < g) return w;
    }
    return w;
}

typedef struct {
    int n;
    seed_t s[2];
    double gas, w;
} products_t;

static void k_ionization(ctx_t* c, part_t* p, int pi, double xc, double yc, products_t* out) {
    const ko_desc* d = c->d;
    const double ef2 = c->e_from_v2[p->sp], v2e = c->v2_from_e[p->sp];
    double B = d->proc[pi].e_th;
    double v[3] = {p->vel * p->u, p->vel * p->v, p->vel * p->w};
    double V[3], g[3], er;
    thermal(c, p, 2, 3, V);
    g[0] = v[0] - V[0]; g[1] = v[1] - V[1]; g[2] = v[2] - V[2];
    er = (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) * ef2;
    for (uint32_t r = 1; er < B && r <= 15; ++r) {
        c->t->counters[KO_C_TARGET_REDRAW] += 1;
        thermal(c, p, 136u + 2u * r, 137u + 2u * r, V);
        g[0] = v[0] - V[0]; g[1] = v[1] - V[1]; g[2] = v[2] - V[2];
        er = (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) * ef2;
    }
    if (er < B) {
        V[0] = V[1] = V[2] = 0.0;
        g[0] = v[0]; g[1] = v[1]; g[2] = v[2];
        er = (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) * ef2;
    }
    double t = er / B;
    double w = beb_sample(c, p, t, &c->t->counters[KO_C_BEB_TRIES]);
    double W = w * B;
    double ef = er - B - W;
    if (ef < 0.0) ef = 0.0;
    double den = er - B;
    double ctf = 1.0, cts = 0.0;
    if (den > 0.0) {
        ctf = sqrt(ef / den);
        cts = sqrt(W / den);
    }
    double gm = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    double gh[3] = {0.0, 0.0, 1.0};
    if (gm > 0.0) {
        double ig = 1.0 / gm;
        gh[0] = g[0] * ig;
        gh[1] = g[1] * ig;
        gh[2] = g[2] * ig;
    }
    pair_t q = draw(d->seed, p->pid, p->lineage, p->s, 1);
    double phi = TWO_PI * q.d1;
    double phis = phi - PI;
    double df[3], ds[3];
    rotate(gh[0], gh[1], gh[2], ctf, phi, df);
    rotate(gh[0], gh[1], gh[2], cts, phis, ds);
    double sf = sqrt(ef * v2e);
    double ss = sqrt(W * v2e);
    double vf[3] = {V[0] + sf * df[0], V[1] + sf * df[1], V[2] + sf * df[2]};
    double vs[3] = {V[0] + ss * ds[0], V[1] + ss * ds[1], V[2] + ss * ds[2]};
    double es = (vs[0] * vs[0] + vs[1] * vs[1] + vs[2] * vs[2]) * ef2;
    const int qi = d->proc[pi].product;   /* the ion species made */
    double eion = (V[0] * V[0] + V[1] * V[1] + V[2] * V[2]) * c->e_from_v2[qi];
    double e0 = p->e;
    set_velocity(p, ef2, vf);
    out->gas = e0 - (p->e + es + eion + B);
    out->w = w;
    /* slow electron (product slot 0) and ion (product slot 1) */
    out->n = 2;
    seed_t* se = &out->s[0];
    se->x = xc; se->y = yc; se->z = p->z;
    double vsm = sqrt(vs[0] * vs[0] + vs[1] * vs[1] + vs[2] * vs[2]);
    if (vsm > 0.0) { double iv = 1.0 / vsm; se->u = vs[0] * iv; se->v = vs[1] * iv; se->w = vs[2] * iv; }
    else { se->u = 0.0; se->v = 0.0; se->w = 1.0; }
    se->e = es; se->sp = 0; se->ir = p->ir; se->iz = p->iz;
    se->lineage = child_lineage(p->lineage, p->s, 0);
    seed_t* si = &out->s[1];
    si->x = xc; si->y = yc; si->z = p->z;
    double Vm = sqrt(V[0] * V[0] + V[1] * V[1] + V[2] * V[2]);
    if (Vm > 0.0) { double iv = 1.0 / Vm; si->u = V[0] * iv; si->v = V[1] * iv; si->w = V[2] * iv; }
    else { si->u = 0.0; si->v = 0.0; si->w = 1.0; }
    si->e = eion; si->sp = qi; si->ir = p->ir; si->iz = p->iz;
    si->lineage = child_lineage(p->lineage, p->s, 1);
}

/* Clustering (Sec. 3.3 "Clustering"): a target particle's velocity is drawn as for elastic
   scattering; the product moves along it with the target particle's momentum, |v'| = (M/m')|V|.
   The product is a new particle at the collision point; its energy comes from the gas. */
static void k_clustering(ctx_t* c, part_t* p, int pi, double xc, double yc, seed_t* out,
                         double* gas) {
    const int q = c->d->proc[pi].product;
    double V[3];
    thermal(c, p, 2, 3, V);
    const double sc = c->conv[pi];
    double vn[3] = {sc * V[0], sc * V[1], sc * V[2]};
    double vm = sqrt(vn[0] * vn[0] + vn[1] * vn[1] + vn[2] * vn[2]);
    out->x = xc; out->y = yc; out->z = p->z;
    if (vm > 0.0) { double iv = 1.0 / vm; out->u = vn[0] * iv; out->v = vn[1] * iv; out->w = vn[2] * iv; }
    else { out->u = 0.0; out->v = 0.0; out->w = 1.0; }
    out->e = (vn[0] * vn[0] + vn[1] * vn[1] + vn[2] * vn[2]) * c->e_from_v2[q];
    out->sp = q; out->ir = p->ir; out->iz = p->iz;
    out->lineage = child_lineage(p->lineage, p->s, 0);
    *gas = -out->e;
}

/* Charge exchange (Sec. 3.3 "Charge exchange"): the projectile continues with the velocity of a
   target particle, drawn as for elastic scattering. */
static void k_charge_exchange(ctx_t* c, part_t* p, double* gas) {
    double V[3];
    thermal(c, p, 2, 3, V);
    double e0 = p->e;
    set_velocity(p, c->e_from_v2[p->sp], V);
    *gas = e0 - p->e;
}

/* ------------------------------------------------------------------ */
/* rates and interaction, shared by both movers                        */
/* ------------------------------------------------------------------ */
/* rate[j] = n_target sigma_j of every process of the particle's species in its current cell
   (eq. 1); returns their sum */
static double rates(ctx_t* c, part_t* p, double* rate) {
    const ko_desc* d = c->d;
    if (p->e != p->e_rates) eval_sigmas(c, p);
    const int np = c->nps[p->sp];
    const int32_t* pidx = c->pidx[p->sp];
    double sum = 0.0;
    for (int j = 0; j < np; ++j) {
        const ko_process* pr = &d->proc[pidx[j]];
        if (pr->target == KO_TARGET_GAS) {
            double n = d->n_gas[p->iz];
            /* three-body clustering: rate k n^2, written as n (n sigma) with sigma = k/v */
            rate[j] = (pr->density_power == 2) ? n * (n * p->sig[j]) : n * p->sig[j];
        } else {
            /* the density field of the partner species (Sec. 2.2) */
            const double* f = d->n_field[pr->partner];
            double nt = f ? f[(size_t)p->ir * d->n_z + (size_t)p->iz] : 0.0;
            rate[j] = nt * p->sig[j];
        }
        sum += rate[j];
    }
    return sum;
}

/* The interaction (Sec. 2.1: chosen with weight sigma_i n_i) at position (xc, yc, p->z), and the
   terminator's checks after it. */
static void interact(ctx_t* c, part_t* p, const double* rate, double sum, double xi, double xc,
                     double yc) {
    const ko_desc* d = c->d;
    ko_tallies* T = c->t;
    const ko_species* S = &d->sp[p->sp];
    const int np = c->nps[p->sp];
    const int32_t* pidx = c->pidx[p->sp];
    double target = xi * sum;
    double run = 0.0;
    int sel = -1, last = -1;
    for (int j = 0; j < np; ++j) {
        run += rate[j];
        if (rate[j] > 0.0) last = j;
        if (sel < 0 && target < run) sel = j;
    }
    if (sel < 0) sel = last;
    int pi = pidx[sel];
    const ko_process* pr = &d->proc[pi];
    T->counters[KO_C_COLL + p->sp] += 1;
    T->counters[KO_C_PROC + pi] += 1;
    p->n_int += 1;
    ev(p, 2, (uint32_t)pi, (uint32_t)(p->ir * d->n_z + p->iz));
    int killed = 0;
    if (pr->kind == KO_ELASTIC) {
        double gas;
        k_elastic(c, p, pi, &gas);
        p->e_gas += gas;
    } else if (pr->kind == KO_EXCITATION) {
        p->e = p->e - pr->e_th;
        p->vel = (p->e > 0.0) ? sqrt(p->e * c->v2_from_e[p->sp]) : 0.0;
        p->e_exc += pr->e_th;
    } else if (pr->kind == KO_IONIZATION) {
        products_t out;
        k_ionization(c, p, pi, xc, yc, &out);
        p->e_bind += pr->e_th;
        p->e_gas += out.gas;
        for (int j = 0; j < out.n; ++j) push(c, &out.s[j]);
    } else if (pr->kind == KO_CHARGE_EXCHANGE) {
        double gas;
        k_charge_exchange(c, p, &gas);
        p->e_gas += gas;
    } else if (pr->kind == KO_CLUSTERING) {
        seed_t prod;
        double gas;
        k_clustering(c, p, pi, xc, yc, &prod, &gas);
        p->e_gas += gas;
        kill(c, p, KO_CONVERTED);
        push(c, &prod);
        killed = 1;
    } else { /* recombination: one deletion logged in the partner's field (Sec. 3.3) */
        T->recomb[((size_t)pr->partner * d->n_r + (size_t)p->ir) * d->n_z + (size_t)p->iz] += 1;
        kill(c, p, KO_RECOMBINED);
        killed = 1;
    }
    if (!killed) {
        if (p->e < S->e_cut) kill(c, p, KO_CUTOFF);
        else if (p->n_int >= S->cap) kill(c, p, KO_CAP);
        else if (!(p->vel > 0.0)) kill(c, p, KO_LIFETIME);
        else if (c->gc) {
            if (gc_set(c, p, xc, yc, 0)) {
                cross_r(c, p, d->n_r, 1);
                kill(c, p, KO_WALL);
            }
        }
    }
}

/* crossing of z-face f in direction dir (1: +z) in the particle's ring: current collector and
   spectrum plane */
static void cross_z(ctx_t* c, part_t* p, int f, int dir) {
    const ko_desc* d = c->d;
    ko_tallies* T = c->t;
    T->counters[KO_C_ZCROSS + p->sp] += 1;
    T->jz[(((size_t)p->sp * d->n_r + (size_t)p->ir) * (d->n_z + 1) + (size_t)f) * 2 + (size_t)dir] += 1;
    ev(p, 3, (uint32_t)dir, (uint32_t)(p->ir * (d->n_z + 1) + f));
    int pl = c->plane_of[f];
    if (pl >= 0) {
        int bin = find_bin(d->sp[p->sp].edges, d->n_bins, p->e);
        T->spectra[(((size_t)p->sp * d->n_planes + (size_t)pl) * 2 + (size_t)dir) * (d->n_bins + 2) + (size_t)bin] += 1;
        ev(p, 5, (uint32_t)(pl * 2 + dir), (uint32_t)bin);
    }
}

/* ------------------------------------------------------------------ */
/* Boris mover (Sec. 3.1 "Boris mover")                                */
/* ------------------------------------------------------------------ */
/* field vector of array `arr` ([field_nr][field_nz] bins of (r, phi, z) components over the
   field's radius and height) at (x, y, z) in Cartesian components; zero outside the binning */
static void field_at(const ko_desc* d, const double* arr, double x, double y, double z, double out[3]) {
    out[0] = out[1] = out[2] = 0.0;
    if (!arr) return;
    double r = sqrt(x * x + y * y);
    if (!(r < d->field_radius) || !(z >= 0.0) || !(z < d->field_length)) return;
    int ir = (int)((r / d->field_radius) * (double)d->field_nr);
    int iz = (int)((z / d->field_length) * (double)d->field_nz);
    if (ir > d->field_nr - 1) ir = d->field_nr - 1;
    if (iz > d->field_nz - 1) iz = d->field_nz - 1;
    const double* f = arr + ((size_t)ir * d->field_nz + (size_t)iz) * 3;
    double cp = 1.0, sp = 0.0;
    if (r > 0.0) { cp = x / r; sp = y / r; }
    out[0] = f[0] * cp - f[1] * sp;
    out[1] = f[0] * sp + f[1] * cp;
    out[2] = f[2];
}

/* one push: half an electric kick, the magnetic rotation with Omega = h B and
   t = 2 Omega / (1 + Omega.Omega), the second half kick (h = q dt / 2m), then x += v dt */
static void boris_push(const ctx_t* c, part_t* p, double dt) {
    const ko_desc* d = c->d;
    double E[3], B[3];
    field_at(d, d->e_field, p->x, p->y, p->z, E);
    if (d->b_field) field_at(d, d->b_field, p->x, p->y, p->z, B);
    else { B[0] = 0.0; B[1] = 0.0; B[2] = d->bz; }
    const double h = c->boris_h[p->sp];
    double v[3] = {p->vel * p->u, p->vel * p->v, p->vel * p->w};
    double vm[3] = {v[0] + h * E[0], v[1] + h * E[1], v[2] + h * E[2]};
    double W[3] = {h * B[0], h * B[1], h * B[2]};
    double f = 2.0 / (1.0 + (W[0] * W[0] + W[1] * W[1] + W[2] * W[2]));
    double t[3] = {f * W[0], f * W[1], f * W[2]};
    double vp[3] = {vm[0] + (vm[1] * W[2] - vm[2] * W[1]),
                    vm[1] + (vm[2] * W[0] - vm[0] * W[2]),
                    vm[2] + (vm[0] * W[1] - vm[1] * W[0])};
    double vq[3] = {vm[0] + (vp[1] * t[2] - vp[2] * t[1]),
                    vm[1] + (vp[2] * t[0] - vp[0] * t[2]),
                    vm[2] + (vp[0] * t[1] - vp[1] * t[0])};
    double vn[3] = {vq[0] + h * E[0], vq[1] + h * E[1], vq[2] + h * E[2]};
    p->x = p->x + vn[0] * dt;
    p->y = p->y + vn[1] * dt;
    p->z = p->z + vn[2] * dt;
    set_velocity(p, c->e_from_v2[p->sp], vn);
}

/* end of a movement: its time to the segment (and energy bin) it was spent in, the work of
   the electric field on it to the ledger */
static void end_movement(ctx_t* c, part_t* p, double e0m, int eb) {
    const ko_desc* d = c->d;
    if (c->dense_s && p->t_cell != 0.0) {
        size_t k = ((((size_t)p->sp * d->n_r + (size_t)p->ir) * d->n_z + (size_t)p->iz) *
                    (size_t)(d->n_dens_bins + 2)) + (size_t)eb;
        nadd(&c->dense_s[k], &c->dense_c[k], p->t_cell);
    }
    flush_time(c, p);
    double work = p->e - e0m;
    if (work != 0.0) {
        ledger_add(c, KO_L_E_FIELD, work);
        hist_add(c, p, 1, -work);
    }
}

static void transport_boris(ctx_t* c, part_t* p) {
    const ko_desc* d = c->d;
    ko_tallies* T = c->t;
    const ko_species* S = &d->sp[p->sp];
    const double dt = d->boris_dt[p->sp];
    double rate[KO_MAX_PROC];
    int moving = 0, eb = 0;
    double dr = 0.0, e0m = 0.0;
    while (p->alive) {
        if (!moving) {
            /* a new distance from the mean free path at the current position, eq. (2) */
            double sum = rates(c, p, rate);
            pair_t q0 = draw(d->seed, p->pid, p->lineage, p->s, 0);
            dr = (sum > 0.0) ? -ko_log(q0.d0 + TWO_M53) / sum : INFINITY;
            moving = 1;
            e0m = p->e;
            eb = c->dense_s ? find_bin(S->dens_edges, d->n_dens_bins, p->e) : 0;
        }
        boris_push(c, p, dt);
        dr -= p->vel * dt;
        p->t_cell += dt;
        p->t_alive += dt;
        T->counters[KO_C_STEP + p->sp] += 1;
        double r = sqrt(p->x * p->x + p->y * p->y);
        if (p->z < 0.0) {
            end_movement(c, p, e0m, eb);
            for (int f = p->iz; f >= 0; --f) cross_z(c, p, f, 0);
            kill(c, p, KO_EXIT_LOW);
        } else if (!(p->z < d->length)) {
            end_movement(c, p, e0m, eb);
            for (int f = p->iz + 1; f <= d->n_z; ++f) cross_z(c, p, f, 1);
            kill(c, p, KO_EXIT_HIGH);
        } else {
            int niz = count_faces_le(c->zf, d->n_z, p->z);
            int nir = count_faces_le(c->rf, d->n_r, r);
            int wall = !(r < d->radius);
            if (wall || niz != p->iz || nir != p->ir) {
                /* left the segment: the movement stops without an interaction */
                end_movement(c, p, e0m, eb);
                moving = 0;
                if (niz > p->iz) for (int f = p->iz + 1; f <= niz; ++f) cross_z(c, p, f, 1);
                else for (int f = p->iz; f > niz; --f) cross_z(c, p, f, 0);
                p->iz = niz;
                int rto = wall ? d->n_r : nir;
                if (rto > p->ir) for (int f = p->ir + 1; f <= rto; ++f) cross_r(c, p, f, 1);
                else for (int f = p->ir; f > rto; --f) cross_r(c, p, f, 0);
                if (wall) kill(c, p, KO_WALL);
                else p->ir = nir;
            } else if (c->dense_s && find_bin(S->dens_edges, d->n_dens_bins, p->e) != eb) {
                /* left the energy bin: the movement stops without an interaction */
                end_movement(c, p, e0m, eb);
                moving = 0;
            } else if (dr < 0.0) {
                /* the drawn distance is used up: interaction here, chosen with the rates at the
                   current energy and segment (none if they all vanished on the way) */
                end_movement(c, p, e0m, eb);
                moving = 0;
                double sum = rates(c, p, rate);
                if (sum > 0.0) {
                    pair_t q = draw(d->seed, p->pid, p->lineage, p->s, 0);
                    interact(c, p, rate, sum, q.d1, p->x, p->y);
                }
            }
        }
        p->s += 1;
        if (p->alive && p->t_alive >= S->lifetime) {
            if (moving) end_movement(c, p, e0m, eb);
            kill(c, p, KO_LIFETIME);
        }
    }
}

/* ------------------------------------------------------------------ */
/* one particle from birth to deletion                                 */
/* ------------------------------------------------------------------ */
static void transport(ctx_t* c, const seed_t* b, uint32_t pid) {
    const ko_desc* d = c->d;
    ko_tallies* T = c->t;
    part_t P;
    memset(&P, 0, sizeof(P));
    part_t* p = &P;
    p->sp = b->sp; p->ir = b->ir; p->iz = b->iz; p->alive = 1;
    p->pid = pid; p->s = 0; p->lineage = b->lineage;
    p->x = b->x; p->y = b->y; p->z = b->z;
    p->u = b->u; p->v = b->v; p->w = b->w; p->e = b->e;
    p->vel = (b->e > 0.0) ? sqrt(b->e * c->v2_from_e[b->sp]) : 0.0;
    p->e_rates = -1.0;
    p->dg = ko_mix64(p->lineage ^ DIGEST0);
    const ko_species* S = &d->sp[p->sp];

    T->counters[KO_C_BIRTH + p->sp] += 1;
    hist_add(c, p, 2, 1.0);
    ev(p, 1, (uint32_t)p->sp, (uint32_t)(p->ir * d->n_z + p->iz));
    if (!S->tracked) { kill(c, p, KO_UNTRACKED); return; }
    if (p->e < S->e_cut) { kill(c, p, KO_CUTOFF); return; }
    if (!(p->vel > 0.0)) { kill(c, p, KO_LIFETIME); return; }
    if (c->gc) {
        if (gc_set(c, p, p->x, p->y, 1)) {
            cross_r(c, p, d->n_r, 1);
            kill(c, p, KO_WALL);
            return;
        }
    }

    if (c->boris) {
        transport_boris(c, p);
        return;
    }
    double rate[KO_MAX_PROC];
    while (p->alive) {
        double sum = rates(c, p, rate);
        pair_t q0 = draw(d->seed, p->pid, p->lineage, p->s, 0);
        double eta = q0.d0 + TWO_M53;
        double xi = q0.d1;
        double dist = (sum > 0.0) ? -ko_log(eta) / sum : INFINITY;

        /* distance to the next face of the current cell */
        double sg = INFINITY;
        int which = 0; /* 1 z-face, 2 r outer, 3 r inner */
        int zface = -1;
        if (p->w > 0.0) {
            zface = p->iz + 1;
            sg = (c->zf[zface] - p->z) / p->w;
            which = 1;
        } else if (p->w < 0.0) {
            zface = p->iz;
            sg = (c->zf[zface] - p->z) / p->w;
            which = 1;
        }
        if (sg < 0.0) sg = 0.0;
        if (!c->gc) {
            double a = p->u * p->u + p->v * p->v;
            if (a > 0.0) {
                double bq = p->x * p->u + p->y * p->v;
                double ro = c->rf[p->ir + 1];
                double cq = p->x * p->x + p->y * p->y - ro * ro;
                double disc = bq * bq - a * cq;
                double so = (-bq + sqrt(fmax(disc, 0.0))) / a;
                if (so < 0.0) so = 0.0;
                if (so < sg) { sg = so; which = 2; }
                if (p->ir > 0 && bq < 0.0) {
                    double ri = c->rf[p->ir];
                    double ci = p->x * p->x + p->y * p->y - ri * ri;
                    double di = bq * bq - a * ci;
                    if (di >= 0.0) {
                        double si = (-bq - sqrt(di)) / a;
                        if (si < 0.0) si = 0.0;
                        if (si < sg) { sg = si; which = 3; }
                    }
                }
            }
        }
        if (dist == INFINITY && sg == INFINITY) { kill(c, p, KO_LIFETIME); break; }

        double l = (dist < sg) ? dist : sg;
        double dt = l / p->vel;
        p->t_cell += dt;
        p->t_alive += dt;
        if (c->dense_s) {
            /* energy-resolved density field (Sec. 3.4): the segment's time in the bin of the
               energy the particle flies with */
            int eb = find_bin(S->dens_edges, d->n_dens_bins, p->e);
            size_t k = ((((size_t)p->sp * d->n_r + (size_t)p->ir) * d->n_z + (size_t)p->iz) *
                        (size_t)(d->n_dens_bins + 2)) + (size_t)eb;
            nadd(&c->dense_s[k], &c->dense_c[k], dt);
        }
        if (c->gc) {
            p->z += l * p->w;
            p->s_path += l;
        } else {
            p->x += l * p->u;
            p->y += l * p->v;
            p->z += l * p->w;
        }
        T->counters[KO_C_STEP + p->sp] += 1;

        if (dist < sg) {
            /* ---- collision ---- */
            double xc = p->x, yc = p->y;
            if (c->gc) {
                double om = c->omega[p->sp], iom = c->inv_om[p->sp];
                double al = -(om * (p->s_path / p->vel));
                double sa, ca;
                ko_sincos(al, &sa, &ca);
                double un = ca * p->u - sa * p->v;
                double vn = sa * p->u + ca * p->v;
                p->u = un;
                p->v = vn;
                xc = p->x - (p->vel * p->v) * iom;
                yc = p->y + (p->vel * p->u) * iom;
            }
            interact(c, p, rate, sum, xi, xc, yc);
        } else if (which == 1) {
            /* ---- z-face ---- */
            int f = zface;
            int dir = (p->w > 0.0) ? 1 : 0;
            p->z = c->zf[f];
            flush_time(c, p);
            cross_z(c, p, f, dir);
            if (f == 0) kill(c, p, KO_EXIT_LOW);
            else if (f == d->n_z) kill(c, p, KO_EXIT_HIGH);
            else p->iz = dir ? f : f - 1;
        } else {
            /* ---- r-face (straight-line mode) ---- */
            int out = (which == 2);
            int f = out ? p->ir + 1 : p->ir;
            double rho = sqrt(p->x * p->x + p->y * p->y);
            if (rho > 0.0) {
                double sc = c->rf[f] / rho;
                p->x = p->x * sc;
                p->y = p->y * sc;
            }
            flush_time(c, p);
            cross_r(c, p, f, out);
            if (f == d->n_r) kill(c, p, KO_WALL);
            else p->ir = out ? f : f - 1;
        }
        p->s += 1;
        if (p->alive && p->t_alive >= S->lifetime) kill(c, p, KO_LIFETIME);
    }
}

/* ------------------------------------------------------------------ */
/* injection (Sec. 3.5)                                                */
/* ------------------------------------------------------------------ */
static void birth(ctx_t* c, uint32_t pid, seed_t* b, int64_t* tries) {
    const ko_desc* d = c->d;
    b->lineage = 0;
    if (d->source == KO_SOURCE_BEAM || d->source == KO_SOURCE_PAIR) {
        b->sp = d->beam_species;
        b->e = d->beam_energy;
        if (d->source == KO_SOURCE_PAIR) {
            b->sp = (int)(pid & 1u);
            b->e = b->sp ? d->beam_energy_1 : d->beam_energy;
        }
        b->x = d->beam_pos[0]; b->y = d->beam_pos[1]; b->z = d->beam_pos[2];
        b->u = d->beam_dir[0]; b->v = d->beam_dir[1]; b->w = d->beam_dir[2];
        b->ir = count_faces_le(c->rf, d->n_r, sqrt(b->x * b->x + b->y * b->y));
        b->iz = count_faces_le(c->zf, d->n_z, b->z);
        return;
    }
    b->sp = 0;
    pair_t q0 = draw(d->seed, pid, 0, BIRTH_STEP, 0);
    pair_t q1 = draw(d->seed, pid, 0, BIRTH_STEP, 1);
    pair_t q2 = draw(d->seed, pid, 0, BIRTH_STEP, 2);
    double wsum = c->zcdf[d->n_z];
    int k;
    double z;
    if (wsum > 0.0) {
        double tt = q0.d0 * wsum;
        k = -1;
        for (int j = 0; j < d->n_z; ++j)
            if (tt < c->zcdf[j + 1]) { k = j; break; }
        if (k < 0) {
            k = d->n_z - 1;
            while (k > 0 && !(d->n_gas[k] > 0.0)) --k;
        }
        z = c->zf[k] + ((tt - c->zcdf[k]) / d->n_gas[k]) * (d->length / (double)d->n_z);
    } else {
        z = q0.d0 * d->length;
        k = count_faces_le(c->zf, d->n_z, z);
    }
    double r = d->radius * sqrt(q0.d1);
    double al = TWO_PI * q1.d0;
    double mu = 2.0 * q1.d1 - 1.0;
    double ph = TWO_PI * q2.d0;
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double sal, cal, sph, cph;
    ko_sincos(al, &sal, &cal);
    ko_sincos(ph, &sph, &cph);
    b->x = r * cal;
    b->y = r * sal;
    b->z = z;
    b->u = st * cph;
    b->v = st * sph;
    b->w = mu;
    b->iz = k;
    b->ir = count_faces_le(c->rf, d->n_r, r);
    double e = 0.0;
    for (uint32_t j = 0; j < 64; ++j) {
        pair_t q = draw(d->seed, pid, 0, BIRTH_STEP, 3u + j);
        e = d->beta_e0 * (q.d0 + TWO_M53);
        *tries += 1;
        if (q.d1 * d->beta_fmax < ko_beta_shape(e, d->beta_e0, d->beta_z)) break;
    }
    b->e = e;
}

int ko_run(const ko_desc* d, int64_t pid_begin, int64_t pid_end, ko_tallies* t) {
    if (!d || !t || pid_begin < 0 || pid_end < pid_begin || pid_end > d->n_primaries ||
        pid_end > 0xFFFFFFFFLL)
        return -1;
    ctx_t c;
    if (ctx_init(&c, d, t) != 0) { ctx_free(&c); return -1; }
    for (int64_t pid = pid_begin; pid < pid_end; ++pid) {
        seed_t b;
        birth(&c, (uint32_t)pid, &b, &t->counters[KO_C_BETA_TRIES]);
        ledger_add(&c, KO_L_E_PRIMARY, b.e);
        if (t->hist) t->hist[(size_t)pid * KO_NHIST + 0] += b.e;
        c.n_stack = 0;
        push(&c, &b);
        while (c.n_stack > 0) {
            seed_t s = c.stack[--c.n_stack];
            transport(&c, &s, (uint32_t)pid);
        }
    }
    size_t nd = (size_t)c.n_species * d->n_r * d->n_z;
    for (size_t k = 0; k < nd; ++k) t->density_time[k] += c.dens_s[k] + c.dens_c[k];
    if (c.dense_s) {
        size_t ne = nd * (size_t)(d->n_dens_bins + 2);
        for (size_t k = 0; k < ne; ++k) t->density_time_e[k] += c.dense_s[k] + c.dense_c[k];
    }
    for (int k = 0; k < KO_NLEDGER; ++k) t->ledger[k] += c.led_s[k] + c.led_c[k];
    ctx_free(&c);
    return 0;
}

/* ------------------------------------------------------------------ */
/* normalised fields: density, eq. (3) with t_sim = N_prim / a (eq. 4), */
/* and currents j = (N+ - N-) / (A t_sim) through segment faces        */
/* ------------------------------------------------------------------ */
int ko_fields(const ko_desc* d, const ko_tallies* t, double n_prim, double activity,
              double* density, double* jz_cur, double* jr_cur) {
    if (!(n_prim > 0.0) || !(activity > 0.0)) return -1;
    const int nr = d->n_r, nz = d->n_z;
    const double t_sim = n_prim / activity;
    const double dz = d->length / (double)nz;
    const int ns = d->n_species ? d->n_species : 2;
    if (ns < 2 || ns > KO_MAX_SPECIES) return -1;
    for (int s = 0; s < ns; ++s) {
        for (int ir = 0; ir < nr; ++ir) {
            double r0 = d->radius * (double)ir / (double)nr;
            double r1 = d->radius * (double)(ir + 1) / (double)nr;
            double ring = PI * (r1 * r1 - r0 * r0);        /* area of the ring */
            double vol = ring * dz;                          /* segment volume */
            for (int iz = 0; iz < nz; ++iz) {
                size_t k = ((size_t)s * nr + ir) * nz + iz;
                double n = t->density_time[k] / (t_sim * vol);
                n -= (double)t->recomb[k] / vol;
                density[k] = n;
            }
            for (int f = 0; f <= nz; ++f) {
                size_t k = ((size_t)s * nr + ir) * (nz + 1) + f;
                double net = (double)(t->jz[2 * k + 1] - t->jz[2 * k]);
                jz_cur[k] = net / (ring * t_sim);
            }
        }
        for (int f = 0; f <= nr; ++f) {
            double rf = d->radius * (double)f / (double)nr;
            double area = TWO_PI * rf * dz;                  /* cylinder face of one z-segment */
            for (int iz = 0; iz < nz; ++iz) {
                size_t k = ((size_t)s * (nr + 1) + f) * nz + iz;
                double net = (double)(t->jr[2 * k + 1] - t->jr[2 * k]);
                jr_cur[k] = (area > 0.0) ? net / (area * t_sim) : 0.0;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* single-step entry points for the oracle's own tests                 */
/* ------------------------------------------------------------------ */
int ko_birth(const ko_desc* d, int64_t pid, double out[8]) {
    ko_tallies dummy;
    memset(&dummy, 0, sizeof(dummy));
    ctx_t c;
    if (ctx_init(&c, d, &dummy) != 0) { ctx_free(&c); return -1; }
    seed_t b;
    int64_t tries = 0;
    birth(&c, (uint32_t)pid, &b, &tries);
    out[0] = b.x; out[1] = b.y; out[2] = b.z;
    out[3] = b.u; out[4] = b.v; out[5] = b.w;
    out[6] = b.e; out[7] = (double)tries;
    ctx_free(&c);
    return 0;
}

int ko_debug_collide(const ko_desc* d, int proc, int64_t pid, uint64_t lineage, uint32_t s,
                     double e, const double dir[3], double out[16]) {
    int64_t counters[KO_NCOUNTERS];
    memset(counters, 0, sizeof(counters));
    ko_tallies dummy;
    memset(&dummy, 0, sizeof(dummy));
    dummy.counters = counters;
    ctx_t c;
    if (proc < 0 || proc >= d->n_proc || ctx_init(&c, d, &dummy) != 0) { ctx_free(&c); return -1; }
    part_t P;
    memset(&P, 0, sizeof(P));
    P.sp = d->proc[proc].species;
    P.pid = (uint32_t)pid; P.s = s; P.lineage = lineage; P.alive = 1;
    P.u = dir[0]; P.v = dir[1]; P.w = dir[2]; P.e = e;
    P.vel = sqrt(e * c.v2_from_e[P.sp]);
    for (int k = 0; k < 16; ++k) out[k] = 0.0;
    const ko_process* pr = &d->proc[proc];
    if (pr->kind == KO_ELASTIC) {
        k_elastic(&c, &P, proc, &out[14]);
    } else if (pr->kind == KO_EXCITATION) {
        P.e = P.e - pr->e_th;
    } else if (pr->kind == KO_IONIZATION) {
        products_t pr2;
        k_ionization(&c, &P, proc, 0.0, 0.0, &pr2);
        out[5] = 2;
        out[6] = pr2.s[0].e; out[7] = pr2.s[0].u; out[8] = pr2.s[0].v; out[9] = pr2.s[0].w;
        out[10] = pr2.s[1].e; out[11] = pr2.s[1].u; out[12] = pr2.s[1].v; out[13] = pr2.s[1].w;
        out[14] = pr2.gas;
        out[15] = pr2.w;
    } else if (pr->kind == KO_CHARGE_EXCHANGE) {
        k_charge_exchange(&c, &P, &out[14]);
    } else if (pr->kind == KO_CLUSTERING) {
        seed_t prod;
        k_clustering(&c, &P, proc, 0.0, 0.0, &prod, &out[14]);
        P.alive = 0;
        out[5] = 1;
        out[10] = prod.e; out[11] = prod.u; out[12] = prod.v; out[13] = prod.w;
    } else {
        P.alive = 0;
    }
    out[0] = P.e; out[1] = P.u; out[2] = P.v; out[3] = P.w; out[4] = P.alive;
    ctx_free(&c);
    return 0;
}

double ko_debug_angle(const ko_desc* d, int proc, double e_cm, double u) {
    if (proc < 0 || proc >= d->n_proc) return -1.0;
    double mu = scatter_mu(&d->proc[proc], e_cm, u);
    return acos(mu);
}

int ko_debug_boris(const ko_desc* d, int sp, const double x[3], const double v[3], int n,
                   double out[6]) {
    ko_tallies dummy;
    memset(&dummy, 0, sizeof(dummy));
    ctx_t c;
    if (ctx_init(&c, d, &dummy) != 0 || !c.boris || sp < 0 || sp >= c.n_species || n < 0) {
        ctx_free(&c);
        return -1;
    }
    part_t P;
    memset(&P, 0, sizeof(P));
    P.sp = sp;
    P.x = x[0]; P.y = x[1]; P.z = x[2];
    set_velocity(&P, c.e_from_v2[sp], v);
    for (int k = 0; k < n; ++k) boris_push(&c, &P, d->boris_dt[sp]);
    out[0] = P.x; out[1] = P.y; out[2] = P.z;
    out[3] = P.vel * P.u; out[4] = P.vel * P.v; out[5] = P.vel * P.w;
    ctx_free(&c);
    return 0;
}

void ko_debug_helix(double charge, double mass, double bz, const double pos[3],
                    const double dir[3], double speed, double path, double out[6]) {
    double om = charge * bz / mass;
    double u = dir[0], v = dir[1];
    double gx = pos[0] + speed * v / om;
    double gy = pos[1] - speed * u / om;
    double al = -(om * (path / speed));
    double sa, ca;
    ko_sincos(al, &sa, &ca);
    double un = ca * u - sa * v;
    double vn = sa * u + ca * v;
    out[0] = gx - speed * vn / om;
    out[1] = gy + speed * un / om;
    out[2] = pos[2] + path * dir[2];
    out[3] = un;
    out[4] = vn;
    out[5] = dir[2];
}

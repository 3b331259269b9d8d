// Device code of libkarl: the particle-history transport of the KARL method (arXiv
// 2503.10263) for gfx950.
//
// One lane carries one particle from birth to deletion (main cycle, Sec. 2.1): free flight
// d = -lambda ln(eta) with lambda from eq. (1), stop without interaction at every segment face
// and redraw (Sec. 3.1 "Movement"), guiding-centre helix in a uniform axial field (Sec. 3.1
// "Drift mover"), interaction chosen with weight sigma_i n_i and performed (Sec. 3.3),
// termination and deletion logging (Sec. 3.2).  A lane whose particle is deleted takes the
// next work item of the generation: a primary id (generation 0) or a secondary produced by
// the previous generation.  Secondaries go to the next generation's queue through one
// wave-aggregated atomic (ballot + mbcnt prefix) per wave.
//
// Layout: particle state lives in registers; cross-section tables, gas density and face
// positions are staged in LDS per workgroup; queues are structure-of-arrays in HBM; tallies
// are FP64/int64 in HBM, updated once per segment visit (time) or crossing (counts);
// per-event counters are kept in registers or LDS and flushed once per workgroup.
//
// Every floating-point expression of the FP64 instantiation is written in the same order as
// the specification of the method so that, compiled without contraction, each operation is
// rounded exactly as the reference evaluation is.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "karl_internal.h"

namespace karl {
namespace {

constexpr double kQE = 1.602176634e-19;   // J per eV (exact)
constexpr double kMEC2 = 510998.95;        // electron rest energy, eV (CODATA 2018)
constexpr double kALPHA = 7.2973525693e-3; // fine-structure constant (CODATA 2018)
constexpr double kPI = 3.14159265358979323846;
constexpr double kTWO_PI = 6.28318530717958647692;
constexpr double kTWO_PI_DEF = 6.28318530717958647692;
constexpr unsigned long long kPHI64 = 0x9E3779B97F4A7C15ull;
constexpr unsigned long long kDIGEST0 = 0x5851F42D4C957F2Dull;
constexpr uint32_t kBIRTH_STEP = 0xFFFFFFFFu;

constexpr int kBlock = 256;
constexpr int kNCnt = KARL_NCOUNTERS;
constexpr int kNLed = KARL_NLEDGER;

// ---------------------------------------------------------------- elementary functions
// FP64 logarithm and sine/cosine built from IEEE basic operations only (fused multiply-add,
// rounded once, among them).  The guiding-centre phase (omega t ~ 1e5 rad) amplifies any
// 1-ulp difference of a transcendental roughly fifty-fold per collision, so these are spelled
// out step by step -- frexp reduction and atanh series for ln, Cody-Waite reduction by pi/2
// in four 26-bit pieces and Taylor series for sin/cos, each series step one fused
// multiply-add -- which any other evaluation of the same steps reproduces exactly.
constexpr double kSqrtHalf = 0.70710678118654757;
constexpr double kLn2Hi = 0.6931471805601177;         // ln 2 to 40 bits (e * hi exact)
constexpr double kLn2Lo = -1.7239444525614835e-13;    // ln 2 - hi
constexpr double kPiO4 = 0.78539816339744828;
constexpr double kTwoOverPi = 0.6366197723675814;
constexpr double kPiO2_1 = 1.5707963407039642;
constexpr double kPiO2_2 = -1.3909067675399456e-08;
constexpr double kPiO2_3 = 6.123233932053594e-17;
constexpr double kPiO2_4 = 6.368317178484799e-25;

// The constants of the FP64 series below, in the order they are used.  The deferred-launch
// kernels (their own unit) read them from a copy in LDS that the launch stages at its start: a
// 64-bit LDS read per use, beside the vector pipeline, where a literal costs two vector moves
// before an accumulating multiply-add (the other single-job kernels keep the literals: there the
// early LDS reads held too many registers).  The batched unit keeps the compiler's hoisting of
// loop invariants, which would hold every coefficient in registers across the transport loop;
// there each one is pinned to a scalar register pair at its use (an empty volatile asm cannot
// be hoisted), and the fused multiply-add takes it as its one scalar operand.
constexpr double kSeriesTab[] = {
    0.04, 0.043478260869565216, 0.047619047619047616, 0.05263157894736842,   // ln: 1/(2n+1),
    0.058823529411764705, 0.06666666666666667, 0.07692307692307693,           // n = 12 .. 1
    0.09090909090909091, 0.1111111111111111, 0.14285714285714285, 0.2, 0.3333333333333333,
    kLn2Hi, kLn2Lo,                                                           // 12, 13
    kTwoOverPi, kPiO2_1, kPiO2_2, kPiO2_3, kPiO2_4,                           // 14 .. 18
    -8.22063524662433e-18, 2.8114572543455206e-15, -7.647163731819816e-13,    // sine: -1/19! ..
    1.6059043836821613e-10, -2.505210838544172e-08, 2.7557319223985893e-06,   // -1/3!, 19 .. 27
    -0.0001984126984126984, 0.008333333333333333, -0.16666666666666666,
    4.110317623312165e-19, -1.5619206968586225e-16, 4.779477332387385e-14,    // cosine: 1/20! ..
    -1.1470745597729725e-11, 2.08767569878681e-09, -2.755731922398589e-07,    // 1/4!, 28 .. 36
    2.48015873015873e-05, -0.001388888888888889, 0.041666666666666664,
};
constexpr int kNSeries = (int)(sizeof(kSeriesTab) / sizeof(double));
#if defined(KARL_BATCHED_UNIT)
__device__ __forceinline__ double KC(int i) {
    double c = kSeriesTab[i];
    asm volatile("" : "+s"(c));
    return c;
}
#elif defined(KARL_DRAIN_UNIT)
__shared__ double s_series[kNSeries];
#define KC(i) (s_series[(i)])
#else
#define KC(i) (kSeriesTab[(i)])
#endif

// a / b, correctly rounded, where both operands are finite, b is nonzero, and the exponents of a
// (unless it is +0), b, 1/b and a/b all lie well inside the normal range: the compiler's division
// without its operand scaling and special-case fix-up, which for such operands change nothing --
// the reciprocal, two Newton steps, the quotient, its residual and the corrected quotient, each
// one rounding, as in the full sequence.  The callers' operands are bounded by construction.
__device__ __forceinline__ double kdiv(double a, double b) {
    double y = __builtin_amdgcn_rcp(b);
    double e = fma(-b, y, 1.0);
    y = fma(y, e, y);
    e = fma(-b, y, 1.0);
    y = fma(y, e, y);
    const double q = a * y;
    const double r = fma(-b, q, a);
    return fma(r, y, q);
}
// FP32 transport state: the hardware reciprocal (build flag), as any division
__device__ __forceinline__ float kdiv(float a, float b) { return a / b; }

__device__ __forceinline__ double klog(double x) {
    if (!(x > 0.0)) return (x == 0.0) ? -INFINITY : NAN;
    if (isinf(x)) return x;
    int e;
    double m = frexp(x, &e);                 // m in [0.5, 1)
    if (m < kSqrtHalf) {
        m = m * 2.0;
        e = e - 1;
    }
    const double f = m - 1.0;
    const double s = kdiv(f, m + 1.0);       // ln m = 2 atanh(s); f in (-0.30, 0.42], m + 1 in [1.7, 2.5)
    const double z = s * s;
    double p = KC(0);                        // coefficients 1/(2n+1), n = 12 .. 1
    p = fma(z, p, KC(1));
    p = fma(z, p, KC(2));
    p = fma(z, p, KC(3));
    p = fma(z, p, KC(4));
    p = fma(z, p, KC(5));
    p = fma(z, p, KC(6));
    p = fma(z, p, KC(7));
    p = fma(z, p, KC(8));
    p = fma(z, p, KC(9));
    p = fma(z, p, KC(10));
    p = fma(z, p, KC(11));
    const double t = 2.0 * s;
    const double lm = fma(t, z * p, t);
    const double de = (double)e;
    return fma(de, KC(12), fma(de, KC(13), lm));
}
// FP32 transport state: natural logarithm from the hardware's single-precision base-2 logarithm
// (its arguments here -- energies, uniforms of at least 2^-24 -- are normal numbers or 0).
__device__ __forceinline__ float klog(float x) { return __builtin_amdgcn_logf(x) * 0.6931471805599453f; }

__device__ __forceinline__ void ksincos(double x, double* sn, double* cs) {
    if (!isfinite(x)) {
        *sn = NAN;
        *cs = NAN;
        return;
    }
    double r = x;
    long long q = 0;
    if (fabs(x) > kPiO4) {
        double xx = x;
        if (fabs(xx) >= 2.0e8) xx = xx - trunc(xx / kTWO_PI_DEF) * kTWO_PI_DEF;
        const double k = floor(fma(xx, KC(14), 0.5));
        r = fma(-k, KC(15), xx);
        r = fma(-k, KC(16), r);
        r = fma(-k, KC(17), r);
        r = fma(-k, KC(18), r);
        q = (long long)k;
    }
    const double z = r * r;
    double ps = KC(19);                      // sine: -1/19! ... -1/3!
    ps = fma(z, ps, KC(20));
    ps = fma(z, ps, KC(21));
    ps = fma(z, ps, KC(22));
    ps = fma(z, ps, KC(23));
    ps = fma(z, ps, KC(24));
    ps = fma(z, ps, KC(25));
    ps = fma(z, ps, KC(26));
    ps = fma(z, ps, KC(27));
    const double sv = fma(r, z * ps, r);
    double pc = KC(28);                      // cosine: 1/20! ... 1/4!
    pc = fma(z, pc, KC(29));
    pc = fma(z, pc, KC(30));
    pc = fma(z, pc, KC(31));
    pc = fma(z, pc, KC(32));
    pc = fma(z, pc, KC(33));
    pc = fma(z, pc, KC(34));
    pc = fma(z, pc, KC(35));
    pc = fma(z, pc, KC(36));
    const double cv = fma(z * z, pc, fma(-0.5, z, 1.0));
    switch (q & 3) {
        case 0: *sn = sv; *cs = cv; break;
        case 1: *sn = cv; *cs = -sv; break;
        case 2: *sn = -sv; *cs = -cv; break;
        default: *sn = -cv; *cs = sv; break;
    }
}
// FP32 transport state: sine and cosine in single precision from the hardware's sine and cosine,
// which take the angle in revolutions.  The angle is first brought to [-1/2, 1/2] revolution
// (x/2pi minus its nearest integer): at the guiding-centre phases of up to ~1e5 rad this adds
// about as much error as the single-precision rounding of x itself (4e-3 rad), and it replaces
// the library's exact large-argument reduction, which every wave holding one such lane ran.
__device__ __forceinline__ void ksincos(float x, float* s, float* c) {
    float r = x * 0.15915494309189535f;
    r = r - rintf(r);
    *s = __builtin_amdgcn_sinf(r);
    *c = __builtin_amdgcn_cosf(r);
}

__device__ __forceinline__ double ksqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float ksqrt(float x) { return sqrtf(x); }
// sqrt(x) for x = 0 or x >= 2^-1000: the compiler's correctly rounded square root without its
// scaling of arguments below 2^-767 -- the reciprocal square root, two Newton steps on the root
// and its half-reciprocal, and the class test that passes +-0 and +inf through.  Without the
// scaling the steps give the same result for every argument from 2^-1011 up (and +0): checked
// bit for bit on 1.3e7 normal numbers over the whole range; they differ only below 2^-1011.
// The callers' arguments are squared norms of positions (m), velocities (m/s) and unit vectors,
// 1 - mu^2 (0 or at least 2^-53) and -2 ln u (at least 2^-52): zero or far above 2^-1000.
__device__ __forceinline__ double ksqrt_n(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y;
    double h = y * 0.5;
    const double r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, x);
    g = fma(d, h, g);
    d = fma(-g, g, x);
    g = fma(d, h, g);
    return __builtin_amdgcn_class(x, 0x260) ? x : g;
}
__device__ __forceinline__ float ksqrt_n(float x) { return sqrtf(x); }
__device__ __forceinline__ double kexp(double x) { return exp(x); }
__device__ __forceinline__ float kexp(float x) { return expf(x); }
__device__ __forceinline__ double kfabs(double x) { return fabs(x); }
__device__ __forceinline__ float kfabs(float x) { return fabsf(x); }
__device__ __forceinline__ double kfmax(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float kfmax(float a, float b) { return fmaxf(a, b); }

template <typename Real> struct Prec;
template <> struct Prec<double> {
    static constexpr double eps = 1.1102230246251565404e-16;  // 2^-53
    // 53-bit uniform in [0,1) from two 32-bit words: ((a >> 5) 2^26 + (b >> 6)) 2^-53.  Every
    // step is exact (an integer below 2^53, then a power of two), so the product and sum are
    // one fused multiply-add with the same result.
    static __device__ __forceinline__ double uni(uint32_t a, uint32_t b, uint32_t) {
        return fma((double)(a >> 5), 67108864.0, (double)(b >> 6)) * eps;
    }
};
template <> struct Prec<float> {
    static constexpr float eps = 5.9604644775390625e-8f;       // 2^-24
    // 24-bit uniform in [0,1) from the high bits of the first word of the pair
    static __device__ __forceinline__ float uni(uint32_t a, uint32_t, uint32_t) {
        return (float)(a >> 8) * eps;
    }
};

// ---------------------------------------------------------------- random numbers
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64 products
// with the Weyl key schedule.  Each round's two three-way exclusive ors are one gfx950
// three-input bit operation each (truth table 0x96 = a ^ b ^ c).
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ U4 philox(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1,
                                     uint32_t c2, uint32_t c3) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const unsigned long long p0 = (unsigned long long)0xD2511F53u * c0;
        const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

template <typename Real> struct Pair { Real d0, d1; };
template <typename Real> struct Vec3 { Real x, y, z; };   // passed by value: stays in registers

// one slot of the draw schedule: key (seed, pid), counter (step, slot, lineage)
template <typename Real>
__device__ __forceinline__ Pair<Real> draw(uint32_t seed, uint32_t pid, unsigned long long lin,
                                           uint32_t s, uint32_t slot) {
    const U4 w = philox(seed, pid, s, slot, (uint32_t)lin, (uint32_t)(lin >> 32));
    return Pair<Real>{Prec<Real>::uni(w.x, w.y, 0u), Prec<Real>::uni(w.z, w.w, 0u)};
}

// SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA 2014)
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

__device__ __forceinline__ unsigned long long child_lineage(unsigned long long parent, uint32_t s,
                                                            uint32_t j) {
    return mix64(parent ^ (kPHI64 * ((((unsigned long long)s) << 3) | (unsigned long long)(j + 1))));
}

__device__ __forceinline__ unsigned long long digest_event(unsigned long long d, uint32_t s,
                                                           uint32_t kind, uint32_t a, uint32_t b) {
    const unsigned long long w = ((unsigned long long)s << 32) |
                                 ((unsigned long long)(kind & 0xFu) << 28) |
                                 ((unsigned long long)(a & 0xFFu) << 20) |
                                 (unsigned long long)(b & 0xFFFFFu);
    return mix64(d ^ w);
}

// ---------------------------------------------------------------- wave helpers
__device__ __forceinline__ unsigned lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ unsigned rank_in(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// Reserve one slot per lane with `want` among the active lanes with a single atomic.
__device__ __forceinline__ unsigned long long wave_reserve(unsigned long long* ctr, bool want) {
    const unsigned long long m = __ballot(want);
    unsigned long long base = 0;
    if (m) {
        const int leader = __ffsll((long long)m) - 1;
        if ((int)lane_id() == leader) base = atomicAdd(ctr, (unsigned long long)__popcll(m));
        base = __shfl(base, leader);
    }
    return base + rank_in(m);
}

// Add 1 to s_cnt[key] for every active lane, one LDS atomic per distinct key in the wave.
__device__ __forceinline__ void wave_count(unsigned long long* s_cnt, int key) {
    bool pending = true;
    for (;;) {
        const unsigned long long mp = __ballot(pending);
        if (!mp) break;
        const int leader = __ffsll((long long)mp) - 1;
        const int k0 = __shfl(key, leader);
        const unsigned long long mk = __ballot(pending && key == k0);
        if ((int)lane_id() == leader) atomicAdd(&s_cnt[k0], (unsigned long long)__popcll(mk));
        if (key == k0) pending = false;
    }
}

__device__ __forceinline__ void add_u64(unsigned long long* p, unsigned long long v) {
    atomicAdd(p, v);
}
__device__ __forceinline__ void add_f64(double* p, double v) { unsafeAtomicAdd(p, v); }

// ---------------------------------------------------------------- state
template <typename Real>
struct Part {
    Real x, y, z, u, v, w, e, vel, s_path;
    double t_alive, t_cell, e_exc, e_bind, e_gas;
    unsigned long long lin, dg;
    uint32_t pid, s;
    int32_t sp, ir, iz, job;
    int64_t n_int;
    bool alive;
    bool start;            // fetched, not yet started
    bool fly;              // guiding-centre mode: the last segment ended on a z-face;
                           // Boris mover: a movement is under way (s_path: its remaining distance)
    Real e0m;              // Boris mover: energy at the start of the movement
    int32_t eb;            // Boris mover: energy bin of the movement (energy-resolved density)
};

template <typename Real>
struct Lds {
    unsigned long long* cnt;   // [KARL_NCOUNTERS]
    double* led;               // [KARL_NLEDGER]
    const int32_t* pidx;       // [4][16]
    const int32_t* kind;       // [16]
    const int32_t* tgt;        // [16] TGT_*
    const Real* eth;           // [16]
    const Real* xs;            // [n_proc][n_e]
    const Real* ngas;          // [n_z]
    const Real* zf;            // [n_z+1]
    const Real* rf;            // [n_r+1]
    const SpeciesConst* sc;    // per-species constants (LDS copy, or the job's in HBM)
    bool direct;               // per-event counts go straight to cnt (wave-aggregated)
};

// Per-lane event counts of one job, added to that job's counters when the lane moves to
// another job and at the end of the launch.
struct LaneCnt {
    uint32_t step0, step1, coll0, coll1, zc0, zc1, rc0, rc1, redraw, beb, beta;
    double e_prim;
};
// The deferred launch's counts: species 0 (which a job defers only when its electrons make no
// products) with one atomic per event like species 2 and 3, so that the launch keeps registers
// for species 1 only.  The interactions per process are counted per lane for the lane's last
// process (flushed when the process changes and at the end of the launch): the deferred species
// have few processes (the H2+ of the full case one), and a register increment replaces the
// wave-aggregated LDS atomic of the other kernels.
struct LaneCntLean : LaneCnt {
    int32_t proc = -1;
    uint32_t proc_n = 0;
};
template <typename LC>
constexpr bool kLeanCnt = __is_same(LC, LaneCntLean);
template <bool kB, typename T, typename F> struct PickT { using type = T; };
template <typename T, typename F> struct PickT<false, T, F> { using type = F; };

// Count one event of kind idx + sp: in a per-lane register (species 0 and 1), with one atomic
// per lane (species 2 and 3), or -- when the lane's counters are not kept per lane -- with one
// atomic per distinct key of the wave.
template <typename Real, typename LC>
__device__ __forceinline__ void count_ev(const Lds<Real>& L, LC& lc, int idx, int sp) {
    if (L.direct) {
        wave_count(L.cnt, idx + sp);
        return;
    }
    if (sp > 1 || (kLeanCnt<LC> && sp == 0)) {
        atomicAdd(&L.cnt[idx + sp], 1ull);
        return;
    }
    switch (idx) {
        case KARL_C_STEP: if (sp) ++lc.step1; else ++lc.step0; break;
        case KARL_C_COLL: if (sp) ++lc.coll1; else ++lc.coll0; break;
        case KARL_C_ZCROSS: if (sp) ++lc.zc1; else ++lc.zc0; break;
        default: if (sp) ++lc.rc1; else ++lc.rc0; break;
    }
}

template <typename Real, typename LC>
__device__ __forceinline__ void count_evn(const Lds<Real>& L, LC& lc, int idx, int sp, uint32_t n) {
    if (L.direct || sp > 1 || (kLeanCnt<LC> && sp == 0)) {
        atomicAdd(&L.cnt[idx + sp], (unsigned long long)n);
        return;
    }
    switch (idx) {
        case KARL_C_STEP: if (sp) lc.step1 += n; else lc.step0 += n; break;
        case KARL_C_COLL: if (sp) lc.coll1 += n; else lc.coll0 += n; break;
        case KARL_C_ZCROSS: if (sp) lc.zc1 += n; else lc.zc0 += n; break;
        default: if (sp) lc.rc1 += n; else lc.rc0 += n; break;
    }
}

template <typename Real>
__device__ __forceinline__ void count_n(const Lds<Real>& L, uint32_t& reg, int idx, uint32_t n) {
    if (L.direct) {
        if (n) atomicAdd(&L.cnt[idx], (unsigned long long)n);
    } else {
        reg += n;
    }
}

__device__ __forceinline__ void count_proc(unsigned long long* cnt, LaneCntLean& lc, int pi) {
    if (pi != lc.proc) {
        if (lc.proc_n) atomicAdd(&cnt[KARL_C_PROC + lc.proc], (unsigned long long)lc.proc_n);
        lc.proc = pi;
        lc.proc_n = 0u;
    }
    ++lc.proc_n;
}

__device__ __forceinline__ void flush_lane(LaneCnt& lc, unsigned long long* cnt, double* led) {
    const uint32_t v[11] = {lc.step0, lc.step1, lc.coll0, lc.coll1, lc.zc0, lc.zc1, lc.rc0, lc.rc1,
                            lc.redraw, lc.beb, lc.beta};
    const int idx[11] = {KARL_C_STEP, KARL_C_STEP + 1, KARL_C_COLL, KARL_C_COLL + 1, KARL_C_ZCROSS,
                         KARL_C_ZCROSS + 1, KARL_C_RCROSS, KARL_C_RCROSS + 1, KARL_C_TARGET_REDRAW,
                         KARL_C_BEB_TRIES, KARL_C_BETA_TRIES};
#pragma unroll
    for (int k = 0; k < 11; ++k)
        if (v[k]) atomicAdd(&cnt[idx[k]], (unsigned long long)v[k]);
    if (lc.e_prim != 0.0) atomicAdd(&led[KARL_L_E_PRIMARY], lc.e_prim);
    lc = LaneCnt{0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u, 0.0};
}

__device__ __forceinline__ void flush_lane(LaneCntLean& lc, unsigned long long* cnt, double* led) {
    if (lc.proc_n) atomicAdd(&cnt[KARL_C_PROC + lc.proc], (unsigned long long)lc.proc_n);
    lc.proc = -1;
    lc.proc_n = 0u;
    flush_lane(static_cast<LaneCnt&>(lc), cnt, led);
}


// ---------------------------------------------------------------- tally helpers
template <typename Real>
__device__ __forceinline__ void flush_time(const DevJob& J, Part<Real>& p) {
    if (p.t_cell != 0.0) {
        add_f64(&J.dens[((size_t)p.sp * J.n_r + (size_t)p.ir) * J.n_z + (size_t)p.iz], p.t_cell);
        p.t_cell = 0.0;
    }
}

template <typename Real>
__device__ __forceinline__ void ev(Part<Real>& p, uint32_t kind, uint32_t a, uint32_t b,
                                   bool on) {
    if (on) p.dg = digest_event(p.dg, p.s, kind, a, b);
}

template <typename Real>
__device__ void kill(const DevJob& J, const Lds<Real>& L, Part<Real>& p, int reason) {
    flush_time(J, p);
    atomicAdd(&L.cnt[KARL_C_DEATH + p.sp * KARL_NREASON + reason], 1ull);
    atomicAdd(&L.led[KARL_L_E_DEATH + p.sp * KARL_NREASON + reason], (double)p.e);
    if (p.t_alive != 0.0) atomicAdd(&L.led[KARL_L_T_ALIVE + p.sp], p.t_alive);
    if (p.e_exc != 0.0) atomicAdd(&L.led[KARL_L_E_EXC], p.e_exc);
    if (p.e_bind != 0.0) atomicAdd(&L.led[KARL_L_E_BIND], p.e_bind);
    if (p.e_gas != 0.0) atomicAdd(&L.led[KARL_L_E_GAS], p.e_gas);
    if (J.flags & KARL_FLAG_DIGESTS) {
        p.dg = digest_event(p.dg, p.s, 6u, (uint32_t)reason, 0u);
        add_u64(&J.digests[p.pid], p.dg);
    }
    if (J.flags & KARL_FLAG_HISTORY) {
        add_f64(&J.hist[(size_t)p.pid * KARL_NHIST + 1], (((double)p.e + p.e_exc) + p.e_bind) + p.e_gas);
        add_f64(&J.hist[(size_t)p.pid * KARL_NHIST + 3], 1.0);
    }
    p.alive = false;
}

template <typename Real, typename LC>
__device__ __forceinline__ void cross_r(const DevJob& J, const Lds<Real>& L, Part<Real>& p, LC& lc,
                                       int f, int dir) {
    count_ev(L, lc, KARL_C_RCROSS, p.sp);
    add_u64(&J.jr[(((size_t)p.sp * (J.n_r + 1) + (size_t)f) * J.n_z + (size_t)p.iz) * 2 + (size_t)dir], 1ull);
    ev(p, 4u, (uint32_t)dir, (uint32_t)(f * J.n_z + p.iz), (J.flags & KARL_FLAG_DIGESTS) != 0);
}

// r-cell k with rf[k] <= r < rf[k+1], clamped to 0..n_r-1, found by walking from a guess
template <typename Real>
__device__ __forceinline__ int r_cell(const Real* rf, int n_r, Real r, int guess) {
    int k = guess;
    while (k + 1 < n_r && rf[k + 1] <= r) ++k;
    while (k > 0 && !(rf[k] <= r)) --k;
    return k;
}

// Guiding centre from position and velocity; returns true if the orbit reaches the wall.
// At birth the r-cell is set from the guiding-centre radius; after a collision every r-face
// between the old and new guiding-centre radius counts as crossed.
// sp: the particle's species (wave-uniform when the caller serves one species per pass)
template <typename Real, typename LC>
__device__ bool gc_set(const DevJob& J, const Lds<Real>& L, Part<Real>& p, LC& lc, Real xp,
                       Real yp, bool at_birth, int sp) {
    const Real iom = (Real)L.sc->inv_om[sp];
    const Real gx = xp + (p.vel * p.v) * iom;
    const Real gy = yp - (p.vel * p.u) * iom;
    const Real rho = ksqrt_n(gx * gx + gy * gy);
    const Real rl = (p.vel * ksqrt_n(p.u * p.u + p.v * p.v)) * kfabs(iom);
    p.x = gx;
    p.y = gy;
    p.s_path = (Real)0;
    const int nir = r_cell(L.rf, J.n_r, rho, p.ir);
    if (at_birth) {
        p.ir = nir;
    } else if (nir != p.ir) {
        flush_time(J, p);
        if (nir > p.ir) {
            for (int f = p.ir + 1; f <= nir; ++f) cross_r(J, L, p, lc, f, 1);
        } else {
            for (int f = p.ir; f > nir; --f) cross_r(J, L, p, lc, f, 0);
        }
        p.ir = nir;
    }
    return rho + rl >= (Real)J.radius;
}

// Rate (m^-1) of process i at interpolation position (k, f) of the energy (eq. 1): the table
// linear over ln E, zero below the threshold, times the target density -- the gas, the partner
// species' field, or the gas twice for three-body reactions, n (n sigma), whose FP32 tables
// are stored divided by p2scale to stay in range.
template <typename Real>
__device__ __forceinline__ Real proc_rate(const DevJob& J, const Lds<Real>& L, int i, Real exs, int k,
                                         Real f, Real n_gas, Real n_fld) {
    Real sig = (Real)0;
    if (!(exs < L.eth[i])) {
        const Real* tb = L.xs + (size_t)i * J.n_e;
        sig = tb[k] + f * (tb[k + 1] - tb[k]);
    }
    const int t = L.tgt[i];
    const Real r = ((t == TGT_FIELD) ? n_fld : n_gas) * sig;
    if (__builtin_expect(t == TGT_GAS2, 0)) return (n_gas * r) * (Real)J.p2scale;
    return r;
}

// density of the field that species sp's field processes target, in cell (ir, iz)
template <typename Real>
__device__ __forceinline__ Real field_density(const DevJob& J, const Lds<Real>& L, int sp, int ir, int iz) {
    const int fo = L.sc->field_of[sp];
    if (fo < 0) return (Real)0;
    return (Real)L.sc->field[fo][(size_t)ir * J.n_z + (size_t)iz];
}

// ---------------------------------------------------------------- kinematics
template <typename Real>
__device__ __forceinline__ void rotate(Real u, Real v, Real w, Real mu, Real phi, Real out[3]) {
    const Real s = ksqrt_n(kfmax((Real)0, (Real)1 - mu * mu));
    Real sp, cp;
    ksincos(phi, &sp, &cp);
    Real a, b, c;
    if (kfabs(w) < (Real)1 - (Real)1e-10) {
        const Real t = ksqrt_n((Real)1 - w * w);
        const Real it = kdiv((Real)1, t);   // t >= 1.4e-5
        a = mu * u + s * (u * w * cp - v * sp) * it;
        b = mu * v + s * (v * w * cp + u * sp) * it;
        c = mu * w - s * t * cp;
    } else {
        a = s * cp;
        b = s * sp;
        c = (w > (Real)0) ? mu : -mu;
    }
    const Real in = kdiv((Real)1, ksqrt_n(a * a + b * b + c * c));   // a unit vector's norm
    out[0] = a * in;
    out[1] = b * in;
    out[2] = c * in;
}

// thermal target velocity from two Box-Muller slots
template <typename Real>
__device__ void thermal(const DevJob& J, const Part<Real>& p, uint32_t sa, uint32_t sb, Real V[3]) {
    const Real sv = (Real)J.sigma_v;
    if (!(sv > (Real)0)) {
        V[0] = V[1] = V[2] = (Real)0;
        return;
    }
    const Pair<Real> a = draw<Real>(J.seed, p.pid, p.lin, p.s, sa);
    const Pair<Real> b = draw<Real>(J.seed, p.pid, p.lin, p.s, sb);
    const Real r1 = ksqrt_n((Real)-2 * klog(a.d0 + Prec<Real>::eps));
    const Real r2 = ksqrt_n((Real)-2 * klog(b.d0 + Prec<Real>::eps));
    const Real a1 = (Real)kTWO_PI * a.d1;
    const Real a2 = (Real)kTWO_PI * b.d1;
    Real s1, c1, s2, c2;
    ksincos(a1, &s1, &c1);
    ksincos(a2, &s2, &c2);
    V[0] = sv * (r1 * c1);
    V[1] = sv * (r1 * s1);
    V[2] = sv * (r2 * c2);
}

template <typename Real>
__device__ __forceinline__ void set_velocity(Part<Real>& p, Real e_from_v2, const Real vv[3]) {
    const Real v2 = vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2];
    p.e = v2 * e_from_v2;
    p.vel = ksqrt_n(v2);
    if (p.vel > (Real)0) {
        const Real iv = kdiv((Real)1, p.vel);
        p.u = vv[0] * iv;
        p.v = vv[1] * iv;
        p.w = vv[2] * iv;
    }
}

// Cosine of the centre-of-mass scattering angle (Sec. 3.3 "Elastic scattering"): isotropic
// without a table or below the composite threshold, else from the piecewise linear density of
// the impact-energy bin: the interval is the last whose cumulative area is <= u times the
// total, and inside it f0 x + (s/2) x^2 = r is solved as x = 2 r / (f0 + sqrt(f0^2 + 2 s r)).
// The table arithmetic is FP64 in both precisions.
template <typename Real>
__device__ Real scatter_mu(const DevJob& J, int pi, Real ecm, Real u) {
    const int nb = J.ang_nb[pi];
    if (nb <= 0 || ecm < (Real)J.e_iso[pi]) return (Real)2 * u - (Real)1;
    const int n = J.ang_n[pi];
    const double* e = J.ang[pi];
    const double* th = e + nb + 1;
    int b = 0;
    while (b < nb - 1 && (double)ecm >= e[b + 1]) ++b;
    const double* c = th + n + (size_t)b * n;
    const double* f = th + n + (size_t)nb * n + (size_t)b * n;
    const double a = (double)u * c[n - 1];
    int lo = 0, hi = n - 2;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (c[mid] <= a) lo = mid;
        else hi = mid - 1;
    }
    const double h = th[lo + 1] - th[lo];
    const double r = a - c[lo];
    const double s = (f[lo + 1] - f[lo]) / h;
    const double den = f[lo] + ksqrt(f[lo] * f[lo] + 2.0 * s * r);
    double x = (r > 0.0 && den > 0.0) ? 2.0 * r / den : 0.0;
    if (x > h) x = h;
    double sn, cs;
    ksincos(th[lo] + x, &sn, &cs);
    return (Real)cs;
}

// V: the target particle's velocity (thermal(), slots 2 and 3 of the step)
template <typename Real>
__device__ double k_elastic(const DevJob& J, const Lds<Real>& L, Part<Real>& p, int pi, Vec3<Real> tv,
                            int s) {
    const Real V[3] = {tv.x, tv.y, tv.z};
    const Real v[3] = {p.vel * p.u, p.vel * p.v, p.vel * p.w};
    const Real g[3] = {v[0] - V[0], v[1] - V[1], v[2] - V[2]};
    const Real gm = ksqrt_n(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    Real gh[3] = {(Real)0, (Real)0, (Real)1};
    if (gm > (Real)0) {
        const Real ig = kdiv((Real)1, gm);
        gh[0] = g[0] * ig;
        gh[1] = g[1] * ig;
        gh[2] = g[2] * ig;
    }
    // centre-of-mass velocity (m v + M V)/(m + M)
    const Real mf = (Real)L.sc->mfrac[s];
    const Real gf = (Real)L.sc->gfrac[s];
    const Real cm[3] = {mf * v[0] + gf * V[0], mf * v[1] + gf * V[1], mf * v[2] + gf * V[2]};
    const Pair<Real> q = draw<Real>(J.seed, p.pid, p.lin, p.s, 1u);
    // the impact energy in the centre-of-mass frame selects the angle distribution
    const Real ecm = (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) * (Real)L.sc->e_from_v2[s] * gf;
    const Real mu = scatter_mu(J, pi, ecm, q.d0);
    const Real phi = (Real)kTWO_PI * q.d1;
    Real gn[3];
    rotate(gh[0], gh[1], gh[2], mu, phi, gn);
    const Real a = gf * gm;
    const Real vn[3] = {cm[0] + a * gn[0], cm[1] + a * gn[1], cm[2] + a * gn[2]};
    const Real e0 = p.e;
    set_velocity(p, (Real)L.sc->e_from_v2[s], vn);
    return (double)(e0 - p.e);
}

// Kim-Rudd BEB secondary-energy distribution (Q = 1) on w = W/B in [0,(t-1)/2]: exact
// rejection from the positive four-term envelope, each term drawn by its closed-form inverse.
template <typename Real>
__device__ Real beb_sample(const DevJob& J, const Part<Real>& p, Real t, uint32_t* tries) {
    if (!(t > (Real)1)) return (Real)0;
    const Real tp1 = t + (Real)1;
    const Real lt = klog(t);
    const Real a4 = (Real)4 / (tp1 * tp1);
    const Real it2 = (Real)1 / (t * t);
    const Real i1 = (t - (Real)1) / tp1;
    const Real i2 = (t - (Real)1) / (t * tp1);
    const Real i3 = (Real)0.5 * lt * ((Real)1 - a4);
    const Real i4 = (Real)0.5 * lt * (a4 - it2);
    const Real c1 = i1, c2 = c1 + i2, c3 = c2 + i3, tot = c3 + i4;
    const Real wmax = (Real)0.5 * (t - (Real)1);
    Real w = (Real)0;
    for (uint32_t k = 0; k < 64u; ++k) {
        const Pair<Real> a = draw<Real>(J.seed, p.pid, p.lin, p.s, 8u + 2u * k);
        const Pair<Real> b = draw<Real>(J.seed, p.pid, p.lin, p.s, 9u + 2u * k);
        const Real pick = a.d0 * tot;
        const Real u = a.d1;
        if (pick < c1) w = (Real)1 / ((Real)1 - u * ((Real)1 - (Real)2 / tp1)) - (Real)1;
        else if (pick < c2) w = t - (Real)1 / ((Real)1 / t + u * ((Real)2 / tp1 - (Real)1 / t));
        else if (pick < c3) w = (Real)1 / ksqrt((Real)1 - u * ((Real)1 - a4)) - (Real)1;
        else w = t - (Real)1 / ksqrt(it2 + u * (a4 - it2));
        if (w < (Real)0) w = (Real)0;
        if (w > wmax) w = wmax;
        const Real x1 = (Real)1 / (w + (Real)1), x2 = (Real)1 / (t - w);
        const Real env = x1 * x1 + x2 * x2 + lt * (x1 * x1 * x1 + x2 * x2 * x2);
        const Real g = env - (x1 + x2) / tp1;
        *tries += 1u;
        if (b.d0 * env < g) return w;
    }
    return w;
}

// allowed beta shape (nonrelativistic Fermi function, massless neutrino)
template <typename Real>
__device__ __forceinline__ Real beta_shape(Real e, Real e0, Real z) {
    if (!(e > (Real)0) || !(e < e0)) return (Real)0;
    const Real wt = e + (Real)kMEC2;
    const Real pm = ksqrt(e * (e + (Real)2 * (Real)kMEC2));
    const Real y = (Real)kTWO_PI * (Real)kALPHA * z * wt / pm;
    const Real q = e0 - e;
    return ((Real)kTWO_PI * (Real)kALPHA * z * wt / ((Real)1 - kexp(-y))) * wt * q * q;
}

// ---------------------------------------------------------------- queue
template <typename Real>
__device__ __forceinline__ void queue_write(const QueueSoA& q, unsigned long long i, Real x, Real y,
                                           Real z, const Real d[3], Real e,
                                           unsigned long long lin, uint32_t pid, uint32_t meta,
                                           uint32_t job) {
    q.x[i] = (double)x;
    q.y[i] = (double)y;
    q.z[i] = (double)z;
    q.u[i] = (double)d[0];
    q.v[i] = (double)d[1];
    q.w[i] = (double)d[2];
    q.e[i] = (double)e;
    q.lin[i] = lin;
    q.pid[i] = pid;
    q.meta[i] = meta;
    q.job[i] = job;
}

__device__ __forceinline__ uint32_t pack_meta(int sp, int ir, int iz) {
    return (uint32_t)sp | ((uint32_t)ir << 2) | ((uint32_t)iz << 13);
}

// Queue slot of a product of species q for the lanes with `want`: the deferred queue for
// species that make no products of their own, else the next generation's.  Both reservations
// are wave-wide, so lanes may differ in q.
template <typename Real>
__device__ __forceinline__ unsigned long long reserve_product(const Lds<Real>& L, const GenArgs& G, int q,
                                                              bool want, bool* deferred) {
    const bool dq = L.sc->defer[q] != 0;
    const unsigned long long sd = wave_reserve(G.qdef_count, want && dq);
    const unsigned long long so = wave_reserve(G.qout_count, want && !dq);
    *deferred = dq;
    return dq ? sd : so;
}

// A product that is never transported (untracked species, or born below the cutoff) is
// counted, logged and deleted at once, exactly as its birth would do.
template <typename Real>
__device__ void product_inline(const DevJob& J, const Lds<Real>& L, int sp, Real e,
                               unsigned long long lin, uint32_t pid, int ir, int iz, int reason) {
    atomicAdd(&L.cnt[KARL_C_BIRTH + sp], 1ull);
    atomicAdd(&L.cnt[KARL_C_DEATH + sp * KARL_NREASON + reason], 1ull);
    atomicAdd(&L.led[KARL_L_E_DEATH + sp * KARL_NREASON + reason], (double)e);
    if (J.flags & KARL_FLAG_DIGESTS) {
        unsigned long long d = mix64(lin ^ kDIGEST0);
        d = digest_event(d, 0u, 1u, (uint32_t)sp, (uint32_t)(ir * J.n_z + iz));
        d = digest_event(d, 0u, 6u, (uint32_t)reason, 0u);
        add_u64(&J.digests[pid], d);
    }
    if (J.flags & KARL_FLAG_HISTORY) {
        add_f64(&J.hist[(size_t)pid * KARL_NHIST + 1], (double)e);
        add_f64(&J.hist[(size_t)pid * KARL_NHIST + 2], 1.0);
        add_f64(&J.hist[(size_t)pid * KARL_NHIST + 3], 1.0);
    }
}

template <typename Real, typename LC>
__device__ void k_ionization(const DevJob& J, const Lds<Real>& L, const GenArgs& G, Part<Real>& p,
                             int pi, Real xc, Real yc, LC& lc, Vec3<Real> tv, int sp) {
    const Real ef2 = (Real)L.sc->e_from_v2[sp];
    const Real v2e = (Real)L.sc->v2_from_e[sp];
    const Real B = L.eth[pi];
    const Real v[3] = {p.vel * p.u, p.vel * p.v, p.vel * p.w};
    Real V[3] = {tv.x, tv.y, tv.z}, g[3];
    g[0] = v[0] - V[0];
    g[1] = v[1] - V[1];
    g[2] = v[2] - V[2];
    Real er = (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) * ef2;
    for (uint32_t r = 1; er < B && r <= 15u; ++r) {
        count_n(L, lc.redraw, KARL_C_TARGET_REDRAW, 1u);
        thermal(J, p, 136u + 2u * r, 137u + 2u * r, V);
        g[0] = v[0] - V[0];
        g[1] = v[1] - V[1];
        g[2] = v[2] - V[2];
        er = (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) * ef2;
    }
    if (er < B) {
        V[0] = V[1] = V[2] = (Real)0;
        g[0] = v[0];
        g[1] = v[1];
        g[2] = v[2];
        er = (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) * ef2;
    }
    const Real t = er / B;
    uint32_t tries = 0u;
    const Real w = beb_sample(J, p, t, &tries);
    count_n(L, lc.beb, KARL_C_BEB_TRIES, tries);
    const Real W = w * B;
    Real ef = er - B - W;
    if (ef < (Real)0) ef = (Real)0;
    const Real den = er - B;
    Real ctf = (Real)1, cts = (Real)0;
    if (den > (Real)0) {
        ctf = ksqrt(ef / den);
        cts = ksqrt(W / den);
    }
    const Real gm = ksqrt_n(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    Real gh[3] = {(Real)0, (Real)0, (Real)1};
    if (gm > (Real)0) {
        const Real ig = kdiv((Real)1, gm);
        gh[0] = g[0] * ig;
        gh[1] = g[1] * ig;
        gh[2] = g[2] * ig;
    }
    const Pair<Real> q = draw<Real>(J.seed, p.pid, p.lin, p.s, 1u);
    const Real phi = (Real)kTWO_PI * q.d1;
    const Real phis = phi - (Real)kPI;
    Real df[3], ds[3];
    rotate(gh[0], gh[1], gh[2], ctf, phi, df);
    rotate(gh[0], gh[1], gh[2], cts, phis, ds);
    const Real sf = ksqrt(ef * v2e);
    const Real ss = ksqrt(W * v2e);
    const Real vf[3] = {V[0] + sf * df[0], V[1] + sf * df[1], V[2] + sf * df[2]};
    const Real vs[3] = {V[0] + ss * ds[0], V[1] + ss * ds[1], V[2] + ss * ds[2]};
    const Real es = (vs[0] * vs[0] + vs[1] * vs[1] + vs[2] * vs[2]) * ef2;
    const int qi = J.product[pi];   // the ion species made (molecular, or atomic if dissociative)
    const Real eion = (V[0] * V[0] + V[1] * V[1] + V[2] * V[2]) * (Real)L.sc->e_from_v2[qi];
    const Real e0 = p.e;
    set_velocity(p, ef2, vf);
    p.e_bind += (double)B;
    p.e_gas += (double)(e0 - (p.e + es + eion + B));

    // products: slow electron (slot 0) and ion (slot qi), born at the collision point
    const unsigned long long lin_e = child_lineage(p.lin, p.s, 0u);
    const unsigned long long lin_i = child_lineage(p.lin, p.s, 1u);
    Real de[3] = {(Real)0, (Real)0, (Real)1};
    const Real vsm = ksqrt(vs[0] * vs[0] + vs[1] * vs[1] + vs[2] * vs[2]);
    if (vsm > (Real)0) {
        const Real iv = (Real)1 / vsm;
        de[0] = vs[0] * iv;
        de[1] = vs[1] * iv;
        de[2] = vs[2] * iv;
    }
    Real di[3] = {(Real)0, (Real)0, (Real)1};
    const Real Vm = ksqrt(V[0] * V[0] + V[1] * V[1] + V[2] * V[2]);
    if (Vm > (Real)0) {
        const Real iv = (Real)1 / Vm;
        di[0] = V[0] * iv;
        di[1] = V[1] * iv;
        di[2] = V[2] * iv;
    }
    bool push_e = true, push_i = true;
    if (!J.sc.tracked[0]) {
        product_inline(J, L, 0, es, lin_e, p.pid, p.ir, p.iz, KARL_UNTRACKED);
        push_e = false;
    } else if (es < (Real)J.sc.e_cut[0]) {
        product_inline(J, L, 0, es, lin_e, p.pid, p.ir, p.iz, KARL_CUTOFF);
        push_e = false;
    }
    if (!L.sc->tracked[qi]) {
        product_inline(J, L, qi, eion, lin_i, p.pid, p.ir, p.iz, KARL_UNTRACKED);
        push_i = false;
    } else if (eion < (Real)L.sc->e_cut[qi]) {
        product_inline(J, L, qi, eion, lin_i, p.pid, p.ir, p.iz, KARL_CUTOFF);
        push_i = false;
    }
    // the electron's destination is uniform (slot 0); the ion's follows its species
    const QueueSoA& qe = J.sc.defer[0] ? G.qdef : G.qout;
    const unsigned long long se = wave_reserve(J.sc.defer[0] ? G.qdef_count : G.qout_count, push_e);
    bool di_def;
    const unsigned long long si = reserve_product(L, G, qi, push_i, &di_def);
    const unsigned long long cap = (unsigned long long)G.capacity;
    if (push_e) {
        if (se < cap) queue_write(qe, se, xc, yc, p.z, de, es, lin_e, p.pid, pack_meta(0, p.ir, p.iz), (uint32_t)p.job);
        else atomicOr(G.status, STATUS_OVERFLOW);
    }
    if (push_i) {
        if (si < cap) queue_write(di_def ? G.qdef : G.qout, si, xc, yc, p.z, di, eion, lin_i, p.pid,
                                  pack_meta(qi, p.ir, p.iz), (uint32_t)p.job);
        else atomicOr(G.status, STATUS_OVERFLOW);
    }
}

// Clustering (Sec. 3.3 "Clustering"): a target particle's velocity V is drawn as for elastic
// scattering and the product (species product[pi]) moves along it with the target particle's
// momentum, |v'| = (M/m')|V|.  The projectile is deleted ("converted"); the product is a new
// particle at the collision point whose energy comes from the gas.
template <typename Real>
__device__ void k_clustering(const DevJob& J, const Lds<Real>& L, const GenArgs& G, Part<Real>& p,
                             int pi, Real xc, Real yc, Vec3<Real> tv) {
    const Real V[3] = {tv.x, tv.y, tv.z};
    const int q = J.product[pi];
    const Real sc = (Real)J.conv[pi];
    const Real vn[3] = {sc * V[0], sc * V[1], sc * V[2]};
    const Real vm = ksqrt(vn[0] * vn[0] + vn[1] * vn[1] + vn[2] * vn[2]);
    Real dn[3] = {(Real)0, (Real)0, (Real)1};
    if (vm > (Real)0) {
        const Real iv = (Real)1 / vm;
        dn[0] = vn[0] * iv;
        dn[1] = vn[1] * iv;
        dn[2] = vn[2] * iv;
    }
    const Real ep = (vn[0] * vn[0] + vn[1] * vn[1] + vn[2] * vn[2]) * (Real)L.sc->e_from_v2[q];
    const unsigned long long lin = child_lineage(p.lin, p.s, 0u);
    const int ir = p.ir, iz = p.iz;
    const Real z = p.z;
    p.e_gas -= (double)ep;
    kill(J, L, p, KARL_CONVERTED);
    bool push = true;
    if (!L.sc->tracked[q]) {
        product_inline(J, L, q, ep, lin, p.pid, ir, iz, KARL_UNTRACKED);
        push = false;
    } else if (ep < (Real)L.sc->e_cut[q]) {
        product_inline(J, L, q, ep, lin, p.pid, ir, iz, KARL_CUTOFF);
        push = false;
    }
    bool dq;
    const unsigned long long si = reserve_product(L, G, q, push, &dq);
    if (push) {
        if (si < (unsigned long long)G.capacity)
            queue_write(dq ? G.qdef : G.qout, si, xc, yc, z, dn, ep, lin, p.pid, pack_meta(q, ir, iz),
                        (uint32_t)p.job);
        else atomicOr(G.status, STATUS_OVERFLOW);
    }
}

// Charge exchange (Sec. 3.3): the projectile continues with the velocity of a target particle,
// drawn as for elastic scattering.
template <typename Real>
__device__ double k_charge_exchange(const DevJob& J, const Lds<Real>& L, Part<Real>& p, Vec3<Real> tv,
                                    int sp) {
    const Real V[3] = {tv.x, tv.y, tv.z};
    const Real e0 = p.e;
    set_velocity(p, (Real)L.sc->e_from_v2[sp], V);
    return (double)(e0 - p.e);
}

// ---------------------------------------------------------------- birth (Sec. 3.5)
template <typename Real, typename LC>
__device__ __forceinline__ void birth(const DevJob& J, const Lds<Real>& L, uint32_t pid, Part<Real>& p,
                      LC& lc) {
    p.lin = 0ull;
    p.pid = pid;
    if (J.source == KARL_SOURCE_BEAM || J.source == KARL_SOURCE_PAIR) {
        p.sp = J.beam_species;
        p.e = (Real)J.beam_e;
        if (J.source == KARL_SOURCE_PAIR) {
            p.sp = (int32_t)(pid & 1u);
            p.e = (Real)(p.sp ? J.beam_e1 : J.beam_e);
        }
        p.x = (Real)J.beam_pos[0];
        p.y = (Real)J.beam_pos[1];
        p.z = (Real)J.beam_pos[2];
        p.u = (Real)J.beam_dir[0];
        p.v = (Real)J.beam_dir[1];
        p.w = (Real)J.beam_dir[2];
        p.ir = J.beam_ir;
        p.iz = J.beam_iz;
        return;
    }
    p.sp = 0;
    const Pair<Real> q0 = draw<Real>(J.seed, pid, 0ull, kBIRTH_STEP, 0u);
    const Pair<Real> q1 = draw<Real>(J.seed, pid, 0ull, kBIRTH_STEP, 1u);
    const Pair<Real> q2 = draw<Real>(J.seed, pid, 0ull, kBIRTH_STEP, 2u);
    const Real* zcdf = (const Real*)J.zcdf;
    const Real wsum = zcdf[J.n_z];
    int k;
    Real z;
    if (wsum > (Real)0) {
        const Real tt = q0.d0 * wsum;
        // first k with tt < zcdf[k+1]
        int lo = 0, hi = J.n_z;   // answer in [lo, hi]; hi = n_z means none
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (tt < zcdf[mid + 1]) hi = mid;
            else lo = mid + 1;
        }
        k = lo;
        if (k >= J.n_z) {
            k = J.n_z - 1;
            while (k > 0 && !(L.ngas[k] > (Real)0)) --k;
        }
        z = L.zf[k] + ((tt - zcdf[k]) / L.ngas[k]) * ((Real)J.length / (Real)J.n_z);
    } else {
        z = q0.d0 * (Real)J.length;
        int kk = 0;
        for (int j = 1; j < J.n_z; ++j)
            if (L.zf[j] <= z) kk = j;
        k = kk;
    }
    const Real r = (Real)J.radius * ksqrt(q0.d1);
    const Real al = (Real)kTWO_PI * q1.d0;
    const Real mu = (Real)2 * q1.d1 - (Real)1;
    const Real ph = (Real)kTWO_PI * q2.d0;
    const Real st = ksqrt(kfmax((Real)0, (Real)1 - mu * mu));
    Real sa, ca, sph, cph;
    ksincos(al, &sa, &ca);
    ksincos(ph, &sph, &cph);
    p.x = r * ca;
    p.y = r * sa;
    p.z = z;
    p.u = st * cph;
    p.v = st * sph;
    p.w = mu;
    p.iz = k;
    p.ir = r_cell(L.rf, J.n_r, r, 0);
    Real e = (Real)0;
    const Real e0 = (Real)J.beta_e0, bz = (Real)J.beta_z, fmax_ = (Real)J.beta_fmax;
    for (uint32_t j = 0; j < 64u; ++j) {
        const Pair<Real> q = draw<Real>(J.seed, pid, 0ull, kBIRTH_STEP, 3u + j);
        e = e0 * (q.d0 + Prec<Real>::eps);
        count_n(L, lc.beta, KARL_C_BETA_TRIES, 1u);
        if (q.d1 * fmax_ < beta_shape(e, e0, bz)) break;
    }
    p.e = e;
}

// common start of every particle (primary or secondary); returns with p.alive set
template <typename Real, typename LC>
__device__ __forceinline__ void start_particle(const DevJob& J, const Lds<Real>& L, Part<Real>& p, LC& lc) {
    const bool dig = (J.flags & KARL_FLAG_DIGESTS) != 0;
    p.s = 0u;
    p.n_int = 0;
    p.t_alive = 0.0;
    p.t_cell = 0.0;
    p.e_exc = p.e_bind = p.e_gas = 0.0;
    p.s_path = (Real)0;
    p.alive = true;
    p.fly = false;
    p.vel = (p.e > (Real)0) ? ksqrt(p.e * (Real)L.sc->v2_from_e[p.sp]) : (Real)0;
    p.dg = mix64(p.lin ^ kDIGEST0);
    atomicAdd(&L.cnt[KARL_C_BIRTH + p.sp], 1ull);
    if (J.flags & KARL_FLAG_HISTORY) add_f64(&J.hist[(size_t)p.pid * KARL_NHIST + 2], 1.0);
    ev(p, 1u, (uint32_t)p.sp, (uint32_t)(p.ir * J.n_z + p.iz), dig);
    if (!L.sc->tracked[p.sp]) { kill(J, L, p, KARL_UNTRACKED); return; }
    if (p.e < (Real)L.sc->e_cut[p.sp]) { kill(J, L, p, KARL_CUTOFF); return; }
    if (!(p.vel > (Real)0)) { kill(J, L, p, KARL_LIFETIME); return; }
    if (J.gc) {
        if (gc_set(J, L, p, lc, p.x, p.y, true, p.sp)) {
            cross_r(J, L, p, lc, J.n_r, 1);
            kill(J, L, p, KARL_WALL);
        }
    }
}

// energy-resolved density field (Sec. 3.4): a flight segment's time in the bin of the energy
// the particle flies with (bin 0 below the first edge, n_dens_bins+1 at or above the last)
__device__ __forceinline__ void add_dense(const DevJob& J, int sp, int ir, int iz, double e, double dt) {
    const int nb = J.n_dens_bins;
    const double* ed = J.dens_edges + (size_t)sp * (nb + 1);
    int bin;
    if (e < ed[0]) {
        bin = 0;
    } else if (!(e < ed[nb])) {
        bin = nb + 1;
    } else {
        int lo = 0, hi = nb;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (ed[mid] <= e) lo = mid;
            else hi = mid;
        }
        bin = lo + 1;
    }
    add_f64(&J.dense[(((size_t)sp * J.n_r + (size_t)ir) * J.n_z + (size_t)iz) * (size_t)(nb + 2) + (size_t)bin], dt);
}

// energy bin of a plane spectrum: 0 below the first edge, n_bins+1 at or above the last
__device__ __forceinline__ int spectrum_bin(const DevJob& J, int sp, double ee) {
    const double* ed = J.edges + (size_t)sp * (J.n_bins + 1);
    if (ee < ed[0]) return 0;
    if (!(ee < ed[J.n_bins])) return J.n_bins + 1;
    int lo = 0, hi = J.n_bins;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ed[mid] <= ee) lo = mid;
        else hi = mid;
    }
    return lo + 1;
}

// crossing of z-face f in direction dir (1: +z) in the particle's ring: current collector and
// spectrum plane (Sec. 2.3, 3.4)
template <typename Real, typename LC>
__device__ __forceinline__ void cross_z(const DevJob& J, const Lds<Real>& L, Part<Real>& p, LC& lc,
                                        int f, int dir, int sp) {
    const bool dig = (J.flags & KARL_FLAG_DIGESTS) != 0;
    count_ev(L, lc, KARL_C_ZCROSS, sp);
    add_u64(&J.jz[(((size_t)sp * J.n_r + (size_t)p.ir) * (J.n_z + 1) + (size_t)f) * 2 + (size_t)dir], 1ull);
    ev(p, 3u, (uint32_t)dir, (uint32_t)(p.ir * (J.n_z + 1) + f), dig);
    const int pl = J.plane_of[f];
    if (pl >= 0) {
        const int bin = spectrum_bin(J, sp, (double)p.e);
        add_u64(&J.spectra[(((size_t)sp * J.n_planes + (size_t)pl) * 2 + (size_t)dir) * (J.n_bins + 2) + (size_t)bin], 1ull);
        ev(p, 5u, (uint32_t)(pl * 2 + dir), (uint32_t)bin, dig);
    }
}

// Counters and digest event of an interaction of process pi.
template <typename Real, typename LC>
__device__ __forceinline__ void count_interaction(const DevJob& J, const Lds<Real>& L, LC& lc,
                                                  Part<Real>& p, int sp, int pi) {
    count_ev(L, lc, KARL_C_COLL, sp);
    if constexpr (kLeanCnt<LC>) count_proc(L.cnt, lc, pi);
    else wave_count(L.cnt, KARL_C_PROC + pi);
    p.n_int += 1;
    ev(p, 2u, (uint32_t)pi, (uint32_t)(p.ir * J.n_z + p.iz), (J.flags & KARL_FLAG_DIGESTS) != 0);
}

// The interaction chosen for process pi (Sec. 2.1, 3.3) at the collision point (xc, yc, p.z),
// after count_interaction: the kinematics of its class and the terminator's checks after it.
template <typename Real, int kDrain, typename LC>
__device__ __forceinline__ void interact(const DevJob& J, const Lds<Real>& L, const GenArgs& G, Part<Real>& p,
                         LC& lc, int sp, int pi, Real xc, Real yc) {
    bool killed = false;
    const int kd = L.kind[pi];
    // every class but excitation and recombination starts from a target particle's velocity
    // (slots 2 and 3 of the step): drawn once here for all of them
    Vec3<Real> tv{(Real)0, (Real)0, (Real)0};
    if (kd != KARL_EXCITATION && kd != KARL_RECOMBINATION) {
        Real V[3];
        thermal(J, p, 2u, 3u, V);
        tv = Vec3<Real>{V[0], V[1], V[2]};
    }
    // energy losses of the collision, added once after it (one update site per ledger keeps
    // the loss accumulators in registers)
    double d_exc = 0.0, d_gas = 0.0;
    switch (kd) {
        case KARL_ELASTIC:
            d_gas = k_elastic(J, L, p, pi, tv, sp);
            break;
        case KARL_EXCITATION: {
            const Real ex = L.eth[pi];
            p.e = p.e - ex;
            p.vel = (p.e > (Real)0) ? ksqrt(p.e * (Real)L.sc->v2_from_e[sp]) : (Real)0;
            d_exc = (double)ex;
            break;
        }
        case KARL_IONIZATION:
            if constexpr (kDrain) {
                // a deferred species makes no products; flag it rather than go on silently
                atomicOr(J.status, STATUS_NUMERIC);
                kill(J, L, p, KARL_LIFETIME);
                killed = true;
            } else {
                k_ionization(J, L, G, p, pi, xc, yc, lc, tv, sp);
            }
            break;
        case KARL_CHARGE_EXCHANGE:
            d_gas = k_charge_exchange(J, L, p, tv, sp);
            break;
        case KARL_CLUSTERING:
            if constexpr (kDrain) {
                atomicOr(J.status, STATUS_NUMERIC);
                kill(J, L, p, KARL_LIFETIME);
            } else {
                k_clustering(J, L, G, p, pi, xc, yc, tv);
            }
            killed = true;
            break;
        default:
            // one deletion logged in the partner's field (Sec. 3.3 "Recombination")
            add_u64(&J.recomb[((size_t)J.partner[pi] * J.n_r + (size_t)p.ir) * J.n_z + (size_t)p.iz], 1ull);
            kill(J, L, p, KARL_RECOMBINED);
            killed = true;
            break;
    }
    if (!killed) {
        p.e_exc += d_exc;
        p.e_gas += d_gas;
        if (p.e < (Real)L.sc->e_cut[sp]) kill(J, L, p, KARL_CUTOFF);
        else if (p.n_int >= L.sc->cap[sp]) kill(J, L, p, KARL_CAP);
        else if (!(p.vel > (Real)0)) kill(J, L, p, KARL_LIFETIME);
        else if (J.gc) {
            if (gc_set(J, L, p, lc, xc, yc, false, sp)) {
                cross_r(J, L, p, lc, J.n_r, 1);
                kill(J, L, p, KARL_WALL);
            }
        }
    }
}

// ---------------------------------------------------------------- Boris mover (Sec. 3.1)
// Field vector of an array over the job's field binning ((r, phi, z) components per (r, z) bin)
// at (x, y, z), in Cartesian components; zero outside the binning.
template <typename Real>
__device__ __forceinline__ void field_at(const DevJob& J, const double* arr, Real x, Real y, Real z,
                                         Real out[3]) {
    out[0] = out[1] = out[2] = (Real)0;
    if (!arr) return;
    const Real r = ksqrt(x * x + y * y);
    if (!(r < (Real)J.field_radius) || !(z >= (Real)0) || !(z < (Real)J.field_length)) return;
    int ir = (int)((r / (Real)J.field_radius) * (Real)J.field_nr);
    int iz = (int)((z / (Real)J.field_length) * (Real)J.field_nz);
    if (ir > J.field_nr - 1) ir = J.field_nr - 1;
    if (iz > J.field_nz - 1) iz = J.field_nz - 1;
    const double* f = arr + ((size_t)ir * J.field_nz + (size_t)iz) * 3;
    Real cp = (Real)1, sn = (Real)0;
    if (r > (Real)0) {
        cp = x / r;
        sn = y / r;
    }
    const Real fr = (Real)f[0], fp = (Real)f[1];
    out[0] = fr * cp - fp * sn;
    out[1] = fr * sn + fp * cp;
    out[2] = (Real)f[2];
}

// One push of time step dt: half an electric kick, the rotation with Omega = h B and
// t = 2 Omega / (1 + Omega.Omega), the second half kick (h = q dt / 2m), then x += v dt.
template <typename Real>
__device__ __forceinline__ void boris_push(const DevJob& J, const Lds<Real>& L, Part<Real>& p, int sp,
                                           Real dt) {
    Real E[3], B[3];
    field_at(J, J.e_fld, p.x, p.y, p.z, E);
    if (J.b_fld) {
        field_at(J, J.b_fld, p.x, p.y, p.z, B);
    } else {
        B[0] = (Real)0;
        B[1] = (Real)0;
        B[2] = (Real)J.bz;
    }
    const Real h = (Real)L.sc->boris_h[sp];
    const Real v[3] = {p.vel * p.u, p.vel * p.v, p.vel * p.w};
    const Real vm[3] = {v[0] + h * E[0], v[1] + h * E[1], v[2] + h * E[2]};
    const Real W[3] = {h * B[0], h * B[1], h * B[2]};
    const Real f = (Real)2 / ((Real)1 + (W[0] * W[0] + W[1] * W[1] + W[2] * W[2]));
    const Real t[3] = {f * W[0], f * W[1], f * W[2]};
    const Real vp[3] = {vm[0] + (vm[1] * W[2] - vm[2] * W[1]),
                        vm[1] + (vm[2] * W[0] - vm[0] * W[2]),
                        vm[2] + (vm[0] * W[1] - vm[1] * W[0])};
    const Real vq[3] = {vm[0] + (vp[1] * t[2] - vp[2] * t[1]),
                        vm[1] + (vp[2] * t[0] - vp[0] * t[2]),
                        vm[2] + (vp[0] * t[1] - vp[1] * t[0])};
    const Real vn[3] = {vq[0] + h * E[0], vq[1] + h * E[1], vq[2] + h * E[2]};
    p.x = p.x + vn[0] * dt;
    p.y = p.y + vn[1] * dt;
    p.z = p.z + vn[2] * dt;
    set_velocity(p, (Real)L.sc->e_from_v2[sp], vn);
}

// energy bin of the energy-resolved density field (0 below the first edge, n_dens_bins+1 at or
// above the last)
__device__ __forceinline__ int dense_bin(const DevJob& J, int sp, double e) {
    const int nb = J.n_dens_bins;
    const double* ed = J.dens_edges + (size_t)sp * (nb + 1);
    if (e < ed[0]) return 0;
    if (!(e < ed[nb])) return nb + 1;
    int lo = 0, hi = nb;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ed[mid] <= e) lo = mid;
        else hi = mid;
    }
    return lo + 1;
}

// End of a Boris movement: its time to the segment (and energy bin) it was spent in, the work
// of the electric field on it to the ledger and the history.
template <typename Real>
__device__ __forceinline__ void end_movement(const DevJob& J, const Lds<Real>& L, Part<Real>& p, int sp) {
    if (J.dense && p.t_cell != 0.0)
        add_f64(&J.dense[(((size_t)sp * J.n_r + (size_t)p.ir) * J.n_z + (size_t)p.iz) * (size_t)(J.n_dens_bins + 2) +
                         (size_t)p.eb], p.t_cell);
    flush_time(J, p);
    const double work = (double)p.e - (double)p.e0m;
    if (work != 0.0) {
        atomicAdd(&L.led[KARL_L_E_FIELD], work);
        if (J.flags & KARL_FLAG_HISTORY) add_f64(&J.hist[(size_t)p.pid * KARL_NHIST + 1], -work);
    }
    p.fly = false;
}

// One transport step of the Boris mover: start a movement if none is under way (a distance
// from the mean free path at the current energy and segment, eq. 2), one push, then the stops
// in the order: outside the domain (deletion), another segment or energy bin (no interaction),
// the drawn distance used up (interaction at the current position).  Returns whether an
// interaction is due, with its process in *pi_out.
template <typename Real, typename LC>
__device__ __forceinline__ bool boris_move(const DevJob& J, const Lds<Real>& L, Part<Real>& p,
                                           LC& lc, int sp, int* pi_out) {
    const int32_t* pidx = L.pidx + sp * KARL_MAX_PROC;
    const int np = L.sc->nps[sp];
    if (!p.fly) {
        const Real exs = p.e * (Real)L.sc->gfrac[sp];
        const Real xl = klog(exs * (Real)L.sc->inv_emin[sp]) * (Real)L.sc->inv_dlog[sp];
        int k;
        Real f;
        if (!(xl > (Real)0)) { k = 0; f = (Real)0; }
        else if (xl >= (Real)(J.n_e - 1)) { k = J.n_e - 2; f = (Real)1; }
        else { k = (int)xl; f = xl - (Real)k; }
        const Real n_gas_cell = L.ngas[p.iz];
        const Real n_fld_cell = field_density<Real>(J, L, sp, p.ir, p.iz);
        Real sum = (Real)0;
        for (int j = 0; j < np; ++j) sum += proc_rate(J, L, pidx[j], exs, k, f, n_gas_cell, n_fld_cell);
        const Pair<Real> q0 = draw<Real>(J.seed, p.pid, p.lin, p.s, 0u);
        p.s_path = (sum > (Real)0) ? -klog(q0.d0 + Prec<Real>::eps) / sum : (Real)INFINITY;
        p.fly = true;
        p.e0m = p.e;
        p.eb = J.dense ? dense_bin(J, sp, (double)p.e) : 0;
    }
    const Real dt = (Real)L.sc->boris_dt[sp];
    boris_push(J, L, p, sp, dt);
    p.s_path -= p.vel * dt;
    p.t_cell += (double)dt;
    p.t_alive += (double)dt;
    count_ev(L, lc, KARL_C_STEP, sp);
    const Real r = ksqrt(p.x * p.x + p.y * p.y);
    if (p.z < (Real)0) {
        end_movement(J, L, p, sp);
        for (int fz = p.iz; fz >= 0; --fz) cross_z(J, L, p, lc, fz, 0, sp);
        kill(J, L, p, KARL_EXIT_LOW);
    } else if (!(p.z < (Real)J.length)) {
        end_movement(J, L, p, sp);
        for (int fz = p.iz + 1; fz <= J.n_z; ++fz) cross_z(J, L, p, lc, fz, 1, sp);
        kill(J, L, p, KARL_EXIT_HIGH);
    } else {
        int niz = p.iz;
        while (niz + 1 < J.n_z && L.zf[niz + 1] <= p.z) ++niz;
        while (niz > 0 && !(L.zf[niz] <= p.z)) --niz;
        const int nir = r_cell(L.rf, J.n_r, r, p.ir);
        const bool wall = !(r < (Real)J.radius);
        if (wall || niz != p.iz || nir != p.ir) {
            // another segment: the movement stops without an interaction
            end_movement(J, L, p, sp);
            if (niz > p.iz) {
                for (int fz = p.iz + 1; fz <= niz; ++fz) cross_z(J, L, p, lc, fz, 1, sp);
            } else {
                for (int fz = p.iz; fz > niz; --fz) cross_z(J, L, p, lc, fz, 0, sp);
            }
            p.iz = niz;
            const int rto = wall ? J.n_r : nir;
            if (rto > p.ir) {
                for (int fr = p.ir + 1; fr <= rto; ++fr) cross_r(J, L, p, lc, fr, 1);
            } else {
                for (int fr = p.ir; fr > rto; --fr) cross_r(J, L, p, lc, fr, 0);
            }
            if (wall) kill(J, L, p, KARL_WALL);
            else p.ir = nir;
        } else if (J.dense && dense_bin(J, sp, (double)p.e) != p.eb) {
            // another energy bin: the movement stops without an interaction
            end_movement(J, L, p, sp);
        } else if (p.s_path < (Real)0) {
            // the drawn distance is used up: interaction here, with the rates at the current
            // energy and segment (none if they all vanished on the way)
            end_movement(J, L, p, sp);
            const Real exs = p.e * (Real)L.sc->gfrac[sp];
            const Real xl = klog(exs * (Real)L.sc->inv_emin[sp]) * (Real)L.sc->inv_dlog[sp];
            int k;
            Real f;
            if (!(xl > (Real)0)) { k = 0; f = (Real)0; }
            else if (xl >= (Real)(J.n_e - 1)) { k = J.n_e - 2; f = (Real)1; }
            else { k = (int)xl; f = xl - (Real)k; }
            const Real n_gas_cell = L.ngas[p.iz];
            const Real n_fld_cell = field_density<Real>(J, L, sp, p.ir, p.iz);
            Real sum = (Real)0;
            for (int j = 0; j < np; ++j) sum += proc_rate(J, L, pidx[j], exs, k, f, n_gas_cell, n_fld_cell);
            if (sum > (Real)0) {
                const Real target = draw<Real>(J.seed, p.pid, p.lin, p.s, 0u).d1 * sum;
                Real run = (Real)0;
                int sel = -1, last = -1;
                for (int j = 0; j < np; ++j) {
                    const Real rate = proc_rate(J, L, pidx[j], exs, k, f, n_gas_cell, n_fld_cell);
                    run += rate;
                    if (rate > (Real)0) last = j;
                    if (sel < 0 && target < run) sel = j;
                }
                if (sel < 0) sel = last;
                *pi_out = pidx[sel];
                count_interaction(J, L, lc, p, sp, pidx[sel]);
                return true;
            }
        }
    }
    return false;
}

// ---------------------------------------------------------------- one flight segment
// kDrain: the launch that runs the deferred queue, whose species have no ionization process
// (the job setup defers exactly those); the ionization branch is left out of that kernel.
// kDrain == 1 also leaves out the energy-resolved density tally (jobs without it), 2 keeps it.
template <typename Real, int kDrain = 0, bool kBoris = false, typename LC>
__device__ void step(const DevJob& J, const Lds<Real>& L, const GenArgs& G, Part<Real>& p,
                     LC& lc) {
    // batched launches serve the lanes of a wave by (job, species): the species is uniform and
    // the process metadata below become scalar loads
    const int sp = L.direct ? __builtin_amdgcn_readfirstlane(p.sp) : p.sp;
    bool coll = false;   // an interaction is due: process pi at (xc, yc, p.z)
    int pi = 0;
    Real xc = (Real)0, yc = (Real)0;
    if constexpr (!kBoris) {
        if (J.boris) {
            // a Boris job in a kernel built without the mover: cannot happen (the host picks the
            // kernel by job); flag it rather than move the particle with the wrong mover
            atomicOr(J.status, STATUS_NUMERIC);
            kill(J, L, p, KARL_LIFETIME);
            return;
        }
    }
    if (kBoris && J.boris) {
        coll = boris_move(J, L, p, lc, sp, &pi);
        xc = p.x;
        yc = p.y;
    } else {
    const bool dig = (J.flags & KARL_FLAG_DIGESTS) != 0;
    p.fly = false;
    // cross sections at the current energy, rates in the current cell (eq. 1)
    const Real exs = p.e * (Real)L.sc->gfrac[sp];
    const Real xl = klog(exs * (Real)L.sc->inv_emin[sp]) *
                    (Real)L.sc->inv_dlog[sp];
    int k;
    Real f;
    if (!(xl > (Real)0)) {
        k = 0;
        f = (Real)0;
    } else if (xl >= (Real)(J.n_e - 1)) {
        k = J.n_e - 2;
        f = (Real)1;
    } else {
        k = (int)xl;
        f = xl - (Real)k;
    }
    const Real n_gas_cell = L.ngas[p.iz];
    // density field of the partner species (Sec. 2.2), for processes that target it
    const Real n_fld_cell = field_density<Real>(J, L, sp, p.ir, p.iz);
    const int np = L.sc->nps[sp];
    const int32_t* pidx = L.pidx + sp * KARL_MAX_PROC;
    Real sum = (Real)0;
    for (int j = 0; j < np; ++j) sum += proc_rate(J, L, pidx[j], exs, k, f, n_gas_cell, n_fld_cell);
    const Pair<Real> q0 = draw<Real>(J.seed, p.pid, p.lin, p.s, 0u);
    const Real eta = q0.d0 + Prec<Real>::eps;
    const Real xi = q0.d1;
    const Real inf = (Real)INFINITY;
    const Real dist = (sum > (Real)0) ? -klog(eta) / sum : inf;

    // distance to the next face of the current segment
    Real sg = inf;
    int which = 0;   // 1 z-face, 2 r outer, 3 r inner
    int zface = -1;
    if (p.w > (Real)0) {
        zface = p.iz + 1;
        sg = (L.zf[zface] - p.z) / p.w;
        which = 1;
    } else if (p.w < (Real)0) {
        zface = p.iz;
        sg = (L.zf[zface] - p.z) / p.w;
        which = 1;
    }
    if (sg < (Real)0) sg = (Real)0;
    if (!J.gc) {
        const Real a = p.u * p.u + p.v * p.v;
        if (a > (Real)0) {
            const Real bq = p.x * p.u + p.y * p.v;
            const Real ro = L.rf[p.ir + 1];
            const Real cq = p.x * p.x + p.y * p.y - ro * ro;
            const Real disc = bq * bq - a * cq;
            Real so = (-bq + ksqrt(kfmax(disc, (Real)0))) / a;
            if (so < (Real)0) so = (Real)0;
            if (so < sg) { sg = so; which = 2; }
            if (p.ir > 0 && bq < (Real)0) {
                const Real ri = L.rf[p.ir];
                const Real ci = p.x * p.x + p.y * p.y - ri * ri;
                const Real di = bq * bq - a * ci;
                if (di >= (Real)0) {
                    Real si = (-bq - ksqrt(di)) / a;
                    if (si < (Real)0) si = (Real)0;
                    if (si < sg) { sg = si; which = 3; }
                }
            }
        }
    }
    if (dist == inf && sg == inf) {
        kill(J, L, p, KARL_LIFETIME);
        return;
    }
    if (dist != dist || sum != sum) atomicOr(J.status, STATUS_NUMERIC);

    const Real l = (dist < sg) ? dist : sg;
    const Real dt = kdiv(l, p.vel);   // l >= 0 (+0 at most), a speed
    p.t_cell += (double)dt;
    p.t_alive += (double)dt;
    if (kDrain != 1 && J.dense) add_dense(J, sp, p.ir, p.iz, (double)p.e, (double)dt);
    if (J.gc) {
        p.z += l * p.w;
        p.s_path += l;
    } else {
        p.x += l * p.u;
        p.y += l * p.v;
        p.z += l * p.w;
    }
    count_ev(L, lc, KARL_C_STEP, sp);

    if (dist < sg) {
        // ---- interaction, chosen with weight sigma_i n_i (Sec. 2.1) ----
        const Real target = xi * sum;
        Real run = (Real)0;
        int sel = -1, last = -1;
        for (int j = 0; j < np; ++j) {
            const Real rate = proc_rate(J, L, pidx[j], exs, k, f, n_gas_cell, n_fld_cell);
            run += rate;
            if (rate > (Real)0) last = j;
            if (sel < 0 && target < run) sel = j;
        }
        if (sel < 0) sel = last;
        pi = pidx[sel];
        count_interaction(J, L, lc, p, sp, pi);
        xc = p.x;
        yc = p.y;
        if (J.gc) {
            const Real om = (Real)L.sc->omega[sp];
            const Real iom = (Real)L.sc->inv_om[sp];
            const Real al = -(om * kdiv(p.s_path, p.vel));
            Real sa, ca;
            ksincos(al, &sa, &ca);
            const Real un = ca * p.u - sa * p.v;
            const Real vn = sa * p.u + ca * p.v;
            p.u = un;
            p.v = vn;
            xc = p.x - (p.vel * p.v) * iom;
            yc = p.y + (p.vel * p.u) * iom;
        }
        // kernels without the Boris mover interact here; with it, the two movers share one site
        if constexpr (!kBoris) interact<Real, kDrain>(J, L, G, p, lc, sp, pi, xc, yc);
        else coll = true;
    } else if (which == 1) {
        // ---- z-face: current collector, spectrum plane, exit ----
        const int fz = zface;
        const int dir = (p.w > (Real)0) ? 1 : 0;
        p.z = L.zf[fz];
        flush_time(J, p);
        cross_z(J, L, p, lc, fz, dir, sp);
        if (fz == 0) kill(J, L, p, KARL_EXIT_LOW);
        else if (fz == J.n_z) kill(J, L, p, KARL_EXIT_HIGH);
        else p.iz = dir ? fz : fz - 1;
        p.fly = J.gc != 0;
    } else {
        // ---- r-face (straight-line transport) ----
        const int out = (which == 2);
        const int fr = out ? p.ir + 1 : p.ir;
        const Real rho = ksqrt(p.x * p.x + p.y * p.y);
        if (rho > (Real)0) {
            const Real sc = L.rf[fr] / rho;
            p.x = p.x * sc;
            p.y = p.y * sc;
        }
        flush_time(J, p);
        cross_r(J, L, p, lc, fr, out);
        if (fr == J.n_r) kill(J, L, p, KARL_WALL);
        else p.ir = out ? fr : fr - 1;
    }
    }
    if constexpr (kBoris) {
        if (coll) interact<Real, kDrain>(J, L, G, p, lc, sp, pi, xc, yc);
    }
    p.s += 1u;
    if (p.alive && p.t_alive >= L.sc->lifetime[sp]) {
        if (kBoris && J.boris && p.fly) end_movement(J, L, p, sp);
        kill(J, L, p, KARL_LIFETIME);
    }
}


// ---------------------------------------------------------------- wave-cooperative flight
// Values of lane j (a wave-uniform index) for every lane.
__device__ __forceinline__ int bc_i(int x, int j) { return __builtin_amdgcn_readlane(x, j); }
__device__ __forceinline__ uint32_t bc_u(uint32_t x, int j) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, j);
}
__device__ __forceinline__ unsigned long long bc_u64(unsigned long long x, int j) {
    const uint32_t lo = bc_u((uint32_t)x, j), hi = bc_u((uint32_t)(x >> 32), j);
    return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ double bc_r(double x, int j) {
    return __longlong_as_double((long long)bc_u64((unsigned long long)__double_as_longlong(x), j));
}
__device__ __forceinline__ float bc_r(float x, int j) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), j));
}

// The flight of the particle in lane j, computed by the whole wave (guiding-centre mode, where
// a flight only meets z-faces).  Lane k takes the k-th flight segment from the particle's
// position: its cell, its own free-path draw (step ordinal s+k: the draws are keyed by step,
// so segment k needs nothing from segments before it), the distance to its far face, and
// whether the draw ends inside the segment.  The particle then crosses every face before the
// first segment with an interaction, the tube end, or 64 faces, with the tallies of each
// crossing made by its lane.  Everything a later step reads is accumulated in step order:
// time alive and path length by a wave-uniform loop over the crossed segments, the event
// digest likewise.  The interaction itself is left to the next regular step, which draws the
// same numbers, so results equal those of segment-by-segment transport.
template <typename Real, typename LC>
__device__ __forceinline__ void coop_flight(const DevJob& J, const Lds<Real>& L, const GenArgs& G, Part<Real>& p,
                            LC& lc, int j) {
    const bool dig = (J.flags & KARL_FLAG_DIGESTS) != 0;
    const int k = (int)lane_id();
    const Real z = bc_r(p.z, j), w = bc_r(p.w, j), e = bc_r(p.e, j), vel = bc_r(p.vel, j);
    const int iz = bc_i(p.iz, j), ir = bc_i(p.ir, j), sp = bc_i(p.sp, j);
    const uint32_t s = bc_u(p.s, j), pid = bc_u(p.pid, j);
    const unsigned long long lin = bc_u64(p.lin, j);
    const int dir = (w > (Real)0) ? 1 : 0;
    const int izk = dir ? iz + k : iz - k;
    const bool inside = izk >= 0 && izk < J.n_z;
    const int izc = inside ? izk : iz;              // lanes past the tube end load valid cells
    const int fz = dir ? izc + 1 : izc;             // far face of segment k
    // rates in the segment's cell at the particle's energy (the arithmetic of step())
    const Real exs = e * (Real)L.sc->gfrac[sp];
    const Real xl = klog(exs * (Real)L.sc->inv_emin[sp]) *
                    (Real)L.sc->inv_dlog[sp];
    int kt;
    Real f;
    if (!(xl > (Real)0)) {
        kt = 0;
        f = (Real)0;
    } else if (xl >= (Real)(J.n_e - 1)) {
        kt = J.n_e - 2;
        f = (Real)1;
    } else {
        kt = (int)xl;
        f = xl - (Real)kt;
    }
    const Real n_gas_cell = L.ngas[izc];
    const Real n_fld_cell = field_density<Real>(J, L, sp, ir, izc);
    const int np = L.sc->nps[sp];
    const int32_t* pidx = L.pidx + sp * KARL_MAX_PROC;
    Real sum = (Real)0;
    for (int q = 0; q < np; ++q) sum += proc_rate(J, L, pidx[q], exs, kt, f, n_gas_cell, n_fld_cell);
    const Pair<Real> q0 = draw<Real>(J.seed, pid, lin, s + (uint32_t)k, 0u);
    const Real eta = q0.d0 + Prec<Real>::eps;
    const Real dist = (sum > (Real)0) ? -klog(eta) / sum : (Real)INFINITY;
    const Real zs = (k == 0) ? z : L.zf[dir ? izc : izc + 1];
    Real sg = (L.zf[fz] - zs) / w;
    if (sg < (Real)0) sg = (Real)0;
    const bool coll = inside && (dist < sg);
    const bool at_end = inside && !coll && (fz == 0 || fz == J.n_z);
    const unsigned long long cmask = __ballot(coll), emask = __ballot(at_end);
    const int kc = cmask ? __ffsll((long long)cmask) - 1 : 64;
    const int ke = emask ? __ffsll((long long)emask) - 1 : 64;
    int m = kc;
    if (ke < kc) m = ke + 1;                       // the tube end comes first
    if (m == 0) {
        if (k == j) p.fly = false;
        return;
    }
    if (k == 0 && G.wave_segments) atomicAdd(G.wave_segments, (unsigned long long)m);
    const Real dt = sg / vel;
    // time alive and path length in step order; a step whose time reaches the lifetime ends
    // the flight (the particle is deleted after that crossing)
    double ta = bc_r(p.t_alive, j);
    Real path = bc_r(p.s_path, j);
    const double life = L.sc->lifetime[sp];
    bool life_end = false;
    for (int kk = 0; kk < m; ++kk) {
        ta += (double)bc_r(dt, kk);
        path += bc_r(sg, kk);
        if (kk != ke && ta >= life) {
            m = kk + 1;
            life_end = true;
            break;
        }
    }
    // tallies of the crossed segments, one lane each
    const int bin = spectrum_bin(J, sp, (double)e);
    if (k < m) {
        if (dist != dist || sum != sum) atomicOr(J.status, STATUS_NUMERIC);
        const double tc = (k == 0) ? bc_r(p.t_cell, j) + (double)dt : (double)dt;
        if (tc != 0.0) add_f64(&J.dens[((size_t)sp * J.n_r + (size_t)ir) * J.n_z + (size_t)izk], tc);
        if (J.dense) add_dense(J, sp, ir, izk, (double)e, (double)dt);
        add_u64(&J.jz[(((size_t)sp * J.n_r + (size_t)ir) * (J.n_z + 1) + (size_t)fz) * 2 + (size_t)dir], 1ull);
        const int pl = J.plane_of[fz];
        if (pl >= 0)
            add_u64(&J.spectra[(((size_t)sp * J.n_planes + (size_t)pl) * 2 + (size_t)dir) * (J.n_bins + 2) + (size_t)bin], 1ull);
    }
    unsigned long long dg = bc_u64(p.dg, j);
    if (dig)
        for (int kk = 0; kk < m; ++kk) {
            const int fk = dir ? iz + kk + 1 : iz - kk;
            dg = digest_event(dg, s + (uint32_t)kk, 3u, (uint32_t)dir, (uint32_t)(ir * (J.n_z + 1) + fk));
            const int pl = J.plane_of[fk];
            if (pl >= 0) dg = digest_event(dg, s + (uint32_t)kk, 5u, (uint32_t)(pl * 2 + dir), (uint32_t)bin);
        }
    if (k == j) {
        const int fl = dir ? iz + m : iz - m + 1;  // the last face crossed
        p.z = L.zf[fl];
        p.t_cell = 0.0;
        p.t_alive = ta;
        p.s_path = path;
        p.dg = dg;
        count_evn(L, lc, KARL_C_STEP, sp, (uint32_t)m);
        count_evn(L, lc, KARL_C_ZCROSS, sp, (uint32_t)m);
        if (ke < 64 && m == ke + 1) {
            p.s = s + (uint32_t)(m - 1);
            kill(J, L, p, fl == 0 ? KARL_EXIT_LOW : KARL_EXIT_HIGH);
            p.s += 1u;
        } else {
            p.iz = dir ? fl : fl - 1;
            p.s = s + (uint32_t)m;
            if (life_end) kill(J, L, p, KARL_LIFETIME);
        }
        p.fly = p.alive && m == 64;
    }
}

// ---------------------------------------------------------------- the kernel
template <typename Real> struct EthOf;
template <> struct EthOf<double> {
    static __device__ __forceinline__ const double* get(const DevJob& J) { return J.e_th; }
};
template <> struct EthOf<float> {
    static __device__ __forceinline__ const float* get(const DevJob& J) { return J.e_th_f; }
};

// Tables and counters of a job read directly from HBM (batched launches: the lanes of a
// workgroup may work for different jobs; the tables stay resident in L2).
template <typename Real>
__device__ __forceinline__ Lds<Real> global_view(const DevJob& J, unsigned long long* cnt, double* led) {
    return Lds<Real>{cnt, led, &J.pidx[0][0], J.kind, J.target, EthOf<Real>::get(J),
                     (const Real*)J.xs, (const Real*)J.n_gas, (const Real*)J.zf, (const Real*)J.rf,
                     &J.sc, true};
}

// Per-wave LDS counter slots of batched launches: each wave keeps the counters and ledger of up
// to kSlots jobs (tagged by job index) and adds a slot to its job's tallies in HBM only when the
// slot is reused for another job or at the end of the launch.
constexpr int kSlots = 4;
constexpr int kSlotWords = kNCnt + kNLed;   // counters and ledger entries, 8 bytes each

__device__ __forceinline__ void slot_flush(const DevJob* jobs, int job, unsigned long long* w) {
    // called by one lane
    const DevJob& J = jobs[job];
    for (int i = 0; i < kNCnt; ++i)
        if (w[i]) {
            add_u64(&J.counters[i], w[i]);
            w[i] = 0ull;
        }
    double* d = (double*)(w + kNCnt);
    for (int i = 0; i < kNLed; ++i)
        if (d[i] != 0.0) {
            add_f64(&J.ledger[i], d[i]);
            d[i] = 0.0;
        }
}

// Load a queued particle into the lane.
template <typename Real, bool kBatched>
__device__ __forceinline__ void load_queued(const GenArgs& G, int64_t idx, Part<Real>& p) {
    const uint32_t meta = G.qin.meta[idx];
    p.sp = (int32_t)(meta & 3u);
    p.ir = (int32_t)((meta >> 2) & 0x7FFu);
    p.iz = (int32_t)(meta >> 13);
    p.x = (Real)G.qin.x[idx];
    p.y = (Real)G.qin.y[idx];
    p.z = (Real)G.qin.z[idx];
    p.u = (Real)G.qin.u[idx];
    p.v = (Real)G.qin.v[idx];
    p.w = (Real)G.qin.w[idx];
    p.e = (Real)G.qin.e[idx];
    p.lin = G.qin.lin[idx];
    p.pid = G.qin.pid[idx];
    p.job = kBatched ? (int32_t)G.qin.job[idx] : 0;
}

// Job choice of batched launches (all 64 lanes of the wave active).  A wave starts on the job
// that holds the item at its share of the launch's items, so that waves are spread over the jobs
// in proportion to their work, and a wave whose job has run out moves to the job with the most
// unfetched items per wave already on it; both keep each wave on few jobs.
__device__ __forceinline__ int first_job(const GenArgs& G, int gwave, int n_waves) {
    int j = 0;
    if (lane_id() == 0) {
        const int64_t t = ((2 * (int64_t)gwave + 1) * G.n_items) / (2 * (int64_t)n_waves);
        int lo = 0, hi = G.n_jobs - 1;   // last job with job_cum <= t
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (G.job_cum[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        j = lo;
        atomicAdd(&G.job_waves[j], 1ull);
    }
    return __shfl(j, 0);
}

__device__ __forceinline__ int pick_job(const GenArgs& G, int leave) {
    if (leave >= 0 && lane_id() == 0) atomicSub(&G.job_waves[leave], 1ull);
    double best = -1.0;
    int bj = -1;
    for (int j = (int)lane_id(); j < G.n_jobs; j += 64) {
        const int64_t rem = G.job_count[j] - (int64_t)__atomic_load_n(&G.job_fetch[j], __ATOMIC_RELAXED);
        if (rem > 0) {
            const double w = (double)__atomic_load_n(&G.job_waves[j], __ATOMIC_RELAXED);
            const double score = (double)rem / (1.0 + w);
            if (score > best) {
                best = score;
                bj = j;
            }
        }
    }
    // wave-wide arg-max, ties to the lower job index: every lane ends with the same pair
    for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const int oj = __shfl_xor(bj, off);
        if (ob > best || (ob == best && (unsigned)oj < (unsigned)bj)) {
            best = ob;
            bj = oj;
        }
    }
    if (bj >= 0 && lane_id() == 0) atomicAdd(&G.job_waves[bj], 1ull);
    return bj;
}

// Give every lane with `need` a work item.  Plain launches take the next items of one global
// counter.  Batched launches keep each wave on one job (wjob) and move it to another job only
// when the current one has no items left, so that the lanes of a wave stay on few jobs.
template <typename Real, bool kBatched>
__device__ __forceinline__ void refill(const GenArgs& G, Part<Real>& p, bool need, bool& done,
                                       int& wjob) {
    if (!kBatched) {
        const unsigned long long idx = wave_reserve(G.fetch, need);
        if (!need) return;
        if (idx >= (unsigned long long)G.n_items) {
            done = true;
            return;
        }
        if (G.mode == 0) {
            p.job = 0;
            p.pid = (uint32_t)(G.pid_begin0 + (int64_t)idx);
        } else {
            load_queued<Real, kBatched>(G, (int64_t)idx, p);
        }
        p.start = true;
        return;
    }
    unsigned long long m = __ballot(need);
    while (m) {
        if (wjob < 0) {
            if (need) done = true;
            return;
        }
        const int leader = __ffsll((long long)m) - 1;
        unsigned long long base = 0;
        if ((int)lane_id() == leader) base = atomicAdd(&G.job_fetch[wjob], (unsigned long long)__popcll(m));
        base = __shfl(base, leader);
        const int64_t avail = G.job_count[wjob] - (int64_t)base;
        const int64_t rank = (int64_t)rank_in(m);
        if (need && rank < avail) {
            const int64_t local = (int64_t)base + rank;
            if (G.mode == 0) {
                p.job = wjob;
                p.pid = (uint32_t)(G.job_first[wjob] + local);
            } else {
                load_queued<Real, kBatched>(G, G.job_first[wjob] + local, p);
            }
            p.start = true;
            need = false;
        }
        m = __ballot(need);
        if (m) wjob = pick_job(G, wjob);
    }
}

// One unit of work for a lane: start its fetched particle, or move it by one flight segment.
template <typename Real, int kDrain = 0, bool kBoris = false, typename LC>
__device__ __forceinline__ void advance(const DevJob& J, const Lds<Real>& L, const GenArgs& G,
                                        Part<Real>& p, LC& lc) {
    if (p.start) {
        p.start = false;
        if (!kDrain && G.mode == 0) {
            birth(J, L, p.pid, p, lc);
            if (L.direct) atomicAdd(&L.led[KARL_L_E_PRIMARY], (double)p.e);
            else lc.e_prim += (double)p.e;
            if (J.flags & KARL_FLAG_HISTORY) add_f64(&J.hist[(size_t)p.pid * KARL_NHIST + 0], (double)p.e);
        }
        start_particle(J, L, p, lc);
    } else {
        step<Real, kDrain, kBoris>(J, L, G, p, lc);
    }
}

// ---------------------------------------------------------------- deferred launch in slices
// Issue priority of a wave (0..3; the immediate operand of s_setprio).
__device__ __forceinline__ void set_wave_prio(uint32_t p) {
    switch (p) {
        case 0: __builtin_amdgcn_s_setprio(0); break;
        case 1: __builtin_amdgcn_s_setprio(1); break;
        case 2: __builtin_amdgcn_s_setprio(2); break;
        default: __builtin_amdgcn_s_setprio(3); break;
    }
}

// Every 64 iterations of a transport loop, the wave takes the issue priority (its slot on the
// SIMD + the period of 2^18 ticks of the 100 MHz clock) mod 4.  A SIMD issues from its oldest
// wave first: left alone, the four waves of a SIMD advance at rates of about 1 : 1.5 : 2 : 2.4,
// so that a particle's progress depends on the waves it happened to run on, and a launch ends
// with a tail of particles that ran on slow ones.  The waves resident on a SIMD hold distinct
// slots (HW_ID bits 3:0), so each period gives them distinct priorities, each period another
// order: over a slice every wave runs at about the mean rate.
__device__ __forceinline__ void rotate_prio(uint32_t& iter) {
    if ((++iter & 63u) == 0u) {
        const uint32_t slot = (uint32_t)__builtin_amdgcn_s_getreg((3 << 11) | 4);   // HW_ID[3:0]
        set_wave_prio(((uint32_t)(__builtin_amdgcn_s_memrealtime() >> 18) + slot) & 3u);
    }
}

// The lanes of the deferred launch claim indices of one counter (G.fetch): index u < n_items is
// item u of the deferred queue, u >= n_items the ring entry u - n_items.  A wave claims only
// indices below n_items + ring_tail, i.e. items written before the launch or ring entries whose
// producer already owns the slot, so that a claimed entry is readable a few instructions after
// its producer took it; the lane then checks its flag once per loop iteration and never spins
// (its producer may be another lane of the same wave).  A wave ends when every index is claimed
// and none of its lanes holds a particle: every later ring entry is claimed by the lane that
// wrote it, which looks for work right after.
__device__ __forceinline__ unsigned long long ld_agent(const unsigned long long* a) {
    return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_acquire(const unsigned long long* a) {
    return __hip_atomic_load(a, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(unsigned long long* a, unsigned long long v) {
    __hip_atomic_store(a, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename Real>
__device__ __forceinline__ void ring_write(RingEntry* e, const Part<Real>& p) {
    e->x = (double)p.x;
    e->y = (double)p.y;
    e->z = (double)p.z;
    e->u = (double)p.u;
    e->v = (double)p.v;
    e->w = (double)p.w;
    e->e = (double)p.e;
    e->vel = (double)p.vel;
    e->s_path = (double)p.s_path;
    e->t_alive = p.t_alive;
    e->t_cell = p.t_cell;
    e->e_exc = p.e_exc;
    e->e_bind = p.e_bind;
    e->e_gas = p.e_gas;
    e->lin = p.lin;
    e->dg = p.dg;
    e->pid = p.pid;
    e->s = p.s;
    e->sp = p.sp;
    e->ir = p.ir;
    e->iz = p.iz;
    e->fly = p.fly ? 1 : 0;
    e->n_int = p.n_int;
}

template <typename Real>
__device__ __forceinline__ void ring_read(const RingEntry* e, Part<Real>& p) {
    p.x = (Real)e->x;
    p.y = (Real)e->y;
    p.z = (Real)e->z;
    p.u = (Real)e->u;
    p.v = (Real)e->v;
    p.w = (Real)e->w;
    p.e = (Real)e->e;
    p.vel = (Real)e->vel;
    p.s_path = (Real)e->s_path;
    p.t_alive = e->t_alive;
    p.t_cell = e->t_cell;
    p.e_exc = e->e_exc;
    p.e_bind = e->e_bind;
    p.e_gas = e->e_gas;
    p.lin = e->lin;
    p.dg = e->dg;
    p.pid = e->pid;
    p.s = e->s;
    p.sp = e->sp;
    p.ir = e->ir;
    p.iz = e->iz;
    p.fly = e->fly != 0;
    p.n_int = e->n_int;
    p.job = 0;
}

// Work for the lanes with `need`: 1 some lane got an index, 0 every index is claimed, -1 the
// wave lost every race for the counter this time.
template <typename Real>
__device__ __forceinline__ int claim(const GenArgs& G, Part<Real>& p, bool need, bool& wait) {
    const unsigned long long m = __ballot(need);
    const int leader = __ffsll((long long)m) - 1;
    const unsigned long long k = (unsigned long long)__popcll(m);
    const unsigned long long n = (unsigned long long)G.n_items;
    unsigned long long base = 0, got = 0;
    int res = -1;
    if ((int)lane_id() == leader) {
        for (int t = 0; t < 16; ++t) {
            const unsigned long long h = ld_agent(G.fetch);
            const unsigned long long total = n + (G.slice_mask ? ld_agent(G.ring_tail) : 0ull);
            if (h >= total) {
                res = 0;
                break;
            }
            const unsigned long long take = (total - h < k) ? total - h : k;
            if (atomicCAS(G.fetch, h, h + take) == h) {
                base = h;
                got = take;
                res = 1;
                break;
            }
        }
    }
    res = bc_i(res, leader);
    if (res <= 0) return res;
    base = bc_u64(base, leader);
    got = bc_u64(got, leader);
    const unsigned long long r = (unsigned long long)rank_in(m);
    if (need && r < got) {
        const unsigned long long u = base + r;
        if (u < n) {
            load_queued<Real, false>(G, (int64_t)u, p);
            p.start = true;
        } else {
            p.lin = u - n;   // the claimed ring index, held in the idle lane's lineage word
            wait = true;
        }
    }
    return 1;
}

// A claimed ring entry, once its producer has written it: the lane resumes the particle.
template <typename Real>
__device__ __forceinline__ void take_ring(const GenArgs& G, Part<Real>& p, bool& wait) {
    const unsigned long long i = p.lin;
    const unsigned long long slot = i % (unsigned long long)G.ring_cap;
    if (ld_acquire(&G.ring_flag[slot]) != 2ull * i + 1ull) return;
    ring_read(&G.ring[slot], p);
    st_release(&G.ring_flag[slot], 2ull * i + 2ull);   // read: the slot may take entry i + ring_cap
    p.alive = true;
    p.start = false;
    wait = false;
}

// Particles of the lanes with `want` go to the end of the ring.  A slot is taken only when its
// last entry has been read; a particle that finds its slot still in use, or keeps losing the
// race for the ring's tail, stays on its lane for another slice.
template <typename Real>
__device__ __forceinline__ void ring_put(const GenArgs& G, Part<Real>& p, bool want) {
    const unsigned long long cap = (unsigned long long)G.ring_cap;
    for (int t = 0; t < 16 && __ballot(want); ++t) {
        if (want) {
            const unsigned long long j = ld_agent(G.ring_tail);
            const unsigned long long slot = j % cap;
            const unsigned long long free_mark = (j < cap) ? 0ull : 2ull * (j - cap) + 2ull;
            if (ld_acquire(&G.ring_flag[slot]) != free_mark) {
                if (ld_agent(G.ring_tail) == j) want = false;
            } else if (atomicCAS(G.ring_tail, j, j + 1ull) == j) {
                ring_write(&G.ring[slot], p);
                st_release(&G.ring_flag[slot], 2ull * j + 1ull);
                p.alive = false;
                want = false;
            }
        }
    }
}

// Waves per SIMD a transport kernel is built for (its register budget is 512 / waves).  The
// deferred kernels and the FP32 batched kernels are held to four, the FP64 batched kernels to
// three: the FP32 batched kernel then keeps 17 registers' worth (68 bytes) in scratch and
// measured 13 % faster than at the three waves its 158 registers allow without; the FP64
// batched kernel keeps 148 bytes and measured 17 % faster than at the two waves of its 222
// registers.  The single-job kernels take what their registers give (FP64 plain 3, FP32 plain
// 4; held to four, the FP64 plain kernel keeps 132 bytes and measured slower).
template <typename Real, bool kBatched, int kDrain>
constexpr int kMinWaves = kDrain ? 4 : kBatched ? (sizeof(Real) == 4 ? 4 : 3) : 1;

// The wave's counter slot of job ju: found among the slot tags, or taken over from the least
// recent job (whose counts are flushed to its tallies first).  Called by all active lanes of a
// wave with the same ju.
__device__ __forceinline__ unsigned long long* job_slot(const DevJob* jobs, unsigned long long* wslots,
                                                       volatile int32_t* wtags, int ju) {
    int slot = -1;
    for (int k = 0; k < kSlots; ++k)
        if (wtags[k] == ju) slot = k;
    if (slot < 0) {
        slot = wtags[kSlots];
        const int old = wtags[slot];
        const unsigned long long mine = __ballot(true);
        if ((int)lane_id() == __ffsll((long long)mine) - 1) {
            if (old >= 0) slot_flush(jobs, old, wslots + (size_t)slot * kSlotWords);
            wtags[slot] = ju;
            wtags[kSlots] = (slot + 1) % kSlots;
        }
        __builtin_amdgcn_wave_barrier();
    }
    return wslots + (size_t)slot * kSlotWords;
}

// kBatched = false: one job (jobs[0]); its tables are staged in LDS and its event counters
// reduced in LDS.  kBatched = true: every lane carries a job index; the lanes of a wave are
// served job by job (one pass per distinct job, normally one) so that the job's parameters are
// read with scalar loads.  kCoop (guiding-centre mode): before each step, the flights of
// particles that just crossed a face are advanced by the whole wave (coop_flight) -- in batched
// launches those of the jobs that chose the wave mapping (DevJob::wave).  kDrain
// (one job): the deferred-queue launch, without the birth and ionization code, which leaves
// the kernel half the registers and twice the waves per SIMD (1: without, 2: with the
// energy-resolved density tally).
template <typename Real, bool kBatched, bool kCoop = false, int kDrain = 0, bool kBoris = false>
__global__ __launch_bounds__(kBlock, (kMinWaves<Real, kBatched, kDrain>)) void transport_kernel(
    const DevJob* __restrict__ jobs, const GenArgs G) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int tid = threadIdx.x;
    Lds<Real> L0;
    if (!kBatched) {
        const DevJob& J = jobs[0];
        unsigned long long* s_cnt = (unsigned long long*)lds_raw;
        double* s_led = (double*)(lds_raw + kNCnt * 8);
        int32_t* s_pidx = (int32_t*)(lds_raw + (kNCnt + kNLed) * 8);
        int32_t* s_kind = s_pidx + kS * KARL_MAX_PROC;
        int32_t* s_tgt = s_kind + KARL_MAX_PROC;
        Real* s_eth = (Real*)(s_tgt + KARL_MAX_PROC);
        Real* s_xs = s_eth + KARL_MAX_PROC;
        Real* s_ngas = s_xs + (size_t)J.n_proc * J.n_e;
        Real* s_zf = s_ngas + J.n_z;
        Real* s_rf = s_zf + (J.n_z + 1);
        // species constants after the tables, at an 8-byte aligned offset of the LDS block
        const size_t sc_off = ((size_t)((unsigned char*)(s_rf + (J.n_r + 1)) - lds_raw) + 7) & ~(size_t)7;
        SpeciesConst* s_sc = (SpeciesConst*)(lds_raw + sc_off);
        for (int i = tid; i < kNCnt; i += blockDim.x) s_cnt[i] = 0ull;
        for (int i = tid; i < kNLed; i += blockDim.x) s_led[i] = 0.0;
        for (int i = tid; i < kS * KARL_MAX_PROC; i += blockDim.x) s_pidx[i] = J.pidx[i / KARL_MAX_PROC][i % KARL_MAX_PROC];
        for (int i = tid; i < KARL_MAX_PROC; i += blockDim.x) {
            s_kind[i] = J.kind[i];
            s_tgt[i] = J.target[i];
            s_eth[i] = (Real)J.e_th[i];
        }
        const Real* g_xs = (const Real*)J.xs;
        for (int i = tid; i < J.n_proc * J.n_e; i += blockDim.x) s_xs[i] = g_xs[i];
        const Real* g_ngas = (const Real*)J.n_gas;
        for (int i = tid; i < J.n_z; i += blockDim.x) s_ngas[i] = g_ngas[i];
        const Real* g_zf = (const Real*)J.zf;
        for (int i = tid; i <= J.n_z; i += blockDim.x) s_zf[i] = g_zf[i];
        const Real* g_rf = (const Real*)J.rf;
        for (int i = tid; i <= J.n_r; i += blockDim.x) s_rf[i] = g_rf[i];
        static_assert(sizeof(SpeciesConst) % 8 == 0, "species constants copied in 8-byte words");
        const unsigned long long* g_sc = (const unsigned long long*)&J.sc;
        for (int i = tid; i < (int)(sizeof(SpeciesConst) / 8); i += blockDim.x)
            ((unsigned long long*)s_sc)[i] = g_sc[i];
#ifdef KARL_DRAIN_UNIT
        for (int i = tid; i < kNSeries; i += blockDim.x) s_series[i] = kSeriesTab[i];
#endif
        __syncthreads();
        L0 = Lds<Real>{s_cnt, s_led, s_pidx, s_kind, s_tgt, s_eth, s_xs, s_ngas, s_zf, s_rf, s_sc, false};
    }

    // batched: this wave's counter slots and their job tags
    const int wid = tid >> 6;
    unsigned long long* wslots = (unsigned long long*)lds_raw + (size_t)wid * kSlots * kSlotWords;
    // per wave: kSlots job tags, then the index of the next slot to take over; kept in LDS so
    // that every lane of the wave sees the same values whichever lanes ran the last pass
    volatile int32_t* wtags =
        (volatile int32_t*)((unsigned long long*)lds_raw + (size_t)(kBlock / 64) * kSlots * kSlotWords) +
        wid * (kSlots + 1);
    if (kBatched) {
        for (int i = (tid & 63); i < kSlots * kSlotWords; i += 64) wslots[i] = 0ull;
        if ((tid & 63) < kSlots) wtags[tid & 63] = -1;
        if ((tid & 63) == kSlots) wtags[kSlots] = 0;
        __builtin_amdgcn_wave_barrier();
    }

    typename PickT<kDrain != 0, LaneCntLean, LaneCnt>::type lc{};
    Part<Real> p;
    p.alive = false;
    p.start = false;
    p.job = 0;
    bool done = false;
    // batched: the wave's current job, first spread over the jobs by wave index
    int wjob = 0;
    if (kBatched) wjob = first_job(G, (int)(blockIdx.x * (kBlock / 64) + wid), (int)(gridDim.x * (kBlock / 64)));
    if constexpr (kDrain != 0) {
        // the deferred launch: every lane's first item is fixed by its thread index (the host
        // starts the counter past them), the rest are claimed; with slices, particles go round
        // through the ring
        const unsigned long long gtid = (unsigned long long)blockIdx.x * kBlock + (unsigned long long)tid;
        if (gtid < (unsigned long long)G.n_items) {
            load_queued<Real, false>(G, (int64_t)gtid, p);
            p.start = true;
        }
        bool wait = false;   // a ring entry is claimed (index in p.lin), not yet readable
        int skip = 0;        // wave-uniform: loop iterations before idle lanes look for work again
        uint32_t iter = 0;   // loop iterations (issue-priority rotation)
        for (;;) {
            rotate_prio(iter);
            if (wait) take_ring(G, p, wait);
            const bool need = !p.alive && !p.start && !wait;
            if (__ballot(need)) {
                const bool busy = __ballot(!need) != 0ull;
                if (!busy || skip == 0) {
                    const int c = claim<Real>(G, p, need, wait);
                    if (c == 0 && !busy) break;   // nothing left to claim, nothing held
                    skip = (c == 1) ? 0 : (c == 0) ? 32 : 4;
                } else {
                    --skip;
                }
            }
            if (p.alive || p.start) advance<Real, kDrain, kBoris>(jobs[0], L0, G, p, lc);
            if (G.slice_mask) {
                // slice ends where the step count plus the (well mixed) low lineage bits is a
                // multiple of the slice: particles that start together still leave the ring's
                // tail and the claim counter a few at a time
                const bool rq = p.alive && p.s != 0u && ((p.s + (uint32_t)p.lin) & G.slice_mask) == 0u;
                if (__ballot(rq)) ring_put<Real>(G, p, rq);
            }
        }
    } else
    for (;;) {
        const bool need = !p.alive && !p.start && !done;
        if (__ballot(need)) refill<Real, kBatched>(G, p, need, done, wjob);
        if (!__ballot(!done)) break;
        if (!kBatched) {
            if (kCoop) {
                unsigned long long cm = __ballot(p.alive && !p.start && p.fly);
                while (cm) {
                    const int j = __ffsll((long long)cm) - 1;
                    cm &= cm - 1ull;
                    coop_flight(jobs[0], L0, G, p, lc, j);
                }
            }
            if (p.alive || p.start) advance<Real, kDrain, kBoris>(jobs[0], L0, G, p, lc);
        } else {
            if constexpr (kCoop) {
                // wave-cooperative flights (coop_flight) of the particles whose job chose the
                // wave mapping: each flight is one job's, whose tables and counter slot the
                // whole wave uses for it
                unsigned long long cm = __ballot(p.alive && !p.start && p.fly && jobs[p.job].wave != 0);
                while (cm) {
                    const int j = __ffsll((long long)cm) - 1;
                    cm &= cm - 1ull;
                    const int ju = bc_i(p.job, j);
                    const DevJob& J = jobs[ju];
                    unsigned long long* sc = job_slot(jobs, wslots, wtags, ju);
                    coop_flight(J, global_view<Real>(J, sc, (double*)(sc + kNCnt)), G, p, lc, j);
                }
            }
            bool todo = p.alive || p.start;
            const int key = kS * p.job + (p.start ? 0 : p.sp);
            for (;;) {
                const unsigned long long m = __ballot(todo);
                if (!m) break;
                const int leader = __ffsll((long long)m) - 1;
                const int k0 = __shfl(key, leader);
                if (todo && key == k0) {
                    const int ju = __builtin_amdgcn_readfirstlane(p.job);
                    const DevJob& J = jobs[ju];
                    unsigned long long* sc = job_slot(jobs, wslots, wtags, ju);
                    advance<Real, 0, kBoris>(J, global_view<Real>(J, sc, (double*)(sc + kNCnt)), G, p, lc);
                    todo = false;
                }
            }
        }
    }

    if (!kBatched) {
        flush_lane(lc, L0.cnt, L0.led);
        __syncthreads();
        const DevJob& J = jobs[0];
        for (int i = tid; i < kNCnt; i += blockDim.x)
            if (L0.cnt[i]) add_u64(&J.counters[i], L0.cnt[i]);
        for (int i = tid; i < kNLed; i += blockDim.x)
            if (L0.led[i] != 0.0) add_f64(&J.ledger[i], L0.led[i]);
    } else {
        __builtin_amdgcn_wave_barrier();
        if ((tid & 63) == 0)
            for (int k = 0; k < kSlots; ++k)
                if (wtags[k] >= 0) slot_flush(jobs, wtags[k], wslots + (size_t)k * kSlotWords);
    }
}

// Normalised fields (Sec. 2.2 eq. 3 with t_sim = N_prim / activity, eq. 4; Sec. 2.3 currents):
// density per species and segment minus the recombinations logged in its field per volume,
// currents through the z-faces of each ring and the r-faces of each z-segment.
__global__ void fields_kernel(const DevJob J, double t_sim, double* density, double* jz_cur,
                              double* jr_cur) {
    const int nr = J.n_r, nz = J.n_z;
    const double dz = J.length / (double)nz;
    const size_t ns = (size_t)J.n_species;
    const size_t n_dens = ns * nr * nz;
    const size_t n_jz = ns * nr * (nz + 1);
    const size_t n_jr = ns * (nr + 1) * nz;
    const size_t total = n_dens + n_jz + n_jr;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (size_t)gridDim.x * blockDim.x) {
        if (t < n_dens) {
            const int s = (int)(t / ((size_t)nr * nz));
            const int ir = (int)((t / nz) % nr);
            const int iz = (int)(t % nz);
            const double r0 = J.radius * (double)ir / (double)nr;
            const double r1 = J.radius * (double)(ir + 1) / (double)nr;
            const double ring = kPI * (r1 * r1 - r0 * r0);
            const double vol = ring * dz;
            (void)s;
            (void)iz;
            double n = J.dens[t] / (t_sim * vol);
            n -= (double)J.recomb[t] / vol;
            density[t] = n;
        } else if (t < n_dens + n_jz) {
            const size_t k = t - n_dens;
            const int ir = (int)((k / (nz + 1)) % nr);
            const double r0 = J.radius * (double)ir / (double)nr;
            const double r1 = J.radius * (double)(ir + 1) / (double)nr;
            const double ring = kPI * (r1 * r1 - r0 * r0);
            const double net = (double)((long long)J.jz[2 * k + 1] - (long long)J.jz[2 * k]);
            jz_cur[k] = net / (ring * t_sim);
        } else {
            const size_t k = t - n_dens - n_jz;
            const int f = (int)((k / nz) % (nr + 1));
            const double rf = J.radius * (double)f / (double)nr;
            const double area = kTWO_PI * rf * dz;
            const double net = (double)((long long)J.jr[2 * k + 1] - (long long)J.jr[2 * k]);
            jr_cur[k] = (area > 0.0) ? net / (area * t_sim) : 0.0;
        }
    }
}

// Target fields for the next cycle (Sec. 2.2, Sec. 3.6): the density of each species from the
// tallies so far, eq. (3) with t_sim = N_prim / activity (eq. 4), negative values set to zero.
__global__ void target_fields_kernel(const DevJob J, double t_sim) {
    const int nr = J.n_r, nz = J.n_z;
    const double dz = J.length / (double)nz;
    const size_t n = (size_t)J.n_species * nr * nz;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const int s = (int)(t / ((size_t)nr * nz));
        const size_t cell = t % ((size_t)nr * nz);
        const int ir = (int)(cell / nz);
        const double r0 = J.radius * (double)ir / (double)nr;
        const double r1 = J.radius * (double)(ir + 1) / (double)nr;
        const double vol = kPI * (r1 * r1 - r0 * r0) * dz;
        double d = J.dens[t] / (t_sim * vol);
        d -= (double)J.recomb[t] / vol;
        if (J.sc.field[s]) J.sc.field[s][cell] = d > 0.0 ? d : 0.0;
    }
}

__global__ void sort_count_kernel(const uint32_t* __restrict__ job, int64_t n,
                                  unsigned long long* counts) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        wave_count(counts, (int)job[i]);
}

__global__ void sort_scan_kernel(const unsigned long long* counts, int32_t n_jobs, int64_t* first,
                                 int64_t* count, unsigned long long* cursor) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int64_t acc = 0;
        for (int j = 0; j < n_jobs; ++j) {
            first[j] = acc;
            count[j] = (int64_t)counts[j];
            cursor[j] = 0ull;
            acc += (int64_t)counts[j];
        }
    }
}

__global__ void sort_scatter_kernel(const QueueSoA in, const QueueSoA out, int64_t n, const int64_t* first,
                                    unsigned long long* cursor) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t j = in.job[i];
        const int64_t d = first[j] + (int64_t)atomicAdd(&cursor[j], 1ull);
        out.x[d] = in.x[i];
        out.y[d] = in.y[i];
        out.z[d] = in.z[i];
        out.u[d] = in.u[i];
        out.v[d] = in.v[i];
        out.w[d] = in.w[i];
        out.e[d] = in.e[i];
        out.lin[d] = in.lin[i];
        out.pid[d] = in.pid[i];
        out.meta[d] = in.meta[i];
        out.job[d] = j;
    }
}

__global__ void fill_u64_kernel(unsigned long long* p, size_t n, unsigned long long value) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = value;
}

}  // namespace

#if defined(KARL_DRAIN_UNIT)
// The deferred-launch kernels, compiled in a unit of their own (see karl_kernels_drain.hip).
hipError_t launch_transport_drain(const DevJob* jobs_dev, bool dense, const GenArgs& g, int precision,
                                  int grid, int block, size_t lds, hipStream_t s) {
    if (precision == KARL_FP32) {
        if (dense)
            hipLaunchKernelGGL((transport_kernel<float, false, false, 2>), dim3(grid), dim3(block), lds, s, jobs_dev, g);
        else
            hipLaunchKernelGGL((transport_kernel<float, false, false, 1>), dim3(grid), dim3(block), lds, s, jobs_dev, g);
    } else {
        if (dense)
            hipLaunchKernelGGL((transport_kernel<double, false, false, 2>), dim3(grid), dim3(block), lds, s, jobs_dev, g);
        else
            hipLaunchKernelGGL((transport_kernel<double, false, false, 1>), dim3(grid), dim3(block), lds, s, jobs_dev, g);
    }
    return hipGetLastError();
}

hipError_t transport_occupancy_drain(int precision, int block, size_t lds, int* blocks_per_cu) {
    if (precision == KARL_FP32)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, transport_kernel<float, false, false, 1>, block, lds);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, transport_kernel<double, false, false, 1>, block, lds);
}
#elif defined(KARL_BATCHED_UNIT)
// The batched kernels, compiled in a unit of their own (see karl_kernels_batched.hip).
// coop: the variant with wave-cooperative flights for the particles of jobs that chose them
// (DevJob::wave; guiding-centre jobs without the Boris mover)
hipError_t launch_transport_batched(const DevJob* jobs_dev, bool boris, bool coop, const GenArgs& g, int precision,
                                    int grid, int block, size_t lds, hipStream_t s) {
    if (precision == KARL_FP32) {
        if (boris)
            hipLaunchKernelGGL((transport_kernel<float, true, false, 0, true>), dim3(grid), dim3(block), lds, s, jobs_dev, g);
        else if (coop)
            hipLaunchKernelGGL((transport_kernel<float, true, true>), dim3(grid), dim3(block), lds, s, jobs_dev, g);
        else
            hipLaunchKernelGGL((transport_kernel<float, true>), dim3(grid), dim3(block), lds, s, jobs_dev, g);
    } else {
        if (boris)
            hipLaunchKernelGGL((transport_kernel<double, true, false, 0, true>), dim3(grid), dim3(block), lds, s, jobs_dev, g);
        else if (coop)
            hipLaunchKernelGGL((transport_kernel<double, true, true>), dim3(grid), dim3(block), lds, s, jobs_dev, g);
        else
            hipLaunchKernelGGL((transport_kernel<double, true>), dim3(grid), dim3(block), lds, s, jobs_dev, g);
    }
    return hipGetLastError();
}

hipError_t transport_occupancy_batched(int precision, bool boris, bool coop, int block, size_t lds, int* blocks_per_cu) {
    if (precision == KARL_FP32)
        return boris ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, transport_kernel<float, true, false, 0, true>, block, lds)
               : coop ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, transport_kernel<float, true, true>, block, lds)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, transport_kernel<float, true>, block, lds);
    return boris ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, transport_kernel<double, true, false, 0, true>, block, lds)
           : coop ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, transport_kernel<double, true, true>, block, lds)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, transport_kernel<double, true>, block, lds);
}
#else
size_t lds_bytes(const DevJob& j, int precision) {
    const size_t rs = precision == KARL_FP32 ? sizeof(float) : sizeof(double);
    size_t b = (size_t)(kNCnt + kNLed) * 8 + (size_t)(kS + 2) * KARL_MAX_PROC * sizeof(int32_t);
    b += rs * KARL_MAX_PROC;
    b += rs * ((size_t)j.n_proc * j.n_e + (size_t)j.n_z + (size_t)(j.n_z + 1) + (size_t)(j.n_r + 1));
    b += 8 + sizeof(SpeciesConst);   // alignment slack and the species constants
    return (b + 15) & ~(size_t)15;
}

hipError_t launch_transport(const DevJob* jobs_dev, bool batched, bool coop, bool drain, bool dense,
                            bool boris, const GenArgs& g, int precision, int grid, int block, size_t lds,
                            hipStream_t s) {
    if (drain && !batched) return launch_transport_drain(jobs_dev, dense, g, precision, grid, block, lds, s);
    if (batched) return launch_transport_batched(jobs_dev, boris, coop, g, precision, grid, block, lds, s);
    if (precision == KARL_FP32) {
        if (coop) {
            hipLaunchKernelGGL((transport_kernel<float, false, true>), dim3(grid), dim3(block), lds, s, jobs_dev, g);
        } else if (boris) {
            hipLaunchKernelGGL((transport_kernel<float, false, false, 0, true>), dim3(grid), dim3(block), lds, s, jobs_dev, g);
        } else {
            hipLaunchKernelGGL((transport_kernel<float, false>), dim3(grid), dim3(block), lds, s, jobs_dev, g);
        }
    } else {
        if (coop) {
            hipLaunchKernelGGL((transport_kernel<double, false, true>), dim3(grid), dim3(block), lds, s, jobs_dev, g);
        } else if (boris) {
            hipLaunchKernelGGL((transport_kernel<double, false, false, 0, true>), dim3(grid), dim3(block), lds, s, jobs_dev, g);
        } else {
            hipLaunchKernelGGL((transport_kernel<double, false>), dim3(grid), dim3(block), lds, s, jobs_dev, g);
        }
    }
    return hipGetLastError();
}

size_t batched_lds_bytes() {
    return (size_t)(kBlock / 64) * (kSlots * kSlotWords * 8 + (kSlots + 1) * 4);
}

hipError_t launch_fields(const DevJob& j, double t_sim, double* density, double* jz, double* jr,
                         hipStream_t s) {
    const size_t ns = (size_t)j.n_species;
    const size_t total = ns * j.n_r * j.n_z + ns * j.n_r * (j.n_z + 1) + ns * (j.n_r + 1) * j.n_z;
    size_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fields_kernel, dim3((unsigned)blocks), dim3(256), 0, s, j, t_sim, density, jz, jr);
    return hipGetLastError();
}

hipError_t launch_target_fields(const DevJob& j, double t_sim, hipStream_t s) {
    const size_t total = (size_t)2 * j.n_r * j.n_z;
    size_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(target_fields_kernel, dim3((unsigned)blocks), dim3(256), 0, s, j, t_sim);
    return hipGetLastError();
}

hipError_t launch_sort_by_job(const QueueSoA& in, const QueueSoA& out, int64_t n, int32_t n_jobs,
                              unsigned long long* counts, int64_t* first, int64_t* count,
                              unsigned long long* cursor, hipStream_t s) {
    hipError_t e = launch_fill_u64(counts, (size_t)n_jobs, 0ull, s);
    if (e != hipSuccess) return e;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(sort_count_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in.job, n, counts);
    hipLaunchKernelGGL(sort_scan_kernel, dim3(1), dim3(64), 0, s, counts, n_jobs, first, count, cursor);
    hipLaunchKernelGGL(sort_scatter_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, out, n, first, cursor);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, size_t n, unsigned long long value, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, value);
    return hipGetLastError();
}

hipError_t transport_occupancy(int precision, bool batched, bool coop, bool drain, bool boris, int block,
                               size_t lds, int* blocks_per_cu) {
    if (drain && !batched) return transport_occupancy_drain(precision, block, lds, blocks_per_cu);
    if (batched) return transport_occupancy_batched(precision, boris, coop, block, lds, blocks_per_cu);
    if (precision == KARL_FP32) {
        if (coop)
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, transport_kernel<float, false, true>, block, lds);
        return boris ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, transport_kernel<float, false, false, 0, true>, block, lds)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, transport_kernel<float, false>, block, lds);
    }
    if (coop)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, transport_kernel<double, false, true>, block, lds);
    return boris ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, transport_kernel<double, false, false, 0, true>, block, lds)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, transport_kernel<double, false>, block, lds);
}

#endif

}  // namespace karl

// C ABI of libkarl (include/karl.h): validation, workspace layout, table upload, and the
// generation loop that drives the transport kernel for one job or a batch of jobs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "karl.h"
#include "karl_internal.h"

namespace {

thread_local char g_err[512] = "";

karl_status fail(karl_status code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_CHECK(expr)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(KARL_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

constexpr double kKB = 1.380649e-23;
constexpr double kPI_HOST = 3.14159265358979323846;
constexpr double kQE = 1.602176634e-19;
constexpr size_t kAlign = 256;
constexpr int kBlock = 256;
constexpr int64_t kDefaultCapacity = int64_t(1) << 22;
constexpr int64_t kDefaultChunk = 65536;
constexpr int64_t kMaxChunk = int64_t(1) << 26;
constexpr size_t kMaxLds = 65536;
constexpr size_t kQueueEntryBytes = 7 * 8 + 8 + 4 + 4 + 4;
constexpr size_t kControlBytes = 64;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Byte offsets of every region of a job's workspace.
struct Layout {
    size_t devjob, xs, n_gas, zf, rf, zcdf, tfield, edges, plane_of, angles, dens_edges, e_fld, b_fld;
    size_t tallies, tally_bytes;
    size_t t_counters, t_ledger, t_dens, t_recomb, t_jz, t_jr, t_spectra, t_digests, t_hist, t_dense;
    size_t snapshot, control, fields, queues, queue_entries;
    size_t ring, ring_flag, ring_cap;   // deferred launch in slices (ring_cap 0: none)
    size_t total;
};

size_t real_size(const karl_job_desc* d) { return d->precision == KARL_FP32 ? 4 : 8; }

// doubles of a process' angle table on the device: edges, theta, cdf and pdf
size_t angle_block(const karl_process_desc& p) {
    if (p.ang_bins <= 0) return 0;
    const size_t nb = (size_t)p.ang_bins, n = (size_t)p.ang_nodes;
    return (nb + 1) + n + 2 * nb * n;
}

size_t angle_doubles(const karl_job_desc* d) {
    size_t n = 0;
    for (int i = 0; i < d->n_proc && i < KARL_MAX_PROC; ++i) n += angle_block(d->proc[i]);
    return n;
}

int species_count(const karl_job_desc* d) { return d->n_species ? d->n_species : 2; }

// some process targets a species' density field (then every species' field gets device storage)
bool uses_fields(const karl_job_desc* d) {
    for (int i = 0; i < d->n_proc && i < KARL_MAX_PROC; ++i)
        if (d->proc[i].target == KARL_TARGET_FIELD) return true;
    return false;
}

Layout make_layout(const karl_job_desc* d) {
    Layout L{};
    const size_t rs = real_size(d);
    const size_t nr = (size_t)d->n_r, nz = (size_t)d->n_z;
    const size_t ns = (size_t)species_count(d);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    L.devjob = take(sizeof(karl::DevJob));
    L.xs = take(rs * (size_t)d->n_proc * (size_t)d->n_e);
    L.n_gas = take(rs * nz);
    L.zf = take(rs * (nz + 1));
    L.rf = take(rs * (nr + 1));
    L.zcdf = take(rs * (nz + 1));
    L.tfield = take(uses_fields(d) ? 8 * ns * nr * nz : 0);
    L.edges = take(8 * ns * ((size_t)d->n_bins + 1));
    L.plane_of = take(4 * (nz + 1));
    L.angles = take(8 * angle_doubles(d));
    L.dens_edges = take(d->n_dens_bins > 0 ? 8 * ns * ((size_t)d->n_dens_bins + 1) : 0);
    const size_t fbins = (size_t)std::max(d->field_nr, 0) * (size_t)std::max(d->field_nz, 0) * 3;
    L.e_fld = take(d->e_field ? 8 * fbins : 0);
    L.b_fld = take(d->b_field ? 8 * fbins : 0);
    // tallies: one contiguous block so that a snapshot is one copy
    size_t t = 0;
    auto tk = [&](size_t bytes) {
        size_t o = t;
        t += (bytes + 7) & ~size_t(7);
        return o;
    };
    const size_t np = (size_t)d->n_primaries;
    L.t_counters = tk(8 * KARL_NCOUNTERS);
    L.t_ledger = tk(8 * KARL_NLEDGER);
    L.t_dens = tk(8 * ns * nr * nz);
    L.t_recomb = tk(8 * ns * nr * nz);
    L.t_jz = tk(8 * ns * nr * (nz + 1) * 2);
    L.t_jr = tk(8 * ns * (nr + 1) * nz * 2);
    L.t_spectra = tk(8 * ns * (size_t)d->n_planes * 2 * ((size_t)d->n_bins + 2));
    L.t_digests = tk((d->flags & KARL_FLAG_DIGESTS) ? 8 * np : 0);
    L.t_hist = tk((d->flags & KARL_FLAG_HISTORY) ? 8 * KARL_NHIST * np : 0);
    L.t_dense = tk(d->n_dens_bins > 0 ? 8 * ns * nr * nz * ((size_t)d->n_dens_bins + 2) : 0);
    L.tally_bytes = t;
    L.tallies = take(t);
    L.snapshot = take(t);
    L.control = take(kControlBytes);
    L.fields = take(8 * (ns * nr * nz + ns * nr * (nz + 1) + ns * (nr + 1) * nz));
    L.queue_entries = (size_t)(d->queue_capacity > 0 ? d->queue_capacity : kDefaultCapacity);
    L.queues = take(4 * L.queue_entries * kQueueEntryBytes);
    L.ring_cap = d->slice_steps > 0 ? (size_t)(d->slice_ring > 0 ? d->slice_ring
                                                                 : (int64_t)L.queue_entries + (1 << 20))
                                    : 0;
    L.ring = take(L.ring_cap * sizeof(karl::RingEntry));
    L.ring_flag = take(8 * L.ring_cap);
    L.total = off;
    return L;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

karl_status validate(const karl_job_desc* d, bool need_workspace) {
    if (!d) return fail(KARL_EINVAL, "descriptor is NULL");
    if (!finite_pos(d->radius) || !finite_pos(d->length))
        return fail(KARL_EINVAL, "radius and length must be finite and positive");
    if (d->n_r < 1 || d->n_r > 2047 || d->n_z < 1 || d->n_z >= (1 << 19))
        return fail(KARL_EINVAL, "grid must have 1 <= n_r <= 2047 and 1 <= n_z < 2^19");
    if (d->n_e < 2 || d->n_e > 1024) return fail(KARL_EINVAL, "n_e must be in 2..1024");
    if (d->n_species != 0 && (d->n_species < 2 || d->n_species > KARL_MAX_SPECIES))
        return fail(KARL_EINVAL, "n_species must be in 2..%d (0: 2)", KARL_MAX_SPECIES);
    const int ns = species_count(d);
    if (d->n_proc < 0 || d->n_proc > KARL_MAX_PROC)
        return fail(KARL_EINVAL, "n_proc must be in 0..%d", KARL_MAX_PROC);
    if (d->n_bins < 1 || d->n_bins > (1 << 20)) return fail(KARL_EINVAL, "n_bins must be in 1..2^20");
    if (d->n_planes < 0 || (d->n_planes > 0 && !d->planes))
        return fail(KARL_EINVAL, "planes missing");
    for (int p = 0; p < d->n_planes; ++p)
        if (d->planes[p] < 0 || d->planes[p] > d->n_z)
            return fail(KARL_EINVAL, "plane %d: z-face index %d outside 0..n_z", p, d->planes[p]);
    if (!d->n_gas) return fail(KARL_EINVAL, "n_gas is NULL");
    for (int k = 0; k < d->n_z; ++k)
        if (!std::isfinite(d->n_gas[k]) || d->n_gas[k] < 0.0)
            return fail(KARL_EINVAL, "n_gas[%d] must be finite and >= 0", k);
    for (int f = 0; f < ns; ++f) {
        const double* fld = d->n_field[f];
        if (fld)
            for (int k = 0; k < d->n_r * d->n_z; ++k)
                if (!std::isfinite(fld[k]) || fld[k] < 0.0)
                    return fail(KARL_EINVAL, "n_field[%d][%d] must be finite and >= 0", f, k);
    }
    if (!std::isfinite(d->t_gas) || d->t_gas < 0.0) return fail(KARL_EINVAL, "t_gas must be >= 0");
    if (!finite_pos(d->m_gas)) return fail(KARL_EINVAL, "m_gas must be positive");
    if (!std::isfinite(d->bz)) return fail(KARL_EINVAL, "bz must be finite");
    for (int s = 0; s < ns; ++s) {
        const karl_species_desc& sp = d->species[s];
        if (!finite_pos(sp.mass)) return fail(KARL_EINVAL, "species %d: mass must be positive", s);
        if (!std::isfinite(sp.charge) || (d->bz != 0.0 && sp.charge == 0.0))
            return fail(KARL_EINVAL, "species %d: charge must be finite and nonzero in a field", s);
        if (!(sp.e_cut >= 0.0) || !(sp.lifetime > 0.0) || sp.cap < 1)
            return fail(KARL_EINVAL, "species %d: e_cut >= 0, lifetime > 0, cap >= 1 required", s);
        if (!finite_pos(sp.xs_emin) || !(sp.xs_emax > sp.xs_emin) || !std::isfinite(sp.xs_emax))
            return fail(KARL_EINVAL, "species %d: need 0 < xs_emin < xs_emax", s);
        if (!sp.edges) return fail(KARL_EINVAL, "species %d: spectrum edges missing", s);
        for (int b = 0; b < d->n_bins; ++b)
            if (!(sp.edges[b] < sp.edges[b + 1]))
                return fail(KARL_EINVAL, "species %d: edges must increase", s);
    }
    int partner_of[KARL_MAX_SPECIES] = {-1, -1, -1, -1};
    for (int i = 0; i < d->n_proc; ++i) {
        const karl_process_desc& p = d->proc[i];
        if (p.kind < KARL_ELASTIC || p.kind > KARL_CLUSTERING)
            return fail(KARL_EINVAL, "process %d: unknown kind %d", i, p.kind);
        if (p.species < 0 || p.species >= ns) return fail(KARL_EINVAL, "process %d: species", i);
        if (p.target != KARL_TARGET_GAS && p.target != KARL_TARGET_FIELD)
            return fail(KARL_EINVAL, "process %d: target", i);
        if (p.kind == KARL_IONIZATION && (p.product < 1 || p.product >= ns))
            return fail(KARL_EINVAL, "process %d: ionization product must be an ion species 1..%d", i, ns - 1);
        if (p.kind == KARL_CLUSTERING && (p.product < 0 || p.product >= ns || p.product == p.species))
            return fail(KARL_EINVAL, "process %d: clustering product must be another species", i);
        if (p.density_power < 0 || p.density_power > 2)
            return fail(KARL_EINVAL, "process %d: density_power must be 0, 1 or 2", i);
        if (p.density_power == 2 && p.target != KARL_TARGET_GAS)
            return fail(KARL_EINVAL, "process %d: density_power 2 needs a gas target", i);
        if ((p.target == KARL_TARGET_FIELD || p.kind == KARL_RECOMBINATION) && (p.partner < 0 || p.partner >= ns))
            return fail(KARL_EINVAL, "process %d: partner species", i);
        if (p.target == KARL_TARGET_FIELD) {
            if (partner_of[p.species] >= 0 && partner_of[p.species] != p.partner)
                return fail(KARL_EINVAL, "process %d: all field processes of species %d must share one partner",
                            i, p.species);
            partner_of[p.species] = p.partner;
        }
        if (!p.xs) return fail(KARL_EINVAL, "process %d: table missing", i);
        if (!std::isfinite(p.e_th) || p.e_th < 0.0) return fail(KARL_EINVAL, "process %d: e_th", i);
        if (p.kind == KARL_IONIZATION && !(p.e_th > 0.0))
            return fail(KARL_EINVAL, "process %d: ionization needs a binding energy > 0", i);
        for (int k = 0; k < d->n_e; ++k)
            if (!std::isfinite(p.xs[k]) || p.xs[k] < 0.0)
                return fail(KARL_EINVAL, "process %d: cross section %d must be finite and >= 0", i, k);
        if (p.ang_bins != 0) {
            if (p.kind != KARL_ELASTIC) return fail(KARL_EINVAL, "process %d: angle table on a non-elastic process", i);
            if (p.ang_bins < 0 || p.ang_bins > 1024 || p.ang_nodes < 2 || p.ang_nodes > 4096)
                return fail(KARL_EINVAL, "process %d: angle table needs 1..1024 bins and 2..4096 nodes", i);
            if (!p.ang_edges || !p.ang_theta || !p.ang_pdf) return fail(KARL_EINVAL, "process %d: angle table missing", i);
            if (!std::isfinite(p.e_iso) || p.e_iso < 0.0) return fail(KARL_EINVAL, "process %d: e_iso", i);
            for (int b = 0; b < p.ang_bins; ++b)
                if (!(p.ang_edges[b] < p.ang_edges[b + 1])) return fail(KARL_EINVAL, "process %d: angle edges must increase", i);
            if (!(p.ang_theta[0] >= 0.0) || !(p.ang_theta[p.ang_nodes - 1] <= kPI_HOST))
                return fail(KARL_EINVAL, "process %d: angle nodes must lie in [0, pi]", i);
            for (int k = 0; k + 1 < p.ang_nodes; ++k)
                if (!(p.ang_theta[k] < p.ang_theta[k + 1])) return fail(KARL_EINVAL, "process %d: angle nodes must increase", i);
            for (int b = 0; b < p.ang_bins; ++b) {
                bool any = false;   // some positive density: the bin has a positive area
                for (int k = 0; k < p.ang_nodes; ++k) {
                    const double f = p.ang_pdf[(size_t)b * p.ang_nodes + k];
                    if (!std::isfinite(f) || f < 0.0) return fail(KARL_EINVAL, "process %d: angle density must be finite and >= 0", i);
                    any = any || f > 0.0;
                }
                if (!any) return fail(KARL_EINVAL, "process %d: angle bin %d has no area", i, b);
            }
        }
    }
    if (d->source == KARL_SOURCE_BETA) {
        if (!finite_pos(d->beta_e0) || !finite_pos(d->beta_fmax) || !std::isfinite(d->beta_z))
            return fail(KARL_EINVAL, "beta source needs e0 > 0 and f_max > 0");
    } else if (d->source == KARL_SOURCE_BEAM || d->source == KARL_SOURCE_PAIR) {
        if (d->beam_species < 0 || d->beam_species >= ns || !std::isfinite(d->beam_energy) ||
            d->beam_energy < 0.0)
            return fail(KARL_EINVAL, "beam needs a species slot and an energy >= 0");
        if (d->source == KARL_SOURCE_PAIR && (!std::isfinite(d->beam_energy_1) || d->beam_energy_1 < 0.0))
            return fail(KARL_EINVAL, "a pair beam needs an ion energy >= 0");
        const double n = std::sqrt(d->beam_dir[0] * d->beam_dir[0] + d->beam_dir[1] * d->beam_dir[1] +
                                   d->beam_dir[2] * d->beam_dir[2]);
        if (!(std::fabs(n - 1.0) < 1e-9)) return fail(KARL_EINVAL, "beam direction must be a unit vector");
        const double r = std::sqrt(d->beam_pos[0] * d->beam_pos[0] + d->beam_pos[1] * d->beam_pos[1]);
        if (!(r < d->radius) || !(d->beam_pos[2] >= 0.0) || !(d->beam_pos[2] <= d->length))
            return fail(KARL_EINVAL, "beam start must lie inside the cylinder");
    } else {
        return fail(KARL_EINVAL, "unknown source %d", d->source);
    }
    if (d->n_dens_bins < 0 || d->n_dens_bins > 4096)
        return fail(KARL_EINVAL, "n_dens_bins must be in 0..4096");
    if (d->mover != KARL_MOVER_DRIFT && d->mover != KARL_MOVER_BORIS)
        return fail(KARL_EINVAL, "mover must be KARL_MOVER_DRIFT or KARL_MOVER_BORIS");
    if (d->mover == KARL_MOVER_DRIFT && (d->e_field || d->b_field))
        return fail(KARL_EINVAL, "field arrays need the Boris mover (the drift mover takes the uniform bz)");
    if (d->e_field || d->b_field) {
        if (d->field_nr < 1 || d->field_nr > 65536 || d->field_nz < 1 || d->field_nz > 65536 ||
            !finite_pos(d->field_radius) || !finite_pos(d->field_length))
            return fail(KARL_EINVAL, "field arrays need 1..65536 bins per axis and a positive radius and height");
        const size_t nb = (size_t)d->field_nr * (size_t)d->field_nz * 3;
        for (const double* a : {d->e_field, d->b_field})
            if (a)
                for (size_t k = 0; k < nb; ++k)
                    if (!std::isfinite(a[k])) return fail(KARL_EINVAL, "field arrays must be finite");
    }
    if (d->mover == KARL_MOVER_BORIS)
        for (int s = 0; s < ns; ++s) {
            const double dt = d->boris_dt[s];
            if (!finite_pos(dt)) return fail(KARL_EINVAL, "species %d: the Boris mover needs a time step > 0", s);
            if (!std::isfinite(d->species[s].lifetime) || !(d->species[s].lifetime / dt <= 2147483648.0))
                return fail(KARL_EINVAL,
                            "species %d: the Boris mover needs a finite lifetime of at most 2^31 time steps", s);
        }
    if (d->n_dens_bins > 0)
        for (int s = 0; s < ns; ++s) {
            const double* e = d->species[s].dens_edges;
            if (!e) return fail(KARL_EINVAL, "species %d: density energy edges missing", s);
            for (int b = 0; b < d->n_dens_bins; ++b)
                if (!(e[b] < e[b + 1])) return fail(KARL_EINVAL, "species %d: density energy edges must increase", s);
        }
    if (d->n_primaries < 0 || d->n_primaries > (int64_t)0xFFFFFFFFLL)
        return fail(KARL_EINVAL, "n_primaries must be in 0..2^32-1");
    if (d->precision != KARL_FP64 && d->precision != KARL_FP32)
        return fail(KARL_EINVAL, "precision must be KARL_FP64 or KARL_FP32");
    if (d->queue_capacity < 0 || d->chunk < 0) return fail(KARL_EINVAL, "negative queue/chunk size");
    if (d->slice_steps < 0 || d->slice_steps > (int64_t(1) << 30) || (d->slice_steps & (d->slice_steps - 1)) != 0)
        return fail(KARL_EINVAL, "slice_steps must be 0 or a power of two up to 2^30");
    if (d->slice_ring < 0 || d->slice_ring > (int64_t(1) << 40))
        return fail(KARL_EINVAL, "slice_ring must be in 0..2^40");
    if (d->mapping != KARL_MAP_AUTO && d->mapping != KARL_MAP_LANE && d->mapping != KARL_MAP_WAVE)
        return fail(KARL_EINVAL, "mapping must be KARL_MAP_AUTO, KARL_MAP_LANE or KARL_MAP_WAVE");
    if (d->precision == KARL_FP32) {
        // FP32 state: the tables and the geometry that the kernels read in single precision must
        // stay finite there (gas densities also summed over the cells, for the birth CDF)
        const double fmax = 3.4028234663852886e38;
        if (d->radius > fmax || d->length > fmax)
            return fail(KARL_EINVAL, "radius and length must be below the FP32 range limit");
        double cum = 0.0;
        for (int k = 0; k < d->n_z; ++k) {
            cum += d->n_gas[k];
            if (!(cum <= fmax))
                return fail(KARL_EINVAL, "n_gas (summed over the cells) must stay below the FP32 range limit");
        }
        for (int i = 0; i < d->n_proc; ++i) {
            const double sc = d->proc[i].density_power == 2 ? std::ldexp(1.0, 100) : 1.0;
            for (int k = 0; k < d->n_e; ++k)
                if (!(d->proc[i].xs[k] * sc <= fmax))
                    return fail(KARL_EINVAL, "process %d: cross section %d beyond the FP32 range limit", i, k);
        }
    }
    {
        // the tables and grid faces are staged in LDS: only their sizes matter here
        karl::DevJob sizes{};
        sizes.n_proc = d->n_proc;
        sizes.n_e = d->n_e;
        sizes.n_z = d->n_z;
        sizes.n_r = d->n_r;
        const size_t lds = karl::lds_bytes(sizes, d->precision);
        if (lds > kMaxLds)
            return fail(KARL_EINVAL, "tables need %zu bytes of LDS per workgroup (max %zu)", lds, kMaxLds);
    }
    if (need_workspace) {
        const Layout L = make_layout(d);
        if (!d->workspace) return fail(KARL_EINVAL, "workspace is NULL");
        if (d->workspace_bytes < L.total)
            return fail(KARL_ENOMEM, "workspace has %llu bytes, job needs %llu",
                        (unsigned long long)d->workspace_bytes, (unsigned long long)L.total);
    }
    return KARL_OK;
}

int count_faces_le(const std::vector<double>& faces, int n, double r) {
    int k = 0;
    for (int j = 1; j < n; ++j)
        if (faces[j] <= r) k = j;
    return k;
}

karl::QueueSoA queue_at(char* base, size_t cap) {
    karl::QueueSoA q;
    size_t o = 0;
    auto d = [&]() {
        double* p = (double*)(base + o);
        o += 8 * cap;
        return p;
    };
    q.x = d(); q.y = d(); q.z = d(); q.u = d(); q.v = d(); q.w = d(); q.e = d();
    q.lin = (unsigned long long*)(base + o);
    o += 8 * cap;
    q.pid = (uint32_t*)(base + o);
    o += 4 * cap;
    q.meta = (uint32_t*)(base + o);
    o += 4 * cap;
    q.job = (uint32_t*)(base + o);
    return q;
}

// Everything needed to run generations: queues, control words, job table, launch shape.
struct Launcher {
    int precision = 0;
    bool batched = false;
    karl::DevJob* jobs_dev = nullptr;       // job table in device memory
    karl::QueueSoA q[2]{};                  // next-generation queues (ping-pong)
    karl::QueueSoA dq[2]{};                 // deferred queues (append / drain)
    unsigned long long* ctl = nullptr;      // [0] fetch [1] qcount [2] status [3..4] dcount [5] job status [6] wave segments [7] ring tail
    int64_t capacity = 0;
    size_t lds = 0;
    int max_blocks = 0;
    int max_blocks_coop = 0;                // single-job launches with wave-cooperative flights
    int max_blocks_drain = 0;               // single-job deferred-queue launches
    bool coop = false;                      // launch the wave-cooperative kernel
    bool dense = false;                     // the job has an energy-resolved density tally
    bool boris = false;                     // a job of the launch uses the Boris mover
    int max_blocks_boris = 0;               // launches of the kernel built with the Boris mover
    uint32_t slice_mask = 0;                // deferred launch in slices: steps per slice - 1
    karl::RingEntry* ring = nullptr;        // its ring of particles between slices
    unsigned long long* ring_flag = nullptr;
    int64_t ring_cap = 0;
    unsigned long long* host_ctl = nullptr; // pinned copy of ctl[1..4] and a scratch word
    bool own_host = false;                  // host_ctl allocated by init (else the caller's)
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double kernel_ms = 0.0;
    int64_t launches = 0, generations = 0, max_queue = 0;
    double drain_ms = 0.0;                  // of kernel_ms: the deferred (drain) launches
    int64_t drain_launches = 0;
    int64_t slices = 0;                     // ring entries written by deferred launches
    // batched launches: per-job item ranges, fetch counters and the queue sort's scratch
    int32_t n_jobs = 1;
    int64_t* job_first = nullptr;
    int64_t* job_count = nullptr;
    int64_t* job_cum = nullptr;
    unsigned long long* job_fetch = nullptr;
    unsigned long long* job_waves = nullptr;
    unsigned long long* sort_counts = nullptr;
    unsigned long long* sort_cursor = nullptr;
    bool ready = false;

    // host_words: caller-provided host memory for the counters read back after each launch
    // (then no pinned memory and no timing events are created: nothing is allocated)
    karl_status init(char* queues, size_t entries, unsigned long long* control, int prec,
                     bool is_batched, size_t lds_bytes, unsigned long long* host_words = nullptr) {
        precision = prec;
        batched = is_batched;
        capacity = (int64_t)entries;
        ctl = control;
        lds = lds_bytes;
        for (int k = 0; k < 2; ++k) {
            q[k] = queue_at(queues + (size_t)k * entries * kQueueEntryBytes, entries);
            dq[k] = queue_at(queues + (size_t)(2 + k) * entries * kQueueEntryBytes, entries);
        }
        int dev = 0;
        HIP_CHECK(hipGetDevice(&dev));
        hipDeviceProp_t prop;
        HIP_CHECK(hipGetDeviceProperties(&prop, dev));
        int per_cu = 0;
        HIP_CHECK(karl::transport_occupancy(prec, is_batched, false, false, false, kBlock, lds, &per_cu));
        if (per_cu < 1) per_cu = 1;
        max_blocks = per_cu * prop.multiProcessorCount;
        max_blocks_coop = max_blocks_drain = max_blocks;
        HIP_CHECK(karl::transport_occupancy(prec, is_batched, false, false, true, kBlock, lds, &per_cu));
        if (per_cu < 1) per_cu = 1;
        max_blocks_boris = per_cu * prop.multiProcessorCount;
        HIP_CHECK(karl::transport_occupancy(prec, is_batched, true, false, false, kBlock, lds, &per_cu));
        if (per_cu < 1) per_cu = 1;
        max_blocks_coop = per_cu * prop.multiProcessorCount;
        if (!is_batched) {
            HIP_CHECK(karl::transport_occupancy(prec, false, false, true, false, kBlock, lds, &per_cu));
            if (per_cu < 1) per_cu = 1;
            max_blocks_drain = per_cu * prop.multiProcessorCount;
        }
        if (host_words) {
            host_ctl = host_words;
            own_host = false;
        } else {
            HIP_CHECK(hipHostMalloc((void**)&host_ctl, 8 * sizeof(unsigned long long), hipHostMallocDefault));
            own_host = true;
            HIP_CHECK(hipEventCreate(&ev0));
            HIP_CHECK(hipEventCreate(&ev1));
            HIP_CHECK(karl::launch_fill_u64(ctl, kControlBytes / 8, 0ull, nullptr));
            HIP_CHECK(hipStreamSynchronize(nullptr));
        }
        ready = true;
        return KARL_OK;
    }

    void release() {
        if (host_ctl && own_host) (void)hipHostFree(host_ctl);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        host_ctl = nullptr;
        ev0 = ev1 = nullptr;
        ready = false;
    }

    void reset_stats() {
        kernel_ms = drain_ms = 0.0;
        launches = generations = max_queue = slices = drain_launches = 0;
    }

    // Run every generation of n primary items (chunk of the item space starting at item_base;
    // for a single job the item i is primary pid_begin0 + i).  Returns with *overflow set if a
    // queue overflowed; *max_gen receives the largest generation.
    karl_status run(const karl::GenArgs& base, int64_t n, hipStream_t s, bool* overflow,
                    int64_t* max_gen) {
        *overflow = false;
        *max_gen = 0;
        int mode = 0;
        int64_t items = n;
        const karl::QueueSoA* in = &q[0];
        int mo = 0;
        int di = 0;
        int64_t ndef = 0;
        unsigned long long* fetch = ctl;
        unsigned long long* qcount = ctl + 1;
        unsigned long long* dcount = ctl + 3;
        HIP_CHECK(karl::launch_fill_u64(dcount, 2, 0ull, s));
        bool drain = false;
        for (;;) {
            if (items == 0) {
                if (ndef == 0) break;
                // the generations are exhausted: drain the deferred queue in one launch
                drain = true;
                in = &dq[di];
                items = ndef;
                mode = 1;
                di ^= 1;
                ndef = 0;
                HIP_CHECK(karl::launch_fill_u64(dcount + di, 1, 0ull, s));
            }
            if (batched && mode == 1) {
                // group the input by job (into the free generation buffer) so that waves can
                // work through one job at a time; the output then reuses buffer 0
                HIP_CHECK(karl::launch_sort_by_job(*in, q[1], items, n_jobs, sort_counts, job_first,
                                                   job_count, sort_cursor, s));
                in = &q[1];
                mo = 0;
            }
            karl::GenArgs g = base;
            g.mode = mode;
            g.n_jobs = batched ? n_jobs : 1;
            g.n_items = items;
            g.fetch = fetch;
            g.job_first = job_first;
            g.job_count = job_count;
            // the job-sorted queue starts of job j at the items of the jobs before it
            g.job_cum = mode == 1 ? job_first : job_cum;
            g.job_fetch = job_fetch;
            g.job_waves = job_waves;
            g.qin = *in;
            g.qout = q[mo];
            g.qout_count = qcount;
            g.qdef = dq[di];
            g.qdef_count = dcount + di;
            g.capacity = capacity;
            g.status = (unsigned int*)(ctl + 2);
            g.wave_segments = ctl + 6;
            HIP_CHECK(karl::launch_fill_u64(fetch, 2, 0ull, s));
            if (batched) {
                HIP_CHECK(karl::launch_fill_u64(job_fetch, (size_t)n_jobs, 0ull, s));
                HIP_CHECK(karl::launch_fill_u64(job_waves, (size_t)n_jobs, 0ull, s));
            }
            const bool use_drain = drain && !batched;
            const bool use_coop = coop && !use_drain && !boris;
            const int64_t cap_blocks = use_drain ? max_blocks_drain : use_coop ? max_blocks_coop
                                       : boris ? max_blocks_boris : max_blocks;
            int64_t blocks = (items + kBlock - 1) / kBlock;
            if (blocks > cap_blocks) blocks = cap_blocks;
            if (use_drain) {
                // every lane starts on the item of its thread index; the claim counter starts
                // after them; with slices, the ring starts empty
                HIP_CHECK(karl::launch_fill_u64(fetch, 1, (unsigned long long)std::min<int64_t>(items, blocks * kBlock), s));
                if (slice_mask) {
                    g.slice_mask = slice_mask;
                    g.ring_cap = ring_cap;
                    g.ring = ring;
                    g.ring_flag = ring_flag;
                    g.ring_tail = ctl + 7;
                    HIP_CHECK(karl::launch_fill_u64(ring_flag, (size_t)ring_cap, 0ull, s));
                    HIP_CHECK(karl::launch_fill_u64(ctl + 7, 1, 0ull, s));
                }
            }
            if (ev0) HIP_CHECK(hipEventRecord(ev0, s));
            HIP_CHECK(karl::launch_transport(jobs_dev, batched, use_coop, use_drain, dense, boris, g, precision,
                                             (int)blocks, kBlock, lds, s));
            if (ev1) HIP_CHECK(hipEventRecord(ev1, s));
            HIP_CHECK(hipMemcpyAsync(host_ctl, qcount, 4 * sizeof(unsigned long long),
                                     hipMemcpyDeviceToHost, s));
            if (use_drain && slice_mask)
                HIP_CHECK(hipMemcpyAsync(host_ctl + 6, ctl + 7, sizeof(unsigned long long),
                                         hipMemcpyDeviceToHost, s));
            HIP_CHECK(hipStreamSynchronize(s));
            if (use_drain && slice_mask) slices += (int64_t)host_ctl[6];
            if (ev0) {
                float ms = 0.f;
                HIP_CHECK(hipEventElapsedTime(&ms, ev0, ev1));
                kernel_ms += ms;
                if (use_drain) {
                    drain_ms += ms;
                    drain_launches += 1;
                }
            }
            launches += 1;
            if (mode == 1) generations += 1;
            const unsigned long long produced = host_ctl[0];
            const unsigned int status = (unsigned int)(host_ctl[1] & 0xFFFFFFFFull);
            ndef = (int64_t)host_ctl[2 + di];
            if (status & karl::STATUS_OVERFLOW) {
                *overflow = true;
                return KARL_OK;
            }
            items = (int64_t)produced;
            *max_gen = std::max(*max_gen, std::max(items, ndef));
            max_queue = std::max(max_queue, std::max(items, ndef));
            mode = 1;
            in = &q[mo];
            if (!batched) mo ^= 1;
        }
        return KARL_OK;
    }

    // after an overflow: clear the fetch/queue counters and the overflow bit
    karl_status clear_overflow(hipStream_t s) {
        HIP_CHECK(karl::launch_fill_u64(ctl, 2, 0ull, s));
        host_ctl[4] = (unsigned long long)((unsigned int)host_ctl[1] & ~karl::STATUS_OVERFLOW);
        HIP_CHECK(hipMemcpyAsync(ctl + 2, &host_ctl[4], sizeof(unsigned int), hipMemcpyHostToDevice, s));
        HIP_CHECK(hipStreamSynchronize(s));
        return KARL_OK;
    }
};

// next chunk: keep the largest generation near half the queue capacity
int64_t next_chunk(int64_t cur, int64_t n_done, int64_t max_gen, int64_t capacity) {
    if (max_gen > 0) {
        const double per_primary = (double)max_gen / (double)n_done;
        const double target = 0.5 * (double)capacity / per_primary;
        return std::max<int64_t>(1, std::min<int64_t>(kMaxChunk, (int64_t)target));
    }
    return std::min<int64_t>(kMaxChunk, std::max<int64_t>(cur, 2 * n_done));
}

struct Job {
    int precision = 0;
    uint32_t flags = 0;
    int64_t n_primaries = 0;
    int n_r = 0, n_z = 0, n_planes = 0, n_bins = 0;
    char* ws = nullptr;
    Layout lay{};
    karl::DevJob dj{};
    Launcher run;
    unsigned int* status = nullptr;
    int64_t chunk = 0;
    int64_t n_transported = 0;   // primaries transported since creation or reset
    bool failed = false;
    int device = 0;
    size_t lds = 0;              // launch shape of the job's own launcher, set up on first use
    int64_t slice_steps = 0;           // deferred launch in slices (0: whole histories)
    int32_t mapping = KARL_MAP_AUTO;   // requested
    int32_t chosen = KARL_MAP_AUTO;    // in use once tuned (or forced)
    double seg_per_int = 0.0;          // flight segments per interaction of the tuning chunk
    double ms_seg[2] = {0.0, 0.0};     // kernel ms per flight segment, lane / wave (last chunk)
};

// The job's own launcher (pinned words, events) is created by its first karl_transport, so that
// jobs transported only in batches hold no host resources whose release synchronizes the device.
karl_status ensure_launcher(Job* j) {
    if (j->run.ready) return KARL_OK;
    unsigned long long* ctl = j->run.ctl;
    karl::DevJob* table = j->run.jobs_dev;
    karl_status s = j->run.init(j->ws + j->lay.queues, j->lay.queue_entries, ctl, j->precision, false, j->lds);
    j->run.jobs_dev = table;
    if (j->lay.ring_cap > 0) {
        j->run.slice_mask = (uint32_t)(j->slice_steps - 1);
        j->run.ring = (karl::RingEntry*)(j->ws + j->lay.ring);
        j->run.ring_flag = (unsigned long long*)(j->ws + j->lay.ring_flag);
        j->run.ring_cap = (int64_t)j->lay.ring_cap;
    }
    return s;
}

struct Batch {
    int32_t max_jobs = 0;
    char* ws = nullptr;
    int64_t* job_first = nullptr;   // device [max_jobs]
    int64_t* job_count = nullptr;   // device [max_jobs]
    int64_t* job_cum = nullptr;     // device [max_jobs]
    int64_t* host_i64 = nullptr;    // pinned staging [3*max_jobs]
    karl::DevJob* host_jobs = nullptr;   // pinned staging of the job table
    Launcher run[2];                // FP64 and FP32 launchers share the queues
    int64_t chunk = kDefaultChunk;
    int device = 0;
};

// job table, per-job first/count/cum/fetch/waves, sort counts and cursors, control words, four queues
size_t batch_layout(int32_t max_jobs, int64_t entries, size_t* o_jobs, size_t* o_perjob,
                    size_t* o_ctl, size_t* o_queues) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    *o_jobs = take(sizeof(karl::DevJob) * (size_t)max_jobs);
    *o_perjob = take(7 * 8 * (size_t)max_jobs);
    *o_ctl = take(kControlBytes);
    *o_queues = take(4 * (size_t)entries * kQueueEntryBytes);
    return off;
}

template <typename T>
std::vector<T> convert(const double* src, size_t n) {
    std::vector<T> out(n);
    for (size_t i = 0; i < n; ++i) out[i] = (T)src[i];
    return out;
}

karl_status upload_real(const Job& j, size_t off, const std::vector<double>& v) {
    char* dst = j.ws + off;
    if (j.precision == KARL_FP32) {
        std::vector<float> f = convert<float>(v.data(), v.size());
        HIP_CHECK(hipMemcpy(dst, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
    } else {
        HIP_CHECK(hipMemcpy(dst, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    return KARL_OK;
}

// flight segments and interactions (all species) counted so far
karl_status read_steps(Job* j, hipStream_t s, int64_t* segs, int64_t* ints) {
    static_assert(KARL_C_COLL == KARL_C_STEP + KARL_MAX_SPECIES, "counter layout");
    unsigned long long c[2 * KARL_MAX_SPECIES] = {};
    HIP_CHECK(hipMemcpyAsync(c, j->dj.counters + KARL_C_STEP, sizeof(c), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    *segs = *ints = 0;
    for (int k = 0; k < KARL_MAX_SPECIES; ++k) {
        *segs += (int64_t)c[k];
        *ints += (int64_t)c[KARL_MAX_SPECIES + k];
    }
    return KARL_OK;
}

// Flights of at least this many segments per interaction run faster with the wave mapping on
// MI355X (measured on the tiny case in a 2.5 T field: 42 segments per interaction +24 % FP32 and
// +36 % FP64 for the wave mapping, 22: -15 % / 0 %, 8.5: -28 % / -8 %, 3: -72 % / -65 %).
constexpr double kWaveRatio = 32.0;
constexpr int64_t kTuneSegments = 100000;   // a tuning chunk must show at least this many

// Transport primaries [b, e) in chunks.  With KARL_MAP_AUTO the first chunk runs with the lane
// mapping and its segments per interaction choose the mapping of the following chunks.
// The launcher, the tally snapshot and the chunk size are arguments: the job's own (queues in
// its workspace) or those of the transport without allocation (queues in the library's array).
karl_status transport_range(Job* j, Launcher& run, char* snap, int64_t& chunk, int64_t b,
                            int64_t pid_end, hipStream_t s) {
    char* tallies = j->ws + j->lay.tallies;
    while (b < pid_end) {
        const int64_t n = std::min<int64_t>(chunk, pid_end - b);
        const bool wave = j->chosen == KARL_MAP_WAVE;
        run.coop = wave;
        int64_t s0 = 0, i0 = 0;
        karl_status st = read_steps(j, s, &s0, &i0);
        if (st != KARL_OK) return st;
        const double k0 = run.kernel_ms;
        HIP_CHECK(hipMemcpyAsync(snap, tallies, j->lay.tally_bytes, hipMemcpyDeviceToDevice, s));
        karl::GenArgs g{};
        g.n_jobs = 1;
        g.pid_begin0 = b;
        bool overflow = false;
        int64_t max_gen = 0;
        st = run.run(g, n, s, &overflow, &max_gen);
        if (st != KARL_OK) {
            j->failed = true;
            return st;
        }
        if (overflow) {
            // undo the partial chunk and retry with half as many primaries
            HIP_CHECK(hipMemcpyAsync(tallies, snap, j->lay.tally_bytes, hipMemcpyDeviceToDevice, s));
            if ((st = run.clear_overflow(s)) != KARL_OK) {
                j->failed = true;
                return st;
            }
            if (n == 1) {
                j->failed = true;
                return fail(KARL_EOVERFLOW, "primary %lld alone overflows a queue of %lld entries",
                            (long long)b, (long long)run.capacity);
            }
            chunk = std::max<int64_t>(1, n / 2);
            continue;
        }
        int64_t s1 = 0, i1 = 0;
        if ((st = read_steps(j, s, &s1, &i1)) != KARL_OK) return st;
        if (s1 > s0 && run.ev0) j->ms_seg[wave ? 1 : 0] = (run.kernel_ms - k0) / (double)(s1 - s0);
        if (j->chosen == KARL_MAP_AUTO && s1 - s0 >= kTuneSegments) {
            j->seg_per_int = (double)(s1 - s0) / (double)std::max<int64_t>(1, i1 - i0);
            j->chosen = j->seg_per_int >= kWaveRatio ? KARL_MAP_WAVE : KARL_MAP_LANE;
        }
        b += n;
        j->n_transported += n;
        chunk = next_chunk(chunk, n, max_gen, run.capacity);
    }
    return KARL_OK;
}

// ---- transport without allocation (karl_transport_noalloc)
// Callers that cannot allocate device memory get their queues, control words and tally
// snapshot from this array, one copy per device, held until the process ends.  In host code
// its name is only a stand-in: the device address comes from hipGetSymbolAddress, once per
// device, and only that address is passed to kernels and copies.
constexpr int kMaxDevices = 64;
constexpr int64_t kNoallocMinEntries = 4096;
static __device__ __align__(256) unsigned char scratch[KARL_NOALLOC_SCRATCH_BYTES];
std::mutex g_noalloc_mu[kMaxDevices];
char* g_noalloc_ptr[kMaxDevices] = {};
Launcher g_noalloc_run[kMaxDevices];
unsigned long long g_noalloc_host[kMaxDevices][8];

// the device address of `scratch` on `dev` (the current device), looked up on first use
karl_status noalloc_scratch(int dev, char** out) {
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(KARL_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                        hipGetErrorString(e));
        g_noalloc_ptr[dev] = (char*)p;
    }
    *out = g_noalloc_ptr[dev];
    return KARL_OK;
}

}  // namespace

extern "C" {

const char* karl_last_error(void) { return g_err; }

// error reporting for the serving layer, which lives in its own translation unit
__attribute__((visibility("hidden"))) karl_status karl_internal_set_error(karl_status code,
                                                                          const char* msg) {
    snprintf(g_err, sizeof(g_err), "%s", msg);
    return code;
}

karl_status karl_workspace_bytes(const karl_job_desc* desc, uint64_t* bytes) {
    if (!bytes) return fail(KARL_EINVAL, "bytes is NULL");
    karl_status st = validate(desc, false);
    if (st != KARL_OK) return st;
    *bytes = make_layout(desc).total;
    return KARL_OK;
}

karl_status karl_create_job(const karl_job_desc* d, void** out) {
    g_err[0] = '\0';
    if (!out) return fail(KARL_EINVAL, "out is NULL");
    *out = nullptr;
    karl_status st = validate(d, true);
    if (st != KARL_OK) return st;
    Job* j = new Job();
    j->precision = d->precision;
    j->flags = d->flags;
    j->n_primaries = d->n_primaries;
    j->n_r = d->n_r;
    j->n_z = d->n_z;
    j->n_planes = d->n_planes;
    j->n_bins = d->n_bins;
    j->ws = (char*)d->workspace;
    j->lay = make_layout(d);
    j->chunk = d->chunk > 0 ? d->chunk : kDefaultChunk;
    j->slice_steps = d->slice_steps;
    j->mapping = d->mapping;
    // flights meet r-faces without a field; the Boris mover has no wave-cooperative flight
    j->chosen = (d->bz == 0.0 || d->mover == KARL_MOVER_BORIS) ? KARL_MAP_LANE : d->mapping;
    const Layout& L = j->lay;
    auto cleanup = [&](karl_status s) {
        j->run.release();
        delete j;
        return s;
    };
#define TRY(expr)                                 \
    do {                                          \
        karl_status s_ = (expr);                  \
        if (s_ != KARL_OK) return cleanup(s_);    \
    } while (0)
#define TRY_HIP(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return cleanup(fail(KARL_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_))); \
    } while (0)

    TRY_HIP(hipGetDevice(&j->device));

    // ---- host-side tables
    const int nz = d->n_z, nr = d->n_r;
    const int ns = species_count(d);
    // three-body tables (k/v, m^5, ~1e-44) are stored scaled by 2^100 in FP32, whose smallest
    // normal number is 1.2e-38; the kernel multiplies the rate by 2^-100 again
    const double p2scale = d->precision == KARL_FP32 ? std::ldexp(1.0, -100) : 1.0;
    std::vector<double> xs((size_t)d->n_proc * d->n_e);
    for (int i = 0; i < d->n_proc; ++i) {
        const double sc = d->proc[i].density_power == 2 ? 1.0 / p2scale : 1.0;
        for (int k = 0; k < d->n_e; ++k) xs[(size_t)i * d->n_e + k] = d->proc[i].xs[k] * sc;
    }
    std::vector<double> ngas(d->n_gas, d->n_gas + nz);
    std::vector<double> zf(nz + 1), rf(nr + 1), zcdf(nz + 1);
    for (int k = 0; k <= nz; ++k) zf[k] = d->length * (double)k / (double)nz;
    for (int k = 0; k <= nr; ++k) rf[k] = d->radius * (double)k / (double)nr;
    zcdf[0] = 0.0;
    for (int k = 0; k < nz; ++k) zcdf[k + 1] = zcdf[k] + d->n_gas[k];
    std::vector<double> edges((size_t)ns * ((size_t)d->n_bins + 1));
    for (int s = 0; s < ns; ++s)
        std::memcpy(&edges[(size_t)s * (d->n_bins + 1)], d->species[s].edges,
                    sizeof(double) * ((size_t)d->n_bins + 1));
    std::vector<int32_t> plane_of(nz + 1, -1);
    for (int p = 0; p < d->n_planes; ++p)
        if (plane_of[d->planes[p]] < 0) plane_of[d->planes[p]] = p;

    TRY(upload_real(*j, L.xs, xs));
    TRY(upload_real(*j, L.n_gas, ngas));
    TRY(upload_real(*j, L.zf, zf));
    TRY(upload_real(*j, L.rf, rf));
    TRY(upload_real(*j, L.zcdf, zcdf));
    if (uses_fields(d)) {
        // one density field per species; absent: 0
        TRY_HIP(karl::launch_fill_u64((unsigned long long*)(j->ws + L.tfield), (size_t)ns * nr * nz, 0ull, nullptr));
        for (int f = 0; f < ns; ++f)
            if (d->n_field[f])
                TRY_HIP(hipMemcpy(j->ws + L.tfield + 8 * (size_t)f * nr * nz, d->n_field[f],
                                  sizeof(double) * (size_t)nr * nz, hipMemcpyHostToDevice));
    }
    TRY_HIP(hipMemcpy(j->ws + L.edges, edges.data(), sizeof(double) * edges.size(), hipMemcpyHostToDevice));
    TRY_HIP(hipMemcpy(j->ws + L.plane_of, plane_of.data(), sizeof(int32_t) * plane_of.size(), hipMemcpyHostToDevice));
    if (d->n_dens_bins > 0) {
        std::vector<double> de((size_t)ns * ((size_t)d->n_dens_bins + 1));
        for (int s = 0; s < ns; ++s)
            std::memcpy(&de[(size_t)s * (d->n_dens_bins + 1)], d->species[s].dens_edges,
                        sizeof(double) * ((size_t)d->n_dens_bins + 1));
        TRY_HIP(hipMemcpy(j->ws + L.dens_edges, de.data(), sizeof(double) * de.size(), hipMemcpyHostToDevice));
    }
    if (d->e_field || d->b_field) {
        const size_t nb = (size_t)d->field_nr * (size_t)d->field_nz * 3;
        if (d->e_field) TRY_HIP(hipMemcpy(j->ws + L.e_fld, d->e_field, 8 * nb, hipMemcpyHostToDevice));
        if (d->b_field) TRY_HIP(hipMemcpy(j->ws + L.b_fld, d->b_field, 8 * nb, hipMemcpyHostToDevice));
    }
    // angle tables with the cumulative areas of the piecewise linear densities (trapezoids,
    // left to right)
    size_t ang_off = 0;
    std::vector<size_t> ang_at(d->n_proc, 0);
    if (angle_doubles(d) > 0) {
        std::vector<double> tab(angle_doubles(d));
        for (int i = 0; i < d->n_proc; ++i) {
            const karl_process_desc& p = d->proc[i];
            ang_at[i] = ang_off;
            if (p.ang_bins <= 0) continue;
            const int nb = p.ang_bins, n = p.ang_nodes;
            double* e = tab.data() + ang_off;
            double* th = e + nb + 1;
            double* cdf = th + n;
            double* pdf = cdf + (size_t)nb * n;
            for (int b = 0; b <= nb; ++b) e[b] = p.ang_edges[b];
            for (int k = 0; k < n; ++k) th[k] = p.ang_theta[k];
            for (int b = 0; b < nb; ++b) {
                const double* f = p.ang_pdf + (size_t)b * n;
                double* c = cdf + (size_t)b * n;
                c[0] = 0.0;
                for (int k = 0; k + 1 < n; ++k) c[k + 1] = c[k] + 0.5 * (f[k] + f[k + 1]) * (th[k + 1] - th[k]);
                for (int k = 0; k < n; ++k) pdf[(size_t)b * n + k] = f[k];
            }
            ang_off += angle_block(p);
        }
        TRY_HIP(hipMemcpy(j->ws + L.angles, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice));
    }

    // ---- device job
    karl::DevJob& J = j->dj;
    J.radius = d->radius;
    J.length = d->length;
    J.n_r = nr;
    J.n_z = nz;
    J.n_e = d->n_e;
    J.n_proc = d->n_proc;
    J.n_bins = d->n_bins;
    J.n_planes = d->n_planes;
    J.boris = d->mover == KARL_MOVER_BORIS ? 1 : 0;
    J.gc = (d->bz != 0.0 && !J.boris) ? 1 : 0;   // the Boris mover follows the particle itself
    J.bz = d->bz;
    J.field_nr = d->field_nr;
    J.field_nz = d->field_nz;
    J.field_radius = d->field_radius;
    J.field_length = d->field_length;
    J.e_fld = d->e_field ? (const double*)(j->ws + L.e_fld) : nullptr;
    J.b_fld = d->b_field ? (const double*)(j->ws + L.b_fld) : nullptr;
    J.source = d->source;
    J.beam_species = d->beam_species;
    J.flags = (int32_t)d->flags;
    J.seed = d->seed;
    J.n_species = ns;
    for (int s = 0; s < karl::kS; ++s) {
        J.sc.nps[s] = 0;
        J.sc.field_of[s] = -1;
        J.sc.defer[s] = 0;
        J.sc.field[s] = nullptr;
        if (s >= ns) {
            // unused slots: harmless values (never selected by a particle)
            J.sc.tracked[s] = 0;
            J.sc.cap[s] = 1;
            J.sc.mass[s] = J.sc.charge[s] = J.sc.e_cut[s] = J.sc.lifetime[s] = J.sc.msum[s] = 0.0;
            J.sc.xs_emin[s] = J.sc.inv_dlog[s] = J.sc.omega[s] = J.sc.mfrac[s] = J.sc.gfrac[s] = 0.0;
            J.sc.inv_emin[s] = J.sc.inv_om[s] = J.sc.e_from_v2[s] = J.sc.v2_from_e[s] = 0.0;
            J.sc.boris_dt[s] = J.sc.boris_h[s] = 0.0;
            continue;
        }
        const karl_species_desc& sp = d->species[s];
        J.sc.tracked[s] = sp.tracked ? 1 : 0;
        J.sc.cap[s] = sp.cap;
        J.sc.mass[s] = sp.mass;
        J.sc.charge[s] = sp.charge;
        J.sc.e_cut[s] = sp.e_cut;
        J.sc.lifetime[s] = sp.lifetime;
        J.sc.msum[s] = sp.mass + d->m_gas;
        J.sc.xs_emin[s] = sp.xs_emin;
        J.sc.inv_dlog[s] = (double)(d->n_e - 1) / std::log(sp.xs_emax / sp.xs_emin);
        J.sc.omega[s] = sp.charge * d->bz / sp.mass;
        const double mt = sp.mass + d->m_gas;
        J.sc.mfrac[s] = sp.mass / mt;
        J.sc.gfrac[s] = d->m_gas / mt;
        J.sc.inv_emin[s] = 1.0 / sp.xs_emin;
        J.sc.inv_om[s] = (J.sc.omega[s] != 0.0) ? 1.0 / J.sc.omega[s] : 0.0;
        J.sc.e_from_v2[s] = 0.5 * sp.mass / kQE;
        J.sc.v2_from_e[s] = 2.0 * kQE / sp.mass;
        J.sc.boris_dt[s] = d->mover == KARL_MOVER_BORIS ? d->boris_dt[s] : 0.0;
        J.sc.boris_h[s] = d->mover == KARL_MOVER_BORIS ? 0.5 * d->boris_dt[s] * sp.charge / sp.mass : 0.0;
    }
    for (int i = 0; i < KARL_MAX_PROC; ++i) {
        const bool has_ang = i < d->n_proc && d->proc[i].ang_bins > 0;
        J.ang[i] = has_ang ? (const double*)(j->ws + L.angles) + ang_at[i] : nullptr;
        J.ang_nb[i] = has_ang ? d->proc[i].ang_bins : 0;
        J.ang_n[i] = has_ang ? d->proc[i].ang_nodes : 0;
        J.e_iso[i] = has_ang ? d->proc[i].e_iso : 0.0;
        const karl_process_desc* pr = i < d->n_proc ? &d->proc[i] : nullptr;
        J.kind[i] = pr ? pr->kind : 0;
        J.target[i] = !pr ? karl::TGT_GAS
                          : pr->target == KARL_TARGET_FIELD ? karl::TGT_FIELD
                          : pr->density_power == 2 ? karl::TGT_GAS2 : karl::TGT_GAS;
        J.product[i] = pr && (pr->kind == KARL_IONIZATION || pr->kind == KARL_CLUSTERING) ? pr->product : 0;
        J.partner[i] = pr && (pr->target == KARL_TARGET_FIELD || pr->kind == KARL_RECOMBINATION) ? pr->partner : 0;
        J.conv[i] = pr && pr->kind == KARL_CLUSTERING ? d->m_gas / d->species[pr->product].mass : 0.0;
        J.e_th[i] = pr ? pr->e_th : 0.0;
        J.e_th_f[i] = (float)J.e_th[i];
    }
    for (int i = 0; i < d->n_proc; ++i) {
        const int s = d->proc[i].species;
        J.pidx[s][J.sc.nps[s]++] = i;
        if (d->proc[i].target == KARL_TARGET_FIELD) J.sc.field_of[s] = d->proc[i].partner;
    }
    // A species without ionization or clustering never produces particles: its particles can
    // wait in the deferred queue and run together in one launch after the other generations.
    for (int s = 0; s < ns; ++s) {
        bool produces = false;
        for (int i = 0; i < d->n_proc; ++i)
            if (d->proc[i].species == s &&
                (d->proc[i].kind == KARL_IONIZATION || d->proc[i].kind == KARL_CLUSTERING))
                produces = true;
        // the drain launch has no Boris mover: Boris jobs keep every particle in the generations
        J.sc.defer[s] = (produces || J.boris) ? 0 : 1;
    }
    J.p2scale = p2scale;
    J.sigma_v = std::sqrt(kKB * d->t_gas / d->m_gas);
    J.m_gas = d->m_gas;
    J.beta_e0 = d->beta_e0;
    J.beta_z = d->beta_z;
    J.beta_fmax = d->beta_fmax;
    J.beam_e = d->beam_energy;
    J.beam_e1 = d->beam_energy_1;
    for (int k = 0; k < 3; ++k) {
        J.beam_pos[k] = d->beam_pos[k];
        J.beam_dir[k] = d->beam_dir[k];
    }
    J.beam_ir = count_faces_le(rf, nr, std::sqrt(d->beam_pos[0] * d->beam_pos[0] + d->beam_pos[1] * d->beam_pos[1]));
    J.beam_iz = count_faces_le(zf, nz, d->beam_pos[2]);
    char* w = j->ws;
    J.xs = w + L.xs;
    J.n_gas = w + L.n_gas;
    J.zf = w + L.zf;
    J.rf = w + L.rf;
    J.zcdf = w + L.zcdf;
    for (int f = 0; f < ns; ++f)
        J.sc.field[f] = uses_fields(d) ? (double*)(w + L.tfield + 8 * (size_t)f * nr * nz) : nullptr;
    J.edges = (const double*)(w + L.edges);
    J.plane_of = (const int32_t*)(w + L.plane_of);
    char* t = w + L.tallies;
    J.counters = (unsigned long long*)(t + L.t_counters);
    J.ledger = (double*)(t + L.t_ledger);
    J.dens = (double*)(t + L.t_dens);
    J.recomb = (unsigned long long*)(t + L.t_recomb);
    J.jz = (unsigned long long*)(t + L.t_jz);
    J.jr = (unsigned long long*)(t + L.t_jr);
    J.spectra = (unsigned long long*)(t + L.t_spectra);
    J.digests = (d->flags & KARL_FLAG_DIGESTS) ? (unsigned long long*)(t + L.t_digests) : nullptr;
    J.hist = (d->flags & KARL_FLAG_HISTORY) ? (double*)(t + L.t_hist) : nullptr;
    J.n_dens_bins = d->n_dens_bins;
    J.dens_edges = d->n_dens_bins > 0 ? (const double*)(w + L.dens_edges) : nullptr;
    J.dense = d->n_dens_bins > 0 ? (double*)(t + L.t_dense) : nullptr;
    unsigned long long* ctl = (unsigned long long*)(w + L.control);
    j->status = (unsigned int*)(ctl + 5);     // the job's own sticky status (NaN met)
    J.status = j->status;

    const size_t lds = karl::lds_bytes(J, d->precision);   // at most kMaxLds (validated)
    TRY_HIP(hipMemcpy(w + L.devjob, &J, sizeof(J), hipMemcpyHostToDevice));
    j->lds = lds;
    j->run.ctl = ctl;
    j->run.dense = d->n_dens_bins > 0;
    j->run.boris = d->mover == KARL_MOVER_BORIS;
    j->run.jobs_dev = (karl::DevJob*)(w + L.devjob);
    TRY_HIP(karl::launch_fill_u64(ctl, kControlBytes / 8, 0ull, nullptr));
    TRY_HIP(karl::launch_fill_u64((unsigned long long*)t, L.tally_bytes / 8, 0ull, nullptr));
    TRY_HIP(hipStreamSynchronize(nullptr));
#undef TRY
#undef TRY_HIP
    *out = j;
    return KARL_OK;
}

karl_status karl_transport(void* job, int64_t pid_begin, int64_t pid_end, void* hip_stream) {
    Job* j = (Job*)job;
    if (!j) return fail(KARL_ESTATE, "job is NULL");
    if (j->failed) return fail(KARL_ESTATE, "job failed earlier; destroy and recreate it");
    if (pid_begin < 0 || pid_end < pid_begin || pid_end > j->n_primaries)
        return fail(KARL_EINVAL, "pid range [%lld, %lld) outside 0..%lld", (long long)pid_begin,
                    (long long)pid_end, (long long)j->n_primaries);
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_CHECK(hipSetDevice(j->device));
    karl_status st = ensure_launcher(j);
    if (st != KARL_OK) return st;
    return transport_range(j, j->run, j->ws + j->lay.snapshot, j->chunk, pid_begin, pid_end, s);
}

karl_status karl_transport_noalloc(void* job, int64_t pid_begin, int64_t pid_end, void* hip_stream) {
    Job* j = (Job*)job;
    if (!j) return fail(KARL_ESTATE, "job is NULL");
    if (j->failed) return fail(KARL_ESTATE, "job failed earlier; destroy and recreate it");
    if (pid_begin < 0 || pid_end < pid_begin || pid_end > j->n_primaries)
        return fail(KARL_EINVAL, "pid range [%lld, %lld) outside 0..%lld", (long long)pid_begin,
                    (long long)pid_end, (long long)j->n_primaries);
    if (j->device < 0 || j->device >= kMaxDevices)
        return fail(KARL_EINVAL, "device %d beyond the %d devices of the no-allocation path",
                    j->device, kMaxDevices);
    // the array holds the control words, a snapshot of the tallies (undo of a chunk whose queue
    // overflowed) and four queues of at least kNoallocMinEntries entries
    const size_t fixed = align_up(kControlBytes) + align_up(j->lay.tally_bytes);
    if (fixed + 4 * (size_t)kNoallocMinEntries * kQueueEntryBytes > KARL_NOALLOC_SCRATCH_BYTES)
        return fail(KARL_EINVAL, "the job's tallies (%zu bytes) leave no room for queues of %lld entries "
                    "in the %zu-byte array of karl_transport_noalloc; use karl_transport",
                    j->lay.tally_bytes, (long long)kNoallocMinEntries, (size_t)KARL_NOALLOC_SCRATCH_BYTES);
    if (pid_end == pid_begin) return KARL_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_CHECK(hipSetDevice(j->device));
    std::lock_guard<std::mutex> lk(g_noalloc_mu[j->device]);
    char* base = nullptr;
    karl_status st = noalloc_scratch(j->device, &base);
    if (st != KARL_OK) return st;
    unsigned long long* ctl = (unsigned long long*)base;
    char* snap = base + align_up(kControlBytes);
    char* queues = snap + align_up(j->lay.tally_bytes);
    const size_t entries = (KARL_NOALLOC_SCRATCH_BYTES - fixed) / (4 * kQueueEntryBytes);
    Launcher& run = g_noalloc_run[j->device];
    run = Launcher{};
    if ((st = run.init(queues, entries, ctl, j->precision, false, j->lds, g_noalloc_host[j->device])) != KARL_OK)
        return st;
    run.jobs_dev = j->run.jobs_dev;
    run.dense = j->run.dense;
    run.boris = j->run.boris;
    // the array keeps the previous call's contents: the control words start at zero
    HIP_CHECK(karl::launch_fill_u64(ctl, kControlBytes / 8, 0ull, s));
    int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(j->chunk, (int64_t)entries / 4));
    return transport_range(j, run, snap, chunk, pid_begin, pid_end, s);
}

karl_status karl_read_tallies(void* job, karl_tallies* out, void* hip_stream) {
    Job* j = (Job*)job;
    if (!j || !out) return fail(KARL_EINVAL, "job or out is NULL");
    HIP_CHECK(hipSetDevice(j->device));
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_CHECK(hipStreamSynchronize(s));
    const karl::DevJob& J = j->dj;
    const size_t nr = (size_t)j->n_r, nz = (size_t)j->n_z, ns = (size_t)J.n_species;
    auto get = [&](void* dst, const void* src, size_t bytes) -> karl_status {
        if (dst && src && bytes) HIP_CHECK(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
        return KARL_OK;
    };
    karl_status st;
    if ((st = get(out->counters, J.counters, 8 * KARL_NCOUNTERS)) != KARL_OK) return st;
    if ((st = get(out->ledger, J.ledger, 8 * KARL_NLEDGER)) != KARL_OK) return st;
    if ((st = get(out->density_time, J.dens, 8 * ns * nr * nz)) != KARL_OK) return st;
    if ((st = get(out->recomb, J.recomb, 8 * ns * nr * nz)) != KARL_OK) return st;
    if ((st = get(out->jz, J.jz, 8 * ns * nr * (nz + 1) * 2)) != KARL_OK) return st;
    if ((st = get(out->jr, J.jr, 8 * ns * (nr + 1) * nz * 2)) != KARL_OK) return st;
    if ((st = get(out->spectra, J.spectra, 8 * ns * (size_t)j->n_planes * 2 * ((size_t)j->n_bins + 2))) != KARL_OK)
        return st;
    if (out->digests) {
        if (!J.digests) return fail(KARL_EINVAL, "digests requested but KARL_FLAG_DIGESTS not set");
        if ((st = get(out->digests, J.digests, 8 * (size_t)j->n_primaries)) != KARL_OK) return st;
    }
    if (out->density_time_e) {
        if (!J.dense) return fail(KARL_EINVAL, "energy-resolved density requested but n_dens_bins is 0");
        if ((st = get(out->density_time_e, J.dense, 8 * ns * nr * nz * ((size_t)J.n_dens_bins + 2))) != KARL_OK)
            return st;
    }
    if (out->hist) {
        if (!J.hist) return fail(KARL_EINVAL, "history ledger requested but KARL_FLAG_HISTORY not set");
        if ((st = get(out->hist, J.hist, 8 * KARL_NHIST * (size_t)j->n_primaries)) != KARL_OK) return st;
    }
    unsigned int status = 0;
    HIP_CHECK(hipMemcpy(&status, j->status, sizeof(status), hipMemcpyDeviceToHost));
    if (status & karl::STATUS_NUMERIC) return fail(KARL_ENUMERIC, "NaN met in the particle state");
    if (j->failed) return fail(KARL_ESTATE, "job failed earlier; tallies are incomplete");
    return KARL_OK;
}

karl_status karl_read_fields(void* job, double activity, double* density, double* jz_current,
                             double* jr_current, void* hip_stream) {
    Job* j = (Job*)job;
    if (!j) return fail(KARL_EINVAL, "job is NULL");
    if (!(activity > 0.0) || !std::isfinite(activity))
        return fail(KARL_EINVAL, "activity must be positive and finite");
    if (j->n_transported <= 0) return fail(KARL_ESTATE, "no primaries transported since the last reset");
    HIP_CHECK(hipSetDevice(j->device));
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t nr = (size_t)j->n_r, nz = (size_t)j->n_z, ns = (size_t)j->dj.n_species;
    const size_t n_dens = ns * nr * nz, n_jz = ns * nr * (nz + 1), n_jr = ns * (nr + 1) * nz;
    double* f = (double*)(j->ws + j->lay.fields);
    const double t_sim = (double)j->n_transported / activity;
    HIP_CHECK(karl::launch_fields(j->dj, t_sim, f, f + n_dens, f + n_dens + n_jz, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (density) HIP_CHECK(hipMemcpy(density, f, 8 * n_dens, hipMemcpyDeviceToHost));
    if (jz_current) HIP_CHECK(hipMemcpy(jz_current, f + n_dens, 8 * n_jz, hipMemcpyDeviceToHost));
    if (jr_current) HIP_CHECK(hipMemcpy(jr_current, f + n_dens + n_jz, 8 * n_jr, hipMemcpyDeviceToHost));
    return KARL_OK;
}

karl_status karl_update_target_fields(void* job, double activity, void* hip_stream) {
    Job* j = (Job*)job;
    if (!j) return fail(KARL_EINVAL, "job is NULL");
    if (!(activity > 0.0) || !std::isfinite(activity))
        return fail(KARL_EINVAL, "activity must be positive and finite");
    if (j->n_transported <= 0) return fail(KARL_ESTATE, "no primaries transported since the last reset");
    if (!j->dj.sc.field[0]) return KARL_OK;   // no process targets a field
    HIP_CHECK(hipSetDevice(j->device));
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_CHECK(karl::launch_target_fields(j->dj, (double)j->n_transported / activity, s));
    HIP_CHECK(hipStreamSynchronize(s));
    return KARL_OK;
}

karl_status karl_reset_tallies(void* job, void* hip_stream) {
    Job* j = (Job*)job;
    if (!j) return fail(KARL_EINVAL, "job is NULL");
    HIP_CHECK(hipSetDevice(j->device));
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_CHECK(karl::launch_fill_u64((unsigned long long*)(j->ws + j->lay.tallies), j->lay.tally_bytes / 8, 0ull, s));
    HIP_CHECK(karl::launch_fill_u64(j->run.ctl, kControlBytes / 8, 0ull, s));
    HIP_CHECK(hipStreamSynchronize(s));
    j->run.reset_stats();
    j->n_transported = 0;
    j->failed = false;
    return KARL_OK;
}

karl_status karl_job_stats(void* job, double* kernel_ms, int64_t* n_launches, int64_t* generations,
                           int64_t* max_queue) {
    Job* j = (Job*)job;
    if (!j) return fail(KARL_EINVAL, "job is NULL");
    if (kernel_ms) *kernel_ms = j->run.kernel_ms;
    if (n_launches) *n_launches = j->run.launches;
    if (generations) *generations = j->run.generations;
    if (max_queue) *max_queue = j->run.max_queue;
    return KARL_OK;
}

karl_status karl_job_drain_stats(void* job, double* kernel_ms, int64_t* n_launches) {
    Job* j = (Job*)job;
    if (!j || !kernel_ms || !n_launches) return fail(KARL_EINVAL, "job and outputs must not be NULL");
    *kernel_ms = j->run.drain_ms;
    *n_launches = j->run.drain_launches;
    return KARL_OK;
}

karl_status karl_job_slices(void* job, int64_t* ring_entries) {
    Job* j = (Job*)job;
    if (!j || !ring_entries) return fail(KARL_EINVAL, "job and ring_entries must not be NULL");
    *ring_entries = j->run.slices;
    return KARL_OK;
}

karl_status karl_job_mapping(void* job, int32_t* mapping, double* segments_per_interaction,
                             double* ms_per_segment_lane, double* ms_per_segment_wave,
                             int64_t* wave_segments) {
    Job* j = (Job*)job;
    if (!j) return fail(KARL_EINVAL, "job is NULL");
    if (mapping) *mapping = j->chosen;
    if (segments_per_interaction) *segments_per_interaction = j->seg_per_int;
    if (ms_per_segment_lane) *ms_per_segment_lane = j->ms_seg[0];
    if (ms_per_segment_wave) *ms_per_segment_wave = j->ms_seg[1];
    if (wave_segments) {
        unsigned long long v = 0ull;
        HIP_CHECK(hipSetDevice(j->device));
        HIP_CHECK(hipMemcpy(&v, j->run.ctl + 6, sizeof(v), hipMemcpyDeviceToHost));
        *wave_segments = (int64_t)v;
    }
    return KARL_OK;
}

karl_status karl_destroy_job(void* job) {
    Job* j = (Job*)job;
    if (!j) return fail(KARL_EINVAL, "job is NULL");
    j->run.release();
    delete j;
    return KARL_OK;
}

// ---------------------------------------------------------------- batches

karl_status karl_batch_workspace_bytes(int32_t max_jobs, int64_t queue_capacity, uint64_t* bytes) {
    if (!bytes || max_jobs < 1 || queue_capacity < 0)
        return fail(KARL_EINVAL, "need max_jobs >= 1, queue_capacity >= 0 and a result pointer");
    size_t a, b, c, d;
    *bytes = batch_layout(max_jobs, queue_capacity > 0 ? queue_capacity : kDefaultCapacity, &a, &b, &c, &d);
    return KARL_OK;
}

karl_status karl_create_batch(int32_t max_jobs, int64_t queue_capacity, void* workspace,
                              uint64_t workspace_bytes, void** out) {
    g_err[0] = '\0';
    if (!out) return fail(KARL_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_jobs < 1 || queue_capacity < 0) return fail(KARL_EINVAL, "need max_jobs >= 1 and queue_capacity >= 0");
    if (!workspace) return fail(KARL_EINVAL, "workspace is NULL");
    const int64_t entries = queue_capacity > 0 ? queue_capacity : kDefaultCapacity;
    size_t o_jobs, o_pj, o_ctl, o_q;
    const size_t need = batch_layout(max_jobs, entries, &o_jobs, &o_pj, &o_ctl, &o_q);
    if (workspace_bytes < need)
        return fail(KARL_ENOMEM, "batch workspace has %llu bytes, needs %llu",
                    (unsigned long long)workspace_bytes, (unsigned long long)need);
    Batch* b = new Batch();
    b->max_jobs = max_jobs;
    b->ws = (char*)workspace;
    int64_t* pj = (int64_t*)(b->ws + o_pj);
    b->job_first = pj;
    b->job_count = pj + max_jobs;
    b->job_cum = pj + 2 * (size_t)max_jobs;
    auto cleanup = [&](karl_status s) {
        b->run[0].release();
        b->run[1].release();
        if (b->host_i64) (void)hipHostFree(b->host_i64);
        if (b->host_jobs) (void)hipHostFree(b->host_jobs);
        delete b;
        return s;
    };
    if (hipGetDevice(&b->device) != hipSuccess) return cleanup(fail(KARL_EDEVICE, "hipGetDevice failed"));
    unsigned long long* ctl = (unsigned long long*)(b->ws + o_ctl);
    for (int p = 0; p < 2; ++p) {
        karl_status st = b->run[p].init(b->ws + o_q, (size_t)entries, ctl, p == 0 ? KARL_FP64 : KARL_FP32,
                                        true, karl::batched_lds_bytes());
        if (st != KARL_OK) return cleanup(st);
        b->run[p].jobs_dev = (karl::DevJob*)(b->ws + o_jobs);
        b->run[p].job_first = pj;
        b->run[p].job_count = pj + max_jobs;
        b->run[p].job_cum = pj + 2 * (size_t)max_jobs;
        b->run[p].job_fetch = (unsigned long long*)(pj + 3 * (size_t)max_jobs);
        b->run[p].job_waves = (unsigned long long*)(pj + 4 * (size_t)max_jobs);
        b->run[p].sort_counts = (unsigned long long*)(pj + 5 * (size_t)max_jobs);
        b->run[p].sort_cursor = (unsigned long long*)(pj + 6 * (size_t)max_jobs);
    }
    if (hipHostMalloc((void**)&b->host_i64, 8 * (3 * (size_t)max_jobs), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&b->host_jobs, sizeof(karl::DevJob) * (size_t)max_jobs, hipHostMallocDefault) != hipSuccess)
        return cleanup(fail(KARL_EDEVICE, "pinned staging allocation failed"));
    *out = b;
    return KARL_OK;
}

karl_status karl_transport_batch(void* batch, void* const* jobs, const int64_t* ranges, int32_t n_jobs,
                                 void* hip_stream) {
    Batch* B = (Batch*)batch;
    if (!B) return fail(KARL_ESTATE, "batch is NULL");
    if (n_jobs < 0 || n_jobs > B->max_jobs)
        return fail(KARL_EINVAL, "n_jobs %d outside 0..%d", n_jobs, B->max_jobs);
    if (n_jobs == 0) return KARL_OK;
    if (!jobs || !ranges) return fail(KARL_EINVAL, "jobs or ranges is NULL");
    const int prec = ((Job*)jobs[0])->precision;
    std::vector<int64_t> offs(n_jobs + 1, 0);      // items of job i: [offs[i], offs[i+1])
    for (int32_t i = 0; i < n_jobs; ++i) {
        Job* j = (Job*)jobs[i];
        if (!j) return fail(KARL_ESTATE, "job %d is NULL", i);
        if (j->failed) return fail(KARL_ESTATE, "job %d failed earlier", i);
        if (j->precision != prec) return fail(KARL_EINVAL, "jobs of one batch share the precision");
        if (j->device != B->device) return fail(KARL_EINVAL, "job %d lives on another device", i);
        const int64_t b = ranges[2 * i], e = ranges[2 * i + 1];
        if (b < 0 || e < b || e > j->n_primaries)
            return fail(KARL_EINVAL, "job %d: pid range [%lld, %lld) invalid", i, (long long)b, (long long)e);
        B->host_jobs[i] = j->dj;
        B->host_jobs[i].wave = j->chosen == KARL_MAP_WAVE ? 1 : 0;
        offs[i + 1] = offs[i] + (e - b);
    }
    const int64_t total = offs[n_jobs];
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_CHECK(hipSetDevice(B->device));
    Launcher& R = B->run[prec == KARL_FP32 ? 1 : 0];
    R.n_jobs = n_jobs;
    // the kernel built with the Boris mover only when a job of the batch needs it
    R.boris = false;
    for (int i = 0; i < n_jobs; ++i) R.boris = R.boris || ((Job*)jobs[i])->dj.boris != 0;
    // the kernel variant with wave-cooperative flights only while a job of the batch uses them
    auto any_wave = [&]() {
        for (int i = 0; i < n_jobs; ++i)
            if (B->host_jobs[i].wave) return true;
        return false;
    };
    R.coop = any_wave();
    HIP_CHECK(hipMemcpyAsync(R.jobs_dev, B->host_jobs, sizeof(karl::DevJob) * (size_t)n_jobs, hipMemcpyHostToDevice, s));
    int64_t c0 = 0;
    while (c0 < total) {
        const int64_t n = std::min<int64_t>(B->chunk, total - c0);
        // the chunk's primaries per job: first id and count
        const int j_lo = (int)(std::upper_bound(offs.begin(), offs.end(), c0) - offs.begin()) - 1;
        const int j_hi = (int)(std::lower_bound(offs.begin(), offs.end(), c0 + n) - offs.begin());
        int64_t cum = 0;
        for (int i = 0; i < n_jobs; ++i) {
            const int64_t lo = std::max(c0, offs[i]), hi = std::min(c0 + n, offs[i + 1]);
            const int64_t cnt = hi > lo ? hi - lo : 0;
            B->host_i64[i] = ranges[2 * i] + (cnt > 0 ? lo - offs[i] : 0);
            B->host_i64[n_jobs + i] = cnt;
            B->host_i64[2 * n_jobs + i] = cum;
            cum += cnt;
        }
        HIP_CHECK(hipMemcpyAsync(B->job_first, B->host_i64, 8 * (size_t)n_jobs, hipMemcpyHostToDevice, s));
        HIP_CHECK(hipMemcpyAsync(B->job_count, B->host_i64 + n_jobs, 8 * (size_t)n_jobs, hipMemcpyHostToDevice, s));
        HIP_CHECK(hipMemcpyAsync(B->job_cum, B->host_i64 + 2 * n_jobs, 8 * (size_t)n_jobs, hipMemcpyHostToDevice, s));
        // snapshot the tallies of the jobs in the chunk for an overflow retry
        for (int i = j_lo; i < j_hi && i < n_jobs; ++i) {
            Job* j = (Job*)jobs[i];
            HIP_CHECK(hipMemcpyAsync(j->ws + j->lay.snapshot, j->ws + j->lay.tallies, j->lay.tally_bytes,
                                     hipMemcpyDeviceToDevice, s));
        }
        karl::GenArgs g{};
        bool overflow = false;
        int64_t max_gen = 0;
        karl_status st = R.run(g, n, s, &overflow, &max_gen);
        if (st != KARL_OK) return st;
        if (overflow) {
            for (int i = j_lo; i < j_hi && i < n_jobs; ++i) {
                Job* j = (Job*)jobs[i];
                HIP_CHECK(hipMemcpyAsync(j->ws + j->lay.tallies, j->ws + j->lay.snapshot, j->lay.tally_bytes,
                                         hipMemcpyDeviceToDevice, s));
            }
            if ((st = R.clear_overflow(s)) != KARL_OK) return st;
            if (n == 1) return fail(KARL_EOVERFLOW, "one primary alone overflows the batch queue");
            B->chunk = std::max<int64_t>(1, n / 2);
            continue;
        }
        // credit the transported primaries to their jobs
        for (int i = j_lo; i < j_hi && i < n_jobs; ++i) {
            const int64_t lo = std::max(c0, offs[i]), hi = std::min(c0 + n, offs[i + 1]);
            if (hi > lo) ((Job*)jobs[i])->n_transported += hi - lo;
        }
        // mapping choice of the jobs still on KARL_MAP_AUTO: once a job's flight segments since
        // creation reach kTuneSegments, its segments per interaction choose the wave mapping for
        // its particles in the following chunks (the crossover measured for single jobs)
        bool changed = false;
        for (int i = j_lo; i < j_hi && i < n_jobs; ++i) {
            Job* j = (Job*)jobs[i];
            if (j->chosen != KARL_MAP_AUTO) continue;
            int64_t segs = 0, ints = 0;
            if ((st = read_steps(j, s, &segs, &ints)) != KARL_OK) return st;
            if (segs < kTuneSegments) continue;
            j->seg_per_int = (double)segs / (double)std::max<int64_t>(1, ints);
            j->chosen = j->seg_per_int >= kWaveRatio ? KARL_MAP_WAVE : KARL_MAP_LANE;
            if (j->chosen == KARL_MAP_WAVE) {
                B->host_jobs[i].wave = 1;
                HIP_CHECK(hipMemcpyAsync(&R.jobs_dev[i].wave, &B->host_jobs[i].wave, sizeof(int32_t),
                                         hipMemcpyHostToDevice, s));
                changed = true;
            }
        }
        if (changed) R.coop = any_wave();
        c0 += n;
        B->chunk = next_chunk(B->chunk, n, max_gen, R.capacity);
    }
    return KARL_OK;
}

karl_status karl_batch_stats(void* batch, double* kernel_ms, int64_t* n_launches, int64_t* generations,
                             int64_t* max_queue) {
    Batch* B = (Batch*)batch;
    if (!B) return fail(KARL_EINVAL, "batch is NULL");
    const Launcher* R[2] = {&B->run[0], &B->run[1]};
    if (kernel_ms) *kernel_ms = R[0]->kernel_ms + R[1]->kernel_ms;
    if (n_launches) *n_launches = R[0]->launches + R[1]->launches;
    if (generations) *generations = R[0]->generations + R[1]->generations;
    if (max_queue) *max_queue = std::max(R[0]->max_queue, R[1]->max_queue);
    return KARL_OK;
}

karl_status karl_batch_wave_segments(void* batch, int64_t* wave_segments) {
    Batch* B = (Batch*)batch;
    if (!B || !wave_segments) return fail(KARL_EINVAL, "batch and wave_segments must not be NULL");
    unsigned long long v = 0ull;
    HIP_CHECK(hipSetDevice(B->device));
    HIP_CHECK(hipMemcpy(&v, B->run[0].ctl + 6, sizeof(v), hipMemcpyDeviceToHost));
    *wave_segments = (int64_t)v;
    return KARL_OK;
}

karl_status karl_destroy_batch(void* batch) {
    Batch* B = (Batch*)batch;
    if (!B) return fail(KARL_EINVAL, "batch is NULL");
    B->run[0].release();
    B->run[1].release();
    if (B->host_i64) (void)hipHostFree(B->host_i64);
    if (B->host_jobs) (void)hipHostFree(B->host_jobs);
    delete B;
    return KARL_OK;
}

}  // extern "C"

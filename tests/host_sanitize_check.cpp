// Test support: the C ABI's host code (descriptor validation, workspace sizing, the error paths
// of every entry point that run before device work) exercised by a program of its own, so that
// the library's host code can be built with AddressSanitizer and UndefinedBehaviorSanitizer
// (device code unchanged).  Needs no GPU: every call here returns before touching a device.
// Prints one line per check and exits 0 when every call returned what it should, 1 otherwise.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "karl.h"

namespace {

int failures = 0;

void expect(bool ok, const char* what) {
    std::printf("%s %s\n", ok ? "ok  " : "FAIL", what);
    if (!ok) ++failures;
}

// A small valid job: electrons and untracked ions in a straight tube, three electron processes.
struct Tiny {
    std::vector<double> n_gas, edges, xs0, xs1, xs2;
    std::vector<int32_t> planes;
    karl_job_desc d;

    Tiny() : n_gas(4, 1e20), edges(33), xs0(16, 1e-20), xs1(16, 5e-21), xs2(16, 2e-21), planes{0, 4} {
        for (int i = 0; i <= 32; ++i) edges[i] = 625.0 * i;
        std::memset(&d, 0, sizeof d);
        d.radius = 0.045;
        d.length = 1.0;
        d.n_r = 1;
        d.n_z = 4;
        d.n_gas = n_gas.data();
        d.t_gas = 80.0;
        d.m_gas = 3.3476e-27;
        d.n_species = 2;
        const double mass[2] = {9.1093837e-31, 3.3466e-27}, charge[2] = {-1.602176634e-19, 1.602176634e-19};
        for (int s = 0; s < 2; ++s) {
            d.species[s].mass = mass[s];
            d.species[s].charge = charge[s];
            d.species[s].e_cut = 1.0;
            d.species[s].lifetime = INFINITY;
            d.species[s].cap = 1000000;
            d.species[s].tracked = s == 0;
            d.species[s].xs_emin = 1.0;
            d.species[s].xs_emax = 2.0e4;
            d.species[s].edges = edges.data();
        }
        d.n_proc = 3;
        d.n_e = 16;
        const double* xs[3] = {xs0.data(), xs1.data(), xs2.data()};
        const int32_t kind[3] = {KARL_ELASTIC, KARL_IONIZATION, KARL_EXCITATION};
        const double eth[3] = {0.0, 15.43, 12.6};
        for (int i = 0; i < 3; ++i) {
            d.proc[i].kind = kind[i];
            d.proc[i].species = 0;
            d.proc[i].target = KARL_TARGET_GAS;
            d.proc[i].product = 1;
            d.proc[i].partner = 1;
            d.proc[i].density_power = 1;
            d.proc[i].e_th = eth[i];
            d.proc[i].xs = xs[i];
        }
        d.source = KARL_SOURCE_BETA;
        d.beta_e0 = 18600.0;
        d.beta_z = 2.0;
        d.beta_fmax = 1.0;
        d.seed = 1;
        d.n_bins = 32;
        d.n_planes = 2;
        d.planes = planes.data();
        d.n_primaries = 100;
        d.precision = KARL_FP64;
        d.queue_capacity = 1024;
        d.mapping = KARL_MAP_AUTO;
    }
};

bool has_message() {
    const char* m = karl_last_error();
    return m != nullptr && std::strlen(m) > 0;
}

// Rejected by sizing and by creation (with a workspace pointer that is never touched), with a
// message, without device work.
void rejected(const char* what, void (*mutate)(karl_job_desc&)) {
    Tiny t;
    mutate(t.d);
    uint64_t bytes = 0;
    const karl_status a = karl_workspace_bytes(&t.d, &bytes);
    t.d.workspace = reinterpret_cast<void*>(uintptr_t(1) << 40);
    t.d.workspace_bytes = uint64_t(1) << 40;
    void* job = nullptr;
    const karl_status b = karl_create_job(&t.d, &job);
    char line[160];
    std::snprintf(line, sizeof line, "rejected: %s (sizing %d, create %d)", what, a, b);
    expect(a == KARL_EINVAL && b == KARL_EINVAL && job == nullptr && has_message(), line);
}

}  // namespace

int main() {
    {
        Tiny t;
        uint64_t bytes = 0;
        expect(karl_workspace_bytes(&t.d, &bytes) == KARL_OK && bytes > 0, "valid descriptor sized");
        t.d.workspace = nullptr;
        void* job = nullptr;
        expect(karl_create_job(&t.d, &job) == KARL_EINVAL && job == nullptr, "no workspace");
        t.d.workspace = reinterpret_cast<void*>(uintptr_t(1) << 40);
        t.d.workspace_bytes = bytes - 1;
        expect(karl_create_job(&t.d, &job) == KARL_ENOMEM && job == nullptr, "workspace one byte short");
    }
    rejected("no grid", [](karl_job_desc& d) { d.n_r = 0; });
    rejected("negative radius", [](karl_job_desc& d) { d.radius = -1.0; });
    rejected("one node", [](karl_job_desc& d) { d.n_e = 1; });
    rejected("1025 nodes", [](karl_job_desc& d) { d.n_e = 1025; });
    rejected("17 processes", [](karl_job_desc& d) { d.n_proc = KARL_MAX_PROC + 1; });
    rejected("unknown process kind", [](karl_job_desc& d) { d.proc[0].kind = 9; });
    rejected("process of a species beyond the job's", [](karl_job_desc& d) { d.proc[0].species = 3; });
    rejected("five species", [](karl_job_desc& d) { d.n_species = KARL_MAX_SPECIES + 1; });
    rejected("unknown precision", [](karl_job_desc& d) { d.precision = 7; });
    rejected("negative primaries", [](karl_job_desc& d) { d.n_primaries = -5; });
    rejected("plane beyond the grid", [](karl_job_desc& d) { const_cast<int32_t*>(d.planes)[1] = 5; });
    rejected("no cross-section table", [](karl_job_desc& d) { d.proc[1].xs = nullptr; });
    rejected("no gas densities", [](karl_job_desc& d) { d.n_gas = nullptr; });
    rejected("NaN gas density", [](karl_job_desc& d) { const_cast<double*>(d.n_gas)[2] = NAN; });
    rejected("slice of three steps", [](karl_job_desc& d) { d.slice_steps = 3; });
    rejected("angle table with one node", [](karl_job_desc& d) {
        static const double e[2] = {0.0, 10.0}, th[1] = {0.0}, pdf[1] = {1.0};
        d.proc[0].ang_bins = 1;
        d.proc[0].ang_nodes = 1;
        d.proc[0].ang_edges = e;
        d.proc[0].ang_theta = th;
        d.proc[0].ang_pdf = pdf;
    });
    rejected("Boris mover without time steps", [](karl_job_desc& d) { d.mover = KARL_MOVER_BORIS; });
    rejected("grid faces beyond the LDS of a workgroup", [](karl_job_desc& d) {
        static std::vector<double> n(8192, 1e20);
        d.n_z = 8192;
        d.n_gas = n.data();
    });
    rejected("FP32 cross section beyond the FP32 range", [](karl_job_desc& d) {
        d.precision = KARL_FP32;
        const_cast<double*>(d.proc[0].xs)[3] = 1e39;
    });
    {
        uint64_t bytes = 0;
        expect(karl_workspace_bytes(nullptr, &bytes) == KARL_EINVAL && has_message(), "null descriptor");
        Tiny t;
        expect(karl_workspace_bytes(&t.d, nullptr) == KARL_EINVAL, "null size output");
        void* job = nullptr;
        expect(karl_create_job(nullptr, &job) == KARL_EINVAL && job == nullptr, "create from null");
        expect(karl_transport(nullptr, 0, 1, nullptr) == KARL_ESTATE, "transport of no job");
        expect(karl_transport_noalloc(nullptr, 0, 1, nullptr) == KARL_ESTATE, "no-alloc transport of no job");
        expect(karl_destroy_job(nullptr) == KARL_EINVAL, "destroy no job");
        int64_t n = -1;
        expect(karl_job_slices(nullptr, &n) == KARL_EINVAL && n == -1, "slices of no job");
        expect(karl_batch_wave_segments(nullptr, &n) == KARL_EINVAL && n == -1, "wave segments of no batch");
        expect(karl_batch_workspace_bytes(0, 1024, &bytes) == KARL_EINVAL, "batch of no jobs");
        expect(karl_batch_workspace_bytes(4, -1, &bytes) == KARL_EINVAL, "batch with a negative queue");
        expect(karl_batch_workspace_bytes(4, 0, &bytes) == KARL_OK && bytes > 0, "batch with the default queue");
        expect(karl_batch_workspace_bytes(4, 1024, &bytes) == KARL_OK && bytes > 0, "batch sized");
        expect(karl_destroy_batch(nullptr) == KARL_EINVAL, "destroy no batch");
        expect(karl_destroy_server(nullptr) == KARL_EINVAL, "destroy no server");
    }
    std::printf("%d failed\n", failures);
    return failures ? 1 : 0;
}

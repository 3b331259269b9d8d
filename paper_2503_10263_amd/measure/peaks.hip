// Achievable peaks of MI355X for the transport's ceilings, measured rather than quoted:
//   copy / triad     HBM bandwidth (BW_ach): 16-byte vector loads and stores over 2 GiB arrays
//   atomics          device-scope atomic additions without return into tally-shaped arrays
//                    (FP64 and int64; 256 KiB .. 2 MiB; uniform random cells, 64 hot cells,
//                    and one private copy per XCD) -- the tallies' ceiling (A_ach)
//   fp64 fma         dependent fused multiply-add chains, 8 per lane -- the FP64 vector rate
//   philox + log     Philox4x32-10 draws turned into two 53-bit uniforms and their logarithms,
//                    the free-path sampling's inner work
// Every kernel is timed with HIP events, best of five launches after one warm-up launch.
// Output: one JSON object on stdout.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>

#define CHECK(x)                                                                        \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) {                                                         \
            fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));             \
            exit(1);                                                                    \
        }                                                                               \
    } while (0)

__global__ void copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void triad_kernel(const double2* __restrict__ b, const double2* __restrict__ c,
                             double2* __restrict__ a, double s, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const double2 x = b[i], y = c[i];
        a[i] = make_double2(x.x + s * y.x, x.y + s * y.y);
    }
}

// cell index of atomic k of thread g: a multiply-xorshift hash, reduced to the pattern's range
__device__ __forceinline__ uint32_t cell_hash(uint32_t g, uint32_t k) {
    uint32_t x = g * 0x9E3779B1u + k * 0x85EBCA77u;
    x ^= x >> 15;
    x *= 0x2C1B3C6Du;
    x ^= x >> 12;
    return x;
}

// pattern 0: uniform over n cells; 1: 64 hot cells; 2: uniform over the copy of the
// workgroup's XCD (workgroups are dispatched to the 8 XCDs round-robin), 8 copies of n cells
template <typename T>
__global__ void atomic_kernel(T* __restrict__ cells, uint32_t n, int pattern, int per_thread) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t base = pattern == 2 ? (size_t)(blockIdx.x & 7u) * n : 0;
    const uint32_t range = pattern == 1 ? 64u : n;
    for (int k = 0; k < per_thread; ++k) {
        const uint32_t idx = cell_hash(g, (uint32_t)k) % range;
        atomicAdd(&cells[base + idx], (T)1);
    }
}

__global__ void fma_kernel(double* __restrict__ out, int iters) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    double x[8];
    for (int c = 0; c < 8; ++c) x[c] = 1.0 + 1e-3 * (double)(c + (g & 7));
    const double a = 0.9999999, b = 1.0e-7;
    for (int i = 0; i < iters; ++i)
        for (int c = 0; c < 8; ++c) x[c] = fma(x[c], a, b);
    double s = 0.0;
    for (int c = 0; c < 8; ++c) s += x[c];
    out[g] = s;
}

__device__ __forceinline__ void philox10(uint32_t k0, uint32_t k1, uint32_t c[4]) {
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = (uint32_t)p1;
        c[2] = n2;
        c[3] = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__global__ void philox_log_kernel(double* __restrict__ out, int draws) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    for (int i = 0; i < draws; ++i) {
        uint32_t c[4] = {(uint32_t)i, 0u, g, 0u};
        philox10(1u, g, c);
        const double u0 = ((double)(c[0] >> 5) * 67108864.0 + (double)(c[1] >> 6)) * 0x1p-53 + 0x1p-53;
        const double u1 = ((double)(c[2] >> 5) * 67108864.0 + (double)(c[3] >> 6)) * 0x1p-53 + 0x1p-53;
        acc += log(u0) + log(u1);
    }
    out[g] = acc;
}

struct Timer {
    hipEvent_t a, b;
    Timer() {
        CHECK(hipEventCreate(&a));
        CHECK(hipEventCreate(&b));
    }
    template <typename F>
    double best_ms(F launch) {
        launch();
        CHECK(hipDeviceSynchronize());
        double best = 1e30;
        for (int r = 0; r < 5; ++r) {
            CHECK(hipEventRecord(a, 0));
            launch();
            CHECK(hipEventRecord(b, 0));
            CHECK(hipEventSynchronize(b));
            float ms = 0.f;
            CHECK(hipEventElapsedTime(&ms, a, b));
            if (ms < best) best = ms;
        }
        return best;
    }
};

int main(int argc, char** argv) {
    if (argc > 2 && strcmp(argv[1], "copy") == 0) {
        // counter calibration: one kind of kernel only (the copy of argv[2] bytes, five times)
        const size_t bytes = (size_t)atoll(argv[2]) & ~(size_t)15;
        uint4 *a = nullptr, *b = nullptr;
        CHECK(hipMalloc(&a, bytes));
        CHECK(hipMalloc(&b, bytes));
        CHECK(hipMemset(a, 1, bytes));
        Timer t;
        const double ms = t.best_ms([&] { copy_kernel<<<4096, 256>>>(a, b, bytes / 16); });
        printf("{\"copy_bytes\": %zu, \"ms\": %.4f, \"GBps\": %.1f}\n", bytes, ms, 2.0 * bytes / (ms * 1e-3) / 1e9);
        return 0;
    }
    int dev = 0;
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, dev));
    const int cus = prop.multiProcessorCount;
    Timer t;
    printf("{\"device\": \"%s\", \"cus\": %d, \"clock_khz\": %d", prop.gcnArchName, cus, prop.clockRate);

    // HBM: copy and triad over 2 GiB per array
    {
        const size_t bytes = (size_t)2 << 30;
        char *a, *b, *c;
        CHECK(hipMalloc(&a, bytes));
        CHECK(hipMalloc(&b, bytes));
        CHECK(hipMalloc(&c, bytes));
        CHECK(hipMemset(b, 0, bytes));
        CHECK(hipMemset(c, 0, bytes));
        // launch shapes: workgroups per CU x threads per workgroup; the best of each kernel counts
        const int shapes[5][2] = {{4, 256}, {16, 256}, {64, 256}, {8, 1024}, {32, 512}};
        double best_copy = 1e30, best_triad = 1e30;
        int sc = 0, st = 0;
        for (int k = 0; k < 5; ++k) {
            const int blocks = cus * shapes[k][0], threads = shapes[k][1];
            const double mc = t.best_ms([&] { copy_kernel<<<blocks, threads>>>((const uint4*)b, (uint4*)a, bytes / 16); });
            const double mt = t.best_ms([&] {
                triad_kernel<<<blocks, threads>>>((const double2*)b, (const double2*)c, (double2*)a, 3.0, bytes / 16);
            });
            if (mc < best_copy) { best_copy = mc; sc = k; }
            if (mt < best_triad) { best_triad = mt; st = k; }
        }
        printf(", \"copy_GBps\": %.1f, \"copy_shape\": [%d, %d], \"triad_GBps\": %.1f, \"triad_shape\": [%d, %d]",
               2.0 * bytes / (best_copy * 1e-3) / 1e9, shapes[sc][0], shapes[sc][1],
               3.0 * bytes / (best_triad * 1e-3) / 1e9, shapes[st][0], shapes[st][1]);
        CHECK(hipFree(a));
        CHECK(hipFree(b));
        CHECK(hipFree(c));
    }

    // atomics into tally-shaped arrays
    {
        const uint32_t sizes_bytes[4] = {256u << 10, 512u << 10, 1u << 20, 2u << 20};
        const char* pat[3] = {"uniform", "hot64", "per_xcd"};
        void* cells = nullptr;
        CHECK(hipMalloc(&cells, (size_t)8 * (2u << 20)));
        const int blocks = cus * 8, threads = 256, per = 256;
        const double n_atomics = (double)blocks * threads * per;
        printf(", \"atomics_per_launch\": %.0f, \"atomics\": [", n_atomics);
        bool first = true;
        for (int type = 0; type < 2; ++type)
            for (int s = 0; s < 4; ++s)
                for (int p = 0; p < 3; ++p) {
                    const uint32_t n = sizes_bytes[s] / 8u;
                    CHECK(hipMemset(cells, 0, (size_t)8 * (2u << 20)));
                    double ms;
                    if (type == 0)
                        ms = t.best_ms([&] { atomic_kernel<double><<<blocks, threads>>>((double*)cells, n, p, per); });
                    else
                        ms = t.best_ms([&] {
                            atomic_kernel<unsigned long long><<<blocks, threads>>>((unsigned long long*)cells, n, p, per);
                        });
                    printf("%s{\"type\": \"%s\", \"bytes\": %u, \"pattern\": \"%s\", \"per_s\": %.4e}",
                           first ? "" : ", ", type == 0 ? "f64" : "i64", sizes_bytes[s], pat[p], n_atomics / (ms * 1e-3));
                    first = false;
                }
        printf("]");
        CHECK(hipFree(cells));
    }

    // vector ALU: FP64 fused multiply-add chains; Philox draws with two logarithms
    {
        const int blocks = cus * 16, threads = 256;
        double* out = nullptr;
        CHECK(hipMalloc(&out, sizeof(double) * (size_t)blocks * threads));
        const int iters = 4096;
        const double ms_fma = t.best_ms([&] { fma_kernel<<<blocks, threads>>>(out, iters); });
        const double flops = 2.0 * 8.0 * iters * (double)blocks * threads;
        const int draws = 256;
        const double ms_ph = t.best_ms([&] { philox_log_kernel<<<blocks, threads>>>(out, draws); });
        printf(", \"fp64_fma_TFLOPs\": %.2f, \"philox_log_draws_per_s\": %.4e", flops / (ms_fma * 1e-3) / 1e12,
               (double)draws * blocks * threads / (ms_ph * 1e-3));
        CHECK(hipFree(out));
    }
    printf("}\n");
    return 0;
}

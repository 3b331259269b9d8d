// Test support, not part of the library: the transport kernels' elementary device arithmetic
// (ln, sin/cos, the divisions and square roots with bounded operands, the FP64 uniform from two
// Philox words, Philox4x32-10, the SplitMix64 finaliser) applied element-wise to host arrays, so
// that the GPU tests can compare each function bit for bit with the host's IEEE arithmetic and
// with the oracle's functions.  Compiled once per kernel unit (-DKARL_DRAIN_UNIT,
// -DKARL_BATCHED_UNIT or neither), since each unit reads the series constants its own way
// (from LDS, from scalar registers, as literals); KARL_TEST_NAME names the entry point.
#include "karl_kernels.hip"

#ifndef KARL_TEST_NAME
#error "KARL_TEST_NAME must name the entry point"
#endif

namespace karl_test {
namespace {   // one copy per unit in the same library

enum Op {
    kDiv64 = 0,      // out0 = kdiv(a, b), out1 = a / b (the compiler's correctly rounded division)
    kSqrt64 = 1,     // out0 = ksqrt_n(a), out1 = sqrt(a) (the compiler's correctly rounded root)
    kLog64 = 2,      // out0 = klog(a)
    kSinCos64 = 3,   // out0, out1 = ksincos(a)
    kLog32 = 4,      // float: out0 = klog(a)
    kSinCos32 = 5,   // float: out0, out1 = ksincos(a)
    kPhilox = 6,     // a: 6 words per element (k0, k1, c0, c1, c2, c3) -> out0: 4 words
    kU53 = 7,        // a: 2 words per element -> out0: the FP64 uniform
    kMix64 = 8,      // a: 64-bit words -> out0: the SplitMix64 finaliser
    kNOps
};

__global__ void arith_kernel(int op, int64_t n, const void* a, const void* b, void* o0, void* o1) {
#ifdef KARL_DRAIN_UNIT
    // the deferred-launch unit reads the series constants from LDS, staged as its kernels do
    for (int i = threadIdx.x; i < karl::kNSeries; i += blockDim.x) karl::s_series[i] = karl::kSeriesTab[i];
    __syncthreads();
#endif
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        switch (op) {
            case kDiv64: {
                const double x = ((const double*)a)[i], y = ((const double*)b)[i];
                ((double*)o0)[i] = karl::kdiv(x, y);
                ((double*)o1)[i] = x / y;
                break;
            }
            case kSqrt64: {
                const double x = ((const double*)a)[i];
                ((double*)o0)[i] = karl::ksqrt_n(x);
                ((double*)o1)[i] = sqrt(x);
                break;
            }
            case kLog64:
                ((double*)o0)[i] = karl::klog(((const double*)a)[i]);
                break;
            case kSinCos64:
                karl::ksincos(((const double*)a)[i], (double*)o0 + i, (double*)o1 + i);
                break;
            case kLog32:
                ((float*)o0)[i] = karl::klog(((const float*)a)[i]);
                break;
            case kSinCos32:
                karl::ksincos(((const float*)a)[i], (float*)o0 + i, (float*)o1 + i);
                break;
            case kPhilox: {
                const uint32_t* w = (const uint32_t*)a + 6 * i;
                const karl::U4 r = karl::philox(w[0], w[1], w[2], w[3], w[4], w[5]);
                uint32_t* out = (uint32_t*)o0 + 4 * i;
                out[0] = r.x;
                out[1] = r.y;
                out[2] = r.z;
                out[3] = r.w;
                break;
            }
            case kU53: {
                const uint32_t* w = (const uint32_t*)a + 2 * i;
                ((double*)o0)[i] = karl::Prec<double>::uni(w[0], w[1], 0u);
                break;
            }
            case kMix64:
                ((unsigned long long*)o0)[i] = karl::mix64(((const unsigned long long*)a)[i]);
                break;
            default:
                break;
        }
    }
}

// bytes per element of (a, b, out0, out1) for each operation
struct Sizes { size_t a, b, o0, o1; };
inline Sizes sizes(int op) {
    switch (op) {
        case kDiv64: return {8, 8, 8, 8};
        case kSqrt64: return {8, 0, 8, 8};
        case kLog64: return {8, 0, 8, 0};
        case kSinCos64: return {8, 0, 8, 8};
        case kLog32: return {4, 0, 4, 0};
        case kSinCos32: return {4, 0, 4, 4};
        case kPhilox: return {24, 0, 16, 0};
        case kU53: return {8, 0, 8, 0};
        case kMix64: return {8, 0, 8, 0};
        default: return {0, 0, 0, 0};
    }
}

}  // namespace
}  // namespace karl_test

// Applies operation `op` to n elements.  a, b, out0, out1: host arrays of the sizes the
// operation names (b, out1 unused by some); the device copies are made and freed here.
// Returns 0, a HIP error code, or -1 for an unknown operation or a negative n.
extern "C" int KARL_TEST_NAME(int op, int64_t n, const void* a, const void* b, void* out0, void* out1) {
    using namespace karl_test;
    if (op < 0 || op >= kNOps || n < 0) return -1;
    if (n == 0) return 0;
    const Sizes s = sizes(op);
    void* d[4] = {nullptr, nullptr, nullptr, nullptr};
    const size_t bytes[4] = {s.a * (size_t)n, s.b * (size_t)n, s.o0 * (size_t)n, s.o1 * (size_t)n};
    hipError_t e = hipSuccess;
    for (int k = 0; k < 4 && e == hipSuccess; ++k)
        if (bytes[k]) e = hipMalloc(&d[k], bytes[k]);
    if (e == hipSuccess) e = hipMemcpy(d[0], a, bytes[0], hipMemcpyHostToDevice);
    if (e == hipSuccess && bytes[1]) e = hipMemcpy(d[1], b, bytes[1], hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        const int64_t blocks = (n + 255) / 256;
        const int grid = (int)(blocks < 4096 ? blocks : 4096);
        hipLaunchKernelGGL(arith_kernel, dim3(grid), dim3(256), 0, 0, op, n, d[0], d[1], d[2], d[3]);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(out0, d[2], bytes[2], hipMemcpyDeviceToHost);
    if (e == hipSuccess && bytes[3]) e = hipMemcpy(out1, d[3], bytes[3], hipMemcpyDeviceToHost);
    for (int k = 0; k < 4; ++k)
        if (d[k]) (void)hipFree(d[k]);
    return (int)e;
}

// fh_probe.hip -- measured ceilings for the rooflines that the benchmark
// reports: HBM bandwidth from a device-to-device copy, the LDS rates of the
// operations the spread is built from (float and double atomic adds, and the
// read-modify-write of complex double and complex float cells), and the
// matrix-core rate of the 16 x 16 x 4 products of the matrix-core spread.
// Each figure is the best of several timed launches over the whole chip.
#include "fh_common.hpp"

namespace fh {
namespace {

// Plain copy, one 16-byte element per thread and step.
__global__ void __launch_bounds__(256) k_probe_copy(const uint4* __restrict__ a, uint4* __restrict__ b, size_t n)
{
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) b[i] = a[i];
}

// Copy with four 16-byte loads in flight per thread (each a coalesced row of
// the block) before the four stores, non-temporal; n a multiple of 4 * 256.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_probe_copy4(const u32x4* __restrict__ a, u32x4* __restrict__ b, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x * 4;
    for (size_t i = blockIdx.x * (size_t)blockDim.x * 4 + threadIdx.x; i < n; i += stride) {
        u32x4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = __builtin_nontemporal_load(a + i + k * blockDim.x);
#pragma unroll
        for (int k = 0; k < 4; ++k) __builtin_nontemporal_store(v[k], b + i + k * blockDim.x);
    }
}

// Every lane adds to its own cell of a 4096-entry LDS table (consecutive
// lanes, consecutive cells: no bank conflicts), 16 independent adds per
// iteration; the result is never read back by the atomics (non-returning).
constexpr int kProbeCells = 4096;
constexpr int kProbeUnroll = 16;

template <class T>
__global__ void __launch_bounds__(256) k_probe_lds_add(int iters, T* __restrict__ out)
{
    __shared__ T s[kProbeCells];
    for (int e = threadIdx.x; e < kProbeCells; e += blockDim.x) s[e] = T(0);
    __syncthreads();
    const T v = T(1);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kProbeUnroll; ++k) atomicAdd(&s[(threadIdx.x + 256 * k) & (kProbeCells - 1)], v);
    }
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = s[blockIdx.x & (kProbeCells - 1)];
}

// Read-modify-write of complex cells (C: double2 or float2), as a run flush
// of the spread does: each lane reads a cell, adds, and writes it back, 8
// cells per iteration (a compiler barrier keeps the values from staying in
// registers from one iteration to the next).
template <class C>
__global__ void __launch_bounds__(256) k_probe_lds_rmw(int iters, double* __restrict__ out)
{
    __shared__ C s[2048];
    for (int e = threadIdx.x; e < 2048; e += blockDim.x) s[e] = C{0, 0};
    __syncthreads();
    for (int i = 0; i < iters; ++i) {
        C v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = s[(threadIdx.x + 256 * k) & 2047];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            v[k].x += 1;
            v[k].y -= 1;
            s[(threadIdx.x + 256 * k) & 2047] = v[k];
        }
        asm volatile("" ::: "memory");
    }
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (double)s[blockIdx.x & 2047].x;
}

// Matrix-core throughput of the 16 x 16 x 4 products the matrix-core spread
// issues (v_mfma_f64_16x16x4f64, v_mfma_f32_16x16x4f32): every wavefront
// keeps 8 independent accumulators and issues 8 products per iteration.
template <class R> struct ProbeMma;
template <> struct ProbeMma<double> {
    typedef double V __attribute__((ext_vector_type(4)));
    __device__ static V mma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};
template <> struct ProbeMma<float> {
    typedef float V __attribute__((ext_vector_type(4)));
    __device__ static V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};

template <class R>
__global__ void __launch_bounds__(256) k_probe_mfma(int iters, double* __restrict__ out)
{
    using V = typename ProbeMma<R>::V;
    V acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = V{R(0), R(0), R(0), R(0)};
    R a = R(1) + R(threadIdx.x) * R(1e-3), b = R(2) - R(threadIdx.x) * R(1e-3);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] = ProbeMma<R>::mma(a, b, acc[k]);
        a += R(1e-7);
    }
    R t = R(0);
#pragma unroll
    for (int k = 0; k < 8; ++k) t += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    if (t == R(-1)) out[blockIdx.x] = (double)t;  // never true; keeps the products live
}

// Best time in ms of `reps` launches of `launch` on the context stream.
template <class F>
fh_status best_ms(fh_ctx* c, int reps, F launch, double* ms)
{
    hipEvent_t e0, e1;
    FH_HIP(hipEventCreate(&e0));
    FH_HIP(hipEventCreate(&e1));
    double best = 1e30;
    hipError_t err = hipSuccess;
    for (int r = 0; r < reps + 1 && err == hipSuccess; ++r) {
        err = hipEventRecord(e0, c->stream);
        if (err == hipSuccess) launch();
        if (err == hipSuccess) err = hipGetLastError();
        if (err == hipSuccess) err = hipEventRecord(e1, c->stream);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float t = 0.0f;
        if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
        if (err == hipSuccess && r > 0) best = std::min(best, (double)t);  // launch 0 warms up
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    FH_HIP(err);
    *ms = best;
    return FH_OK;
}

}  // namespace
}  // namespace fh

using namespace fh;

extern "C" fh_status fh_probe_ceilings(fh_ctx* c, double* out)
{
    try {
        FH_ARG(c && out, FH_ERR_INVALID_ARG, "NULL argument");
        FH_HIP(hipSetDevice(c->device));
        FH_HIP(hipStreamSynchronize(c->stream));
        // HBM: copy 1 GiB into another 1 GiB
        const size_t bytes = size_t(1) << 30;
        void* a = nullptr;
        void* b = nullptr;
        FH_TRY(dev_alloc(c, bytes, &a));
        fh_status s = dev_alloc(c, bytes, &b);
        if (s != FH_OK) {
            (void)dev_free(c, a);
            return s;
        }
        const size_t n16 = bytes / 16;
        const unsigned grid = (unsigned)c->cu_count * 16;
        double ms = 0.0, ms4 = 0.0;
        s = best_ms(c, 5, [&] {
            hipLaunchKernelGGL(k_probe_copy, dim3(grid), dim3(256), 0, c->stream, static_cast<const uint4*>(a),
                               static_cast<uint4*>(b), n16);
        }, &ms);
        if (s == FH_OK)
            s = best_ms(c, 5, [&] {
                hipLaunchKernelGGL(k_probe_copy4, dim3((unsigned)c->cu_count * 8), dim3(256), 0, c->stream,
                                   static_cast<const u32x4*>(a), static_cast<u32x4*>(b), n16);
            }, &ms4);
        (void)hipStreamSynchronize(c->stream);
        (void)dev_free(c, a);
        (void)dev_free(c, b);
        FH_TRY(s);
        // the faster of the two copies
        out[0] = 2.0 * (double)bytes / (std::min(ms, ms4) * 1e-3) / 1e9;

        // LDS atomics and read-modify-write: 8 blocks of 256 threads per CU
        const unsigned lgrid = (unsigned)c->cu_count * 8;
        void* sink = nullptr;
        FH_TRY(dev_alloc(c, sizeof(double) * lgrid, &sink));
        const int iters = 256;
        const double ops = (double)lgrid * 256.0 * iters * kProbeUnroll;
        s = best_ms(c, 5, [&] {
            hipLaunchKernelGGL((k_probe_lds_add<float>), dim3(lgrid), dim3(256), 0, c->stream, iters,
                               static_cast<float*>(sink));
        }, &ms);
        if (s == FH_OK) out[1] = ops * sizeof(float) / (ms * 1e-3) / 1e9;
        if (s == FH_OK)
            s = best_ms(c, 5, [&] {
                hipLaunchKernelGGL((k_probe_lds_add<double>), dim3(lgrid), dim3(256), 0, c->stream, iters,
                                   static_cast<double*>(sink));
            }, &ms);
        if (s == FH_OK) out[2] = ops * sizeof(double) / (ms * 1e-3) / 1e9;
        if (s == FH_OK)
            s = best_ms(c, 5, [&] {
                hipLaunchKernelGGL((k_probe_lds_rmw<double2>), dim3(lgrid), dim3(256), 0, c->stream, iters,
                                   static_cast<double*>(sink));
            }, &ms);
        // 8 cells of 16 bytes read and written per lane and iteration
        if (s == FH_OK) out[3] = (double)lgrid * 256.0 * iters * 8 * 32.0 / (ms * 1e-3) / 1e9;
        if (s == FH_OK)
            s = best_ms(c, 5, [&] {
                hipLaunchKernelGGL((k_probe_lds_rmw<float2>), dim3(lgrid), dim3(256), 0, c->stream, iters,
                                   static_cast<double*>(sink));
            }, &ms);
        // 8 cells of 8 bytes read and written per lane and iteration
        if (s == FH_OK) out[4] = (double)lgrid * 256.0 * iters * 8 * 16.0 / (ms * 1e-3) / 1e9;
        // matrix cores: 8 products of 16 x 16 x 4 (2 x 1024 flops) per
        // wavefront and iteration, 4 wavefronts per block
        const double mflop = (double)lgrid * 4.0 * iters * 8 * 2048.0;
        if (s == FH_OK)
            s = best_ms(c, 5, [&] {
                hipLaunchKernelGGL((k_probe_mfma<double>), dim3(lgrid), dim3(256), 0, c->stream, iters,
                                   static_cast<double*>(sink));
            }, &ms);
        if (s == FH_OK) out[5] = mflop / (ms * 1e-3) / 1e12;
        if (s == FH_OK)
            s = best_ms(c, 5, [&] {
                hipLaunchKernelGGL((k_probe_mfma<float>), dim3(lgrid), dim3(256), 0, c->stream, iters,
                                   static_cast<double*>(sink));
            }, &ms);
        if (s == FH_OK) out[6] = mflop / (ms * 1e-3) / 1e12;
        (void)hipStreamSynchronize(c->stream);
        (void)dev_free(c, sink);
        return s;
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

// fh_nsli.hip -- the non-singular line integral (appendix, eq. nsli).
//
// For a counter-clockwise vector line rule (X_i, Y_i, W_i, V_i) on the
// boundary and a target (xi, eta), with r_i = (X_i - xi, Y_i - eta),
//   u_ap = (1/2pi) sum_i (1 - exp(i pi r_i^2/(lambda z))) (r_i x ds_i)/r_i^2,
// r x ds = r_x V - r_y W, a term being zero when r_i^2 = 0.  The integrand is
// bounded as the target reaches the boundary, so one formula serves targets
// inside, outside and on it.  With t = r^2/(2 lambda z) turns reduced to
// f = t - rint(t),
//   (1 - exp(2 pi i f))/r^2 = (2 sin(pi f)/r^2) (sin(pi f) - i cos(pi f)),
// which keeps full relative accuracy as r -> 0 (the subtraction the paper's
// error analysis discusses never happens).
//
// Deep-shadow option (the appendix's remark, with eq. li): for a target at
// least `far` from every node,
//   u_ap = u_geom - (1/2pi) sum_i exp(i pi r_i^2/(lambda z)) (r_i x ds_i)/r_i^2,
// u_geom the nearest integer to the winding number (1/2pi) sum (r x ds)/r^2
// evaluated with the same rule; the sum of exp(.) terms is the winding sum
// minus the NSLI sum, so one pass accumulates both.
//
// The work is O(n M) FP64 arithmetic with a few bytes per target: every
// thread owns targets and walks all boundary nodes (read as wavefront-uniform
// scalar loads), so the kernel is bound by FP64 VALU throughput.  When the
// targets alone give fewer than two workgroups per CU, the nodes are split
// into groups whose partial sums a second kernel adds in a fixed order.
#include <algorithm>
#include <mutex>

#include "fh_common.hpp"

namespace fh {
namespace {

constexpr int kNsliBlock = 256;

// Device scratch of the allocation-free edge integral (fh_field_nsli_noalloc):
// the node groups' partial sums, 4 groups M doubles, at most 32 MiB.  Each
// device holds its own copy until the process ends; every call on a device
// shares it.  Host code never uses the array's name as an address: the
// device's copy is found with hipGetSymbolAddress on the first call there.
constexpr size_t kNsliScratchDoubles = size_t(4) << 20;
static __device__ __align__(256) double scratch[kNsliScratchDoubles];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kScratchDevices] = {};

// The address of this device's scratch (the device must be current).
fh_status scratch_for(int device, double** out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    FH_ARG(device >= 0 && device < kScratchDevices, FH_ERR_UNSUPPORTED, "device %d beyond the %d supported", device,
           kScratchDevices);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        FH_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        FH_ARG(p != nullptr, FH_ERR_HIP, "no device address for the scratch array");
        g_scratch_ptr[device] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[device];
    return FH_OK;
}
constexpr double kNsliTiny = 1e-280;  // floor of r^2 before its reciprocal

struct NsliParams {
    const double* X;
    const double* Y;
    const double* W;
    const double* V;
    int64_t n;
    const double* xi;
    const double* eta;
    int64_t M;
    double inv2lz;  // 1/(2 lambda z)
    double far2;    // far^2 (deep-shadow form when shadow != 0)
    int shadow;
    int occulter;
    int groups;     // node groups (grid y)
    int64_t per;    // nodes per group
    double* part;   // groups > 1: partial sums, [4][groups][M]
};

struct NsliAcc {
    double sre, sim, wnd, d2;
};

__device__ __forceinline__ double rcp_f64(double x)
{
    // hardware reciprocal estimate, then two Newton steps
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// Taylor coefficients of sin(pi f) = f sum_k s_k f^(2k) and
// cos(pi f) = sum_k c_k f^(2k): s_k = (-1)^k pi^(2k+1)/(2k+1)!,
// c_k = (-1)^k pi^(2k)/(2k)!.  On |f| <= 1/2 the first 11 and 12 terms leave
// a truncation error below 1e-18 (the next terms are (pi/2)^23/23! and
// (pi/2)^24/24!), so the sums are good to rounding.
constexpr int kSinTerms = 11, kCosTerms = 12;
struct PiSeries {
    double s[kSinTerms];
    double c[kCosTerms];
    constexpr PiSeries() : s(), c()
    {
        const double pi2 = kPi * kPi;
        double t = kPi;
        for (int k = 0; k < kSinTerms; ++k) {
            s[k] = t;
            t *= -pi2 / ((2.0 * k + 2.0) * (2.0 * k + 3.0));
        }
        t = 1.0;
        for (int k = 0; k < kCosTerms; ++k) {
            c[k] = t;
            t *= -pi2 / ((2.0 * k + 1.0) * (2.0 * k + 2.0));
        }
    }
};
constexpr PiSeries kPiSeries{};

// sin(pi f) and cos(pi f) for |f| <= 1/2 (Horner in f^2).
__device__ __forceinline__ void sincospi_half(double f, double& sn, double& cs)
{
    const double f2 = f * f;
    double ps = kPiSeries.s[kSinTerms - 1];
#pragma unroll
    for (int k = kSinTerms - 2; k >= 0; --k) ps = fma(ps, f2, kPiSeries.s[k]);
    double pc = kPiSeries.c[kCosTerms - 1];
#pragma unroll
    for (int k = kCosTerms - 2; k >= 0; --k) pc = fma(pc, f2, kPiSeries.c[k]);
    sn = f * ps;
    cs = pc;
}

// One node's term.  The accumulators hold half the NSLI sum (the factor 2 of
// the half-angle form is applied once at the end).  r^2 is floored at a tiny
// value before the reciprocal: a target on a node has r x ds = 0 there, so
// its term is 0; nearer than 1e-140 the term is below any rounding.
__device__ __forceinline__ void nsli_term(double bx, double by, double bw, double bv, double xi, double eta,
                                          double inv2lz, NsliAcc& a)
{
    const double rx = bx - xi, ry = by - eta;
    const double r2 = fma(rx, rx, ry * ry);
    a.d2 = fmin(a.d2, r2);
    const double cr = fma(rx, bv, -(ry * bw));
    const double t = r2 * inv2lz;
    const double f = t - rint(t);
    double sn, cs;
    sincospi_half(f, sn, cs);
    const double c = cr * rcp_f64(fmax(r2, kNsliTiny));
    const double h = sn * c;
    a.sre = fma(h, sn, a.sre);
    a.sim = fma(-h, cs, a.sim);
    a.wnd += c;
}

template <class OUT>
__device__ __forceinline__ void nsli_store(const NsliParams& p, int64_t k, const NsliAcc& a, OUT* __restrict__ u)
{
    // sre, sim hold half of the NSLI sum (see nsli_term)
    constexpr double inv2pi = 0.5 / kPi, invpi = 1.0 / kPi;
    double re, im = a.sim * invpi;
    if (p.shadow && a.d2 >= p.far2) {
        const double geom = rint(a.wnd * inv2pi);
        re = geom - a.wnd * inv2pi + a.sre * invpi;
    } else {
        re = a.sre * invpi;
    }
    if (p.occulter) {
        re = 1.0 - re;
        im = -im;
    }
    u[2 * k] = (OUT)re;
    u[2 * k + 1] = (OUT)im;
}

// TPT targets per thread, at k = base + t * kNsliBlock.
template <int TPT, class OUT>
__global__ void __launch_bounds__(kNsliBlock) k_nsli(NsliParams p, OUT* __restrict__ u)
{
    const int64_t base = (int64_t)blockIdx.x * (kNsliBlock * TPT) + threadIdx.x;
    const int g = blockIdx.y;
    const int64_t i0 = (int64_t)g * p.per;
    const int64_t i1 = min(p.n, i0 + p.per);
    double xi[TPT], eta[TPT];
    NsliAcc acc[TPT];
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        const int64_t k = base + (int64_t)t * kNsliBlock;
        const int64_t kk = k < p.M ? k : p.M - 1;  // tail lanes compute a copy, store nothing
        xi[t] = p.xi[kk];
        eta[t] = p.eta[kk];
        acc[t] = NsliAcc{0.0, 0.0, 0.0, __builtin_inf()};
    }
    const double* __restrict__ X = p.X;
    const double* __restrict__ Y = p.Y;
    const double* __restrict__ W = p.W;
    const double* __restrict__ V = p.V;
#pragma unroll 2
    for (int64_t i = i0; i < i1; ++i) {
        const double bx = X[i], by = Y[i], bw = W[i], bv = V[i];
#pragma unroll
        for (int t = 0; t < TPT; ++t) nsli_term(bx, by, bw, bv, xi[t], eta[t], p.inv2lz, acc[t]);
    }
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
        const int64_t k = base + (int64_t)t * kNsliBlock;
        if (k >= p.M) continue;
        if (p.groups == 1) {
            nsli_store(p, k, acc[t], u);
        } else {
            const int64_t s = (int64_t)p.groups * p.M;
            double* q = p.part + (int64_t)g * p.M + k;
            q[0] = acc[t].sre;
            q[s] = acc[t].sim;
            q[2 * s] = acc[t].wnd;
            q[3 * s] = acc[t].d2;
        }
    }
}

// Adds the node groups' partial sums in group order and stores the field.
template <class OUT>
__global__ void __launch_bounds__(kNsliBlock) k_nsli_finish(NsliParams p, OUT* __restrict__ u)
{
    const int64_t k = (int64_t)blockIdx.x * kNsliBlock + threadIdx.x;
    if (k >= p.M) return;
    const int64_t s = (int64_t)p.groups * p.M;
    NsliAcc a{0.0, 0.0, 0.0, __builtin_inf()};
    for (int g = 0; g < p.groups; ++g) {
        const double* q = p.part + (int64_t)g * p.M + k;
        a.sre += q[0];
        a.sim += q[s];
        a.wnd += q[2 * s];
        a.d2 = fmin(a.d2, q[3 * s]);
    }
    nsli_store(p, k, a, u);
}

template <class OUT>
__global__ void k_nsli_empty(int64_t M, int occulter, OUT* __restrict__ u)
{
    const int64_t k = (int64_t)blockIdx.x * kNsliBlock + threadIdx.x;
    if (k >= M) return;
    u[2 * k] = (OUT)(occulter ? 1.0 : 0.0);
    u[2 * k + 1] = (OUT)0.0;
}

inline unsigned nsli_blocks(int64_t n, int per) { return (unsigned)std::max<int64_t>(1, (n + per - 1) / per); }

constexpr int kNsliTpt = 2;

template <class OUT>
fh_status nsli_launch(fh_ctx* c, NsliParams p, OUT* u)
{
    if (p.n == 0) {
        hipLaunchKernelGGL(k_nsli_empty<OUT>, dim3(nsli_blocks(p.M, kNsliBlock)), dim3(kNsliBlock), 0, c->stream,
                           p.M, p.occulter, u);
        FH_HIP(hipGetLastError());
        return FH_OK;
    }
    const unsigned bx = nsli_blocks(p.M, kNsliBlock * kNsliTpt);
    if (p.groups == 1) {
        hipLaunchKernelGGL((k_nsli<kNsliTpt, OUT>), dim3(bx, 1), dim3(kNsliBlock), 0, c->stream, p, u);
    } else {
        hipLaunchKernelGGL((k_nsli<kNsliTpt, OUT>), dim3(bx, p.groups), dim3(kNsliBlock), 0, c->stream, p, u);
        hipLaunchKernelGGL(k_nsli_finish<OUT>, dim3(nsli_blocks(p.M, kNsliBlock)), dim3(kNsliBlock), 0, c->stream,
                           p, u);
    }
    FH_HIP(hipGetLastError());
    return FH_OK;
}

// Node groups: split the nodes only when the targets alone give fewer than
// two workgroups per CU (then aim at four), at least 64 nodes each;
// otherwise the partial sums would cost a second pass for nothing.  Returns
// the number of non-empty groups and the nodes per group (at least 1, also
// for an empty rule).
void nsli_groups(const fh_ctx* c, int64_t n, int64_t M, int* groups_out, int64_t* per_out)
{
    const int64_t bx = (M + kNsliBlock * kNsliTpt - 1) / (kNsliBlock * kNsliTpt);
    int groups = 1;
    if (bx < 2LL * c->cu_count && n > 128)
        groups = (int)std::min<int64_t>({(4LL * c->cu_count + bx - 1) / bx, n / 64, 1024});
    groups = std::max(groups, 1);
    const int64_t per = std::max<int64_t>(1, (n + groups - 1) / groups);
    *groups_out = (int)std::max<int64_t>(1, (n + per - 1) / per);
    *per_out = per;
}

fh_status nsli_check(const fh_ctx* c, const double* X, const double* Y, const double* W, const double* V, int64_t n,
                     double lambda, double z, int64_t M, const double* xi, const double* eta, double far,
                     const void* u)
{
    FH_ARG(c, FH_ERR_INVALID_ARG, "NULL context");
    FH_ARG(n >= 0 && M >= 0, FH_ERR_INVALID_ARG, "negative size");
    FH_ARG(n < ((int64_t)1 << 40) && M < ((int64_t)1 << 40), FH_ERR_INVALID_ARG, "size too large");
    FH_ARG(n == 0 || (X && Y && W && V), FH_ERR_INVALID_ARG, "NULL boundary array");
    FH_ARG(M == 0 || (xi && eta && u), FH_ERR_INVALID_ARG, "NULL target or output array");
    FH_ARG(std::isfinite(lambda) && std::isfinite(z) && std::isfinite(far), FH_ERR_NONFINITE,
           "lambda, z or far not finite");
    FH_ARG(lambda * z > 0, FH_ERR_NONPOSITIVE_LZ, "lambda * z must be positive");
    FH_ARG(far >= 0, FH_ERR_INVALID_ARG, "far must be >= 0");
    return FH_OK;
}

NsliParams nsli_params(const double* X, const double* Y, const double* W, const double* V, int64_t n, double lambda,
                       double z, int64_t M, const double* xi, const double* eta, double far, int32_t occulter,
                       int groups, int64_t per)
{
    NsliParams p{};
    p.X = X; p.Y = Y; p.W = W; p.V = V;
    p.n = n;
    p.xi = xi; p.eta = eta;
    p.M = M;
    p.inv2lz = 1.0 / (2.0 * lambda * z);
    p.far2 = far * far;
    p.shadow = far > 0;
    p.occulter = occulter != 0;
    p.groups = groups;
    p.per = per;
    p.part = nullptr;
    return p;
}

}  // namespace
}  // namespace fh

using namespace fh;

extern "C" {

fh_status fh_field_nsli(fh_ctx* c, const double* X, const double* Y, const double* W, const double* V, int64_t n,
                        double lambda, double z, int64_t M, const double* xi, const double* eta, double far,
                        int32_t occulter, void* u, fh_memspace mem)
{
    try {
        FH_TRY(nsli_check(c, X, Y, W, V, n, lambda, z, M, xi, eta, far, u));
        FH_ARG(mem == FH_MEM_HOST || mem == FH_MEM_DEVICE, FH_ERR_INVALID_ARG, "bad memspace");
        if (M == 0) return FH_OK;
        FH_HIP(hipSetDevice(c->device));
        const bool mixed = c->prec == FH_MIXED;
        const size_t usz = (mixed ? sizeof(float) : sizeof(double)) * 2 * (size_t)M;
        int groups;
        int64_t per;
        nsli_groups(c, n, M, &groups, &per);

        size_t need = 0;
        if (groups > 1) need += aligned_bytes(sizeof(double) * 4 * (size_t)groups * M);
        if (mem == FH_MEM_HOST)
            need += 4 * aligned_bytes(sizeof(double) * std::max<int64_t>(n, 1)) +
                    2 * aligned_bytes(sizeof(double) * M) + aligned_bytes(usz);
        FH_TRY(arena_reserve(c, need));
        NsliParams p = nsli_params(X, Y, W, V, n, lambda, z, M, xi, eta, far, occulter, groups, per);
        p.part = groups > 1 ? c->arena.take<double>(4 * (size_t)groups * M) : nullptr;
        void* dout = u;
        if (mem == FH_MEM_HOST) {
            const double* h[4] = {X, Y, W, V};
            const double* d[4] = {nullptr, nullptr, nullptr, nullptr};
            for (int k = 0; k < 4; ++k) {
                double* b = c->arena.take<double>(std::max<int64_t>(n, 1));
                if (n > 0) FH_HIP(hipMemcpyAsync(b, h[k], sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
                d[k] = b;
            }
            p.X = d[0]; p.Y = d[1]; p.W = d[2]; p.V = d[3];
            double* dxi = c->arena.take<double>(M);
            double* deta = c->arena.take<double>(M);
            FH_HIP(hipMemcpyAsync(dxi, xi, sizeof(double) * M, hipMemcpyHostToDevice, c->stream));
            FH_HIP(hipMemcpyAsync(deta, eta, sizeof(double) * M, hipMemcpyHostToDevice, c->stream));
            p.xi = dxi;
            p.eta = deta;
            dout = c->arena.take<char>(usz);
        }
        if (mixed)
            FH_TRY(nsli_launch(c, p, static_cast<float*>(dout)));
        else
            FH_TRY(nsli_launch(c, p, static_cast<double*>(dout)));
        if (mem == FH_MEM_HOST) {
            FH_HIP(hipMemcpyAsync(u, dout, usz, hipMemcpyDeviceToHost, c->stream));
            FH_HIP(hipStreamSynchronize(c->stream));
        }
        return FH_OK;
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_field_nsli_noalloc(fh_ctx* c, const double* X, const double* Y, const double* W, const double* V,
                                int64_t n, double lambda, double z, int64_t M, const double* xi, const double* eta,
                                double far, int32_t occulter, void* u)
{
    try {
        FH_TRY(nsli_check(c, X, Y, W, V, n, lambda, z, M, xi, eta, far, u));
        if (M == 0) return FH_OK;
        FH_HIP(hipSetDevice(c->device));
        int groups;
        int64_t per;
        nsli_groups(c, n, M, &groups, &per);
        NsliParams p = nsli_params(X, Y, W, V, n, lambda, z, M, xi, eta, far, occulter, groups, per);
        if (groups > 1) {
            const size_t want = 4 * (size_t)groups * (size_t)M;
            FH_ARG(want <= kNsliScratchDoubles, FH_ERR_UNSUPPORTED,
                   "the edge integral's partial sums need %zu bytes (%d node groups x %lld targets), beyond the "
                   "%zu-byte device scratch of the allocation-free call",
                   want * sizeof(double), groups, (long long)M, kNsliScratchDoubles * sizeof(double));
            FH_TRY(scratch_for(c->device, &p.part));
        }
        if (c->prec == FH_MIXED)
            FH_TRY(nsli_launch(c, p, static_cast<float*>(u)));
        else
            FH_TRY(nsli_launch(c, p, static_cast<double*>(u)));
        return FH_OK;
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

}  // extern "C"

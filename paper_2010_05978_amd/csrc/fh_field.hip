// fh_field.hip -- the field evaluation path on the device.
//
// For an areal rule (x_j, y_j, w_j) the field of eq. faq is evaluated through
// the factorisation of eq. split:
//   1. strengths c_j = exp(i pi |x_j|^2/(lambda z)) w_j, with any pre-phase for
//      translated grids or type-3 centring folded into the same FP64 phase,
//      which is carried in turns and reduced before sincospi;
//   2. a 2D NUFFT -- type 1 onto the uniform target grid (sec. 2.2) or type 3
//      to scattered targets (eq. nufft3, sec. 2.1) -- made of
//        bin:     counting sort of the nodes into T x T fine-grid tiles,
//        spread:  exponential-of-semicircle kernel into a (T+W-1)^2 LDS tile
//                 per work item with LDS atomics, flushed once per tile cell,
//        FFT:     rocFFT on the fine grid,
//        finish:  deconvolution by the kernel's Fourier transform (type 1), or
//                 precorrection, a second FFT and kernel interpolation at the
//                 targets (type 3);
//   3. the target chirp exp(i pi |xi_k|^2/(lambda z))/(i lambda z), and
//      u_oc = 1 - u_ap for occulters (eq. bab).
#include <algorithm>
#include <cstring>

#include "fh_common.hpp"

namespace fh {
namespace {

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)std::max<int64_t>(1, (n + bs - 1) / bs); }

template <class R> struct V2;
template <> struct V2<float> { using T = float2; };
template <> struct V2<double> { using T = double2; };

// --------------------------------------------------------- device helpers
__device__ __forceinline__ int find_inst(const InstParams* t, int n, int64_t j)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t[mid].node_off <= j) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Fine-grid coordinate g -> first stencil cell (wrapped to [0, nf)) and the
// offset d = cell - g in [-W/2, -W/2 + 1).  Non-finite g is mapped to cell 0
// and flagged, so no index is ever out of range.
__device__ __forceinline__ void cell_of(double g, int nf, int W, int& cell, double& d, bool& ok)
{
    const double fnf = (double)nf;
    double gm = g - fnf * floor(g / fnf);
    ok = (gm >= 0.0) && (gm <= fnf);
    if (!ok) gm = 0.0;
    const double l0 = ceil(gm - 0.5 * W);
    d = l0 - gm;
    int i = (int)l0;
    if (i < 0) i += nf;
    if (i >= nf) i -= nf;
    cell = i;
}

template <class R, int W>
__device__ __forceinline__ void es_weights(R d, R beta, R* k)
{
    const R s = R(2) / R(W);
#pragma unroll
    for (int a = 0; a < W; ++a) {
        const R z = (d + R(a)) * s;
        const R q = R(1) - z * z;
        if constexpr (sizeof(R) == 4)
            k[a] = __expf(beta * (__fsqrt_rn(fmaxf(q, 0.0f)) - 1.0f));
        else
            k[a] = exp(beta * (sqrt(fmax(q, 0.0)) - 1.0));
    }
}

__device__ __forceinline__ double cheb_inv_phi(const InvPhiCheb& ch, double theta)
{
    const double u = theta / ch.theta_max;
    const double s = 2.0 * u * u - 1.0;
    double b1 = 0.0, b2 = 0.0;
    for (int j = ch.deg; j >= 1; --j) {
        const double b0 = 2.0 * s * b1 - b2 + ch.c[j];
        b2 = b1;
        b1 = b0;
    }
    return s * b1 - b2 + ch.c[0];
}

// ----------------------------------------------------------------- fills
__global__ void k_zero16(uint4* __restrict__ p, size_t n)
{
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

template <class R>
__global__ void k_fill_field(R* __restrict__ u, int64_t M, R re)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= M) return;
    u[2 * k] = re;
    u[2 * k + 1] = R(0);
}

// ------------------------------------------------------------------- bin
// Rank of each lane's key among all increments of cnt[key]: one atomic per
// distinct key in the wavefront (quadrature nodes arrive in spoke order, so a
// wavefront touches only a few tiles, and the crowded tiles near the origin
// would otherwise serialise thousands of same-address atomics).
__device__ __forceinline__ int wave_rank(int* __restrict__ cnt, int key, bool valid)
{
    const int lane = (int)__lane_id();
    uint64_t remaining = __ballot(valid);
    int rank = 0;
    while (remaining) {
        const int leader = __ffsll((unsigned long long)remaining) - 1;
        const int lkey = __shfl(key, leader);
        const uint64_t same = __ballot(valid && key == lkey) & remaining;
        int base = 0;
        if (lane == leader) base = atomicAdd(&cnt[lkey], __popcll(same));
        base = __shfl(base, leader);
        if ((same >> lane) & 1ull) rank = base + __popcll(same & ((1ull << lane) - 1ull));
        remaining &= ~same;
    }
    return rank;
}

__global__ void __launch_bounds__(256) k_bin_count(InstParams p0, const InstParams* __restrict__ table, int ninst,
                                                   int64_t Ntot, GridGeom gg, int* __restrict__ cnt,
                                                   int* __restrict__ rank)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool valid = j < Ntot;
    int tile = 0;
    if (valid) {
        const InstParams ip = table ? table[find_inst(table, ninst, j)] : p0;
        const int64_t jj = j - ip.node_off;
        const double x = ip.x[jj], y = ip.y[jj];
        int l1, l2;
        double d1, d2;
        bool ok1, ok2;
        cell_of((x - ip.cx) * ip.s1, gg.nf1, gg.W, l1, d1, ok1);
        cell_of((y - ip.cy) * ip.s2, gg.nf2, gg.W, l2, d2, ok2);
        tile = ip.tile_off + (l2 / gg.T) * gg.ntx + (l1 / gg.T);
    }
    const int r = wave_rank(cnt, tile, valid);
    if (valid) rank[j] = r;
}

// One block: exclusive scan of tile counts -> tile offsets, and the list of
// spread work items (tile, [start, end)) with at most P points each.
__global__ void __launch_bounds__(1024) k_scan_tiles(const int* __restrict__ cnt, int ntiles, int P,
                                                     int* __restrict__ off, Sub* __restrict__ subs,
                                                     int* __restrict__ nsub_out)
{
    __shared__ int sa[1024];
    __shared__ int sb[1024];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int chunk = (ntiles + nt - 1) / nt;
    const int t0 = min(ntiles, tid * chunk), t1 = min(ntiles, t0 + chunk);
    int a = 0, b = 0;
    for (int t = t0; t < t1; ++t) {
        const int c = cnt[t];
        a += c;
        b += (c + P - 1) / P;
    }
    sa[tid] = a;
    sb[tid] = b;
    __syncthreads();
    for (int o = 1; o < nt; o <<= 1) {
        const int va = tid >= o ? sa[tid - o] : 0;
        const int vb = tid >= o ? sb[tid - o] : 0;
        __syncthreads();
        sa[tid] += va;
        sb[tid] += vb;
        __syncthreads();
    }
    int ea = sa[tid] - a, eb = sb[tid] - b;
    for (int t = t0; t < t1; ++t) {
        const int c = cnt[t];
        off[t] = ea;
        const int ns = (c + P - 1) / P;
        for (int s = 0; s < ns; ++s) {
            Sub w;
            w.tile = t;
            w.start = ea + s * P;
            w.end = min(ea + (s + 1) * P, ea + c);
            subs[eb + s] = w;
        }
        ea += c;
        eb += ns;
    }
    if (tid == nt - 1) *nsub_out = sb[nt - 1];
}

// Strength (FP64 phase in turns, reduced), stencil offsets, and the sorted
// position of each node.
template <class R>
__global__ void k_bin_place(InstParams p0, const InstParams* __restrict__ table, int ninst, int64_t Ntot,
                            GridGeom gg, const int* __restrict__ off, const int* __restrict__ rank,
                            uint32_t* __restrict__ cell, typename V2<R>::T* __restrict__ dd,
                            typename V2<R>::T* __restrict__ cc)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= Ntot) return;
    const InstParams ip = table ? table[find_inst(table, ninst, j)] : p0;
    const int64_t jj = j - ip.node_off;
    const double x = ip.x[jj], y = ip.y[jj];
    double w = ip.w[jj];
    int l1, l2;
    double d1, d2;
    bool ok1, ok2;
    cell_of((x - ip.cx) * ip.s1, gg.nf1, gg.W, l1, d1, ok1);
    cell_of((y - ip.cy) * ip.s2, gg.nf2, gg.W, l2, d2, ok2);
    if (!(ok1 && ok2)) w = 0.0;
    const int tile = ip.tile_off + (l2 / gg.T) * gg.ntx + (l1 / gg.T);
    const double t = ((x * x + y * y) * ip.pa + (x * ip.px + y * ip.py)) + ip.pc;
    const double f = t - rint(t);
    double s, c;
    sincospi(2.0 * f, &s, &c);
    const int pos = off[tile] + rank[j];
    cell[pos] = (uint32_t)l1 | ((uint32_t)l2 << 16);
    typename V2<R>::T dv, cv;
    dv.x = (R)d1;
    dv.y = (R)d2;
    cv.x = (R)(w * c);
    cv.y = (R)(w * s);
    dd[pos] = dv;
    cc[pos] = cv;
}

// ----------------------------------------------------------------- spread
// Add a padded L x L LDS tile (split re/im planes) into the periodic fine
// grid at origin (ox, oy); empty cells are skipped.
template <class R>
__device__ __forceinline__ void flush_tile(const R* sre, const R* sim, int L, R* __restrict__ g, int ox, int oy,
                                           int nf1, int nf2)
{
    const int LL = L * L;
    for (int e = threadIdx.x; e < LL; e += blockDim.x) {
        const R vr = sre[e], vi = sim[e];
        if (vr != R(0) || vi != R(0)) {
            const int jy = e / L, ix = e - jy * L;
            int gx = ox + ix;
            if (gx >= nf1) gx -= nf1;
            int gy = oy + jy;
            if (gy >= nf2) gy -= nf2;
            R* dst = g + 2 * ((size_t)gy * nf1 + gx);
            atomicAdd(dst, vr);
            atomicAdd(dst + 1, vi);
        }
    }
}

// One work item (tile, point range) per loop trip of a block; each thread
// spreads whole points into the block's LDS tile (split re/im planes) with
// LDS atomics; the tile is then added once into the fine grid.
template <class R, int W>
__global__ void __launch_bounds__(256) k_spread(const Sub* __restrict__ subs, const int* __restrict__ nsub_ptr,
                                                const uint32_t* __restrict__ cell,
                                                const typename V2<R>::T* __restrict__ dd,
                                                const typename V2<R>::T* __restrict__ cc,
                                                R* __restrict__ grid, GridGeom gg, int tiles_per_inst, R beta)
{
    extern __shared__ unsigned char smem_raw[];
    R* sre = reinterpret_cast<R*>(smem_raw);
    const int L = gg.L, LL = L * L;
    R* sim = sre + LL;
    const int nsub = *nsub_ptr;
    for (int s = blockIdx.x; s < nsub; s += gridDim.x) {
        const Sub sb = subs[s];
        const int inst = sb.tile / tiles_per_inst;
        const int tl = sb.tile - inst * tiles_per_inst;
        const int ty = tl / gg.ntx, tx = tl - ty * gg.ntx;
        const int ox = tx * gg.T, oy = ty * gg.T;
        for (int e = threadIdx.x; e < LL; e += blockDim.x) {
            sre[e] = R(0);
            sim[e] = R(0);
        }
        __syncthreads();
        for (int p = sb.start + (int)threadIdx.x; p < sb.end; p += blockDim.x) {
            const uint32_t cp = cell[p];
            const int l1 = (int)(cp & 0xffffu) - ox;
            const int l2 = (int)(cp >> 16) - oy;
            const typename V2<R>::T dv = dd[p];
            const typename V2<R>::T cv = cc[p];
            R k1[W], k2[W];
            es_weights<R, W>(dv.x, beta, k1);
            es_weights<R, W>(dv.y, beta, k2);
#pragma unroll
            for (int b = 0; b < W; ++b) {
                const R vr = cv.x * k2[b], vi = cv.y * k2[b];
                R* rr = sre + (l2 + b) * L + l1;
                R* ri = sim + (l2 + b) * L + l1;
#pragma unroll
                for (int a = 0; a < W; ++a) {
                    atomicAdd(rr + a, vr * k1[a]);
                    atomicAdd(ri + a, vi * k1[a]);
                }
            }
        }
        __syncthreads();
        flush_tile(sre, sim, L, grid + (size_t)inst * gg.nf1 * gg.nf2 * 2, ox, oy, gg.nf1, gg.nf2);
        __syncthreads();
    }
}

// Uniform (scalar) copy of lane q's value.
__device__ __forceinline__ int lane_val(int v, int q) { return __builtin_amdgcn_readlane(v, q); }
__device__ __forceinline__ float lane_val(float v, int q)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), q));
}
__device__ __forceinline__ double lane_val(double v, int q)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), q);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), q);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wavefront-per-point spread.  A wavefront loads 64 points and stages their
// 2W kernel values in LDS; it then walks the points one at a time with its
// lanes laid over the W x W stencil (ceil(W^2/64) passes), so the LDS atomics
// of one instruction never share an address however tightly the points
// cluster (the dilation rule crowds nodes near the origin).
template <class R, int W>
__global__ void __launch_bounds__(256) k_spread_wave(const Sub* __restrict__ subs, const int* __restrict__ nsub_ptr,
                                                     const uint32_t* __restrict__ cell,
                                                     const typename V2<R>::T* __restrict__ dd,
                                                     const typename V2<R>::T* __restrict__ cc,
                                                     R* __restrict__ grid, GridGeom gg, int tiles_per_inst, R beta)
{
    constexpr int KS = 2 * W + 1;               // staging stride per point
    constexpr int NPASS = (W * W + 63) / 64;    // stencil passes per point
    extern __shared__ unsigned char smem_raw[];
    R* sre = reinterpret_cast<R*>(smem_raw);
    const int L = gg.L, LL = L * L;
    R* sim = sre + LL;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    R* kb = sim + LL + wv * 64 * KS;
    int pa[NPASS], pb[NPASS];
    bool pv[NPASS];
#pragma unroll
    for (int p = 0; p < NPASS; ++p) {
        const int e = lane + 64 * p;
        pv[p] = e < W * W;
        pa[p] = pv[p] ? e % W : 0;
        pb[p] = pv[p] ? e / W : 0;
    }
    const int nsub = *nsub_ptr;
    for (int s = blockIdx.x; s < nsub; s += gridDim.x) {
        const Sub sb = subs[s];
        const int inst = sb.tile / tiles_per_inst;
        const int tl = sb.tile - inst * tiles_per_inst;
        const int ty = tl / gg.ntx, tx = tl - ty * gg.ntx;
        const int ox = tx * gg.T, oy = ty * gg.T;
        for (int e = threadIdx.x; e < LL; e += blockDim.x) {
            sre[e] = R(0);
            sim[e] = R(0);
        }
        __syncthreads();
        for (int base = sb.start + wv * 64; base < sb.end; base += nw * 64) {
            const int p = base + lane;
            int l1 = 0, l2 = 0;
            R cr = R(0), ci = R(0);
            if (p < sb.end) {
                const uint32_t cp = cell[p];
                l1 = (int)(cp & 0xffffu) - ox;
                l2 = (int)(cp >> 16) - oy;
                const typename V2<R>::T dv = dd[p];
                const typename V2<R>::T cv = cc[p];
                cr = cv.x;
                ci = cv.y;
                R k[W];
                es_weights<R, W>(dv.x, beta, k);
#pragma unroll
                for (int a = 0; a < W; ++a) kb[lane * KS + a] = k[a];
                es_weights<R, W>(dv.y, beta, k);
#pragma unroll
                for (int b = 0; b < W; ++b) kb[lane * KS + W + b] = k[b];
            }
            // LDS traffic of one wavefront is processed in order; the fences
            // keep the compiler from moving the staging reads above the writes.
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int np = min(64, sb.end - base);
            for (int q = 0; q < np; ++q) {
                const int ql1 = lane_val(l1, q), ql2 = lane_val(l2, q);
                const R qr = lane_val(cr, q), qi = lane_val(ci, q);
                const R* kq = kb + q * KS;
#pragma unroll
                for (int pp = 0; pp < NPASS; ++pp) {
                    if (pv[pp]) {
                        const R kv = kq[pa[pp]] * kq[W + pb[pp]];
                        const int idx = (ql2 + pb[pp]) * L + ql1 + pa[pp];
                        atomicAdd(sre + idx, qr * kv);
                        atomicAdd(sim + idx, qi * kv);
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        __syncthreads();
        flush_tile(sre, sim, L, grid + (size_t)inst * gg.nf1 * gg.nf2 * 2, ox, oy, gg.nf1, gg.nf2);
        __syncthreads();
    }
}

// --------------------------------------------------------- type-1 finish
struct EpiInst {
    double inv2lz;  // 1/(2 lambda z): target chirp in turns
    double invlz;   // 1/(lambda z)
    int occ;
    int pad_;
};

struct EpiParams {
    int n1, n2, nf1, nf2;
    double h1, h2, xc, yc;
    const double* iphi1;
    const double* iphi2;
};

template <class R>
__global__ void k_epilogue(const R* __restrict__ F, R* __restrict__ u, EpiParams ep, EpiInst e0,
                           const EpiInst* __restrict__ table)
{
    const int k1i = blockIdx.x * blockDim.x + threadIdx.x;
    const int k2i = blockIdx.y;
    const int inst = blockIdx.z;
    if (k1i >= ep.n1) return;
    const EpiInst ei = table ? table[inst] : e0;
    const int k1 = k1i - ep.n1 / 2, k2 = k2i - ep.n2 / 2;
    const int i1 = k1 < 0 ? k1 + ep.nf1 : k1;
    const int i2 = k2 < 0 ? k2 + ep.nf2 : k2;
    const size_t fbase = (size_t)inst * ep.nf1 * ep.nf2;
    const typename V2<R>::T fv = reinterpret_cast<const typename V2<R>::T*>(F)[fbase + (size_t)i2 * ep.nf1 + i1];
    const double sc = ep.iphi1[k1i] * ep.iphi2[k2i];
    const double vr = (double)fv.x * sc, vi = (double)fv.y * sc;
    const double xi = ep.xc + ep.h1 * k1, eta = ep.yc + ep.h2 * k2;
    const double t = (xi * xi + eta * eta) * ei.inv2lz;
    const double f = t - rint(t);
    double s, c;
    sincospi(2.0 * f, &s, &c);
    double re = (s * vr + c * vi) * ei.invlz;
    double im = (s * vi - c * vr) * ei.invlz;
    if (ei.occ) {
        re = 1.0 - re;
        im = -im;
    }
    typename V2<R>::T out;
    out.x = (R)re;
    out.y = (R)im;
    reinterpret_cast<typename V2<R>::T*>(u)[(size_t)inst * ep.n1 * ep.n2 + (size_t)k2i * ep.n1 + k1i] = out;
}

// --------------------------------------------------------- type-3 finish
// Precorrect the spread grid b (modes l' in [-nf/2, nf/2)) by 1/Phi and
// embed it in the upsampled grid G (every entry of G is written).
template <class R>
__global__ void k_t3_precorrect(const R* __restrict__ b, int nf1, int nf2, R* __restrict__ G, int m1, int m2,
                                const double* __restrict__ ip1, const double* __restrict__ ip2)
{
    const int i1 = blockIdx.x * blockDim.x + threadIdx.x;
    const int i2 = blockIdx.y;
    if (i1 >= m1) return;
    const int k1 = i1 < m1 / 2 ? i1 : i1 - m1;
    const int k2 = i2 < m2 / 2 ? i2 : i2 - m2;
    typename V2<R>::T v;
    v.x = R(0);
    v.y = R(0);
    if (k1 >= -(nf1 / 2) && k1 < nf1 - nf1 / 2 && k2 >= -(nf2 / 2) && k2 < nf2 - nf2 / 2) {
        const int s1 = k1 < 0 ? k1 + nf1 : k1;
        const int s2 = k2 < 0 ? k2 + nf2 : k2;
        const typename V2<R>::T bv = reinterpret_cast<const typename V2<R>::T*>(b)[(size_t)s2 * nf1 + s1];
        const double sc = ip1[k1 + nf1 / 2] * ip2[k2 + nf2 / 2];
        v.x = (R)(bv.x * sc);
        v.y = (R)(bv.y * sc);
    }
    reinterpret_cast<typename V2<R>::T*>(G)[(size_t)i2 * m1 + i1] = v;
}

struct T3Params {
    int m1, m2;                // upsampled grid
    double xic, etac;          // target centre
    double g1, g2;             // interpolation grid coordinate per unit (xi - xic)
    double th1, th2;           // theta per unit (xi - xic) for the 1/Phi correction
    double inv2lz, invlz;      // target chirp (turns) and 1/(lambda z)
    double Cx, Cy;             // source centre (post-phase exp(-i s.C))
    int occ;
    InvPhiCheb ch1, ch2;
};

template <class R, int W>
__global__ void __launch_bounds__(256) k_t3_interp(const R* __restrict__ G, const double* __restrict__ xi,
                                                   const double* __restrict__ eta, int64_t M, R beta,
                                                   T3Params tp, R* __restrict__ u)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= M) return;
    const double X = xi[k], Y = eta[k];
    int l1, l2;
    double d1, d2;
    bool ok1, ok2;
    cell_of((X - tp.xic) * tp.g1, tp.m1, W, l1, d1, ok1);
    cell_of((Y - tp.etac) * tp.g2, tp.m2, W, l2, d2, ok2);
    R k1[W], k2[W];
    es_weights<R, W>((R)d1, beta, k1);
    es_weights<R, W>((R)d2, beta, k2);
    const typename V2<R>::T* Gv = reinterpret_cast<const typename V2<R>::T*>(G);
    R sr = 0, si = 0;
#pragma unroll
    for (int b = 0; b < W; ++b) {
        int row = l2 + b;
        if (row >= tp.m2) row -= tp.m2;
        const typename V2<R>::T* gr = Gv + (size_t)row * tp.m1;
        R ar = 0, ai = 0;
#pragma unroll
        for (int a = 0; a < W; ++a) {
            int col = l1 + a;
            if (col >= tp.m1) col -= tp.m1;
            const typename V2<R>::T gv = gr[col];
            ar += gv.x * k1[a];
            ai += gv.y * k1[a];
        }
        sr += ar * k2[b];
        si += ai * k2[b];
    }
    const double corr = cheb_inv_phi(tp.ch1, (X - tp.xic) * tp.th1) * cheb_inv_phi(tp.ch2, (Y - tp.etac) * tp.th2);
    const double vr = (double)sr * corr, vi = (double)si * corr;
    const double t = (X * X + Y * Y) * tp.inv2lz - (X * tp.Cx + Y * tp.Cy) * tp.invlz;
    const double f = t - rint(t);
    double s, c;
    sincospi(2.0 * f, &s, &c);
    double re = (s * vr + c * vi) * tp.invlz;
    double im = (s * vi - c * vr) * tp.invlz;
    if (!(ok1 && ok2)) {
        re = __builtin_nan("");
        im = __builtin_nan("");
    }
    if (tp.occ) {
        re = 1.0 - re;
        im = -im;
    }
    u[2 * k] = (R)re;
    u[2 * k + 1] = (R)im;
}

// ---------------------------------------------------------------- bbox
__global__ void __launch_bounds__(256) k_bbox_partial(const double* __restrict__ x, const double* __restrict__ y,
                                                      int64_t n, double* __restrict__ part)
{
    double v[4] = {INFINITY, -INFINITY, INFINITY, -INFINITY};
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double a = x[i], b = y[i];
        bad |= !(isfinite(a) && isfinite(b));
        v[0] = fmin(v[0], a);
        v[1] = fmax(v[1], a);
        v[2] = fmin(v[2], b);
        v[3] = fmax(v[3], b);
    }
    __shared__ double s[4][256];
    __shared__ int sbad;
    if (threadIdx.x == 0) sbad = 0;
    for (int q = 0; q < 4; ++q) s[q][threadIdx.x] = v[q];
    __syncthreads();
    if (bad) atomicOr(&sbad, 1);
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + o]);
            s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][threadIdx.x + o]);
            s[2][threadIdx.x] = fmin(s[2][threadIdx.x], s[2][threadIdx.x + o]);
            s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int q = 0; q < 4; ++q) part[5 * blockIdx.x + q] = s[q][0];
        part[5 * blockIdx.x + 4] = sbad ? 1.0 : 0.0;
    }
}

__global__ void __launch_bounds__(256) k_bbox_final(const double* __restrict__ part, int nparts,
                                                    double* __restrict__ out)
{
    __shared__ double s[5][256];
    double v[5] = {INFINITY, -INFINITY, INFINITY, -INFINITY, 0.0};
    for (int p = threadIdx.x; p < nparts; p += blockDim.x) {
        v[0] = fmin(v[0], part[5 * p]);
        v[1] = fmax(v[1], part[5 * p + 1]);
        v[2] = fmin(v[2], part[5 * p + 2]);
        v[3] = fmax(v[3], part[5 * p + 3]);
        v[4] = fmax(v[4], part[5 * p + 4]);
    }
    for (int q = 0; q < 5; ++q) s[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const int t = threadIdx.x;
            s[0][t] = fmin(s[0][t], s[0][t + o]);
            s[1][t] = fmax(s[1][t], s[1][t + o]);
            s[2][t] = fmin(s[2][t], s[2][t + o]);
            s[3][t] = fmax(s[3][t], s[3][t + o]);
            s[4][t] = fmax(s[4][t], s[4][t + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 5; ++q) out[q] = s[q][0];
}

// ------------------------------------------------------- launch helpers
constexpr size_t kLdsBudget = 64 * 1024;

template <class R, int W>
void launch_spread_w(fh_ctx* c, unsigned grid, const Sub* subs, const int* nsub, const uint32_t* cell,
                     const void* dd, const void* cc, R* fine, const GridGeom& gg, int tpi, double beta)
{
    const size_t tile = 2 * sizeof(R) * (size_t)gg.L * gg.L;
    if (gg.method == 1) {
        hipLaunchKernelGGL((k_spread<R, W>), dim3(grid), dim3(256), tile, c->stream, subs, nsub, cell,
                           (const typename V2<R>::T*)dd, (const typename V2<R>::T*)cc, fine, gg, tpi, (R)beta);
        return;
    }
    const size_t per_wave = sizeof(R) * 64 * (2 * W + 1);
    int nw = 4;
    while (nw > 1 && tile + nw * per_wave > kLdsBudget) --nw;
    hipLaunchKernelGGL((k_spread_wave<R, W>), dim3(grid), dim3(64 * nw), tile + nw * per_wave, c->stream, subs,
                       nsub, cell, (const typename V2<R>::T*)dd, (const typename V2<R>::T*)cc, fine, gg, tpi,
                       (R)beta);
}

template <class R>
fh_status launch_spread(fh_ctx* c, unsigned grid, const Sub* subs, const int* nsub, const uint32_t* cell,
                        const void* dd, const void* cc, R* fine, const GridGeom& gg, int tpi, double beta)
{
    FH_ARG(2 * sizeof(R) * (size_t)gg.L * gg.L + sizeof(R) * 64 * (2 * gg.W + 1) <= kLdsBudget,
           FH_ERR_UNSUPPORTED, "spread tile %d with width %d exceeds the LDS budget", gg.T, gg.W);
    switch (gg.W) {
#define FH_SPREAD_CASE(w) \
    case w: launch_spread_w<R, w>(c, grid, subs, nsub, cell, dd, cc, fine, gg, tpi, beta); break;
        FH_SPREAD_CASE(2) FH_SPREAD_CASE(3) FH_SPREAD_CASE(4) FH_SPREAD_CASE(5) FH_SPREAD_CASE(6)
        FH_SPREAD_CASE(7) FH_SPREAD_CASE(8) FH_SPREAD_CASE(9) FH_SPREAD_CASE(10) FH_SPREAD_CASE(11)
        FH_SPREAD_CASE(12) FH_SPREAD_CASE(13) FH_SPREAD_CASE(14) FH_SPREAD_CASE(15) FH_SPREAD_CASE(16)
        FH_SPREAD_CASE(17) FH_SPREAD_CASE(18) FH_SPREAD_CASE(19) FH_SPREAD_CASE(20)
#undef FH_SPREAD_CASE
    default: set_error("kernel width %d unsupported", gg.W); return FH_ERR_UNSUPPORTED;
    }
    FH_HIP(hipGetLastError());
    return FH_OK;
}

template <class R>
fh_status launch_interp(fh_ctx* c, int W, const R* G, const double* xi, const double* eta, int64_t M,
                        double beta, const T3Params& tp, R* u)
{
    const unsigned g = nblocks(M, 256);
    switch (W) {
#define FH_INTERP_CASE(w)                                                                           \
    case w:                                                                                        \
        hipLaunchKernelGGL((k_t3_interp<R, w>), dim3(g), dim3(256), 0, c->stream, G, xi, eta, M, (R)beta, \
                           tp, u);                                                                 \
        break;
        FH_INTERP_CASE(2) FH_INTERP_CASE(3) FH_INTERP_CASE(4) FH_INTERP_CASE(5) FH_INTERP_CASE(6)
        FH_INTERP_CASE(7) FH_INTERP_CASE(8) FH_INTERP_CASE(9) FH_INTERP_CASE(10) FH_INTERP_CASE(11)
        FH_INTERP_CASE(12) FH_INTERP_CASE(13) FH_INTERP_CASE(14) FH_INTERP_CASE(15) FH_INTERP_CASE(16)
        FH_INTERP_CASE(17) FH_INTERP_CASE(18) FH_INTERP_CASE(19) FH_INTERP_CASE(20)
#undef FH_INTERP_CASE
    default: set_error("kernel width %d unsupported", W); return FH_ERR_UNSUPPORTED;
    }
    FH_HIP(hipGetLastError());
    return FH_OK;
}

// ------------------------------------------------------ spread pipeline
// Buffers of one binned spread, carved from the arena.
struct SpreadBufs {
    int* cnt;
    int* off;
    int* rank;
    uint32_t* cell;
    void* dd;
    void* cc;
    Sub* subs;
    int* nsub;
    int64_t max_sub;
};

size_t spread_bytes(int64_t Ntot, int ntiles_total, int P, size_t rsize)
{
    const int64_t max_sub = Ntot / P + std::min<int64_t>(Ntot, ntiles_total) + 1;
    return 2 * aligned_bytes(sizeof(int) * (size_t)ntiles_total) + aligned_bytes(sizeof(int) * Ntot) +
           aligned_bytes(sizeof(uint32_t) * Ntot) + 2 * aligned_bytes(2 * rsize * Ntot) +
           aligned_bytes(sizeof(Sub) * max_sub) + aligned_bytes(sizeof(int));
}

SpreadBufs spread_carve(fh_ctx* c, int64_t Ntot, int ntiles_total, int P, size_t rsize)
{
    SpreadBufs b;
    b.max_sub = Ntot / P + std::min<int64_t>(Ntot, ntiles_total) + 1;
    b.cnt = c->arena.take<int>(ntiles_total);
    b.off = c->arena.take<int>(ntiles_total);
    b.rank = c->arena.take<int>(Ntot);
    b.cell = c->arena.take<uint32_t>(Ntot);
    b.dd = c->arena.take<char>(2 * rsize * Ntot);
    b.cc = c->arena.take<char>(2 * rsize * Ntot);
    b.subs = c->arena.take<Sub>(b.max_sub);
    b.nsub = c->arena.take<int>(1);
    return b;
}

// Zero the fine grid(s) and tile counters, bin, and spread.
template <class R>
fh_status run_spread(fh_ctx* c, const InstParams& p0, const InstParams* table, int ninst, int64_t Ntot,
                     const GridGeom& gg, int ntiles_total, const SpreadBufs& b, R* fine, size_t fine_bytes,
                     double beta)
{
    FH_TRY(launch_zero(c, b.cnt, sizeof(int) * ntiles_total));
    FH_TRY(launch_zero(c, fine, fine_bytes));
    if (Ntot > 0) {
        hipLaunchKernelGGL(k_bin_count, dim3(nblocks(Ntot, 256)), dim3(256), 0, c->stream, p0, table, ninst,
                           Ntot, gg, b.cnt, b.rank);
    }
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, c->stream, b.cnt, ntiles_total, gg.P, b.off,
                       b.subs, b.nsub);
    if (Ntot > 0) {
        hipLaunchKernelGGL((k_bin_place<R>), dim3(nblocks(Ntot, 256)), dim3(256), 0, c->stream, p0, table,
                           ninst, Ntot, gg, b.off, b.rank, b.cell, (typename V2<R>::T*)b.dd,
                           (typename V2<R>::T*)b.cc);
    }
    FH_HIP(hipGetLastError());
    timing_mark(c, 1);
    if (Ntot > 0) {
        const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(b.max_sub, (int64_t)c->cu_count * 8));
        FH_TRY(launch_spread<R>(c, grid, b.subs, b.nsub, b.cell, b.dd, b.cc, fine, gg,
                                ntiles_total / std::max(ninst, 1), beta));
    }
    timing_mark(c, 2);
    return FH_OK;
}

// Spread method and work-item size: the wavefront-per-point spread is the
// default (robust to the dense clusters of dilation rules); small work items
// spread one crowded tile over many CUs.
void spread_defaults(const fh_ctx* c, GridGeom& g)
{
    g.method = c->opt.spread_method > 0 ? c->opt.spread_method : 2;
    g.P = c->opt.max_subproblem > 0 ? c->opt.max_subproblem : (g.method == 2 ? 256 : 1024);
}

fh_status check_lz(double lambda, double z)
{
    FH_ARG(std::isfinite(lambda) && std::isfinite(z), FH_ERR_NONFINITE, "lambda or z not finite");
    FH_ARG(lambda * z > 0 && std::isfinite(lambda * z), FH_ERR_NONPOSITIVE_LZ, "lambda * z must be > 0");
    return FH_OK;
}

// Shared geometry of a type-1 call on an n1 x n2 target grid.
struct T1Plan {
    EsKernel k;
    GridGeom gg;
    int ntiles;
};

T1Plan plan_t1(fh_ctx* c, int n1, int n2)
{
    T1Plan p;
    p.k = choose_kernel(c, std::max(n1, n2));
    const int W = p.k.w;
    const int need1 = std::max((int)std::ceil(p.k.sigma * n1), 2 * W);
    const int need2 = std::max((int)std::ceil(p.k.sigma * n2), 2 * W);
    int T = pick_tile(c, std::min(need1, need2));
    if (c->prec == FH_FP64 && T > 32) T = 32;
    GridGeom& g = p.gg;
    g.T = T;
    g.W = W;
    g.L = T + W - 1;
    g.nf1 = next_fft_size(std::max(need1, T + W), T);
    g.nf2 = next_fft_size(std::max(need2, T + W), T);
    g.ntx = g.nf1 / T;
    g.nty = g.nf2 / T;
    spread_defaults(c, g);
    p.ntiles = g.ntx * g.nty;
    return p;
}

InstParams inst_t1(const fh_quad* q, double lambda, double z, double h1, double h2, double xc, double yc,
                   const GridGeom& g)
{
    const double lz = lambda * z;
    InstParams ip{};
    ip.x = q->x;
    ip.y = q->y;
    ip.w = q->w;
    ip.N = q->N;
    ip.node_off = 0;
    ip.tile_off = 0;
    // source chirp with the pre-phase of a grid centred at (xc, yc):
    // pi (|x|^2 - 2 (xc x + yc y)) / (lambda z), in turns
    ip.pa = 0.5 / lz;
    ip.px = -xc / lz;
    ip.py = -yc / lz;
    ip.pc = 0.0;
    // rescaled node x~ = 2 pi h x/(lambda z), in fine-grid cells of 2 pi/nf
    ip.cx = 0.0;
    ip.cy = 0.0;
    ip.s1 = h1 * g.nf1 / lz;
    ip.s2 = h2 * g.nf2 / lz;
    return ip;
}

template <class R>
fh_status field_grid_impl(fh_ctx* c, const fh_quad* q, double lambda, double z, int n1, int n2, double h1,
                          double h2, double xc, double yc, int occ, void* u, fh_memspace mem)
{
    const int64_t M = (int64_t)n1 * n2;
    const size_t rs = sizeof(R);
    const double lz = lambda * z;
    T1Plan pl = plan_t1(c, n1, n2);
    const GridGeom& gg = pl.gg;
    const int64_t N = q->N;
    const size_t fine_bytes = 2 * rs * (size_t)gg.nf1 * gg.nf2;
    const size_t out_bytes = 2 * rs * (size_t)M;
    const double* ip1 = nullptr;
    const double* ip2 = nullptr;
    FH_TRY(iphi_table(c, pl.k, n1, gg.nf1, &ip1));
    FH_TRY(iphi_table(c, pl.k, n2, gg.nf2, &ip2));
    FftPlan* fp = nullptr;
    FH_TRY(fft_plan(c, gg.nf1, gg.nf2, 1, &fp));
    size_t need = aligned_bytes(fine_bytes) + spread_bytes(N, pl.ntiles, gg.P, rs) +
                  (mem == FH_MEM_HOST ? aligned_bytes(out_bytes) : 0);
    FH_TRY(arena_reserve(c, need));
    R* fine = c->arena.take<R>(2 * (size_t)gg.nf1 * gg.nf2);
    SpreadBufs sb = spread_carve(c, N, pl.ntiles, gg.P, rs);
    R* dout = mem == FH_MEM_HOST ? c->arena.take<R>(2 * M) : static_cast<R*>(u);

    c->timing_kind = 0;
    timing_mark(c, 0);
    if (N == 0) {
        hipLaunchKernelGGL((k_fill_field<R>), dim3(nblocks(M, 256)), dim3(256), 0, c->stream, dout, M,
                           (R)(occ ? 1.0 : 0.0));
        FH_HIP(hipGetLastError());
        for (int i = 1; i <= 5; ++i) timing_mark(c, i);
    } else {
        InstParams ip = inst_t1(q, lambda, z, h1, h2, xc, yc, gg);
        FH_TRY(run_spread<R>(c, ip, nullptr, 1, N, gg, pl.ntiles, sb, fine, fine_bytes, pl.k.beta));
        FH_TRY(fft_exec(c, fp, fine));
        timing_mark(c, 3);
        EpiParams ep{n1, n2, gg.nf1, gg.nf2, h1, h2, xc, yc, ip1, ip2};
        EpiInst e0{0.5 / lz, 1.0 / lz, occ ? 1 : 0, 0};
        hipLaunchKernelGGL((k_epilogue<R>), dim3(nblocks(n1, 256), n2, 1), dim3(256), 0, c->stream, fine, dout,
                           ep, e0, (const EpiInst*)nullptr);
        FH_HIP(hipGetLastError());
        timing_mark(c, 4);
        timing_mark(c, 5);
    }
    if (mem == FH_MEM_HOST) {
        FH_HIP(hipMemcpyAsync(u, dout, out_bytes, hipMemcpyDeviceToHost, c->stream));
        FH_HIP(hipStreamSynchronize(c->stream));
    }
    return FH_OK;
}

// Type-3 plan of one dimension: sources in [C - X, C + X], targets in
// [ctr - Sx, ctr + Sx] (target-plane units; frequency s = 2 pi xi/(lambda z)).
struct T3Dim {
    double C, ctr;
    int nf, m;          // spread grid and upsampled grid
    double gamma;
    double s;           // spread-grid cells per unit (x - C)
    double g;           // upsampled-grid cells per unit (xi - ctr)
    double th;          // theta per unit (xi - ctr)
    double theta_max;
};

T3Dim plan_t3_dim(double xmin, double xmax, double tmin, double tmax, double lz, const EsKernel& k, int T)
{
    T3Dim d;
    const int W = k.w;
    const double sig = k.sigma;
    d.C = 0.5 * (xmin + xmax);
    const double X = std::max(0.5 * (xmax - xmin), 0.0);
    d.ctr = 0.5 * (tmin + tmax);
    const double S = 2.0 * kPi * std::max(0.5 * (tmax - tmin), 0.0) / lz;
    const double need = 2.0 * sig * X * S / kPi + W + 1;
    d.nf = next_fft_size(std::max({(int)std::ceil(need), 2 * W, T + W}), T);
    if (S > 0)
        d.gamma = d.nf / (2.0 * sig * S);
    else
        d.gamma = std::max(X, 1e-300) * d.nf / (kPi * (d.nf - W - 1));
    if (X == 0 && S == 0) d.gamma = 1.0;
    d.m = next_fft_size(std::max((int)std::ceil(sig * d.nf), 2 * W + 2), 2);
    d.s = d.nf / (2.0 * kPi * d.gamma);
    d.th = 4.0 * kPi * kPi * d.gamma / (lz * d.nf);
    d.g = d.th * d.m / (2.0 * kPi);
    d.theta_max = std::max(S * d.gamma * 2.0 * kPi / d.nf, 1e-6);
    return d;
}

template <class R>
fh_status field_points_impl(fh_ctx* c, const fh_quad* q, double lambda, double z, int64_t M, const double* xi,
                            const double* eta, int occ, void* u, fh_memspace mem)
{
    const size_t rs = sizeof(R);
    const double lz = lambda * z;
    const int64_t N = q->N;
    if (M == 0) return FH_OK;
    // target bounding box
    double tb[4];
    if (mem == FH_MEM_HOST) {
        tb[0] = tb[2] = INFINITY;
        tb[1] = tb[3] = -INFINITY;
        for (int64_t k = 0; k < M; ++k) {
            FH_ARG(std::isfinite(xi[k]) && std::isfinite(eta[k]), FH_ERR_NONFINITE, "target %lld not finite",
                   (long long)k);
            tb[0] = std::min(tb[0], xi[k]);
            tb[1] = std::max(tb[1], xi[k]);
            tb[2] = std::min(tb[2], eta[k]);
            tb[3] = std::max(tb[3], eta[k]);
        }
    } else {
        FH_TRY(device_bbox(c, xi, eta, M, tb));
    }
    if (N == 0) {
        size_t need = mem == FH_MEM_HOST ? aligned_bytes(2 * rs * M) : 0;
        FH_TRY(arena_reserve(c, need));
        R* dout = mem == FH_MEM_HOST ? c->arena.take<R>(2 * M) : static_cast<R*>(u);
        hipLaunchKernelGGL((k_fill_field<R>), dim3(nblocks(M, 256)), dim3(256), 0, c->stream, dout, M,
                           (R)(occ ? 1.0 : 0.0));
        FH_HIP(hipGetLastError());
        if (mem == FH_MEM_HOST) {
            FH_HIP(hipMemcpyAsync(u, dout, 2 * rs * M, hipMemcpyDeviceToHost, c->stream));
            FH_HIP(hipStreamSynchronize(c->stream));
        }
        return FH_OK;
    }
    double sb[4];
    FH_TRY(quad_bbox(c, q, sb));
    FH_ARG(std::isfinite(sb[0]) && std::isfinite(sb[1]) && std::isfinite(sb[2]) && std::isfinite(sb[3]),
           FH_ERR_NONFINITE, "quadrature nodes not finite");
    EsKernel k = choose_kernel(c, 0);
    const int T0 = c->opt.tile > 0 ? c->opt.tile : 16;
    T3Dim d1 = plan_t3_dim(sb[0], sb[1], tb[0], tb[1], lz, k, T0);
    T3Dim d2 = plan_t3_dim(sb[2], sb[3], tb[2], tb[3], lz, k, T0);
    FH_ARG((int64_t)d1.m * d2.m <= (int64_t)1 << 31, FH_ERR_UNSUPPORTED,
           "type-3 fine grid %d x %d too large (space-bandwidth product too big)", d1.m, d2.m);
    FH_ARG(d1.nf <= 65535 && d2.nf <= 65535, FH_ERR_UNSUPPORTED, "type-3 spread grid too large");
    GridGeom gg;
    gg.T = T0;
    gg.W = k.w;
    gg.L = T0 + k.w - 1;
    gg.nf1 = d1.nf;
    gg.nf2 = d2.nf;
    gg.ntx = d1.nf / T0;
    gg.nty = d2.nf / T0;
    spread_defaults(c, gg);
    const int ntiles = gg.ntx * gg.nty;

    const double* ip1 = nullptr;
    const double* ip2 = nullptr;
    FH_TRY(iphi_table(c, k, d1.nf, d1.m, &ip1));
    FH_TRY(iphi_table(c, k, d2.nf, d2.m, &ip2));
    FftPlan* fp = nullptr;
    FH_TRY(fft_plan(c, d1.m, d2.m, 1, &fp));
    const size_t fine_bytes = 2 * rs * (size_t)d1.nf * d2.nf;
    const size_t up_bytes = 2 * rs * (size_t)d1.m * d2.m;
    size_t need = aligned_bytes(fine_bytes) + aligned_bytes(up_bytes) + spread_bytes(N, ntiles, gg.P, rs);
    if (mem == FH_MEM_HOST) need += 2 * aligned_bytes(sizeof(double) * M) + aligned_bytes(2 * rs * M);
    FH_TRY(arena_reserve(c, need));
    R* fine = c->arena.take<R>(2 * (size_t)d1.nf * d2.nf);
    R* up = c->arena.take<R>(2 * (size_t)d1.m * d2.m);
    SpreadBufs sbuf = spread_carve(c, N, ntiles, gg.P, rs);
    const double* dxi = xi;
    const double* deta = eta;
    R* dout = static_cast<R*>(u);
    if (mem == FH_MEM_HOST) {
        double* a = c->arena.take<double>(M);
        double* b = c->arena.take<double>(M);
        FH_HIP(hipMemcpyAsync(a, xi, sizeof(double) * M, hipMemcpyHostToDevice, c->stream));
        FH_HIP(hipMemcpyAsync(b, eta, sizeof(double) * M, hipMemcpyHostToDevice, c->stream));
        dxi = a;
        deta = b;
        dout = c->arena.take<R>(2 * M);
    }

    InstParams ip{};
    ip.x = q->x;
    ip.y = q->y;
    ip.w = q->w;
    ip.N = N;
    // chirp and pre-phase exp(-i D.(x - C)), D = 2 pi (target centre)/(lambda z)
    ip.pa = 0.5 / lz;
    ip.px = -d1.ctr / lz;
    ip.py = -d2.ctr / lz;
    ip.pc = (d1.ctr * d1.C + d2.ctr * d2.C) / lz;
    ip.cx = d1.C;
    ip.cy = d2.C;
    ip.s1 = d1.s;
    ip.s2 = d2.s;

    c->timing_kind = 1;
    timing_mark(c, 0);
    FH_TRY(run_spread<R>(c, ip, nullptr, 1, N, gg, ntiles, sbuf, fine, fine_bytes, k.beta));
    hipLaunchKernelGGL((k_t3_precorrect<R>), dim3(nblocks(d1.m, 256), d2.m), dim3(256), 0, c->stream, fine,
                       d1.nf, d2.nf, up, d1.m, d2.m, ip1, ip2);
    FH_HIP(hipGetLastError());
    FH_TRY(fft_exec(c, fp, up));
    timing_mark(c, 3);
    T3Params tp;
    tp.m1 = d1.m;
    tp.m2 = d2.m;
    tp.xic = d1.ctr;
    tp.etac = d2.ctr;
    tp.g1 = d1.g;
    tp.g2 = d2.g;
    tp.th1 = d1.th;
    tp.th2 = d2.th;
    tp.inv2lz = 0.5 / lz;
    tp.invlz = 1.0 / lz;
    tp.Cx = d1.C;
    tp.Cy = d2.C;
    tp.occ = occ ? 1 : 0;
    inv_phi_cheb(k, d1.theta_max, &tp.ch1);
    inv_phi_cheb(k, d2.theta_max, &tp.ch2);
    FH_TRY(launch_interp<R>(c, k.w, up, dxi, deta, M, k.beta, tp, dout));
    timing_mark(c, 4);
    timing_mark(c, 5);
    if (mem == FH_MEM_HOST) {
        FH_HIP(hipMemcpyAsync(u, dout, 2 * rs * M, hipMemcpyDeviceToHost, c->stream));
        FH_HIP(hipStreamSynchronize(c->stream));
    }
    return FH_OK;
}

fh_status check_grid(int n1, int n2, double h1, double h2, double xc, double yc)
{
    FH_ARG(n1 > 0 && n2 > 0, FH_ERR_INVALID_ARG, "grid sizes must be positive");
    FH_ARG(n1 % 2 == 0 && n2 % 2 == 0, FH_ERR_ODD_GRID, "grid sizes must be even (got %d x %d)", n1, n2);
    FH_ARG(std::isfinite(h1) && std::isfinite(h2) && std::isfinite(xc) && std::isfinite(yc), FH_ERR_NONFINITE,
           "grid spacing or centre not finite");
    FH_ARG(h1 > 0 && h2 > 0, FH_ERR_INVALID_ARG, "grid spacing must be positive");
    return FH_OK;
}

// ------------------------------------------------------------- batched
struct BatchKey {
    std::string s;
};

template <class R>
fh_status field_grid_batch_impl(fh_ctx* c, int B, const fh_quad* const* qs, const double* lambda,
                                const double* z, int n1, int n2, double h1, double h2, double xc, double yc,
                                const int32_t* occ, void* u)
{
    const size_t rs = sizeof(R);
    T1Plan pl = plan_t1(c, n1, n2);
    const GridGeom& gg = pl.gg;
    const int ntiles_total = pl.ntiles * B;
    FH_ARG((int64_t)pl.ntiles * B < ((int64_t)1 << 31), FH_ERR_UNSUPPORTED, "too many tiles in batch");
    std::vector<InstParams> inst(B);
    std::vector<EpiInst> epi(B);
    int64_t Ntot = 0;
    for (int b = 0; b < B; ++b) {
        inst[b] = inst_t1(qs[b], lambda[b], z[b], h1, h2, xc, yc, gg);
        inst[b].node_off = Ntot;
        inst[b].tile_off = b * pl.ntiles;
        Ntot += qs[b]->N;
        const double lz = lambda[b] * z[b];
        epi[b] = EpiInst{0.5 / lz, 1.0 / lz, occ[b] ? 1 : 0, 0};
    }
    FH_ARG(Ntot < ((int64_t)1 << 31), FH_ERR_UNSUPPORTED, "batch has %lld nodes; at most 2^31 - 1",
           (long long)Ntot);
    const double* ip1 = nullptr;
    const double* ip2 = nullptr;
    FH_TRY(iphi_table(c, pl.k, n1, gg.nf1, &ip1));
    FH_TRY(iphi_table(c, pl.k, n2, gg.nf2, &ip2));
    FftPlan* fp = nullptr;
    FH_TRY(fft_plan(c, gg.nf1, gg.nf2, B, &fp));
    const size_t fine_bytes = 2 * rs * (size_t)gg.nf1 * gg.nf2 * B;
    size_t need = aligned_bytes(fine_bytes) + spread_bytes(Ntot, ntiles_total, gg.P, rs) +
                  aligned_bytes(sizeof(InstParams) * B) + aligned_bytes(sizeof(EpiInst) * B);
    FH_TRY(arena_reserve(c, need));
    R* fine = c->arena.take<R>(2 * (size_t)gg.nf1 * gg.nf2 * B);
    SpreadBufs sb = spread_carve(c, Ntot, ntiles_total, gg.P, rs);
    InstParams* dinst = c->arena.take<InstParams>(B);
    EpiInst* depi = c->arena.take<EpiInst>(B);
    FH_HIP(hipMemcpyAsync(dinst, inst.data(), sizeof(InstParams) * B, hipMemcpyHostToDevice, c->stream));
    FH_HIP(hipMemcpyAsync(depi, epi.data(), sizeof(EpiInst) * B, hipMemcpyHostToDevice, c->stream));

    // The graph is keyed by everything that is baked into its kernel
    // arguments: arena base, sizes, node counts and grid parameters.
    char key[256];
    snprintf(key, sizeof(key), "%p|%zu|%d|%lld|%d|%d|%d|%d|%d|%a|%a|%a|%a|%d", (void*)c->arena.base,
             c->arena.cap, B, (long long)Ntot, n1, n2, gg.nf1, gg.nf2, gg.W, h1, h2, xc, yc, gg.T * 1000 + gg.P);
    std::string k2(key);
    for (int b = 0; b < B; ++b) k2 += "|" + std::to_string(qs[b]->N);
    k2 += "|" + std::to_string((uintptr_t)u);
    const bool use_graph = !c->timing && std::getenv("FH_NO_GRAPH") == nullptr;
    auto run = [&]() -> fh_status {
        InstParams p0{};
        FH_TRY(run_spread<R>(c, p0, dinst, B, Ntot, gg, ntiles_total, sb, fine, fine_bytes, pl.k.beta));
        FH_TRY(fft_exec(c, fp, fine));
        timing_mark(c, 3);
        EpiParams ep{n1, n2, gg.nf1, gg.nf2, h1, h2, xc, yc, ip1, ip2};
        EpiInst e0{};
        hipLaunchKernelGGL((k_epilogue<R>), dim3(nblocks(n1, 256), n2, B), dim3(256), 0, c->stream, fine,
                           static_cast<R*>(u), ep, e0, (const EpiInst*)depi);
        FH_HIP(hipGetLastError());
        timing_mark(c, 4);
        timing_mark(c, 5);
        return FH_OK;
    };
    if (!use_graph) {
        c->timing_kind = 3;
        timing_mark(c, 0);
        return run();
    }
    auto it = c->graph_cache.find(k2);
    if (it == c->graph_cache.end()) {
        GraphEntry ge;
        FH_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        fh_status s = run();
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->stream, &g);
        if (s != FH_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (e != hipSuccess || !g) {
            // capture failed (e.g. a library call that cannot be captured):
            // fall back to eager launches
            (void)hipGetLastError();
            return run();
        }
        ge.graph = g;
        FH_HIP(hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0));
        it = c->graph_cache.emplace(k2, ge).first;
    }
    FH_HIP(hipGraphLaunch(it->second.exec, c->stream));
    return FH_OK;
}

}  // namespace

// ----------------------------------------------------- shared launchers
fh_status launch_zero(fh_ctx* c, void* p, size_t bytes)
{
    const size_t n16 = (bytes + 15) / 16;
    if (n16 == 0) return FH_OK;
    const unsigned g = (unsigned)std::min<size_t>((n16 + 255) / 256, (size_t)c->cu_count * 16);
    hipLaunchKernelGGL(k_zero16, dim3(g), dim3(256), 0, c->stream, static_cast<uint4*>(p), n16);
    FH_HIP(hipGetLastError());
    return FH_OK;
}

fh_status device_bbox(fh_ctx* c, const double* x, const double* y, int64_t n, double* bb)
{
    if (n <= 0) {
        bb[0] = bb[1] = bb[2] = bb[3] = 0.0;
        return FH_OK;
    }
    const int parts = 512;
    if (!c->bbox_dev) {
        void* p = nullptr;
        FH_TRY(dev_alloc(c, sizeof(double) * (5 * parts + 8), &p));
        c->bbox_dev = static_cast<double*>(p);
    }
    if (!c->bbox_host) {
        void* h = nullptr;
        FH_HIP(hipHostMalloc(&h, sizeof(double) * 8, 0));
        c->bbox_host = static_cast<double*>(h);
    }
    double* dv = c->bbox_dev;
    double* hv = c->bbox_host;
    const unsigned g = (unsigned)std::min<int64_t>(parts, (n + 255) / 256);
    hipLaunchKernelGGL(k_bbox_partial, dim3(g), dim3(256), 0, c->stream, x, y, n, dv);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(256), 0, c->stream, dv, (int)g, dv + 5 * parts);
    FH_HIP(hipGetLastError());
    FH_HIP(hipMemcpyAsync(hv, dv + 5 * parts, sizeof(double) * 5, hipMemcpyDeviceToHost, c->stream));
    FH_HIP(hipStreamSynchronize(c->stream));
    for (int q = 0; q < 4; ++q) bb[q] = hv[q];
    FH_ARG(hv[4] == 0.0, FH_ERR_NONFINITE, "non-finite coordinate among %lld points", (long long)n);
    return FH_OK;
}

}  // namespace fh

using namespace fh;

extern "C" {

fh_status fh_field_grid(fh_ctx* c, const fh_quad* q, double lambda, double z, int32_t n1, int32_t n2, double h1,
                        double h2, double xc, double yc, int32_t occulter, void* u, fh_memspace mem)
{
    try {
        FH_ARG(c && q && u, FH_ERR_INVALID_ARG, "NULL argument");
        FH_ARG(q->ctx == c, FH_ERR_INVALID_ARG, "quadrature belongs to another context");
        FH_ARG(mem == FH_MEM_HOST || mem == FH_MEM_DEVICE, FH_ERR_INVALID_ARG, "bad memspace");
        FH_TRY(check_lz(lambda, z));
        FH_TRY(check_grid(n1, n2, h1, h2, xc, yc));
        FH_ARG(q->N < ((int64_t)1 << 31), FH_ERR_UNSUPPORTED, "at most 2^31 - 1 nodes per call");
        FH_HIP(hipSetDevice(c->device));
        if (c->prec == FH_FP64)
            return field_grid_impl<double>(c, q, lambda, z, n1, n2, h1, h2, xc, yc, occulter, u, mem);
        return field_grid_impl<float>(c, q, lambda, z, n1, n2, h1, h2, xc, yc, occulter, u, mem);
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_field_points(fh_ctx* c, const fh_quad* q, double lambda, double z, int64_t M, const double* xi,
                          const double* eta, int32_t occulter, void* u, fh_memspace mem)
{
    try {
        FH_ARG(c && q, FH_ERR_INVALID_ARG, "NULL argument");
        FH_ARG(q->ctx == c, FH_ERR_INVALID_ARG, "quadrature belongs to another context");
        FH_ARG(M >= 0, FH_ERR_INVALID_ARG, "M must be >= 0");
        FH_ARG(M == 0 || (xi && eta && u), FH_ERR_INVALID_ARG, "NULL target or output array");
        FH_ARG(mem == FH_MEM_HOST || mem == FH_MEM_DEVICE, FH_ERR_INVALID_ARG, "bad memspace");
        FH_TRY(check_lz(lambda, z));
        FH_ARG(q->N < ((int64_t)1 << 31), FH_ERR_UNSUPPORTED, "at most 2^31 - 1 nodes per call");
        FH_HIP(hipSetDevice(c->device));
        if (c->prec == FH_FP64)
            return field_points_impl<double>(c, q, lambda, z, M, xi, eta, occulter, u, mem);
        return field_points_impl<float>(c, q, lambda, z, M, xi, eta, occulter, u, mem);
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_field_grid_batch(fh_ctx* c, int32_t B, const fh_quad* const* q, const double* lambda,
                              const double* z, int32_t n1, int32_t n2, double h1, double h2, double xc, double yc,
                              const int32_t* occulter, void* u)
{
    try {
        FH_ARG(c && q && lambda && z && occulter && u, FH_ERR_INVALID_ARG, "NULL argument");
        FH_ARG(B >= 1, FH_ERR_INVALID_ARG, "B must be >= 1");
        FH_TRY(check_grid(n1, n2, h1, h2, xc, yc));
        for (int b = 0; b < B; ++b) {
            FH_ARG(q[b] && q[b]->ctx == c, FH_ERR_INVALID_ARG, "quadrature %d NULL or from another context", b);
            FH_TRY(check_lz(lambda[b], z[b]));
        }
        FH_HIP(hipSetDevice(c->device));
        if (c->prec == FH_FP64)
            return field_grid_batch_impl<double>(c, B, q, lambda, z, n1, n2, h1, h2, xc, yc, occulter, u);
        return field_grid_batch_impl<float>(c, B, q, lambda, z, n1, n2, h1, h2, xc, yc, occulter, u);
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

}  // extern "C"

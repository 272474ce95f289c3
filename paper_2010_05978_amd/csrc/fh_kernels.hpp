// fh_kernels.hpp -- device kernels and host launch helpers shared by the
// forward field path (fh_field.hip) and its adjoint (fh_adjoint.hip).
//
// Binning: counting sort of nodes into T x T fine-grid tiles.  Spread: the
// exponential-of-semicircle (ES) kernel into a (T+W-1)^2 LDS tile per work
// item, written to one slot per work item.  Reduce: every fine-grid cell sums
// the slots that cover it.  Type-1 finish: transpose/pad between the two FFT
// passes and the deconvolving epilogue.  Type-3 finish: precorrection and
// interpolation.  Plus bounding boxes and fills.
#pragma once
#include <algorithm>
#include <cstring>

#include "fh_common.hpp"
#include "fh_fft.hpp"

namespace fh {
namespace {

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)std::max<int64_t>(1, (n + bs - 1) / bs); }

template <class R> struct V2;
template <> struct V2<float> { using T = float2; };
template <> struct V2<double> { using T = double2; };

constexpr int kMaxSubPerTile = 2048;  // work items per tile before items grow
constexpr int kMergeG = 16;           // slots summed per merge group
constexpr int kMergeLevels = 2;       // 16 * 16 * 16 >= kMaxSubPerTile
constexpr size_t kLdsBudget = 64 * 1024;
constexpr size_t kCuLds = 160 * 1024;  // LDS per CU

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

// Instance of every kChunk-th node: chunk[c] = instance of node
// min(c kChunk, Ntot - 1), for c = 0 .. ceil(Ntot / kChunk), written once per
// call by k_chunk_inst.  A block of consecutive nodes [j0, j1] with j0 a
// multiple of kChunk reads the instance of j0 and an upper bound, the
// instance of node j1 + 1 (or of the last node): when the two agree every
// node of the block lies in that instance, else a node searches between them.
constexpr int kChunk = 256;

__global__ void k_chunk_inst(const InstParams* __restrict__ t, int n, int64_t Ntot, int* __restrict__ chunk)
{
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t nc = (Ntot + kChunk - 1) / kChunk;
    if (c > nc) return;
    chunk[c] = find_inst(t, n, min(c * kChunk, Ntot - 1));
}

__device__ __forceinline__ int node_inst(const InstParams* t, int64_t j, int2 ab)
{
    if (ab.x == ab.y) return __builtin_amdgcn_readfirstlane(ab.x);
    int lo = ab.x, hi = ab.y;
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

// Node -> (x cell, y cell, offsets); y is relative to the instance's window.
__device__ __forceinline__ bool node_cell(const InstParams& ip, const GridGeom& gg, double x, double y, int& l1,
                                          int& l2, double& d1, double& d2)
{
    bool ok1, ok2;
    cell_of((x - ip.cx) * ip.s1, gg.nf1, gg.W, l1, d1, ok1);
    cell_of((y - ip.cy) * ip.s2 - (double)ip.sh2, gg.nf2, gg.W, l2, d2, ok2);
    bool ok = ok1 && ok2;
    if (!gg.wrap_y && l2 > gg.rows - gg.W) ok = false;  // outside the window
    if (!ok) {
        l1 = 0;
        l2 = 0;
    }
    return ok;
}

// ES kernel values k[a] = phi((d + a) 2/W), a < W, for the first-cell offset
// d in [-W/2, -W/2 + 1): by the polynomial table when there is one (uniform
// coefficients, W independent Horner chains), else directly.
template <class R, int W>
__device__ __forceinline__ void es_weights(R d, R beta, const R* __restrict__ poly, R* k)
{
    if (poly) {
        constexpr int NP = poly_np(W);
        const R t = R(2) * d + R(W - 1);
#pragma unroll
        for (int a = 0; a < W; ++a) k[a] = poly[a];
#pragma unroll
        for (int j = 1; j < NP; ++j) {
#pragma unroll
            for (int a = 0; a < W; ++a) k[a] = k[a] * t + poly[j * W + a];
        }
        return;
    }
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

// One kernel value phi((d + a) 2/W) (a may vary across lanes).
template <class R, int W>
__device__ __forceinline__ R es_one(R d, int a, R beta, const R* __restrict__ poly)
{
    if (poly) {
        constexpr int NP = poly_np(W);
        const R t = R(2) * d + R(W - 1);
        R v = poly[a];
#pragma unroll
        for (int j = 1; j < NP; ++j) v = v * t + poly[j * W + a];
        return v;
    }
    const R z = (d + R(a)) * (R(2) / R(W));
    const R q = R(1) - z * z;
    if constexpr (sizeof(R) == 4)
        return __expf(beta * (__fsqrt_rn(fmaxf(q, 0.0f)) - 1.0f));
    else
        return exp(beta * (sqrt(fmax(q, 0.0)) - 1.0));
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
// Block-aggregated counting: the wavefronts of a block first combine their
// per-tile counts in a small LDS hash table (open addressing), then one
// global atomic per distinct tile of the block reserves the block's
// positions; a group whose tile finds the table full takes one global atomic
// of its own.  When every node of a rule falls in a couple of tiles (a
// starshade seen on a coarse pupil grid), this turns one same-address atomic
// chain per wavefront into one per block.  (A table of twice the block's
// nodes, which never fills, measured no faster on the batch's 6-cell tiles:
// 0.68 against 0.63 ms.)  A batch's nodes spread over many tiles and the
// kernel waits on memory: 256-thread blocks, four times as many per CU,
// hide more of it (whole binning 1.50 against 1.57 ms on the 256-shape
// batch), and four nodes per thread more still (1.44 ms; mixed 1.23 ->
// 1.11 ms).
constexpr int kBinBlock = 1024;      // one rule: its nodes may crowd a few tiles
constexpr int kBinBlockBatch = 256;  // a batch: spread over many tiles, latency bound
constexpr int kBinNodesBatch = 4;    // nodes per thread in a batch
constexpr int kBinKeyBits = 7;       // hash table of one rule's 1024-node block
constexpr int kBinKeyBitsBatch = 9;  // and of a batch's 1024-node block
constexpr int kBinProbes = 16;       // slots a lookup tries before its global atomic

// A thread takes NPT nodes, BS apart (each load coalesced): the block's chain
// of latencies (instance lookup, node loads, the table, the global atomics)
// is paid once for BS NPT nodes.  A lookup tries at most kBinProbes slots; a
// group whose tile finds none takes a global atomic of its own.
template <int BS, int NPT, int KB>
__global__ void __launch_bounds__(BS) k_bin_count(InstParams p0, const InstParams* __restrict__ table,
                                                  const int* __restrict__ chunk, int64_t Ntot, GridGeom gg,
                                                  int* __restrict__ cnt, int* __restrict__ rank,
                                                  uint32_t* __restrict__ key, int* __restrict__ vals)
{
    constexpr int NK = 1 << KB;
    static_assert((BS * NPT) % kChunk == 0, "a block starts at a chunk");
    __shared__ int s_key[NK];
    __shared__ int s_cnt[NK];
    __shared__ int s_base[NK];
    for (int e = threadIdx.x; e < NK; e += BS) {
        s_key[e] = -1;
        s_cnt[e] = 0;
    }
    const int64_t j0 = blockIdx.x * (int64_t)(BS * NPT);
    int2 ib = make_int2(0, 0);
    if (table) {
        const int64_t j1 = min(j0 + (int64_t)(BS * NPT), Ntot) - 1;
        ib = make_int2(chunk[j0 / kChunk], chunk[(j1 + kChunk) / kChunk]);
    }
    __syncthreads();
    const int lane = (int)__lane_id();
    int tile[NPT];
    bool valid[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int64_t j = j0 + (int64_t)k * BS + threadIdx.x;
        valid[k] = j < Ntot;
        tile[k] = 0;
        if (valid[k]) {
            const InstParams ip = table ? table[node_inst(table, j, ib)] : p0;
            const int64_t jj = j - ip.node_off;
            int l1, l2;
            double d1, d2;
            node_cell(ip, gg, ip.x[jj], ip.y[jj], l1, l2, d1, d2);
            tile[k] = ip.tile_off + (l2 / gg.T) * gg.ntx + (l1 / gg.T);
            if (key) {
                key[j] = (uint32_t)tile[k];
                vals[j] = (int)j;
            }
        }
    }
    uint64_t mine[NPT];
    int leader[NPT], slot[NPT], off[NPT], gbase[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        // groups of lanes with one tile; the lowest lane leads each group
        uint64_t remaining = __ballot(valid[k]);
        mine[k] = 0;
        leader[k] = lane;
        while (remaining) {
            const int l = __ffsll((unsigned long long)remaining) - 1;
            const int lkey = __shfl(tile[k], l);
            const uint64_t same = __ballot(valid[k] && tile[k] == lkey) & remaining;
            if ((same >> lane) & 1ull) {
                mine[k] = same;
                leader[k] = l;
            }
            remaining &= ~same;
        }
        slot[k] = -1;
        off[k] = 0;
        gbase[k] = 0;
        if (valid[k] && leader[k] == lane) {
            int h = (int)(((unsigned)tile[k] * 2654435761u) >> (32 - KB));
            for (int probe = 0; probe < kBinProbes; ++probe) {
                const int prev = atomicCAS(&s_key[h], -1, tile[k]);
                if (prev == -1 || prev == tile[k]) {
                    slot[k] = h;
                    break;
                }
                h = (h + 1) & (NK - 1);
            }
            if (slot[k] >= 0)
                off[k] = atomicAdd(&s_cnt[slot[k]], __popcll(mine[k]));
            else
                gbase[k] = atomicAdd(&cnt[tile[k]], __popcll(mine[k]));
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < NK; e += BS)
        if (s_key[e] >= 0) s_base[e] = atomicAdd(&cnt[s_key[e]], s_cnt[e]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        int base = 0;
        if (valid[k] && leader[k] == lane) base = slot[k] >= 0 ? s_base[slot[k]] + off[k] : gbase[k];
        base = __shfl(base, leader[k]);
        if (valid[k]) rank[j0 + (int64_t)k * BS + threadIdx.x] = base + __popcll(mine[k] & ((1ull << lane) - 1ull));
    }
}

// Points per work item of a tile holding c points: at least P, and large
// enough that the tile makes at most kMaxSubPerTile items, so a crowded tile
// is spread by many CUs while its slots stay few enough to merge.
__host__ __device__ __forceinline__ int tile_item_points(int c, int P)
{
    return max(P, (c + kMaxSubPerTile - 1) / kMaxSubPerTile);
}

// Exclusive scan of tile counts -> tile offsets (points) and, per tile, the
// first work item and the item count; the items themselves are written by
// k_bin_place.  Blocks of 1024 threads take 4096 consecutive tiles (4 per
// thread); with more than one block, k_scan_sums first totals every block
// and each block of k_scan_tiles adds the totals of the blocks before it.
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 4;
constexpr int kScanChunk = kScanThreads * kScanPer;

// Inclusive scan of (a, b) over a block of 1024 threads (wavefront shuffles,
// then the 16 wavefront totals); tot receives the block totals.
__device__ __forceinline__ void block_scan2(int& a, int& b, int* wa, int* wb, int& ta, int& tb)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int va = __shfl_up(a, o), vb = __shfl_up(b, o);
        if (lane >= o) {
            a += va;
            b += vb;
        }
    }
    if (lane == 63) {
        wa[wv] = a;
        wb[wv] = b;
    }
    __syncthreads();
    if (wv == 0) {
        int xa = lane < 16 ? wa[lane] : 0, xb = lane < 16 ? wb[lane] : 0;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            const int va = __shfl_up(xa, o), vb = __shfl_up(xb, o);
            if (lane >= o) {
                xa += va;
                xb += vb;
            }
        }
        if (lane < 16) {
            wa[lane] = xa;
            wb[lane] = xb;
        }
    }
    __syncthreads();
    if (wv > 0) {
        a += wa[wv - 1];
        b += wb[wv - 1];
    }
    ta = wa[15];
    tb = wb[15];
}

__device__ __forceinline__ int tile_items(int c, int P)
{
    return (c + tile_item_points(c, P) - 1) / tile_item_points(c, P);
}

__global__ void __launch_bounds__(kScanThreads) k_scan_sums(const int* __restrict__ cnt, int ntiles, int P,
                                                            int* __restrict__ bsum)
{
    __shared__ int wa[16], wb[16];
    const int t0 = blockIdx.x * kScanChunk + threadIdx.x * kScanPer;
    int a = 0, b = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const int c = t0 + k < ntiles ? cnt[t0 + k] : 0;
        a += c;
        b += tile_items(c, P);
    }
    int ta, tb;
    block_scan2(a, b, wa, wb, ta, tb);
    if (threadIdx.x == 0) {
        bsum[2 * blockIdx.x] = ta;
        bsum[2 * blockIdx.x + 1] = tb;
    }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(const int* __restrict__ cnt, int ntiles, int P,
                                                             const int* __restrict__ bsum,
                                                             int* __restrict__ off, int* __restrict__ tsub,
                                                             int* __restrict__ nsub_out, int* __restrict__ zero_out)
{
    // the counter of the tile reduce's list starts at zero
    if (zero_out && blockIdx.x == 0 && threadIdx.x == 0) *zero_out = 0;
    __shared__ int wa[16], wb[16];
    // totals of the blocks before this one
    int base_a = 0, base_b = 0;
    if (blockIdx.x > 0) {
        int sa = 0, sb = 0;
        for (int k = threadIdx.x; k < (int)blockIdx.x; k += kScanThreads) {
            sa += bsum[2 * k];
            sb += bsum[2 * k + 1];
        }
        block_scan2(sa, sb, wa, wb, base_a, base_b);
        __syncthreads();
    }
    const int t0 = blockIdx.x * kScanChunk + threadIdx.x * kScanPer;
    int c[kScanPer];
    int a = 0, b = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        c[k] = t0 + k < ntiles ? cnt[t0 + k] : 0;
        a += c[k];
        b += tile_items(c[k], P);
    }
    int ia = a, ib = b, ta, tb;
    block_scan2(ia, ib, wa, wb, ta, tb);
    int ea = ia - a + base_a, eb = ib - b + base_b;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (t0 + k >= ntiles) break;
        const int ns = tile_items(c[k], P);
        off[t0 + k] = ea;
        tsub[2 * (t0 + k)] = eb;
        tsub[2 * (t0 + k) + 1] = ns;
        ea += c[k];
        eb += ns;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *nsub_out = base_b + tb;
}

// Stable binning: after the sort by tile (ties in node order), the node at
// sorted position pos ranks pos - off[tile] within its tile.
__global__ void k_rank_sorted(const uint32_t* __restrict__ key_sorted, const int* __restrict__ vals_sorted,
                              int64_t Ntot, const int* __restrict__ off, int* __restrict__ rank)
{
    const int64_t pos = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (pos >= Ntot) return;
    rank[vals_sorted[pos]] = (int)(pos - off[key_sorted[pos]]);
}

// Strength (FP64 phase in turns, reduced, times the node's source term when
// the rule has one), stencil offsets, and the sorted position of each node.
// A thread takes kPlaceNodes nodes, 256 apart: first every node's loads and
// strength, then its tile's offset and count, then the stores, so that each
// round of memory latency covers all of them.  The register allocator is
// held to five waves per SIMD (93 registers in FP64 instead of 101 and four
// waves: FP64 binning 1.33 -> 1.30 ms on the batch).
constexpr int kPlaceNodes = 4;

template <class R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) k_bin_place(InstParams p0, const InstParams* __restrict__ table,
                                                   const int* __restrict__ chunk, int64_t Ntot, GridGeom gg,
                                                   const int* __restrict__ cnt, const int* __restrict__ off,
                                                   const int* __restrict__ tsub, const int* __restrict__ rank,
                                                   uint32_t* __restrict__ cell, typename V2<R>::T* __restrict__ dd,
                                                   typename V2<R>::T* __restrict__ cc, Sub* __restrict__ subs)
{
    constexpr int NPT = kPlaceNodes;
    static_assert((256 * NPT) % kChunk == 0, "a block starts at a chunk");
    const int64_t j0 = blockIdx.x * (int64_t)(256 * NPT);
    int2 ib = make_int2(0, 0);
    if (table) {
        const int64_t j1 = min(j0 + (int64_t)(256 * NPT), Ntot) - 1;
        ib = make_int2(chunk[j0 / kChunk], chunk[(j1 + kChunk) / kChunk]);
    }
    bool ok[NPT];
    int tile[NPT], rk[NPT];
    uint32_t cl[NPT];
    typename V2<R>::T dv[NPT], cv[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int64_t j = j0 + (int64_t)k * 256 + threadIdx.x;
        ok[k] = j < Ntot;
        tile[k] = 0;
        rk[k] = 0;
        cl[k] = 0;
        dv[k] = typename V2<R>::T{R(0), R(0)};
        cv[k] = typename V2<R>::T{R(0), R(0)};
        if (!ok[k]) continue;
        const InstParams ip = table ? table[node_inst(table, j, ib)] : p0;
        const int64_t jj = j - ip.node_off;
        const double x = ip.x[jj], y = ip.y[jj];
        double w = ip.w[jj];
        int l1, l2;
        double d1, d2;
        if (!node_cell(ip, gg, x, y, l1, l2, d1, d2)) w = 0.0;
        tile[k] = ip.tile_off + (l2 / gg.T) * gg.ntx + (l1 / gg.T);
        const double t = ((x * x + y * y) * ip.pa + (x * ip.px + y * ip.py)) + ip.pc;
        const double f = t - rint(t);
        double sn, cs;
        sincospi(2.0 * f, &sn, &cs);
        double cr = w * cs, ci = w * sn;
        if (ip.src && jj < ip.N) {
            // the node's source term multiplies its strength (jj < N always
            // holds: j lies in this instance's node range)
            const double sr = ip.src[2 * jj], si = ip.src[2 * jj + 1];
            const double tr = cr * sr - ci * si;
            ci = cr * si + ci * sr;
            cr = tr;
        }
        rk[k] = rank[j];
        cl[k] = (uint32_t)l1 | ((uint32_t)l2 << 16);
        dv[k].x = (R)d1;
        dv[k].y = (R)d2;
        cv[k].x = (R)cr;
        cv[k].y = (R)ci;
    }
    int o[NPT], ct[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        o[k] = ok[k] ? off[tile[k]] : 0;
        ct[k] = ok[k] ? cnt[tile[k]] : 0;
    }
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        if (!ok[k]) continue;
        const int pos = o[k] + rk[k];
        cell[pos] = cl[k];
        dd[pos] = dv[k];
        cc[pos] = cv[k];
        // the point that opens a work item of its tile writes the item
        const int Pt = tile_item_points(ct[k], gg.P);
        if (rk[k] % Pt == 0) {
            Sub it;
            it.tile = tile[k];
            it.start = pos;
            it.end = min(pos + Pt, o[k] + ct[k]);
            subs[tsub[2 * tile[k]] + rk[k] / Pt] = it;
        }
    }
}

// ----------------------------------------------------------------- spread
// Work item s covers the points [start, end) of one tile; its padded L x L
// complex tile is written to slot s (interleaved re/im).
template <class R>
__device__ __forceinline__ void tile_origin(const Sub& sb, const GridGeom& gg, int tpi, int& ox, int& oy)
{
    const int inst = sb.tile / tpi;
    const int tl = sb.tile - inst * tpi;
    const int ty = tl / gg.ntx, tx = tl - ty * gg.ntx;
    ox = tx * gg.T;
    oy = ty * gg.T;
}

// Thread per point: the threads of a block spread whole points into one
// shared LDS tile with atomics (order of same-cell additions unspecified).
template <class R, int W>
__global__ void __launch_bounds__(256) k_spread_thread(const Sub* __restrict__ subs, const int* __restrict__ nsub_ptr,
                                                       const uint32_t* __restrict__ cell,
                                                       const typename V2<R>::T* __restrict__ dd,
                                                       const typename V2<R>::T* __restrict__ cc,
                                                       typename V2<R>::T* __restrict__ slots, GridGeom gg, int tpi,
                                                       R beta, const R* __restrict__ poly)
{
    extern __shared__ unsigned char smem_raw[];
    R* sre = reinterpret_cast<R*>(smem_raw);
    const int L = gg.L, LL = L * L;
    R* sim = sre + LL;
    const int nsub = *nsub_ptr;
    for (int s = blockIdx.x; s < nsub; s += gridDim.x) {
        const Sub sb = subs[s];
        int ox, oy;
        tile_origin<R>(sb, gg, tpi, ox, oy);
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
            es_weights<R, W>(dv.x, beta, poly, k1);
            es_weights<R, W>(dv.y, beta, poly, k2);
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
        typename V2<R>::T* slot = slots + (size_t)s * LL;
        for (int e = threadIdx.x; e < LL; e += blockDim.x) {
            typename V2<R>::T v;
            v.x = sre[e];
            v.y = sim[e];
            slot[e] = v;
        }
        __syncthreads();
    }
}

// LDS order point: keeps the compiler from moving LDS accesses of this
// wavefront across it (the hardware already completes them in order).
__device__ __forceinline__ void wave_lds_order()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// NV (1 or 2) wavefronts per work item, lanes over the stencil.  Each
// wavefront owns an LDS tile (no sharing: LDS float atomics serialise badly
// when points cluster).  The block loads 64 points at a time and stages their
// 2W kernel values and strength in LDS (with two wavefronts, one evaluates
// the kernel along x and the other along y), then wavefront v walks its
// share of the 64 (a contiguous half when NV = 2) one point at a time with
// lane (a, b) holding stencil cell (a, b) (ceil(W^2/64) passes).  Consecutive
// points with the same first cell form a run (nodes in spoke order share one
// for tens of points near the origin), summed in registers and added to the
// tile once.  The tile values under a run are read when the run starts and
// the sums written back when it ends, so the read's latency is covered by
// the run's own points rather than stalling the wavefront; the LDS
// operations of one wavefront complete in issue order, so a run's read sees
// the previous run's write.  Lanes past W^2 in the last pass read and write a
// spare cell after the tile instead of branching (each lane's cell address
// is one multiply-add from the run's cell), the staged values of a
// trip of points are all read before the first is added, and points past
// the end of the item are staged as zeros, so the only branch per point is
// the (wavefront-uniform) start of a run.  The slot receives the sum of the
// NV tiles in wavefront order.  For a given order of the item's points the
// summation order is fixed (the order of points within a tile comes from the
// binning's atomic counters, so it, and the last bits of the sums, can change
// from call to call).  ATOMIC adds each run with non-returning LDS atomics
// instead of the read and write.
template <class R, int W, bool ATOMIC, int NV>
__global__ void __launch_bounds__(64 * NV) k_spread_wave(const Sub* __restrict__ subs,
                                                         const int* __restrict__ nsub_ptr,
                                                         const uint32_t* __restrict__ cell,
                                                         const typename V2<R>::T* __restrict__ dd,
                                                         const typename V2<R>::T* __restrict__ cc,
                                                         typename V2<R>::T* __restrict__ slots, GridGeom gg,
                                                         int tpi, R beta, const R* __restrict__ poly)
{
    static_assert(NV == 1 || NV == 2, "one or two wavefronts per work item");
    using C = typename V2<R>::T;
    constexpr int KS = 2 * W + 2;             // staged reals per point
    constexpr int NPASS = (W * W + 63) / 64;  // stencil passes per point
    constexpr int U = sizeof(R) == 8 ? 4 : 8; // points per trip
    constexpr int QW = 64 / NV;               // points of a batch per wavefront
    constexpr int NP = poly_np(W);        // coefficients per kernel polynomial
    constexpr int KG = 64 / W;                // lane groups evaluating the kernel
    extern __shared__ unsigned char smem_raw[];
    const int L = gg.L, LL = L * L;
    // the wavefront index, marked wavefront-uniform for the compiler (the
    // share bounds and run starts derived from it stay scalar)
    const int wv = NV == 1 ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    // LDS: each wavefront's 64 kernel arguments first (at a fixed address),
    // then NV tiles of LL cells and a spare cell each, then the staging of 64
    // points
    constexpr int TTC = (NV * 64 * (int)sizeof(R) + (int)sizeof(C) - 1) / (int)sizeof(C);
    R* tt = reinterpret_cast<R*>(smem_raw) + wv * 64;
    C* tiles = reinterpret_cast<C*>(smem_raw) + TTC;
    C* tile = tiles + wv * (LL + 1);
    R* kb = reinterpret_cast<R*>(tiles + NV * (LL + 1));
    // the block's first work item is loaded without waiting for the item
    // count (the grid never exceeds the item capacity)
    const Sub first = subs[blockIdx.x];
    const bool has_poly = poly != nullptr;
    // kernel values by lanes over the value index: lane (kg, ka), ka =
    // lane % W, keeps the coefficients of cell ka's polynomial in registers
    // (loaded once) and evaluates it at points kg, kg + KG, ... of a batch.
    // A coefficient shared by all lanes would cost a full 64-lane LDS or
    // scalar-load delivery per use; held per lane it costs nothing.
    const int ka = lane % W, kg = lane / W;
    R coef[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) coef[j] = has_poly ? poly[j * W + ka] : R(0);
    // lane (a, b) of pass p: its kernel values, and the LDS byte offset of
    // its cell for a run at tile cell c, tb[p] + tm[p] c (lanes past W^2:
    // the spare cell whatever c)
    int pa[NPASS], pb[NPASS];
    uint32_t tb[NPASS], tm[NPASS];
#pragma unroll
    for (int p = 0; p < NPASS; ++p) {
        const int e = lane + 64 * p;
        const bool valid = e < W * W;
        pa[p] = valid ? e % W : 0;
        pb[p] = valid ? e / W : 0;
        const C* cp = tile + (valid ? pb[p] * L + pa[p] : LL);
        tb[p] = (uint32_t)(reinterpret_cast<const unsigned char*>(cp) - smem_raw);
        tm[p] = valid ? (uint32_t)sizeof(C) : 0u;
    }
    // the first item's tile is cleared while the item and its count load
    for (int e = lane; e < LL; e += 64) tile[e] = C{R(0), R(0)};
    const int nsub = *nsub_ptr;
    for (int s = blockIdx.x; s < nsub; s += gridDim.x) {
        if (s != (int)blockIdx.x)
            for (int e = lane; e < LL; e += 64) tile[e] = C{R(0), R(0)};
        const Sub sb = s == (int)blockIdx.x ? first : subs[s];
        int ox, oy;
        tile_origin<R>(sb, gg, tpi, ox, oy);
        const uint32_t org = (uint32_t)ox | ((uint32_t)oy << 16);
        // the run before the first point: cell 0 with zero sums (its write
        // stores zeros over zeros)
        int cur = 0;
        R accr[NPASS], acci[NPASS];
        C bs[NPASS];  // tile values under the current run
#pragma unroll
        for (int pp = 0; pp < NPASS; ++pp) {
            accr[pp] = acci[pp] = R(0);
            bs[pp] = C{R(0), R(0)};
        }
        for (int base = sb.start; base < sb.end; base += 64) {
            const int p = base + lane;
            const bool live = p < sb.end;
            int cl = 0;
            R* kp = kb + lane * KS;
            // points past the item stage zeros (they add exact zeros)
            C dv{R(0), R(0)}, cv{R(0), R(0)};
            if (live) {
                // tile-relative first cell as an LDS index (x, y < T)
                const uint32_t rel = cell[p] - org;
                cl = (int)(rel >> 16) * L + (int)(rel & 0xffffu);
                dv = dd[p];
                // the strength is loaded with the offsets, not after the
                // kernel values (its latency would add to theirs)
                if (wv == NV - 1) cv = cc[p];
            }
            if (wv == NV - 1) {
                kp[2 * W] = cv.x;
                kp[2 * W + 1] = cv.y;
            }
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                if (NV == 2 && d != wv) continue;
                const R off = d == 0 ? dv.x : dv.y;
                if (has_poly) {
                    // the batch's polynomial arguments (es_weights' t), then
                    // the evaluations (es_weights' Horner steps, in order)
                    tt[lane] = R(2) * off + R(W - 1);
                    wave_lds_order();
#pragma unroll
                    for (int r = 0; r < (64 + KG - 1) / KG; ++r) {
                        const int q = r * KG + kg;
                        if (kg < KG && q < 64) {
                            const R t = tt[q];
                            R k = coef[0];
#pragma unroll
                            for (int j = 1; j < NP; ++j) k = k * t + coef[j];
                            kb[q * KS + d * W + ka] = base + q < sb.end ? k : R(0);
                        }
                    }
                    // tt is rewritten for the next dimension or batch
                    wave_lds_order();
                } else {
                    R k[W];
                    es_weights<R, W>(off, beta, nullptr, k);
#pragma unroll
                    for (int a = 0; a < W; ++a) kp[d * W + a] = live ? k[a] : R(0);
                }
            }
            __syncthreads();
            const int np = min(64, sb.end - base);
            const int qs = wv * QW, qe = min(np, qs + QW);
            for (int q0 = qs; q0 < qe; q0 += U) {
                // all LDS reads of the trip first (fixed offsets from one base)
                R ka[U][NPASS], kc[U][NPASS], vr[U], vi[U];
                int cq[U];
                const R* kt = kb + q0 * KS;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    cq[u] = lane_val(cl, q0 + u);
                    const R* kq = kt + u * KS;
#pragma unroll
                    for (int pp = 0; pp < NPASS; ++pp) {
                        ka[u][pp] = kq[pa[pp]];
                        kc[u][pp] = kq[W + pb[pp]];
                    }
                    vr[u] = kq[2 * W];
                    vi[u] = kq[2 * W + 1];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    // points of the trip past the wavefront's share add
                    // zeros to the current run (they were staged as zeros)
                    // or are never reached (a share is a whole number of
                    // trips); neither starts a run
                    const int c = q0 + u < qe ? cq[u] : cur;
                    if (c != cur) {
                        // the sums of the run that ends
#pragma unroll
                        for (int pp = 0; pp < NPASS; ++pp) {
                            C* e = reinterpret_cast<C*>(smem_raw + (tb[pp] + tm[pp] * (uint32_t)cur));
                            if constexpr (ATOMIC) {
                                // no return value: the wavefront does not wait for the LDS
                                atomicAdd(&e->x, accr[pp]);
                                atomicAdd(&e->y, acci[pp]);
                            } else {
                                *e = C{bs[pp].x + accr[pp], bs[pp].y + acci[pp]};
                            }
                            accr[pp] = acci[pp] = R(0);
                        }
                        // every pass's write precedes the new run's reads:
                        // the two runs' stencils may overlap across passes,
                        // and another lane may read a cell this lane wrote
                        // (the order point keeps the compiler from moving
                        // those reads above the writes)
                        if constexpr (!ATOMIC) {
                            wave_lds_order();
#pragma unroll
                            for (int pp = 0; pp < NPASS; ++pp)
                                bs[pp] = *reinterpret_cast<const C*>(smem_raw + (tb[pp] + tm[pp] * (uint32_t)c));
                        }
                        cur = c;
                    }
#pragma unroll
                    for (int pp = 0; pp < NPASS; ++pp) {
                        const R kv = ka[u][pp] * kc[u][pp];
                        accr[pp] += vr[u] * kv;
                        acci[pp] += vi[u] * kv;
                    }
                }
            }
            // the next batch rewrites the staging
            __syncthreads();
        }
#pragma unroll
        for (int pp = 0; pp < NPASS; ++pp) {
            C* e = reinterpret_cast<C*>(smem_raw + (tb[pp] + tm[pp] * (uint32_t)cur));
            if constexpr (ATOMIC) {
                atomicAdd(&e->x, accr[pp]);
                atomicAdd(&e->y, acci[pp]);
            } else {
                *e = C{bs[pp].x + accr[pp], bs[pp].y + acci[pp]};
            }
        }
        __syncthreads();
        C* slot = slots + (size_t)s * LL;
        for (int e = threadIdx.x; e < LL; e += 64 * NV) {
            C v = tiles[e];
            if constexpr (NV == 2) {
                const C v1 = tiles[LL + 1 + e];
                v.x += v1.x;
                v.y += v1.y;
            }
            slot[e] = v;
        }
        // the tiles are cleared for the next item
        __syncthreads();
    }
}

// Register-tile spread (method 4), for tiles of TT = 8 or 16 cells.  A block
// of NW wavefronts takes one work item at a time; each wavefront keeps a
// padded L x L tile (L = TT + W - 1) in registers, lane (x, bank) owning
// column x of the rows [bank RB, bank RB + RB).  The block stages PC points
// at a time in LDS (kernel values along x, kernel values along y inside a
// zero border wide enough for every row a lane owns, strength and first
// cell), and wavefront v adds points v, v + NW, ...: every lane adds
// strength x kx[x - cx] x ky[y - cy] to its RB cells, with reads at fixed
// offsets from one base and no branches (lanes outside the stencil add
// zeros).  At the end of the item the NW tiles are summed through LDS in a
// fixed order into the item's slot.
template <int TT, int W>
struct RegTile {
    static constexpr int L = TT + W - 1;
    static constexpr int NB = 64 / L;                // banks (rows split over NB lane groups)
    static constexpr int RB = (L + NB - 1) / NB;     // rows per bank
    static constexpr int PADL = TT - 1;              // y - cy >= -(TT - 1)
    static constexpr int KYP = PADL + NB * RB;       // padded y values per point
    static constexpr int PC = 32;                    // points staged at a time
    static constexpr int NW = 4;                     // wavefronts per block
};

template <class R, int TT, int W>
constexpr size_t reg_spread_lds()
{
    using RT = RegTile<TT, W>;
    return sizeof(R) * ((size_t)RT::PC * (W + RT::KYP + 2)) + 2 * sizeof(int) * RT::PC +
           2 * sizeof(R) * (size_t)RT::NW * RT::L * RT::L;
}

template <class R, int W, int TT>
__global__ void __launch_bounds__(256) k_spread_reg(const Sub* __restrict__ subs, const int* __restrict__ nsub_ptr,
                                                    const uint32_t* __restrict__ cell,
                                                    const typename V2<R>::T* __restrict__ dd,
                                                    const typename V2<R>::T* __restrict__ cc,
                                                    typename V2<R>::T* __restrict__ slots, GridGeom gg, int tpi,
                                                    R beta, const R* __restrict__ poly)
{
    using C = typename V2<R>::T;
    using RT = RegTile<TT, W>;
    constexpr int L = RT::L, NB = RT::NB, RB = RT::RB, KYP = RT::KYP, PC = RT::PC, NW = RT::NW, LL = L * L;
    static_assert(NB >= 1, "tile too wide for one wavefront");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R* skx = reinterpret_cast<R*>(smem_raw);
    R* sky = skx + PC * W;
    R* scr = sky + PC * KYP;
    R* sci = scr + PC;
    R* stile = sci + PC;                            // NW tiles, planar re/im
    int* scx = reinterpret_cast<int*>(stile + 2 * NW * LL);
    int* scy = scx + PC;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int bank = lane / L;
    const int x = lane - bank * L;                // column (lanes past NB L repeat bank NB - 1's rows)
    const int y0 = min(bank, NB - 1) * RB;
    // the y border stays zero; only the W middle values of a point change
    for (int e = tid; e < PC * KYP; e += 64 * NW) sky[e] = R(0);
    const int nsub = *nsub_ptr;
    for (int s = blockIdx.x; s < nsub; s += gridDim.x) {
        const Sub sb = subs[s];
        int ox, oy;
        tile_origin<R>(sb, gg, tpi, ox, oy);
        const uint32_t org = (uint32_t)ox | ((uint32_t)oy << 16);
        R accr[RB], acci[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) accr[j] = acci[j] = R(0);
        for (int base = sb.start; base < sb.end; base += PC) {
            const int np = min(PC, sb.end - base);
            __syncthreads();
            if (tid < np) {
                const int p = base + tid;
                const uint32_t rel = cell[p] - org;  // tile-relative first cell (x, y < TT)
                const C dv = dd[p];
                const C cv = cc[p];
                R k[W];
                es_weights<R, W>(dv.x, beta, poly, k);
#pragma unroll
                for (int a = 0; a < W; ++a) skx[tid * W + a] = k[a];
                es_weights<R, W>(dv.y, beta, poly, k);
#pragma unroll
                for (int b = 0; b < W; ++b) sky[tid * KYP + RT::PADL + b] = k[b];
                scr[tid] = cv.x;
                sci[tid] = cv.y;
                scx[tid] = (int)(rel & 0xffffu);
                scy[tid] = (int)(rel >> 16);
            }
            __syncthreads();
            for (int q = wv; q < np; q += NW) {
                const int ax = x - scx[q];
                const bool in = (unsigned)ax < (unsigned)W;
                const R kx = skx[q * W + (in ? ax : 0)];
                const R vr = in ? scr[q] * kx : R(0);
                const R vi = in ? sci[q] * kx : R(0);
                const R* ky = sky + q * KYP + RT::PADL + y0 - scy[q];
#pragma unroll
                for (int j = 0; j < RB; ++j) {
                    const R w = ky[j];
                    accr[j] += vr * w;
                    acci[j] += vi * w;
                }
            }
            // the y values of the next chunk overwrite this chunk's
            __syncthreads();
            if (tid < np)
#pragma unroll
                for (int b = 0; b < W; ++b) sky[tid * KYP + RT::PADL + b] = R(0);
        }
        // sum the NW register tiles in wavefront order into the slot
        if (lane < NB * L) {
#pragma unroll
            for (int j = 0; j < RB; ++j)
                if (y0 + j < L) {
                    stile[wv * 2 * LL + (y0 + j) * L + x] = accr[j];
                    stile[wv * 2 * LL + LL + (y0 + j) * L + x] = acci[j];
                }
        }
        __syncthreads();
        C* slot = slots + (size_t)s * LL;
        for (int e = tid; e < LL; e += 64 * NW) {
            R vr = R(0), vi = R(0);
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                vr += stile[w * 2 * LL + e];
                vi += stile[w * 2 * LL + LL + e];
            }
            slot[e] = C{vr, vi};
        }
    }
}

// Matrix-core spread (method 5).  A work item's padded tile is a sum of
// rank-one terms, one per point p: (c_p ky_p)(kx_p)^T, with ky_p and kx_p the
// kernel values placed at the point's first cell (zero elsewhere), i.e. the
// matrix product G = A^T B over the item's points with A[p][y] = c_p
// ky_p(y - cy_p) and B[p][x] = kx_p(x - cx_p).  Each wavefront takes one item
// and holds its tile, zero-extended to (16 NB)^2 cells, in matrix-core
// accumulators: NB x NB blocks of 16 x 16, a real and an imaginary one each,
// updated four points at a time by v_mfma_{f64,f32}_16x16x4 (lane l supplies
// A[row l % 16][point l / 16] and B[point l / 16][column l % 16]).
//
// The operands are read from zero-padded rows of kx and c ky (real and
// imaginary) staged in LDS for MS points at a time, so that a lane reads its
// value with no bounds test: each point's shifted row base is staged too.  The kernel values
// are evaluated by lanes over the value index with the polynomial table (as
// the wavefront spread does), the y values multiplied by the strength there.
// A point costs the same whatever its neighbours; the wavefront spread
// instead merges runs of points that share a first cell, which wins where
// points crowd.  Points are summed in their staged order, four at a time (the
// order of a tile's points comes from the binning's atomic counters).  The
// slot receives the L x L corner of the accumulators.
template <class R> struct MfmaAcc;
template <> struct MfmaAcc<double> {
    typedef double V __attribute__((ext_vector_type(4)));
    __device__ static V mma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    // output v of lane l holds row (l / 16) + 4 v, column l % 16
    __device__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <> struct MfmaAcc<float> {
    typedef float V __attribute__((ext_vector_type(4)));
    __device__ static V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    // output v of lane l holds row 4 (l / 16) + v, column l % 16
    __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

constexpr int kMfmaWaves = 4;  // wavefronts (items) per block

// Operand rows in LDS: the x values of the MS staged points lie in one array,
// point q's W values at positions q P + T - 1 .. q P + T + W - 2 and zeros
// elsewhere; the real and imaginary y rows (times the strength) follow in two
// arrays of the same layout.  Lane i of the block b reads position
// q P + T - 1 - cx + 16 b + i, which stays inside point q's window
// [q P, q P + 16 NB + T - 2]: that window holds no other point's values when
// the period P is at least 16 NB (and the tile side L <= 16 NB).  P is odd so
// that consecutive points start in different LDS banks.
__host__ __device__ inline int mfma_period(int NB) { return 16 * NB + 1; }
__host__ __device__ inline int mfma_rows(int NB, int T, int MS) { return MS * mfma_period(NB) + T; }

// LDS bytes of one wavefront's staging of MS points: three operand arrays,
// the strengths and the polynomial arguments (2 reals each per point), and
// two row offsets per point.
__host__ __device__ inline size_t mfma_wave_lds(int NB, int T, int MS, size_t rsize)
{
    return (3 * (size_t)mfma_rows(NB, T, MS) + 4 * (size_t)MS) * rsize + 2 * (size_t)MS * sizeof(int);
}

// The register allocator is asked for eight waves per SIMD in FP32 (61
// registers; seven by default: batch spread 0.93 -> 0.88 ms) and four in
// FP64, where the mirrored-pair evaluation would otherwise take 130
// registers and three waves (2.40 -> 2.22 ms with four; five spill).
template <class R, int W, int NB, int MS>
__global__ void __launch_bounds__(64 * kMfmaWaves) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 8 : 4))) k_spread_mfma(const Sub* __restrict__ subs,
                                                                 const int* __restrict__ nsub_ptr,
                                                                 const uint32_t* __restrict__ cell,
                                                                 const typename V2<R>::T* __restrict__ dd,
                                                                 const typename V2<R>::T* __restrict__ cc,
                                                                 typename V2<R>::T* __restrict__ slots, GridGeom gg,
                                                                 int tpi, R beta, const R* __restrict__ poly)
{
    using C = typename V2<R>::T;
    using M = MfmaAcc<R>;
    using V = typename M::V;
    constexpr int NP = poly_np(W);  // coefficients per kernel polynomial
    constexpr int KG = 64 / W;          // lane groups evaluating kernel values (no table)
    constexpr int NPAIR = poly_npair(W), NE = poly_ne(W), NO = poly_no(W);
    constexpr int KGP = 64 / NPAIR;     // lane groups evaluating mirrored pairs (table)
    static_assert(W <= 16 * NB, "the padded tile must fit the blocks");
    static_assert(MS % 16 == 0 && MS <= 64, "points are staged in sixteens, one per lane at most");
    extern __shared__ unsigned char smem_raw[];
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int T = gg.T, L = gg.L;
    const int P = mfma_period(NB), AL = mfma_rows(NB, T, MS);
    unsigned char* wbase = smem_raw + (size_t)wv * mfma_wave_lds(NB, T, MS, sizeof(R));
    R* rows = reinterpret_cast<R*>(wbase);  // x values, y values (real), y values (imaginary)
    R* ctab = rows + 3 * AL;                // strengths, 2 reals per point
    R* ttab = ctab + 2 * MS;                // polynomial arguments: x of each point, then y
    int* shx = reinterpret_cast<int*>(ttab + 2 * MS);  // byte offset of q P + T - 1 - cx
    int* shy = shx + MS;                                // byte offset of q P + T - 1 - cy
    const int nsub = *nsub_ptr;
    const int k4 = lane >> 4, i16 = lane & 15;
    // With the table, lane (pg, pp), pp = lane % NPAIR, holds the even and
    // odd parts of cell pp's polynomial and evaluates cells pp and W - 1 - pp
    // at arguments pg, pg + KGP, ... (measured against a cell per lane, which
    // needs fewer registers: FP32 1.045 -> 0.93 ms, FP64 2.40 -> 2.22 ms once
    // held to four waves).  Without it, lane (kg, ka), ka = lane % W,
    // evaluates phi itself for cell ka at arguments kg, kg + KG, ...
    const bool has_poly = poly != nullptr;
    const int ka = lane % W, kg = lane / W;
    const int pp = lane % NPAIR, pg = lane / NPAIR;
    R ce[NE], co[NO];
#pragma unroll
    for (int j = 0; j < NE; ++j) ce[j] = has_poly ? poly[NP * W + j * NPAIR + pp] : R(0);
#pragma unroll
    for (int j = 0; j < NO; ++j) co[j] = has_poly ? poly[NP * W + (NE + j) * NPAIR + pp] : R(0);
    // rows start at zero; staging only ever writes their W middle positions
    for (int e = lane; e < 3 * AL; e += 64) rows[e] = R(0);
    const uint32_t lane_off = (uint32_t)(i16 * sizeof(R));
    for (int s = blockIdx.x * kMfmaWaves + wv; s < nsub; s += gridDim.x * kMfmaWaves) {
        const Sub sb = subs[s];
        int ox, oy;
        tile_origin<R>(sb, gg, tpi, ox, oy);
        const uint32_t org = (uint32_t)ox | ((uint32_t)oy << 16);
        V are[NB][NB], aim[NB][NB];
#pragma unroll
        for (int br = 0; br < NB; ++br)
#pragma unroll
            for (int bc = 0; bc < NB; ++bc) {
                are[br][bc] = V{R(0), R(0), R(0), R(0)};
                aim[br][bc] = V{R(0), R(0), R(0), R(0)};
            }
        for (int base = sb.start; base < sb.end; base += MS) {
            // stage: lane q < MS loads point base + q (zero strength past the
            // item's end: such points add nothing)
            if (lane < MS) {
                const int p = base + lane;
                C dv{R(0), R(0)}, cv{R(0), R(0)};
                int cx = 0, cy = 0;
                if (p < sb.end) {
                    const uint32_t rel = cell[p] - org;  // tile-relative first cell (x, y < T)
                    cx = (int)(rel & 0xffffu);
                    cy = (int)(rel >> 16);
                    dv = dd[p];
                    cv = cc[p];
                }
                ctab[2 * lane] = cv.x;
                ctab[2 * lane + 1] = cv.y;
                ttab[lane] = R(2) * dv.x + R(W - 1);
                ttab[MS + lane] = R(2) * dv.y + R(W - 1);
                shx[lane] = (int)(sizeof(R) * (lane * P + T - 1 - cx));
                shy[lane] = (int)(sizeof(R) * (AL + lane * P + T - 1 - cy));
            }
            wave_lds_order();
            // the kernel values: arguments 0..MS-1 are the points' x, the
            // next MS their y (times the strength)
            if (has_poly) {
#pragma unroll
                for (int r = 0; r < (2 * MS + KGP - 1) / KGP; ++r) {
                    const int qq = r * KGP + pg;
                    if (pg < KGP && qq < 2 * MS) {
                        const R t = ttab[qq], s2 = t * t;
                        R e = ce[0], o = co[0];
#pragma unroll
                        for (int j = 1; j < NE; ++j) e = e * s2 + ce[j];
#pragma unroll
                        for (int j = 1; j < NO; ++j) o = o * s2 + co[j];
                        const R lo = e + t * o, hi = e - t * o;  // cells pp and W - 1 - pp
                        const bool two = 2 * pp != W - 1;
                        const int q = qq < MS ? qq : qq - MS;
                        R* row = rows + q * P + T - 1;
                        if (qq < MS) {
                            row[pp] = lo;
                            if (two) row[W - 1 - pp] = hi;
                        } else {
                            const R cr = ctab[2 * q], ci = ctab[2 * q + 1];
                            row[AL + pp] = cr * lo;
                            row[2 * AL + pp] = ci * lo;
                            if (two) {
                                row[AL + W - 1 - pp] = cr * hi;
                                row[2 * AL + W - 1 - pp] = ci * hi;
                            }
                        }
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < (2 * MS + KG - 1) / KG; ++r) {
                    const int qq = r * KG + kg;
                    if (kg < KG && qq < 2 * MS) {
                        const R t = ttab[qq];
                        const R k = es_one<R, W>((t - R(W - 1)) * R(0.5), ka, beta, nullptr);
                        const int q = qq < MS ? qq : qq - MS;
                        R* row = rows + q * P + T - 1 + ka;
                        if (qq < MS) {
                            row[0] = k;
                        } else {
                            row[AL] = ctab[2 * q] * k;
                            row[2 * AL] = ctab[2 * q + 1] * k;
                        }
                    }
                }
            }
            wave_lds_order();
            const int np = min(MS, sb.end - base);
#pragma unroll
            for (int h = 0; h < MS / 16; ++h) {
                if (16 * h >= np) break;  // wavefront-uniform
                // four points per product, the operands of all sixteen read
                // first (points past np carry zero strength)
                R bx[4][NB], ar[4][NB], ai[4][NB];
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int q = 16 * h + 4 * g + k4;
                    const unsigned char* px = reinterpret_cast<const unsigned char*>(rows) + shx[q] + lane_off;
                    const unsigned char* py = reinterpret_cast<const unsigned char*>(rows) + shy[q] + lane_off;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        bx[g][b] = reinterpret_cast<const R*>(px)[16 * b];
                        ar[g][b] = reinterpret_cast<const R*>(py)[16 * b];
                        ai[g][b] = reinterpret_cast<const R*>(py)[16 * b + AL];
                    }
                }
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    if (16 * h + 4 * g >= np) break;  // wavefront-uniform
#pragma unroll
                    for (int br = 0; br < NB; ++br)
#pragma unroll
                        for (int bc = 0; bc < NB; ++bc) {
                            are[br][bc] = M::mma(ar[g][br], bx[g][bc], are[br][bc]);
                            aim[br][bc] = M::mma(ai[g][br], bx[g][bc], aim[br][bc]);
                        }
                }
            }
            // the next stage rewrites the staging
            wave_lds_order();
        }
        C* slot = slots + (size_t)s * L * L;
#pragma unroll
        for (int br = 0; br < NB; ++br)
#pragma unroll
            for (int bc = 0; bc < NB; ++bc)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int y = 16 * br + M::row(lane, v), x = 16 * bc + i16;
                    if (x < L && y < L) slot[y * L + x] = C{are[br][bc][v], aim[br][bc][v]};
                }
    }
}

// Points staged per wavefront at a time.
template <class R> constexpr int mfma_stage() { return 16; }

// LDS bytes of one matrix-core spread block: the staging of each wavefront.
inline size_t mfma_spread_lds(int NB, int T, size_t rsize)
{
    return (size_t)kMfmaWaves * mfma_wave_lds(NB, T, rsize == 8 ? mfma_stage<double>() : mfma_stage<float>(), rsize);
}

// ----------------------------------------------------------------- reduce
// A tile with cnt work items is merged in levels: level l sums, for every
// item r (its index within the tile) divisible by G^l, the slots r + k G^(l-1)
// (k < G, inside the tile) into slot r.  A tile takes merge_levels(cnt)
// levels, which leaves at most G heads, at stride G^levels, for the reduce.
// Groups are disjoint within a level and the order of every sum is fixed.
__host__ __device__ __forceinline__ int merge_levels(int cnt)
{
    int l = 0;
    for (int span = kMergeG; cnt > span && l < kMergeLevels; span *= kMergeG) ++l;
    return l;
}

// A block takes kMergeChunk consecutive work items at a time: a thread per
// item checks whether the item heads a group at this level (most items do
// not: only crowded tiles merge) and the block lists those in LDS; then its
// threads sum the listed groups, a thread per (group, slot element).  The
// chunk is small so that the consecutive heads of one crowded tile spread
// over many blocks.
constexpr int kMergeChunk = 32;

template <class R>
__global__ void __launch_bounds__(256) k_merge_slots(typename V2<R>::T* __restrict__ slots,
                                                     const Sub* __restrict__ subs, const int* __restrict__ nsub_ptr,
                                                     const int* __restrict__ tsub, int LL, int level)
{
    using C = typename V2<R>::T;
    __shared__ int s_item[kMergeChunk];
    __shared__ int s_nk[kMergeChunk];
    __shared__ int s_n;
    const int nsub = *nsub_ptr;
    int stride = 1;
    for (int l = 1; l < level; ++l) stride *= kMergeG;
    const int span = stride * kMergeG;
    const size_t st = (size_t)stride * LL;
    const FastDiv dLL = fast_div((unsigned)LL);
    for (int i0 = blockIdx.x * kMergeChunk; i0 < nsub; i0 += gridDim.x * kMergeChunk) {
        if (threadIdx.x == 0) s_n = 0;
        __syncthreads();
        const int i = i0 + (int)threadIdx.x;
        if (threadIdx.x < kMergeChunk && i < nsub) {
            const int t = subs[i].tile;
            const int first = tsub[2 * t], cnt = tsub[2 * t + 1];
            const int r = i - first;
            if (merge_levels(cnt) >= level && r % span == 0) {
                const int m = atomicAdd(&s_n, 1);
                s_item[m] = i;
                s_nk[m] = min(kMergeG, (cnt - r + stride - 1) / stride);
            }
        }
        __syncthreads();
        const int n = s_n;
        for (int w = threadIdx.x; w < n * LL; w += blockDim.x) {
            const int m = (int)fdiv((unsigned)w, dLL), e = w - m * LL;
            const int nk = s_nk[m];
            C* sp = slots + (size_t)s_item[m] * LL + e;
            // all loads of the group in flight at once, then summed in order
            C v[kMergeG];
#pragma unroll
            for (int k = 0; k < kMergeG; ++k) v[k] = k < nk ? sp[k * st] : C{R(0), R(0)};
            C acc = v[0];
#pragma unroll
            for (int k = 1; k < kMergeG; ++k) {
                acc.x += v[k].x;
                acc.y += v[k].y;
            }
            sp[0] = acc;
        }
        __syncthreads();
    }
}

// Fine-grid cell (gx, gy) of tile (tx, ty) is covered by the padded tiles of
// (tx - dx, ty - dy) for every dx, dy >= 0 with i + dx T < L and j + dy T < L
// (periodic in x, and in y when the window is the whole grid; a padded tile
// reaches ceil((W-1)/T) tiles on; one reached through the wrap of a period
// whose last tile is partial sits padx (pady) cells closer).  Each thread sums, in item order, the
// merged slots of those tiles at its cell and writes the cell: every cell of
// the held rows is written, zeros included.
// The (first, count) pairs of all covering tiles are loaded at once, then
// the first kRedU merged slots of every covering tile, and only then summed
// (covering tiles in (dy, dx) order, slots in item order; any further slots
// of a tile follow its first kRedU), so a tile costs two memory latencies
// rather than two per covering tile.  REACH = (L - 1)/T; KC cells per thread.
constexpr int kRedU = 2;

// Rows held for instance b and its first row in F: its own window when the
// batch holds ragged windows (rwin), else gg.rows each, one after another.
__device__ __forceinline__ int2 inst_rows(const int2* __restrict__ rwin, const GridGeom& gg, int b)
{
    return rwin ? rwin[b] : make_int2(gg.rows, b * gg.rows);
}

template <class R, int REACH, int KC>
__global__ void __launch_bounds__(256) k_reduce_tiles(const typename V2<R>::T* __restrict__ slots,
                                                      const int* __restrict__ tsub, GridGeom gg, int tpi,
                                                      int ntiles_total, R* __restrict__ F, int* __restrict__ cnt,
                                                      const int2* __restrict__ rwin)
{
    using C = typename V2<R>::T;
    constexpr int NC = (REACH + 1) * (REACH + 1);  // covering tiles
    const int T = gg.T, TT = T * T;
    const int L = gg.L, LL = L * L;
    C* Fv = reinterpret_cast<C*>(F);
    int ci[KC], cj[KC];
    bool cv[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        const int e = threadIdx.x + k * blockDim.x;
        cv[k] = e < TT;
        ci[k] = cv[k] ? e % T : 0;
        cj[k] = cv[k] ? e / T : 0;
    }
    for (int tile = blockIdx.x; tile < ntiles_total; tile += gridDim.x) {
        // the binning counters of the call are spent: leave them at zero
        // for the next one
        if (threadIdx.x == 0) cnt[tile] = 0;
        const int b = tile / tpi, tl = tile - b * tpi;
        const int ty = tl / gg.ntx, tx = tl - ty * gg.ntx;
        // cells of this tile inside the grid (the last tile of a row or
        // column may be partial; an instance may hold fewer rows)
        const int2 rw = inst_rows(rwin, gg, b);
        const int wx = min(T, gg.nf1 - tx * T), wy = min(T, rw.x - ty * T);
        if (wy <= 0) continue;
        // covering tile i = (dy, dx): its first merged slot, slot stride
        // and number of merged slots (0 where no tile reaches), and the
        // shift of its padded cells when it wraps around the period
        int first[NC], stride[NC], heads[NC], sx[NC], sy[NC];
        bool any = false;
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const int dy = i / (REACH + 1), dx = i % (REACH + 1);
            int sty = ty - dy;
            const bool ok = sty >= 0 || gg.wrap_y;
            sy[i] = sty < 0 ? gg.pady : 0;
            if (sty < 0) sty = ((sty % gg.nty) + gg.nty) % gg.nty;
            sx[i] = tx - dx < 0 ? gg.padx : 0;
            const int stx = (((tx - dx) % gg.ntx) + gg.ntx) % gg.ntx;
            const int t = b * tpi + sty * gg.ntx + stx;
            const int n = ok ? tsub[2 * t + 1] : 0;
            first[i] = ok ? tsub[2 * t] : 0;
            int st = 1;
            for (int l = merge_levels(n); l > 0; --l) st *= kMergeG;
            stride[i] = st;
            heads[i] = (n + st - 1) / st;
            any = any || n > 0;
        }
        C* out = Fv + ((size_t)rw.y + (size_t)ty * T) * gg.nf1 + (size_t)tx * T;
        if (!any) {
            for (int e = threadIdx.x; e < TT; e += blockDim.x)
                if (e % T < wx && e / T < wy) out[(size_t)(e / T) * gg.nf1 + e % T] = C{R(0), R(0)};
            continue;
        }
        // the first kRedU slots of every covering tile at each cell
        C r[KC][NC][kRedU];
#pragma unroll
        for (int q = 0; q < KC; ++q)
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                const int dy = i / (REACH + 1), dx = i % (REACH + 1);
                const int lx = ci[q] + dx * T - sx[i], ly = cj[q] + dy * T - sy[i];
                const bool in = cv[q] && lx < L && ly < L;
                const C* sp = slots + (size_t)first[i] * LL + (in ? ly * L + lx : 0);
#pragma unroll
                for (int u = 0; u < kRedU; ++u)
                    r[q][i][u] = in && u < heads[i] ? sp[(size_t)u * stride[i] * LL] : C{R(0), R(0)};
            }
#pragma unroll
        for (int q = 0; q < KC; ++q) {
            R ar = R(0), ai = R(0);
#pragma unroll
            for (int i = 0; i < NC; ++i) {
#pragma unroll
                for (int u = 0; u < kRedU; ++u) {
                    ar += r[q][i][u].x;
                    ai += r[q][i][u].y;
                }
                if (heads[i] > kRedU) {
                    // merged slots past the first kRedU (clustered tiles)
                    const int dy = i / (REACH + 1), dx = i % (REACH + 1);
                    const int lx = ci[q] + dx * T - sx[i], ly = cj[q] + dy * T - sy[i];
                    const bool in = cv[q] && lx < L && ly < L;
                    const size_t st = (size_t)stride[i] * LL;
                    const C* sp = slots + (size_t)first[i] * LL + (in ? ly * L + lx : 0);
                    for (int k = kRedU; k < heads[i]; k += 4) {
                        C v[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) v[u] = in && k + u < heads[i] ? sp[(k + u) * st] : C{R(0), R(0)};
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            ar += v[u].x;
                            ai += v[u].y;
                        }
                    }
                }
            }
            if (cv[q] && ci[q] < wx && cj[q] < wy) out[(size_t)cj[q] * gg.nf1 + ci[q]] = C{ar, ai};
        }
    }
}

// Cell-parallel form of the tile reduce, for small tiles (whose blocks of one
// tile would leave most lanes idle): a thread per fine-grid cell, 64 x 4
// cells per block (x fastest, so the stores of a row are contiguous), grid z
// the instance.  A cell of a tile that no padded tile reaches is zero;
// otherwise the thread finds the covering tiles and sums their merged slots
// in the same order as k_reduce_tiles: covering tiles in (dy, dx) order,
// slots in item order.
// Tiles that some padded tile reaches (any of their covering tiles holds work
// items), appended to a list: most of a batch's fine grids are empty, and the
// list reduce visits only these.  One atomic per wavefront reserves its
// entries (the list's order does not matter: every cell is summed by one
// thread in a fixed order).  Also leaves the binning counters at zero for
// the next call.
template <int REACH>
__global__ void __launch_bounds__(256) k_tile_active(const int* __restrict__ tsub, GridGeom gg, int tpi,
                                                     int ntiles_total, int* __restrict__ list,
                                                     int* __restrict__ nlist, int* __restrict__ cnt)
{
    const int tile = blockIdx.x * blockDim.x + threadIdx.x;
    int any = 0;
    if (tile < ntiles_total) {
        cnt[tile] = 0;
        const int b = tile / tpi, tl = tile - b * tpi;
        const int ty = tl / gg.ntx, tx = tl - ty * gg.ntx;
#pragma unroll
        for (int i = 0; i < (REACH + 1) * (REACH + 1); ++i) {
            const int dy = i / (REACH + 1), dx = i % (REACH + 1);
            int sty = ty - dy;
            if (sty < 0 && !gg.wrap_y) continue;
            if (sty < 0) sty = ((sty % gg.nty) + gg.nty) % gg.nty;
            const int stx = (((tx - dx) % gg.ntx) + gg.ntx) % gg.ntx;
            any |= tsub[2 * (b * tpi + sty * gg.ntx + stx) + 1];
        }
    }
    const uint64_t m = __ballot(any != 0);
    if (!m) return;
    const int lane = (int)__lane_id();
    const int lead = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane == lead) base = atomicAdd(nlist, __popcll(m));
    base = __shfl(base, lead);
    if (any) list[base + __popcll(m & ((1ull << lane) - 1ull))] = tile;
}

// Merged slots of a tile with n work items: (first item, number of merged
// slots, item stride between them).
__device__ __forceinline__ int4 tile_heads(int first, int n)
{
    int st = 1;
    for (int l = merge_levels(n); l > 0; --l) st *= kMergeG;
    return make_int4(first, (n + st - 1) / st, st, 0);
}

// Sum at cell (ci, cj) of tile (tx, ty) of one instance: the merged slots of
// the tiles whose padded tiles cover it, covering tiles in (dy, dx) order,
// slots in item order (the order of k_reduce_tiles).  head(ty', tx') gives
// tile_heads of tile (tx', ty'), where tx' is already wrapped into [0, ntx)
// and ty' may be negative (wrapped by head, when the grid wraps in y).
template <class R, int REACH, int U = kRedU, class Head>
__device__ __forceinline__ typename V2<R>::T reduce_cell(const typename V2<R>::T* __restrict__ slots,
                                                         const GridGeom& gg, int tx, int ty, int ci, int cj,
                                                         const Head& head)
{
    using C = typename V2<R>::T;
    constexpr int NC = (REACH + 1) * (REACH + 1);
    const int T = gg.T, L = gg.L, LL = L * L;
    int first[NC], stride[NC], heads[NC], off[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        const int dy = i / (REACH + 1), dx = i % (REACH + 1);
        const int sty = ty - dy;
        const int sy = sty < 0 ? gg.pady : 0;
        const bool okr = sty >= 0 || gg.wrap_y;
        int stx = tx - dx, sx = 0;
        if (stx < 0) {
            stx += gg.ntx;
            sx = gg.padx;
            if (stx < 0) stx = ((stx % gg.ntx) + gg.ntx) % gg.ntx;
        }
        const int lx = ci + dx * T - sx, ly = cj + dy * T - sy;
        const bool in = okr && lx < L && ly < L;
        const int4 h = in ? head(sty, stx) : make_int4(0, 0, 1, 0);
        first[i] = h.x;
        heads[i] = h.y;
        stride[i] = h.z;
        off[i] = in ? ly * L + lx : 0;
    }
    C r[NC][U];
#pragma unroll
    for (int i = 0; i < NC; ++i)
#pragma unroll
        for (int u = 0; u < U; ++u)
            r[i][u] = u < heads[i] ? slots[((size_t)first[i] + (size_t)u * stride[i]) * LL + off[i]] : C{R(0), R(0)};
    R ar = R(0), ai = R(0);
#pragma unroll
    for (int i = 0; i < NC; ++i) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ar += r[i][u].x;
            ai += r[i][u].y;
        }
        for (int q = U; q < heads[i]; ++q) {
            const C v = slots[((size_t)first[i] + (size_t)q * stride[i]) * LL + off[i]];
            ar += v.x;
            ai += v.y;
        }
    }
    return C{ar, ai};
}

// Tile heads straight from the scan's table (tiles of instance b).
struct TsubHead {
    const int* tsub;
    int base, ntx, nty;
    __device__ int4 operator()(int sty, int stx) const
    {
        if (sty < 0) sty = ((sty % nty) + nty) % nty;
        const int t = base + sty * ntx + stx;
        return tile_heads(tsub[2 * t], tsub[2 * t + 1]);
    }
};

// Tile reduce over the listed tiles (the rest of the fine grid was filled
// with zeros): persistent blocks walk the cells of the listed tiles, 256 at
// a time, a thread per cell (reduce_cell); cells of a partial last tile
// outside the grid are skipped.  The 256 cells of a step touch at most
// kRedTiles listed tiles: the heads of their covering tiles are looked up
// once, into LDS, and the cells read them there, so a cell waits on one
// round of global loads (its slots) rather than two.  (Tiles are at least
// 4 x 4 cells; a step that still spanned more than kRedTiles tiles would look
// the heads up from the scan's table, cell by cell.)
constexpr int kRedTiles = 256 / 16 + 2;

template <int REACH>
struct ListHead {
    const int4* tab;  // (REACH + 1)^2 heads per listed tile of the step, (dy, dx) order
    int tx, ty, ntx;
    __device__ int4 operator()(int sty, int stx) const
    {
        int dx = tx - stx;
        if (dx < 0) dx += ntx;
        return tab[(ty - sty) * (REACH + 1) + dx];
    }
};

template <class R, int REACH>
__global__ void __launch_bounds__(256) k_reduce_list(const typename V2<R>::T* __restrict__ slots,
                                                     const int* __restrict__ tsub, const int* __restrict__ list,
                                                     const int* __restrict__ nlist, GridGeom gg, int tpi,
                                                     R* __restrict__ F, const int2* __restrict__ rwin)
{
    using C = typename V2<R>::T;
    constexpr int NC = (REACH + 1) * (REACH + 1);
    __shared__ int4 s_head[kRedTiles * NC];
    const int T = gg.T, TT = T * T;
    const int nl = *nlist;
    const int64_t ncell = (int64_t)nl * TT;
    for (int64_t e0 = blockIdx.x * (int64_t)blockDim.x; e0 < ncell; e0 += (int64_t)gridDim.x * blockDim.x) {
        const int k0 = (int)(e0 / TT);
        const int nt = min((int)((e0 + blockDim.x - 1) / TT), nl - 1) - k0 + 1;
        const bool staged = nt <= kRedTiles;
        for (int h = threadIdx.x; staged && h < nt * NC; h += blockDim.x) {
            const int kk = h / NC, i = h - kk * NC;
            const int dy = i / (REACH + 1), dx = i - dy * (REACH + 1);
            const int tile = list[k0 + kk];
            const int b = tile / tpi, tl = tile - b * tpi;
            const int ty = tl / gg.ntx, tx = tl - ty * gg.ntx;
            int sty = ty - dy;
            int4 hv = make_int4(0, 0, 1, 0);
            if (sty >= 0 || gg.wrap_y) {
                if (sty < 0) sty = ((sty % gg.nty) + gg.nty) % gg.nty;
                const int stx = (((tx - dx) % gg.ntx) + gg.ntx) % gg.ntx;
                const int t = b * tpi + sty * gg.ntx + stx;
                hv = tile_heads(tsub[2 * t], tsub[2 * t + 1]);
            }
            s_head[h] = hv;
        }
        __syncthreads();
        const int64_t e = e0 + threadIdx.x;
        if (e < ncell) {
            const int k = (int)(e / TT), c = (int)(e - (int64_t)k * TT);
            const int tile = list[k];
            const int b = tile / tpi, tl = tile - b * tpi;
            const int ty = tl / gg.ntx, tx = tl - ty * gg.ntx;
            const int cj = c / T, ci = c - cj * T;
            const int2 rw = inst_rows(rwin, gg, b);
            if (tx * T + ci < gg.nf1 && ty * T + cj < rw.x)
                reinterpret_cast<C*>(F)[((size_t)rw.y + ty * T + cj) * gg.nf1 + tx * T + ci] =
                    staged ? reduce_cell<R, REACH>(slots, gg, tx, ty, ci, cj,
                                                   ListHead<REACH>{s_head + (k - k0) * NC, tx, ty, gg.ntx})
                           : reduce_cell<R, REACH>(slots, gg, tx, ty, ci, cj,
                                                   TsubHead{tsub, b * tpi, gg.ntx, gg.nty});
        }
        __syncthreads();
    }
}

// Tile heads of the tile rows [ty_lo, ty_lo + nt) of one instance, copied
// to LDS (rows before 0 wrap when the grid wraps in y, else are empty).
struct LdsHead {
    const int4* tab;
    int ty_lo, ntx;
    __device__ int4 operator()(int sty, int stx) const { return tab[(sty - ty_lo) * ntx + stx]; }
};

// Tile reduce by strips: workgroup (ty S + sl, b) writes every cell of slice
// sl (of S) of tile row ty of instance b (rows ty T + sl RB .. of the rows
// ty T .. min(ty T + T, its rows) - 1, RB = ceil(T / S); all nf1 columns,
// row-major, so a step's 256 writes are contiguous), zeros included: no zero
// fill and no list of reached tiles.  Slices (S > 1) give a single large
// grid workgroups enough to fill the chip.  It first copies to LDS the heads of
// the REACH + 1 tile rows that cover the strip, then a flag per tile column:
// whether any covering tile holds points; cells under none are written as
// zeros without a load.  The sums are those of reduce_cell, in its order.
// Slice 0 also clears the binning counters of its tile row for the next
// call; a tile row past the instance's window has no cells.  A cell loads the
// first merged slot of each covering tile at once (U = 1: most tiles hold
// one work item), which leaves registers for four waves per SIMD in FP64
// instead of three (reduce 1.03 -> 0.99 ms on the batch).
__host__ __device__ inline size_t reduce_strips_lds(int reach, int ntx)
{
    return (size_t)(reach + 1) * ntx * sizeof(int4) + (size_t)ntx * sizeof(int);
}

template <class R, int REACH>
__global__ void __launch_bounds__(256) k_reduce_strips(const typename V2<R>::T* __restrict__ slots,
                                                       const int* __restrict__ tsub, GridGeom gg, int tpi,
                                                       R* __restrict__ F, int* __restrict__ cnt,
                                                       const int2* __restrict__ rwin, int S)
{
    using C = typename V2<R>::T;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int ty = blockIdx.x / S, sl = blockIdx.x - ty * S, b = blockIdx.y;
    const int T = gg.T, ntx = gg.ntx;
    int4* tab = reinterpret_cast<int4*>(lds_raw);                    // (REACH + 1) x ntx heads
    int* act = reinterpret_cast<int*>(lds_raw + (size_t)(REACH + 1) * ntx * sizeof(int4));
    if (sl == 0)
        for (int tx = threadIdx.x; tx < ntx; tx += blockDim.x) cnt[b * tpi + ty * ntx + tx] = 0;
    const int2 rw = inst_rows(rwin, gg, b);
    const int RB = (T + S - 1) / S;
    const int y0 = ty * T, ys = y0 + sl * RB;
    if (ys >= min(y0 + T, rw.x)) return;
    const int ty_lo = ty - REACH;
    for (int e = threadIdx.x; e < (REACH + 1) * ntx; e += blockDim.x) {
        const int k = e / ntx, tx = e - k * ntx;
        int sty = ty_lo + k;
        int4 h = make_int4(0, 0, 1, 0);
        if (sty >= 0 || gg.wrap_y) {
            if (sty < 0) sty = ((sty % gg.nty) + gg.nty) % gg.nty;
            const int t = b * tpi + sty * ntx + tx;
            h = tile_heads(tsub[2 * t], tsub[2 * t + 1]);
        }
        tab[e] = h;
    }
    __syncthreads();
    for (int tx = threadIdx.x; tx < ntx; tx += blockDim.x) {
        int any = 0;
#pragma unroll
        for (int dx = 0; dx <= REACH; ++dx) {
            const int stx = (((tx - dx) % ntx) + ntx) % ntx;
#pragma unroll
            for (int k = 0; k <= REACH; ++k) any |= tab[k * ntx + stx].y;
        }
        act[tx] = any;
    }
    __syncthreads();
    const int nrow = min(min(RB, y0 + T - ys), rw.x - ys), nf1 = gg.nf1;
    const LdsHead head{tab, ty_lo, ntx};
    const FastDiv dT = fast_div((unsigned)T);
    for (int r = 0; r < nrow; ++r) {
        C* Fr = reinterpret_cast<C*>(F) + ((size_t)rw.y + ys + r) * nf1;
        for (int x = threadIdx.x; x < nf1; x += blockDim.x) {
            const int tx = (int)fdiv((unsigned)x, dT);
            C v{R(0), R(0)};
            if (act[tx]) v = reduce_cell<R, REACH, 1>(slots, gg, tx, ty, x - tx * T, ys - y0 + r, head);
            Fr[x] = v;
        }
    }
}

// Tile rows whose heads a group of C fine-grid rows starting at r0 needs,
// and the table's byte offset in LDS (after the rows and the twiddles,
// 16-byte aligned).
__host__ __device__ inline int t1_rows_table_rows(int C, int T, int reach) { return (C - 1) / T + 2 + reach; }
__host__ __device__ inline size_t t1_rows_table_offset(int C, int n, int ntw, size_t csize)
{
    return (csize * (lds_span(n, C) + ntw) + 15) / 16 * 16;
}

// Tile reduce fused with the first FFT pass of type 1.  Workgroup (group g,
// instance b) takes the C fine-grid rows [g C, g C + C) of the band: it
// copies the heads of the tile rows covering them to LDS, each cell sums its
// covering slots (reduce_cell) straight into LDS, the rows are transformed
// there (length nf1), and only the n1 needed columns k1 mod nf1,
// k1 in [-n1/2, n1/2), are written to G (B x rows x n1, row stride n1, in k1
// order).  The fine grid itself is never stored.  The binning counters of
// the tile rows that start in this group's rows are left at zero for the
// next call.  Every cell looks up its covering tiles, so this pays where
// the tiles are large (a padded tile reaching one tile on) or the grid is
// densely covered; the list reduce into a stored grid visits only the
// reached tiles.
template <class R, int MAXE, int NT, bool R7, int REACH>
__global__ void __launch_bounds__(NT) k_t1_rows(const typename V2<R>::T* __restrict__ slots,
                                                const int* __restrict__ tsub, GridGeom gg, int tpi, int C,
                                                int groups, LdsFftPlan plan, int n1, R* __restrict__ G,
                                                int* __restrict__ cnt)
{
    using C2 = typename V2<R>::T;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    C2* buf = reinterpret_cast<C2*>(lds_raw);
    const int g = xcd_group(groups);
    if (g >= groups) return;
    const int b = blockIdx.y;
    const int nf1 = plan.n, T = gg.T;
    const int r0 = g * C;
    const int nr = min(C, gg.rows - r0);
    // heads of the covering tile rows, after the FFT's data and twiddles
    const int ty_lo = r0 / T - REACH;
    const int nt = t1_rows_table_rows(C, T, REACH);
    int4* tab = reinterpret_cast<int4*>(lds_raw + t1_rows_table_offset(C, nf1, plan.ntw, sizeof(C2)));
    for (int e = threadIdx.x; e < nt * gg.ntx; e += NT) {
        const int k = e / gg.ntx, tx = e - k * gg.ntx;
        int sty = ty_lo + k;
        int4 h = make_int4(0, 0, 1, 0);
        if (sty < gg.nty && (sty >= 0 || gg.wrap_y)) {
            if (sty < 0) sty = ((sty % gg.nty) + gg.nty) % gg.nty;
            const int t = b * tpi + sty * gg.ntx + tx;
            h = tile_heads(tsub[2 * t], tsub[2 * t + 1]);
        }
        tab[e] = h;
    }
    // tile rows ty with r0 <= ty T < r0 + nr
    const int ty0 = (r0 + T - 1) / T, ty1 = (r0 + nr + T - 1) / T;
    for (int e = threadIdx.x; e < (ty1 - ty0) * gg.ntx; e += NT) cnt[b * tpi + ty0 * gg.ntx + e] = 0;
    __syncthreads();
    const LdsHead head{tab, ty_lo, gg.ntx};
    const FastDiv dT = fast_div((unsigned)T), dn = fast_div((unsigned)nf1);
    for (int e = threadIdx.x; e < C * nf1; e += NT) {
        const int rr = (int)fdiv((unsigned)e, dn), x = e - rr * nf1;
        C2 v{R(0), R(0)};
        if (rr < nr) {
            const int y = r0 + rr;
            const int tx = (int)fdiv((unsigned)x, dT), ty = (int)fdiv((unsigned)y, dT);
            v = reduce_cell<R, REACH, 1>(slots, gg, tx, ty, x - tx * T, y - ty * T, head);
        }
        buf[lds_pad(e)] = v;
    }
    __syncthreads();
    lds_fft<MAXE, NT, R7>(buf, plan, C, buf + lds_span(nf1, C));
    C2* Gv = reinterpret_cast<C2*>(G) + ((size_t)b * gg.rows + r0) * n1;
    for (int e = threadIdx.x; e < nr * n1; e += NT) {
        const int rr = e / n1, k1i = e - rr * n1;
        const int k1 = k1i - n1 / 2;
        Gv[e] = buf[lds_pad(rr * nf1 + (k1 < 0 ? k1 + nf1 : k1))];
    }
}

// --------------------------------------------------------- type-1 finish
struct EpiInst {
    double inv2lz;  // 1/(2 lambda z): target chirp in turns
    double invlz;   // 1/(lambda z)
    int occ;
    int sh2;        // row shift of the instance's window
    int rows;       // rows held for the instance (its window)
    int roff;       // its first row in the band array
};

struct EpiParams {
    int n1, n2, nf1, nf2;
    double h1, h2, xc, yc;
    const double* iphi1;
    const double* iphi2;
};

// Z[b][c][r] = F[b][r][k1 mod nf1] with k1 = c - n1/2 for r < rows, 0 beyond:
// the n1 needed columns after the first FFT pass, transposed and padded to
// the full period for the second pass.
template <class R>
__global__ void __launch_bounds__(256) k_transpose_pad(const R* __restrict__ F, R* __restrict__ Z, int n1, int nf1,
                                                       int nf2, int rows)
{
    using C2 = typename V2<R>::T;
    __shared__ C2 t[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32, b = blockIdx.z;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const C2* Fv = reinterpret_cast<const C2*>(F) + (size_t)b * rows * nf1;
    for (int k = ty; k < 32; k += 8) {
        const int r = r0 + k, cidx = c0 + tx;
        C2 v;
        v.x = R(0);
        v.y = R(0);
        if (r < rows && cidx < n1) {
            int col = cidx - n1 / 2;
            if (col < 0) col += nf1;
            v = Fv[(size_t)r * nf1 + col];
        }
        t[k][tx] = v;
    }
    __syncthreads();
    C2* Zv = reinterpret_cast<C2*>(Z) + (size_t)b * n1 * nf2;
    for (int k = ty; k < 32; k += 8) {
        const int cidx = c0 + k, r = r0 + tx;
        if (cidx < n1 && r < nf2) Zv[(size_t)cidx * nf2 + r] = t[tx][k];
    }
}

// u[b][k2][k1] from Z[b][k1 + n1/2][k2 mod nf2]: deconvolve by the kernel
// transform, undo the window shift, apply the target chirp and 1/(i lambda z),
// and Babinet.  All factors but 1/(i lambda z) separate into a column factor
// E1[k1] = exp(i pi xi^2/(lambda z)) / Phi1 and a row factor
// E2[k2] = exp(i pi eta^2/(lambda z) - 2 pi i k2 sh2/nf2) / Phi2, computed
// once per block (each phase reduced in turns in FP64 before sincospi).
template <class R>
__global__ void __launch_bounds__(256) k_epilogue_t1(const R* __restrict__ Z, R* __restrict__ u, EpiParams ep,
                                                     EpiInst e0, const EpiInst* __restrict__ table)
{
    using C2 = typename V2<R>::T;
    __shared__ C2 t[32][33];
    __shared__ double2 E1[32], E2[32];
    const int k10 = blockIdx.x * 32, k20 = blockIdx.y * 32, b = blockIdx.z;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const EpiInst ei = table ? table[b] : e0;
    if (threadIdx.x < 64) {
        const bool row = threadIdx.x >= 32;
        const int ki = (row ? k20 : k10) + tx;
        const int n = row ? ep.n2 : ep.n1;
        double2 f = make_double2(0.0, 0.0);
        if (ki < n) {
            const int k = ki - n / 2;
            const double x = row ? ep.yc + ep.h2 * k : ep.xc + ep.h1 * k;
            double tt = x * x * ei.inv2lz;
            if (row) {
                // window shift: F_full[k2] = exp(-2 pi i k2 sh2/nf2) F_window[k2]
                long long km = k % ep.nf2;
                if (km < 0) km += ep.nf2;
                long long sm = ei.sh2 % ep.nf2;
                if (sm < 0) sm += ep.nf2;
                tt = (tt - rint(tt)) - (double)((km * sm) % ep.nf2) / (double)ep.nf2;
            }
            const double ph = tt - rint(tt);
            double sn, cs;
            sincospi(2.0 * ph, &sn, &cs);
            const double sc = row ? ep.iphi2[ki] : ep.iphi1[ki];
            f = make_double2(cs * sc, sn * sc);
        }
        (row ? E2 : E1)[tx] = f;
    }
    const C2* Zv = reinterpret_cast<const C2*>(Z) + (size_t)b * ep.n1 * ep.nf2;
    for (int k = ty; k < 32; k += 8) {
        const int cidx = k10 + k, k2i = k20 + tx;
        if (cidx < ep.n1 && k2i < ep.n2) {
            int r = k2i - ep.n2 / 2;
            if (r < 0) r += ep.nf2;
            t[k][tx] = Zv[(size_t)cidx * ep.nf2 + r];
        }
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int k2i = k20 + k, k1i = k10 + tx;
        if (k1i >= ep.n1 || k2i >= ep.n2) continue;
        const C2 fv = t[tx][k];
        const double2 a = E1[tx], c = E2[k];
        const double ar = a.x * c.x - a.y * c.y, ai = a.x * c.y + a.y * c.x;
        const double wr = (double)fv.x * ar - (double)fv.y * ai;
        const double wi = (double)fv.x * ai + (double)fv.y * ar;
        // times 1/(i lambda z)
        double re = wi * ei.invlz;
        double im = -wr * ei.invlz;
        if (ei.occ) {
            re = 1.0 - re;
            im = -im;
        }
        C2 out;
        out.x = (R)re;
        out.y = (R)im;
        reinterpret_cast<C2*>(u)[((size_t)b * ep.n2 + k2i) * ep.n1 + k1i] = out;
    }
}

// Row factors of the type-1 epilogue, once per call: for instance b and
// output row k2, E2 = exp(i pi eta^2/(lambda z) - 2 pi i k2 sh2/nf2)/Phi2(k2)
// with each phase reduced in turns before sincospi.
__global__ void __launch_bounds__(256) k_t1_rowfactors(EpiParams ep, EpiInst e0, const EpiInst* __restrict__ table,
                                                       double2* __restrict__ E2)
{
    const int k2i = blockIdx.x * blockDim.x + threadIdx.x, b = blockIdx.y;
    if (k2i >= ep.n2) return;
    const EpiInst ei = table ? table[b] : e0;
    const int nf2 = ep.nf2;
    const int sm = (int)(((long long)ei.sh2 % nf2 + nf2) % nf2);
    const int k2 = k2i - ep.n2 / 2;
    const double y = ep.yc + ep.h2 * k2;
    double tt = y * y * ei.inv2lz;
    const unsigned km = (unsigned)(k2 < 0 ? k2 + nf2 : k2);
    const unsigned ph = (km * (unsigned)sm) % (unsigned)nf2;
    tt = (tt - rint(tt)) - (double)ph / (double)nf2;
    tt -= rint(tt);
    double sn, cs;
    sincospi(2.0 * tt, &sn, &cs);
    const double sc = ep.iphi2[k2i];
    E2[(size_t)b * ep.n2 + k2i] = make_double2(cs * sc, sn * sc);
}

// Type-1 second pass and epilogue in one kernel.  Workgroup (group g,
// instance b) takes the C output columns k1 + n1/2 in [g C, g C + C): it
// loads their band of `rows` values from F (after the first pass over the
// rows; row stride ldf, and either the full nf1 columns, column k1 at
// k1 mod nf1, or with `compact` only the n1 needed ones in k1 order),
// zero-pads each to nf2 in LDS, transforms, and writes
// u[b][k2][k1] = epilogue(column value at k2 mod nf2) for every k2, with the
// factors of k_epilogue_t1: its column factors here, its row factors from
// k_t1_rowfactors.
template <class R, int MAXE, int NT, bool R7>
__global__ void __launch_bounds__(NT) k_t1_cols(const R* __restrict__ F, R* __restrict__ u, int rows, int ldf,
                                                            int compact, int C, int groups, LdsFftPlan plan, EpiParams ep,
                                                            EpiInst e0, const EpiInst* __restrict__ table,
                                                            const double2* __restrict__ E2all)
{
    using C2 = typename V2<R>::T;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    C2* buf = reinterpret_cast<C2*>(lds_raw);
    __shared__ double2 E1[16];
    const int g = xcd_group(groups);
    if (g >= groups) return;
    const int b = blockIdx.y;
    const EpiInst ei = table ? table[b] : e0;
    const int nf2 = plan.n;
    const int col0 = g * C;
    const int ncol = min(C, ep.n1 - col0);
    // column factors: target chirp over 1/Phi
    if ((int)threadIdx.x < C) {
        double2 f = make_double2(0.0, 0.0);
        const int ki = col0 + threadIdx.x;
        if (ki < ep.n1) {
            const double x = ep.xc + ep.h1 * (ki - ep.n1 / 2);
            double tt = x * x * ei.inv2lz;
            tt -= rint(tt);
            double sn, cs;
            sincospi(2.0 * tt, &sn, &cs);
            const double sc = ep.iphi1[ki];
            f = make_double2(cs * sc, sn * sc);
        }
        E1[threadIdx.x] = f;
    }
    // band of the C columns (adjacent lanes read adjacent columns of a row)
    const C2* Fv = reinterpret_cast<const C2*>(F) + (size_t)ei.roff * ldf;
    const int rb = min(ei.rows, rows);
    const FastDiv dC = fast_div((unsigned)C);
    for (int e = threadIdx.x; e < C * rb; e += NT) {
        const int r = (int)fdiv((unsigned)e, dC), c = e - r * C;
        C2 v;
        v.x = R(0);
        v.y = R(0);
        if (c < ncol) {
            int col = col0 + c;
            if (!compact) {
                col -= ep.n1 / 2;
                if (col < 0) col += ep.nf1;
            }
            v = Fv[(size_t)r * ldf + col];
        }
        buf[lds_pad(c * nf2 + r)] = v;
    }
    // the zero padding below the band, column by column
    const int nz = nf2 - rb;
    if (nz > 0) {
        const FastDiv dz = fast_div((unsigned)nz);
        for (int e = threadIdx.x; e < C * nz; e += NT) {
            const int c = (int)fdiv((unsigned)e, dz);
            C2 v;
            v.x = R(0);
            v.y = R(0);
            buf[lds_pad(c * nf2 + rb + (e - c * nz))] = v;
        }
    }
    __syncthreads();
    lds_fft<MAXE, NT, R7>(buf, plan, C, buf + lds_span(plan.n, C));
    // epilogue: C lanes write C consecutive outputs of a row, with the row
    // factors of k_t1_rowfactors and the column factors above
    const double2* E2 = E2all + (size_t)b * ep.n2;
    C2* uv = reinterpret_cast<C2*>(u) + (size_t)b * ep.n2 * ep.n1;
    for (int e = threadIdx.x; e < ep.n2 * C; e += NT) {
        const int k2i = (int)fdiv((unsigned)e, dC), c = e - k2i * C;
        if (c >= ncol) continue;
        const int k2 = k2i - ep.n2 / 2;
        const int r = k2 < 0 ? k2 + nf2 : k2;
        const C2 fv = buf[lds_pad(c * nf2 + r)];
        const double2 er = E2[k2i];
        const double2 a = E1[c];
        const double ar = a.x * er.x - a.y * er.y, ai = a.x * er.y + a.y * er.x;
        const double wr = (double)fv.x * ar - (double)fv.y * ai;
        const double wi = (double)fv.x * ai + (double)fv.y * ar;
        // times 1/(i lambda z)
        double re = wi * ei.invlz;
        double im = -wr * ei.invlz;
        if (ei.occ) {
            re = 1.0 - re;
            im = -im;
        }
        C2 out;
        out.x = (R)re;
        out.y = (R)im;
        uv[(size_t)k2i * ep.n1 + col0 + c] = out;
    }
}

// Type-3 precorrection and row pass.  Workgroup g takes the C rows
// [g C, g C + C) of the m1 x m2 upsampled grid G: entry (k1, k2) is
// b[k2 mod nf2][k1 mod nf1] / (Phi1 Phi2) for modes inside the spread grid
// (-nf/2 <= k < nf - nf/2), zero outside; each row is transformed and
// written back to G.
template <class R, int MAXE, int NT, bool R7>
__global__ void __launch_bounds__(NT) k_t3_rows(const R* __restrict__ bgrid, int nf1, int nf2,
                                                            R* __restrict__ G, int m1, int m2, int C, int groups,
                                                            LdsFftPlan plan, const double* __restrict__ ip1,
                                                            const double* __restrict__ ip2)
{
    using C2 = typename V2<R>::T;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    C2* buf = reinterpret_cast<C2*>(lds_raw);
    const int g = xcd_group(groups);
    if (g >= groups) return;
    const int row0 = g * C;
    const int nrow = min(C, m2 - row0);
    const C2* bv = reinterpret_cast<const C2*>(bgrid);
    for (int e = threadIdx.x; e < C * m1; e += NT) {
        const int c = e / m1, i1 = e - c * m1;
        C2 v;
        v.x = R(0);
        v.y = R(0);
        if (c < nrow) {
            const int i2 = row0 + c;
            const int k1 = i1 < m1 / 2 ? i1 : i1 - m1;
            const int k2 = i2 < m2 / 2 ? i2 : i2 - m2;
            if (k1 >= -(nf1 / 2) && k1 < nf1 - nf1 / 2 && k2 >= -(nf2 / 2) && k2 < nf2 - nf2 / 2) {
                const int s1 = k1 < 0 ? k1 + nf1 : k1;
                const int s2 = k2 < 0 ? k2 + nf2 : k2;
                const C2 x = bv[(size_t)s2 * nf1 + s1];
                const double sc = ip1[k1 + nf1 / 2] * ip2[k2 + nf2 / 2];
                v.x = (R)(x.x * sc);
                v.y = (R)(x.y * sc);
            }
        }
        buf[lds_pad(e)] = v;
    }
    __syncthreads();
    lds_fft<MAXE, NT, R7>(buf, plan, C, buf + lds_span(plan.n, C));
    C2* Gv = reinterpret_cast<C2*>(G);
    for (int e = threadIdx.x; e < nrow * m1; e += NT) Gv[(size_t)row0 * m1 + e] = buf[lds_pad(e)];
}

// Type-3 column pass, in place: workgroup g transforms the C columns
// [g C, g C + C) of G (length m2 each).
template <class R, int MAXE, int NT, bool R7>
__global__ void __launch_bounds__(NT) k_t3_cols(R* __restrict__ G, int m1, int m2, int C, int groups,
                                                            LdsFftPlan plan)
{
    using C2 = typename V2<R>::T;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    C2* buf = reinterpret_cast<C2*>(lds_raw);
    const int g = xcd_group(groups);
    if (g >= groups) return;
    const int col0 = g * C;
    const int ncol = min(C, m1 - col0);
    C2* Gv = reinterpret_cast<C2*>(G);
    for (int e = threadIdx.x; e < C * m2; e += NT) {
        const int i2 = e / C, c = e - i2 * C;
        C2 v;
        v.x = R(0);
        v.y = R(0);
        if (c < ncol) v = Gv[(size_t)i2 * m1 + col0 + c];
        buf[lds_pad(c * m2 + i2)] = v;
    }
    __syncthreads();
    lds_fft<MAXE, NT, R7>(buf, plan, C, buf + lds_span(plan.n, C));
    for (int e = threadIdx.x; e < C * m2; e += NT) {
        const int i2 = e / C, c = e - i2 * C;
        if (c < ncol) Gv[(size_t)i2 * m1 + col0 + c] = buf[lds_pad(c * m2 + i2)];
    }
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
    int m1, m2;             // upsampled grid
    double xic, etac;       // target centre
    double g1, g2;          // interpolation grid coordinate per unit (xi - xic)
    double th1, th2;        // theta per unit (xi - xic) for the 1/Phi correction
    double inv2lz, invlz;   // target chirp (turns) and 1/(lambda z)
    double Cx, Cy;          // source centre (post-phase exp(-i s.C))
    double box[4];          // targets the grids were planned for; others give NaN
    int occ;
    InvPhiCheb ch1, ch2;
};

// Sum over aligned groups of GS lanes; lane 0 of each group gets the total,
// always with the same association.  GS = 16 and 8 use DPP row operations
// (no LDS round trip); other sizes use shuffles.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int GS, class R>
__device__ __forceinline__ R group_sum(R v)
{
    if constexpr (GS == 16) {
        v += dpp_f<0x128>(v);  // row_ror:8
        v += dpp_f<0x124>(v);  // row_ror:4
        v += dpp_f<0x122>(v);  // row_ror:2
        v += dpp_f<0x121>(v);  // row_ror:1
    } else if constexpr (GS == 8) {
        v += dpp_f<0x141>(v);  // row_half_mirror: lane i + lane 7 - i
        v += dpp_f<0x4e>(v);   // quad_perm [2,3,0,1]
        v += dpp_f<0xb1>(v);   // quad_perm [1,0,3,2]
    } else {
#pragma unroll
        for (int off = GS / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, GS);
    }
    return v;
}

// Lanes per target in the interpolation: one stencil row per lane.
template <int W>
constexpr int interp_group() { return W <= 8 ? 8 : (W <= 16 ? 16 : 32); }

// Wavefront per 64 targets; a target outside tp.box, or with a non-finite
// coordinate, gets NaN.  Lane l first handles target l of the chunk on
// its own: stencil cell, the 2W kernel values (staged in LDS), and the
// 1/Phi correction, chirp and 1/(i lambda z) factor.  The wavefront then
// gathers in trips of 64/GS targets: GS lanes per target, lane r taking
// stencil column r down all W rows (so each load instruction reads, per
// target, one contiguous run of the row: a few cache lines rather than one
// line per lane), all W loads in flight; the column is weighted down its
// rows, then by its own kernel value, and summed over the group by a fixed
// butterfly.  Lane l finally scales its target's sum and writes it.
template <class R, int W>
__global__ void __launch_bounds__(64) k_t3_interp(const R* __restrict__ G, const double* __restrict__ xi,
                                                  const double* __restrict__ eta, int64_t M, R beta,
                                                  const R* __restrict__ poly, T3Params tp, int tpw,
                                                  R* __restrict__ u, const int* __restrict__ perm)
{
    using C = typename V2<R>::T;
    constexpr int GS = interp_group<W>();
    constexpr int NT = 64 / GS;
    constexpr int KS = 2 * W + 1;
    __shared__ R ks[64 * KS];
    __shared__ uint32_t cs[64];
    __shared__ C res[64];
    const int lane = threadIdx.x, g = lane / GS, r = lane % GS;
    const C* Gv = reinterpret_cast<const C*>(G);
    for (int64_t base = blockIdx.x * (int64_t)tpw; base < M; base += (int64_t)gridDim.x * tpw) {
        const int64_t t = base + lane;
        const bool live = lane < tpw && t < M;
        const int64_t k = live ? t : 0;
        const double X = xi[k], Y = eta[k];
        const bool inbox = X >= tp.box[0] && X <= tp.box[1] && Y >= tp.box[2] && Y <= tp.box[3];
        int l1, l2;
        double d1, d2;
        bool ok1, ok2;
        cell_of((X - tp.xic) * tp.g1, tp.m1, W, l1, d1, ok1);
        cell_of((Y - tp.etac) * tp.g2, tp.m2, W, l2, d2, ok2);
        cs[lane] = (uint32_t)l1 | ((uint32_t)l2 << 16);
        {
            R kv[W];
            es_weights<R, W>((R)d1, beta, poly, kv);
#pragma unroll
            for (int a = 0; a < W; ++a) ks[lane * KS + a] = kv[a];
            es_weights<R, W>((R)d2, beta, poly, kv);
#pragma unroll
            for (int b = 0; b < W; ++b) ks[lane * KS + W + b] = kv[b];
        }
        // output factor: 1/Phi correction times the target chirp over i lambda z
        const double corr =
            cheb_inv_phi(tp.ch1, (X - tp.xic) * tp.th1) * cheb_inv_phi(tp.ch2, (Y - tp.etac) * tp.th2);
        const double ph = (X * X + Y * Y) * tp.inv2lz - (X * tp.Cx + Y * tp.Cy) * tp.invlz;
        double sn, cn;
        sincospi(2.0 * (ph - rint(ph)), &sn, &cn);
        const double fr = sn * corr * tp.invlz, fi = -cn * corr * tp.invlz;
        wave_lds_order();
        const int nq = (int)min<int64_t>(tpw, M - base);
        // gathers of the next trip are issued before the current one is
        // summed, alternating between two register buffers; the gather has
        // no branches (inactive lanes read a valid entry and get weight
        // zero), so the loads can stay in flight
        const int rr = min(r, W - 1);
        C bufA[W], bufB[W];
        auto gather = [&](int q, C* gv) {
            const uint32_t cp = cs[min(q, nq - 1)];
            int col = (int)(cp & 0xffffu) + rr;
            col = col >= tp.m1 ? col - tp.m1 : col;
            const int row0 = (int)(cp >> 16);
            const C* gc = Gv + col;
#pragma unroll
            for (int b = 0; b < W; ++b) {
                const int row = row0 + b;
                gv[b] = gc[(size_t)(row >= tp.m2 ? row - tp.m2 : row) * tp.m1];
            }
        };
        auto trip_sum = [&](int q, const C* gv) {
            const R* kq = ks + min(q, nq - 1) * KS;
            R sr = R(0), si = R(0);
#pragma unroll
            for (int b = 0; b < W; ++b) {
                sr += gv[b].x * kq[W + b];
                si += gv[b].y * kq[W + b];
            }
            const R kx = (q < nq && r < W) ? kq[rr] : R(0);
            sr = group_sum<GS>(sr * kx);
            si = group_sum<GS>(si * kx);
            if (r == 0 && q < nq) res[q] = C{sr, si};
        };
        gather(g, bufA);
        for (int j = 0; j < nq; j += 2 * NT) {
            gather(j + NT + g, bufB);
            trip_sum(j + g, bufA);
            if (j + NT >= nq) break;
            gather(j + 2 * NT + g, bufA);
            trip_sum(j + NT + g, bufB);
        }
        wave_lds_order();
        if (live) {
            const C v = res[lane];
            double re = (double)v.x * fr - (double)v.y * fi;
            double im = (double)v.x * fi + (double)v.y * fr;
            if (!(ok1 && ok2 && inbox)) {
                re = __builtin_nan("");
                im = __builtin_nan("");
            }
            if (tp.occ) {
                re = 1.0 - re;
                im = -im;
            }
            // a sorted target set writes back to the caller's order
            const int64_t ko = perm ? (int64_t)perm[k] : k;
            u[2 * ko] = (R)re;
            u[2 * ko + 1] = (R)im;
        }
        wave_lds_order();
    }
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
// Wavefronts per work item of the wavefront spread: two when their two tiles
// fit the LDS budget with the staging.
inline int spread_waves(const GridGeom& gg, size_t rsize)
{
    const size_t tile = 2 * rsize * ((size_t)gg.L * gg.L + 1);
    return 2 * tile + spread_staging_bytes(gg.W, rsize) <= kLdsBudget ? 2 : 1;
}

// LDS bytes of one spread block.
inline size_t spread_lds(const GridGeom& gg, size_t rsize)
{
    if (gg.method == 5) return mfma_spread_lds(gg.L <= 16 ? 1 : 2, gg.T, rsize);
    if (gg.method == 4) {
        // staging of 32 points (W + KYP + 2 reals and 2 ints each) and the 4
        // wavefront tiles (see RegTile and reg_spread_lds)
        const int L = gg.L, NB = 64 / L, RB = (L + NB - 1) / NB;
        const size_t kyp = (size_t)(gg.T - 1 + NB * RB);
        return 32 * (rsize * ((size_t)gg.W + kyp + 2) + 2 * sizeof(int)) + 2 * rsize * 4 * (size_t)L * L;
    }
    const size_t tile = 2 * rsize * (size_t)gg.L * gg.L;
    if (gg.method == 1) return tile;
    return (size_t)spread_waves(gg, rsize) * (tile + 2 * rsize) + spread_staging_bytes(gg.W, rsize);
}

template <class R, int W>
void launch_spread_w(fh_ctx* c, unsigned grid, const Sub* subs, const int* nsub, const uint32_t* cell,
                     const void* dd, const void* cc, typename V2<R>::T* slots, const GridGeom& gg, int tpi,
                     double beta, const void* poly)
{
    using C2 = typename V2<R>::T;
    const size_t tile = sizeof(C2) * (size_t)gg.L * gg.L;
    if (gg.method == 1) {
        hipLaunchKernelGGL((k_spread_thread<R, W>), dim3(grid), dim3(256), tile, c->stream, subs, nsub, cell,
                           (const C2*)dd, (const C2*)cc, slots, gg, tpi, (R)beta, (const R*)poly);
        return;
    }
    if (gg.method == 5) {
        // (T + W - 1) <= 32: two 16-cell blocks per dimension, else one
        if constexpr (W <= 16) {
            if (gg.L <= 16) {
                hipLaunchKernelGGL((k_spread_mfma<R, W, 1, mfma_stage<R>()>), dim3(grid), dim3(64 * kMfmaWaves),
                                   mfma_spread_lds(1, gg.T, sizeof(R)), c->stream, subs, nsub, cell, (const C2*)dd,
                                   (const C2*)cc, slots, gg, tpi, (R)beta, (const R*)poly);
                return;
            }
        }
            hipLaunchKernelGGL((k_spread_mfma<R, W, 2, mfma_stage<R>()>), dim3(grid), dim3(64 * kMfmaWaves), mfma_spread_lds(2, gg.T, sizeof(R)),
                               c->stream, subs, nsub, cell, (const C2*)dd, (const C2*)cc, slots, gg, tpi, (R)beta,
                               (const R*)poly);
        return;
    }
    if (gg.method == 4) {
        if (gg.T == 16)
            hipLaunchKernelGGL((k_spread_reg<R, W, 16>), dim3(grid), dim3(256), (reg_spread_lds<R, 16, W>()),
                               c->stream, subs, nsub, cell, (const C2*)dd, (const C2*)cc, slots, gg, tpi, (R)beta,
                               (const R*)poly);
        else
            hipLaunchKernelGGL((k_spread_reg<R, W, 8>), dim3(grid), dim3(256), (reg_spread_lds<R, 8, W>()),
                               c->stream, subs, nsub, cell, (const C2*)dd, (const C2*)cc, slots, gg, tpi, (R)beta,
                               (const R*)poly);
        return;
    }
    // the tiles with their spare cells, the point staging and the kernel
    // coefficients (spread_lds)
    const int nv = spread_waves(gg, sizeof(R));
    const size_t lds = spread_lds(gg, sizeof(R));
    const bool at = gg.method == 3;
#define FH_WAVE_LAUNCH(A, N)                                                                                      \
    hipLaunchKernelGGL((k_spread_wave<R, W, A, N>), dim3(grid), dim3(64 * N), lds, c->stream, subs, nsub, cell,  \
                       (const C2*)dd, (const C2*)cc, slots, gg, tpi, (R)beta, (const R*)poly)
    if (nv == 2) {
        if (at)
            FH_WAVE_LAUNCH(true, 2);
        else
            FH_WAVE_LAUNCH(false, 2);
    } else {
        if (at)
            FH_WAVE_LAUNCH(true, 1);
        else
            FH_WAVE_LAUNCH(false, 1);
    }
#undef FH_WAVE_LAUNCH
}

template <class R>
fh_status launch_spread(fh_ctx* c, unsigned grid, const Sub* subs, const int* nsub, const uint32_t* cell,
                        const void* dd, const void* cc, typename V2<R>::T* slots, const GridGeom& gg, int tpi,
                        double beta, const void* poly)
{
    FH_ARG(spread_lds(gg, sizeof(R)) <= kLdsBudget, FH_ERR_UNSUPPORTED,
           "spread tile %d with width %d exceeds the LDS budget", gg.T, gg.W);
    switch (gg.W) {
#define FH_SPREAD_CASE(w) \
    case w: launch_spread_w<R, w>(c, grid, subs, nsub, cell, dd, cc, slots, gg, tpi, beta, poly); break;
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

// Targets per wavefront: 64 (the per-target setup then uses every lane),
// halved (down to one gather trip's worth) while that leaves fewer than
// about 4 wavefronts per CU, so that small target sets still spread their
// gather trips over many wavefronts.
template <class R>
fh_status launch_interp(fh_ctx* c, int W, const R* G, const double* xi, const double* eta, int64_t M,
                        double beta, const void* poly, const T3Params& tp, R* u, const int* perm)
{
    const int per_trip = W <= 8 ? 8 : (W <= 16 ? 4 : 2);
    int tpw = 64;
    while (tpw > per_trip && M / tpw < (int64_t)c->cu_count * 4) tpw /= 2;
    switch (W) {
#define FH_INTERP_CASE(w)                                                                           \
    case w:                                                                                        \
        hipLaunchKernelGGL((k_t3_interp<R, w>), dim3(std::min<int64_t>(nblocks(M, tpw), 1 << 20)), dim3(64), 0, \
                           c->stream, G, xi, eta, M, (R)beta, (const R*)poly, tp, tpw, u, perm); \
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
    int* cnt;       // points per tile
    int* off;       // first sorted point of each tile
    int* tsub;      // per tile: first work item, number of work items
    int* rank;      // rank of each node within its tile
    uint32_t* cell; // sorted: packed first stencil cell (x | y << 16)
    void* dd;       // sorted: stencil offsets (2 reals)
    void* cc;       // sorted: strengths (complex)
    Sub* subs;      // work items
    int* nsub;      // number of work items (device)
    int* bsum;      // per scan block: points and work items
    void* slots;    // one padded L x L complex tile per work item
    int* list;      // tiles some padded tile reaches (list reduce), and their count
    int* nlist;
    int* chunk;     // instance of every kChunk-th node (batches)
    // stable binning only: tile keys and node indices, before and after the
    // sort, and the sort's scratch
    uint32_t* key;
    uint32_t* key_sorted;
    int* vals;
    int* vals_sorted;
    void* sort_tmp;
    size_t sort_bytes;
    int64_t max_sub;
};


// Type-1 geometry: kernel, fine grid and tiling.
struct T1Plan {
    EsKernel k;
    GridGeom gg;
};

size_t spread_bytes(const fh_ctx* c, int64_t Ntot, const GridGeom& gg, int ntiles_total, size_t rsize)
{
    const int64_t max_sub = Ntot / gg.P + std::min<int64_t>(Ntot, ntiles_total) + 1;
    const size_t sort = c->opt.deterministic
                            ? 4 * aligned_bytes(sizeof(int) * (size_t)Ntot) + aligned_bytes(tile_sort_bytes(Ntot))
                            : 0;
    return sort + aligned_bytes(sizeof(int) * (size_t)ntiles_total) + aligned_bytes(2 * sizeof(int) * ntiles_total) +
           aligned_bytes(2 * sizeof(int) * (size_t)(ntiles_total / kScanChunk + 1)) +
           aligned_bytes(sizeof(int) * Ntot) + aligned_bytes(sizeof(uint32_t) * Ntot) +
           2 * aligned_bytes(2 * rsize * Ntot) + aligned_bytes(sizeof(Sub) * max_sub) + aligned_bytes(sizeof(int)) +
           aligned_bytes(2 * rsize * (size_t)gg.L * gg.L * max_sub) + aligned_bytes(sizeof(int) * (size_t)ntiles_total) +
           aligned_bytes(sizeof(int)) + aligned_bytes(sizeof(int) * (size_t)(Ntot / kChunk + 2));
}

SpreadBufs spread_carve(fh_ctx* c, int64_t Ntot, const GridGeom& gg, int ntiles_total, size_t rsize)
{
    SpreadBufs b;
    b.max_sub = Ntot / gg.P + std::min<int64_t>(Ntot, ntiles_total) + 1;
    b.cnt = c->tile_cnt;  // persistent, zero between calls (counters_ready)
    b.off = c->arena.take<int>(ntiles_total);
    b.tsub = c->arena.take<int>(2 * (size_t)ntiles_total);
    b.rank = c->arena.take<int>(Ntot);
    b.cell = c->arena.take<uint32_t>(Ntot);
    b.dd = c->arena.take<char>(2 * rsize * Ntot);
    b.cc = c->arena.take<char>(2 * rsize * Ntot);
    b.subs = c->arena.take<Sub>(b.max_sub);
    b.nsub = c->arena.take<int>(1);
    b.bsum = c->arena.take<int>(2 * (size_t)(ntiles_total / kScanChunk + 1));
    b.slots = c->arena.take<char>(2 * rsize * (size_t)gg.L * gg.L * b.max_sub);
    b.list = c->arena.take<int>((size_t)ntiles_total);
    b.nlist = c->arena.take<int>(1);
    b.chunk = c->arena.take<int>((size_t)(Ntot / kChunk + 2));
    b.key = b.key_sorted = nullptr;
    b.vals = b.vals_sorted = nullptr;
    b.sort_tmp = nullptr;
    b.sort_bytes = 0;
    if (c->opt.deterministic) {
        b.key = c->arena.take<uint32_t>(Ntot);
        b.key_sorted = c->arena.take<uint32_t>(Ntot);
        b.vals = c->arena.take<int>(Ntot);
        b.vals_sorted = c->arena.take<int>(Ntot);
        b.sort_bytes = tile_sort_bytes(Ntot);
        b.sort_tmp = c->arena.take<char>(b.sort_bytes);
    }
    return b;
}

// How many tiles on a padded tile reaches, also through the wrap of the
// period, where a partial last tile brings the next tiles closer.
inline int tile_reach(const GridGeom& gg)
{
    return (gg.L - 1 + std::max(gg.padx, gg.wrap_y ? gg.pady : 0)) / gg.T;
}

// Bin and spread into slots, then merge the slots of each tile's work items
// (the reduce follows: reduce_grid, or the type-1 row pass that fuses it).
template <class R>
fh_status spread_items(fh_ctx* c, const InstParams& p0, const InstParams* table, int ninst, int64_t Ntot,
                       const GridGeom& gg, const SpreadBufs& b, double beta, const void* poly)
{
    const int tpi = gg.ntx * gg.nty;
    const int ntiles_total = tpi * ninst;
    // the counters are zero on entry (counters_ready) and k_reduce_tiles
    // zeroes them again; until it is enqueued they count as dirty
    c->tile_cnt_dirty = true;
    if (Ntot > 0) {
        if (table)
            hipLaunchKernelGGL(k_chunk_inst, dim3(nblocks(Ntot / kChunk + 2, 256)), dim3(256), 0, c->stream, table,
                               ninst, Ntot, b.chunk);
        if (table)
            hipLaunchKernelGGL((k_bin_count<kBinBlockBatch, kBinNodesBatch, kBinKeyBitsBatch>),
                               dim3(nblocks(Ntot, kBinBlockBatch * kBinNodesBatch)), dim3(kBinBlockBatch), 0,
                               c->stream, p0, table, (const int*)b.chunk, Ntot, gg, b.cnt, b.rank, b.key, b.vals);
        else
            hipLaunchKernelGGL((k_bin_count<kBinBlock, 1, kBinKeyBits>), dim3(nblocks(Ntot, kBinBlock)),
                               dim3(kBinBlock), 0, c->stream, p0, table, (const int*)b.chunk, Ntot, gg, b.cnt,
                               b.rank, b.key, b.vals);
        if (b.key) {
            int bits = 1;
            while (bits < 32 && ((int64_t)1 << bits) < ntiles_total) ++bits;
            FH_TRY(tile_sort(c, b.key, b.key_sorted, b.vals, b.vals_sorted, Ntot, bits, b.sort_tmp, b.sort_bytes));
        }
    }
    const int nscan = std::max(1, (ntiles_total + kScanChunk - 1) / kScanChunk);
    if (nscan > 1)
        hipLaunchKernelGGL(k_scan_sums, dim3(nscan), dim3(kScanThreads), 0, c->stream, b.cnt, ntiles_total, gg.P,
                           b.bsum);
    hipLaunchKernelGGL(k_scan_tiles, dim3(nscan), dim3(kScanThreads), 0, c->stream, b.cnt, ntiles_total, gg.P,
                       b.bsum, b.off, b.tsub, b.nsub, b.nlist);
    if (Ntot > 0 && b.key)
        hipLaunchKernelGGL(k_rank_sorted, dim3(nblocks(Ntot, 256)), dim3(256), 0, c->stream, b.key_sorted,
                           b.vals_sorted, Ntot, b.off, b.rank);
    if (Ntot > 0) {
        hipLaunchKernelGGL((k_bin_place<R>), dim3(nblocks(Ntot, 256 * kPlaceNodes)), dim3(256), 0, c->stream, p0, table,
                           (const int*)b.chunk, Ntot, gg, b.cnt, b.off, b.tsub, b.rank, b.cell, (typename V2<R>::T*)b.dd,
                           (typename V2<R>::T*)b.cc, b.subs);
    }
    FH_HIP(hipGetLastError());
    timing_mark(c, 1);
    if (Ntot > 0) {
        // one block per work item up to a few waves of the whole chip
        // (wavefront blocks: as many as fit in LDS, at most 32 per CU)
        const int64_t per_cu = gg.method == 1 ? 8 : std::min<int64_t>(32, kCuLds / spread_lds(gg, sizeof(R)));
        // (the matrix-core spread takes kMfmaWaves items per block)
        const int64_t items_per_block = gg.method == 5 ? kMfmaWaves : 1;
        const unsigned grid = (unsigned)std::max<int64_t>(
            1, std::min<int64_t>((b.max_sub + items_per_block - 1) / items_per_block,
                                 (int64_t)c->cu_count * std::max<int64_t>(1, per_cu) * 4));
        FH_TRY(launch_spread<R>(c, grid, b.subs, b.nsub, b.cell, b.dd, b.cc, (typename V2<R>::T*)b.slots, gg, tpi,
                                beta, poly));
    }
    timing_mark(c, 2);
    if (Ntot > 0) {
        const int64_t LL = (int64_t)gg.L * gg.L;
        const unsigned mgrid =
            (unsigned)std::max<int64_t>(1, std::min<int64_t>((b.max_sub + kMergeChunk - 1) / kMergeChunk,
                                                            (int64_t)c->cu_count * 16));
        for (int level = 1; level <= kMergeLevels; ++level)
            hipLaunchKernelGGL((k_merge_slots<R>), dim3(mgrid), dim3(256), 0, c->stream,
                               (typename V2<R>::T*)b.slots, b.subs, b.nsub, b.tsub, (int)LL, level);
        FH_HIP(hipGetLastError());
    }
    return FH_OK;
}

// Reduce the merged slots into F: B instances x rows x nf1, or with rwin
// (device, one (rows, first row) per instance) each instance's own rows one
// after another, total_rows in all.
template <class R>
fh_status reduce_grid(fh_ctx* c, int ninst, const GridGeom& gg, const SpreadBufs& b, R* F,
                      const int2* rwin = nullptr, int64_t total_rows = -1)
{
    if (total_rows < 0) total_rows = (int64_t)ninst * gg.rows;
    const int tpi = gg.ntx * gg.nty;
    const int ntiles_total = tpi * ninst;
    const unsigned rgrid = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>(ntiles_total, (int64_t)c->cu_count * 16));
    const int reach = tile_reach(gg);
    const int TT = gg.T * gg.T;
    const unsigned rthreads = (unsigned)std::min(256, TT);
    FH_ARG(reach >= 1 && reach <= (TT > 256 ? 1 : 2) && TT <= 1024, FH_ERR_UNSUPPORTED,
           "tile %d with width %d", gg.T, gg.W);
#define FH_REDUCE(RE, K)                                                                                     \
    hipLaunchKernelGGL((k_reduce_tiles<R, RE, K>), dim3(rgrid), dim3(rthreads), 0, c->stream,                \
                       (const typename V2<R>::T*)b.slots, b.tsub, gg, tpi, ntiles_total, F, b.cnt, rwin)
#define FH_REDUCE_CELLS(RE)                                                                                  \
    do {                                                                                                     \
        hipLaunchKernelGGL((k_tile_active<RE>), dim3(nblocks(ntiles_total, 256)), dim3(256), 0, c->stream,   \
                           b.tsub, gg, tpi, ntiles_total, b.list, b.nlist, b.cnt);                           \
        hipLaunchKernelGGL((k_reduce_list<R, RE>), dim3(lgrid), dim3(256), 0, c->stream,                      \
                           (const typename V2<R>::T*)b.slots, b.tsub, (const int*)b.list, (const int*)b.nlist, \
                           gg, tpi, F, rwin);                                                                \
    } while (0)
    // Tiles under 128 cells (the matrix-core spread's), and grids of 4M
    // cells or more (mostly empty in a batch), are reduced a thread per cell:
    // by strips of one tile row (one launch, every cell written once) when
    // the strip's heads fit in LDS, else from the list of reached tiles after
    // a zero fill (three launches).  Small grids of larger tiles take one
    // launch, a tile per block.
    const bool by_cell = TT < 128 || (int64_t)ntiles_total * TT >= ((int64_t)1 << 22);
    const size_t slds = reduce_strips_lds(reach, gg.ntx);
    const bool strips = by_cell && slds <= kLdsBudget && ninst <= 65535;
    const unsigned lgrid = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((int64_t)c->cu_count * 8, ((int64_t)ntiles_total * TT + 255) / 256));
    if (strips) {
        // slices per tile row: enough workgroups for 8 per CU, at most a row each
        const int64_t nstrip = (int64_t)gg.nty * ninst;
        const int S = (int)std::min<int64_t>(gg.T, std::max<int64_t>(1, (8 * (int64_t)c->cu_count + nstrip - 1) / nstrip));
        const dim3 sgrid((unsigned)(gg.nty * S), (unsigned)ninst);
        if (reach == 1)
            hipLaunchKernelGGL((k_reduce_strips<R, 1>), sgrid, dim3(256), slds, c->stream,
                               (const typename V2<R>::T*)b.slots, b.tsub, gg, tpi, F, b.cnt, rwin, S);
        else
            hipLaunchKernelGGL((k_reduce_strips<R, 2>), sgrid, dim3(256), slds, c->stream,
                               (const typename V2<R>::T*)b.slots, b.tsub, gg, tpi, F, b.cnt, rwin, S);
    } else if (by_cell) {
        FH_TRY(launch_zero(c, F, 2 * sizeof(R) * (size_t)total_rows * gg.nf1));
        if (reach == 1) FH_REDUCE_CELLS(1);
        else FH_REDUCE_CELLS(2);
    } else if (TT > 256) {
        // T = 32: a padded tile reaches one tile on for every width
        FH_REDUCE(1, 4);
    } else {
        if (reach == 1) FH_REDUCE(1, 1);
        else FH_REDUCE(2, 1);
    }
#undef FH_REDUCE
#undef FH_REDUCE_CELLS
    FH_HIP(hipGetLastError());
    c->tile_cnt_dirty = false;
    return FH_OK;
}

// Bin, spread into slots, and reduce into F (as reduce_grid).
template <class R>
fh_status run_spread(fh_ctx* c, const InstParams& p0, const InstParams* table, int ninst, int64_t Ntot,
                     const GridGeom& gg, const SpreadBufs& b, R* F, double beta, const void* poly,
                     const int2* rwin = nullptr, int64_t total_rows = -1)
{
    FH_TRY(spread_items<R>(c, p0, table, ninst, Ntot, gg, b, beta, poly));
    return reduce_grid<R>(c, ninst, gg, b, F, rwin, total_rows);
}

fh_status check_lz(double lambda, double z)
{
    FH_ARG(std::isfinite(lambda) && std::isfinite(z), FH_ERR_NONFINITE, "lambda or z not finite");
    FH_ARG(lambda * z > 0 && std::isfinite(lambda * z), FH_ERR_NONPOSITIVE_LZ, "lambda * z must be > 0");
    return FH_OK;
}

fh_status check_grid(int n1, int n2, double h1, double h2, double xc, double yc)
{
    FH_ARG(n1 > 0 && n2 > 0, FH_ERR_INVALID_ARG, "grid sizes must be positive");
    FH_ARG(n1 % 2 == 0 && n2 % 2 == 0, FH_ERR_ODD_GRID, "grid sizes must be even (got %d x %d)", n1, n2);
    FH_ARG(std::isfinite(h1) && std::isfinite(h2) && std::isfinite(xc) && std::isfinite(yc), FH_ERR_NONFINITE,
           "grid spacing or centre not finite");
    FH_ARG(h1 > 0 && h2 > 0, FH_ERR_INVALID_ARG, "grid spacing must be positive");
    FH_ARG(n1 <= 32768 && n2 <= 32768, FH_ERR_UNSUPPORTED, "grid sides up to 32768");
    return FH_OK;
}

// Spread method: the option when set, else auto_method (the wavefront spread
// for type 3, whose grids are small and points crowd; t1_method for type 1).
// The work-item size is set per call.
void spread_defaults(const fh_ctx* c, GridGeom& g, int auto_method = 2)
{
    g.method = c->opt.spread_method > 0 ? c->opt.spread_method : auto_method;
    // the thread-per-point spread adds to a shared tile with atomics in no
    // fixed order
    if (g.method == 1 && c->opt.deterministic) g.method = 2;
    // the register tile needs T = 8 or 16, a padded tile row within one
    // wavefront and its four tiles within the LDS budget
    if (g.method == 4 && !((g.T == 8 || g.T == 16) && g.L <= 64 &&
                           spread_lds(g, c->prec == FH_FP64 ? 8 : 4) <= kLdsBudget))
        g.method = 2;
    // the matrix-core spread holds at most 32 x 32 cells, and its staging
    // must fit the LDS budget
    if (g.method == 5 && (g.L > 32 || mfma_spread_lds(g.L <= 16 ? 1 : 2, g.T, c->prec == FH_FP64 ? 8 : 4) > kLdsBudget))
        g.method = 2;
    g.P = c->opt.max_subproblem > 0 ? c->opt.max_subproblem : 0;
}

// Points per work item for Ntot nodes: the option when set, else enough for
// about 96 work items per CU (at least 64 points): small rules then spread
// over the whole chip, and large batches do not pay one slot per few hundred
// points.  A tile's items still hold at least count / kMaxSubPerTile points.
void size_items(const fh_ctx* c, GridGeom& g, int64_t Ntot)
{
    if (c->opt.max_subproblem > 0) {
        g.P = c->opt.max_subproblem;
        return;
    }
    const int64_t target = (int64_t)c->cu_count * 96;
    g.P = (int)std::min<int64_t>(1 << 24, std::max<int64_t>(64, (Ntot + target - 1) / target));
}

// Type-1 geometry for an n1 x n2 grid and N nodes in all (N < 0: not
// known); the row window is set per call.
T1Plan plan_t1(fh_ctx* c, int n1, int n2, int64_t N)
{
    T1Plan p;
    p.k = choose_kernel(c, std::max(n1, n2));
    if (!p.k.clamped) es_poly_attach(c, p.k);
    const int W = p.k.w;
    const int need1 = std::max((int)std::ceil(p.k.sigma * n1), 2 * W);
    const int need2 = std::max((int)std::ceil(p.k.sigma * n2), 2 * W);
    int method = t1_method(c, W, N);
    int T = pick_tile(c, std::min(need1, need2), W, N);
    if (c->prec == FH_FP64 && T > 32) T = 32;
    GridGeom& g = p.gg;
    g.T = T;
    g.W = W;
    g.L = T + W - 1;
    // power-of-two tiles divide the grid; other tiles (the matrix-core
    // spread's 16-cell padded tiles) leave a partial last tile and keep the
    // grid lengths of 16-cell tiles
    const int step = (T & (T - 1)) == 0 ? T : 16;
    g.nf1 = next_fft_size(std::max(need1, T + W), step);
    g.nf2 = next_fft_size(std::max(need2, T + W), step);
    g.ntx = (g.nf1 + T - 1) / T;
    g.nty = (g.nf2 + T - 1) / T;
    g.rows = g.nf2;
    g.wrap_y = 1;
    g.padx = g.ntx * T - g.nf1;
    g.pady = g.nty * T - g.nf2;
    // the tile reduce follows a padded tile at most two tiles on (one for
    // tiles over 256 cells); a partial last tile brings the wrapped ones
    // closer, so a tile that does not divide the grid falls back to 16
    if ((T & (T - 1)) != 0 && (g.L - 1 + std::max(g.padx, g.pady)) / T > (T * T > 256 ? 1 : 2)) {
        T = 16;
        g.T = T;
        g.L = T + W - 1;
        g.ntx = g.nf1 / T;
        g.nty = g.nf2 / T;
        g.padx = g.pady = 0;
        // a 16-cell tile's padded tile takes 2 x 2 blocks of matrix-core
        // products, four times the work: the chosen spread becomes the
        // wavefront spread unless the caller asked for this one
        if (c->opt.spread_method <= 0) method = 2;
    }
    spread_defaults(c, g, method);
    return p;
}

// Rows of the fine grid an instance's nodes can reach: first row (shift) and
// count, from the rule's bounding box in y (s2 > 0).
void window_rows(const double* bb, double s2, int W, int& lo, int& span)
{
    lo = (int)std::floor(bb[2] * s2 - 0.5 * W) - 1;
    const int hi = (int)std::ceil(bb[3] * s2 - 0.5 * W) + W + 1;
    span = hi - lo;
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
    // source chirp with the pre-phase of a grid centred at (xc, yc):
    // pi (|x|^2 - 2 (xc x + yc y)) / (lambda z), in turns; a point source at
    // distance D adds pi |x|^2/(lambda D) (its incident wave)
    ip.pa = 0.5 / lz + (q->D > 0.0 ? 0.5 / (lambda * q->D) : 0.0);
    ip.src = q->src;
    ip.px = -xc / lz;
    ip.py = -yc / lz;
    ip.pc = 0.0;
    // rescaled node x~ = 2 pi h x/(lambda z), in fine-grid cells of 2 pi/nf
    ip.s1 = h1 * g.nf1 / lz;
    ip.s2 = h2 * g.nf2 / lz;
    return ip;
}

}  // namespace
}  // namespace fh

// fh_adjoint.hip -- vector-Jacobian products of the grid field.
//
// For a real loss L with cotangent g_k = dL/dRe(u_k) + i dL/dIm(u_k) at the
// grid targets xi_k, and a_k = s conj(g_k) (s = -1 for an occulter, since
// u_oc = 1 - u_ap), the derivatives of the quadrature sum of eq. faq are
//   dL/dw_j = Re[G_j/(i lambda z)],
//   dL/dx_j = (2 pi w_j/(lambda z)^2) Re[x_j G_j - Hx_j],  y likewise,
// with G_j = sum_k a_k E_kj, Hx_j = sum_k a_k E_kj xi_k, Hy_j likewise, and
// E_kj = exp(i pi |xi_k - x_j|^2/(lambda z)).  Expanding the square as in eq.
// split, with xi_k = (xc, yc) + (h1 k1, h2 k2):
//   G_j = P_j sum_k b_k exp(-i (k1 x~_j + k2 y~_j)),  b_k = a_k exp(i pi |xi_k|^2/(lambda z)),
// P_j = exp(i pi (|x_j|^2 - 2 (xc x_j + yc y_j))/(lambda z)) (the forward
// strength phase), and x~ = 2 pi h1 x/(lambda z) as in the type-1 transform.
// So G, Hx, Hy are three type-2 NUFFTs with coefficients b, xi b, eta b that
// share one set of kernel weights at each node: deconvolve, a first FFT pass
// over the n1 needed columns, a transpose that keeps only the fine-grid rows
// the nodes can reach, a second pass over those rows, and an ES-kernel gather
// at the nodes.  The starshade product then chains (dL/dx, dL/dy, dL/dw)
// through the perturbed petal construction to the edge coefficients.
#include "fh_kernels.hpp"

namespace fh {
namespace {

struct AdjParams {
    int n1, n2, nf1, nf2, rows, sh2;
    double h1, h2, xc, yc;
    double inv2lz;
    double sign;  // +1 aperture, -1 occulter
    const double* iphi1;
    const double* iphi2;
};

// Zt[ch][c][r] (c = k1 + n1/2, r = k2 mod nf2, zero where |k2| is beyond the
// grid) from the cotangent g[k2 + n2/2][k1 + n1/2]: channels b, xi b, eta b,
// deconvolved by the kernel transform.
template <class R>
__global__ void __launch_bounds__(256) k_adj_prep(const R* __restrict__ gu, R* __restrict__ Zt, AdjParams ap)
{
    using C2 = typename V2<R>::T;
    __shared__ C2 t[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const C2* g = reinterpret_cast<const C2*>(gu);
    for (int k = ty; k < 32; k += 8) {
        const int r = r0 + k, k1i = c0 + tx;
        const int k2 = r < ap.nf2 / 2 ? r : r - ap.nf2;
        C2 v;
        v.x = R(0);
        v.y = R(0);
        if (r < ap.nf2 && k1i < ap.n1 && k2 >= -(ap.n2 / 2) && k2 < ap.n2 - ap.n2 / 2)
            v = g[(size_t)(k2 + ap.n2 / 2) * ap.n1 + k1i];
        t[k][tx] = v;
    }
    __syncthreads();
    C2* Z = reinterpret_cast<C2*>(Zt);
    const size_t plane = (size_t)ap.n1 * ap.nf2;
    for (int k = ty; k < 32; k += 8) {
        const int k1i = c0 + k, r = r0 + tx;
        if (k1i >= ap.n1 || r >= ap.nf2) continue;
        const int k2 = r < ap.nf2 / 2 ? r : r - ap.nf2;
        C2 b0, b1, b2;
        b0.x = b0.y = b1.x = b1.y = b2.x = b2.y = R(0);
        if (k2 >= -(ap.n2 / 2) && k2 < ap.n2 - ap.n2 / 2) {
            const C2 gv = t[tx][k];
            const int k1 = k1i - ap.n1 / 2;
            const double xi = ap.xc + ap.h1 * k1, eta = ap.yc + ap.h2 * k2;
            // a = s conj(g); b = a exp(i pi |xi|^2/lz) / (Phi(k1) Phi(k2))
            const double ar = ap.sign * (double)gv.x, ai = -ap.sign * (double)gv.y;
            const double tt = (xi * xi + eta * eta) * ap.inv2lz;
            const double f = tt - rint(tt);
            double s, c;
            sincospi(2.0 * f, &s, &c);
            const double sc = ap.iphi1[k1i] * ap.iphi2[k2 + ap.n2 / 2];
            const double br = (ar * c - ai * s) * sc, bi = (ar * s + ai * c) * sc;
            b0.x = (R)br;
            b0.y = (R)bi;
            b1.x = (R)(xi * br);
            b1.y = (R)(xi * bi);
            b2.x = (R)(eta * br);
            b2.y = (R)(eta * bi);
        }
        const size_t o = (size_t)k1i * ap.nf2 + r;
        Z[o] = b0;
        Z[plane + o] = b1;
        Z[2 * plane + o] = b2;
    }
}

// F1[ch][row][col] = Zt[ch][k1 + n1/2][(sh2 + row) mod nf2] for the fine-grid
// columns col = k1 mod nf1 of the grid's modes, zero for the other columns.
template <class R>
__global__ void __launch_bounds__(256) k_adj_transpose(const R* __restrict__ Zt, R* __restrict__ F1, AdjParams ap)
{
    using C2 = typename V2<R>::T;
    __shared__ C2 t[32][33];
    const int col0 = blockIdx.x * 32, row0 = blockIdx.y * 32, ch = blockIdx.z;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const C2* Z = reinterpret_cast<const C2*>(Zt) + (size_t)ch * ap.n1 * ap.nf2;
    for (int k = ty; k < 32; k += 8) {
        const int col = col0 + k, row = row0 + tx;
        const int k1 = col < ap.nf1 / 2 ? col : col - ap.nf1;
        C2 v;
        v.x = R(0);
        v.y = R(0);
        if (col < ap.nf1 && row < ap.rows && k1 >= -(ap.n1 / 2) && k1 < ap.n1 - ap.n1 / 2) {
            int r = (ap.sh2 + row) % ap.nf2;
            if (r < 0) r += ap.nf2;
            v = Z[(size_t)(k1 + ap.n1 / 2) * ap.nf2 + r];
        }
        t[k][tx] = v;
    }
    __syncthreads();
    C2* F = reinterpret_cast<C2*>(F1) + (size_t)ch * ap.rows * ap.nf1;
    for (int k = ty; k < 32; k += 8) {
        const int row = row0 + k, col = col0 + tx;
        if (row < ap.rows && col < ap.nf1) F[(size_t)row * ap.nf1 + col] = t[tx][k];
    }
}

// Gather the three channels at each node with the ES kernel, then form the
// node gradients (written, or with ACC added to what the outputs hold).  A
// wavefront takes up to 64 nodes at a time: lane l first finds node l's
// stencil cell and its 2W kernel values (staged in LDS); the wavefront then
// gathers in trips of 64/GS nodes, GS lanes per node, lane r taking stencil
// column r down all W rows of the three channels (3W loads in flight, and
// each load instruction reads, per node, a contiguous run of a row rather
// than one line per lane, as the type-3 interpolation does); the column is
// weighted down its rows, then by its own kernel value, and summed over the
// group by a fixed butterfly.  Lane l finally forms node l's gradients.
template <class R, int W, bool ACC>
__global__ void __launch_bounds__(64) k_adj_gather(const R* __restrict__ F1, InstParams ip, GridGeom gg, R beta,
                                                   const R* __restrict__ poly, double lz, int tpw,
                                                   double* __restrict__ gx, double* __restrict__ gy,
                                                   double* __restrict__ gw)
{
    using C = typename V2<R>::T;
    constexpr int GS = interp_group<W>();
    constexpr int NT = 64 / GS;
    constexpr int KS = 2 * W + 1;
    __shared__ R ks[64 * KS];
    __shared__ uint32_t cs[64];
    __shared__ C res[3][64];
    const int lane = threadIdx.x, g = lane / GS, r = lane % GS;
    const C* F = reinterpret_cast<const C*>(F1);
    const size_t plane = (size_t)gg.rows * gg.nf1;
    for (int64_t base = blockIdx.x * (int64_t)tpw; base < ip.N; base += (int64_t)gridDim.x * tpw) {
        const int64_t j = base + lane;
        const bool live = lane < tpw && j < ip.N;
        const int64_t k = live ? j : 0;
        const double x = ip.x[k], y = ip.y[k];
        int l1, l2;
        double d1, d2;
        const bool ok = node_cell(ip, gg, x, y, l1, l2, d1, d2);
        if (!ok) {
            // a node outside the window: gathered from cell 0 with any
            // weights, its gradients are zero
            l1 = l2 = 0;
            d1 = d2 = 0.0;
        }
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
        wave_lds_order();
        const int nq = (int)min<int64_t>(tpw, ip.N - base);
        const int rr = min(r, W - 1);
        for (int q0 = 0; q0 < nq; q0 += NT) {
            const int q = q0 + g, qq = min(q, nq - 1);
            const uint32_t cp = cs[qq];
            int col = (int)(cp & 0xffffu) + rr;
            col = col >= gg.nf1 ? col - gg.nf1 : col;
            const int row0 = (int)(cp >> 16);
            C v0[W], v1[W], v2[W];
#pragma unroll
            for (int b = 0; b < W; ++b) {
                int row = row0 + b;
                if (row >= gg.rows) row -= gg.rows;  // periodic only when the rows are the whole period
                const size_t e = (size_t)row * gg.nf1 + col;
                v0[b] = F[e];
                v1[b] = F[plane + e];
                v2[b] = F[2 * plane + e];
            }
            const R* kq = ks + qq * KS;
            R s0r = 0, s0i = 0, s1r = 0, s1i = 0, s2r = 0, s2i = 0;
#pragma unroll
            for (int b = 0; b < W; ++b) {
                const R kb = kq[W + b];
                s0r += v0[b].x * kb;
                s0i += v0[b].y * kb;
                s1r += v1[b].x * kb;
                s1i += v1[b].y * kb;
                s2r += v2[b].x * kb;
                s2i += v2[b].y * kb;
            }
            const R kx = (q < nq && r < W) ? kq[rr] : R(0);
            s0r = group_sum<GS>(s0r * kx);
            s0i = group_sum<GS>(s0i * kx);
            s1r = group_sum<GS>(s1r * kx);
            s1i = group_sum<GS>(s1i * kx);
            s2r = group_sum<GS>(s2r * kx);
            s2i = group_sum<GS>(s2i * kx);
            if (r == 0 && q < nq) {
                res[0][q] = C{s0r, s0i};
                res[1][q] = C{s1r, s1i};
                res[2][q] = C{s2r, s2i};
            }
        }
        wave_lds_order();
        if (live) {
            double ox = 0.0, oy = 0.0, ow = 0.0;
            if (ok) {
                const C t0 = res[0][lane], t1 = res[1][lane], t2 = res[2][lane];
                // P_j = exp(2 pi i t), t = the forward strength phase in turns
                const double t = ((x * x + y * y) * ip.pa + (x * ip.px + y * ip.py)) + ip.pc;
                const double f = t - rint(t);
                double sn, c;
                sincospi(2.0 * f, &sn, &c);
                const double Gr = c * (double)t0.x - sn * (double)t0.y, Gi = sn * (double)t0.x + c * (double)t0.y;
                const double Hxr = c * (double)t1.x - sn * (double)t1.y;
                const double Hyr = c * (double)t2.x - sn * (double)t2.y;
                const double fac = 2.0 * kPi * ip.w[k] / (lz * lz);
                ow = Gi / lz;
                ox = fac * (x * Gr - Hxr);
                oy = fac * (y * Gr - Hyr);
            }
            if (ACC) {
                gx[j] += ox;
                gy[j] += oy;
                gw[j] += ow;
            } else {
                gx[j] = ox;
                gy[j] = oy;
                gw[j] = ow;
            }
        }
        wave_lds_order();
    }
}

// The same gradients when the three channels' cells that the nodes reach
// fit in LDS (a rule whose nodes crowd a few cells, as a starshade does on a
// pupil grid): each block first copies that window -- every held row, the
// span1 columns from (col0 mod nf1) on -- into LDS, then a thread per node
// gathers its W x W cells of each channel from there.  The window comes
// from the rule's bounding box (with a cell of margin), so every node's
// stencil lies inside it; reads are clamped to the window all the same.
template <class R, int W, bool ACC>
__global__ void __launch_bounds__(256) k_adj_gather_lds(const R* __restrict__ F1, InstParams ip, GridGeom gg, R beta,
                                                        const R* __restrict__ poly, double lz, int col0, int span1,
                                                        double* __restrict__ gx, double* __restrict__ gy,
                                                        double* __restrict__ gw)
{
    using C = typename V2<R>::T;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    C* win = reinterpret_cast<C*>(lds_raw);
    const C* F = reinterpret_cast<const C*>(F1);
    const size_t plane = (size_t)gg.rows * gg.nf1;
    const int wplane = gg.rows * span1;
    for (int e = threadIdx.x; e < 3 * wplane; e += blockDim.x) {
        const int ch = e / wplane, rem = e - ch * wplane;
        const int row = rem / span1, wc = rem - row * span1;
        int col = (col0 + wc) % gg.nf1;
        if (col < 0) col += gg.nf1;
        win[e] = F[ch * plane + (size_t)row * gg.nf1 + col];
    }
    __syncthreads();
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < ip.N; j += (int64_t)gridDim.x * blockDim.x) {
        const double x = ip.x[j], y = ip.y[j];
        int l1, l2;
        double d1, d2;
        double ox = 0.0, oy = 0.0, ow = 0.0;
        if (node_cell(ip, gg, x, y, l1, l2, d1, d2)) {
            R k1[W];
            es_weights<R, W>((R)d1, beta, poly, k1);
            int wc0 = (l1 - col0) % gg.nf1;
            if (wc0 < 0) wc0 += gg.nf1;
            wc0 = min(wc0, span1 - W);
            const int r0 = min(l2, gg.rows - W);
            // the row kernel values too, once per node (a row index into the
            // table inside the loop made the compiler keep the whole table in
            // registers); the rows are unrolled, each row's loads issued
            // after the previous row's sums
            R k2[W];
            es_weights<R, W>((R)d2, beta, poly, k2);
            R t0r = 0, t0i = 0, t1r = 0, t1i = 0, t2r = 0, t2i = 0;
#pragma unroll
            for (int b = 0; b < W; ++b) {
                const C* wr = win + (r0 + b) * span1 + wc0;
                R a0r = 0, a0i = 0, a1r = 0, a1i = 0, a2r = 0, a2i = 0;
#pragma unroll
                for (int a = 0; a < W; ++a) {
                    const C v0 = wr[a], v1 = wr[wplane + a], v2 = wr[2 * wplane + a];
                    a0r += v0.x * k1[a];
                    a0i += v0.y * k1[a];
                    a1r += v1.x * k1[a];
                    a1i += v1.y * k1[a];
                    a2r += v2.x * k1[a];
                    a2i += v2.y * k1[a];
                }
                const R kb = k2[b];
                __builtin_amdgcn_sched_barrier(0);
                t0r += a0r * kb;
                t0i += a0i * kb;
                t1r += a1r * kb;
                t1i += a1i * kb;
                t2r += a2r * kb;
                t2i += a2i * kb;
            }
            // P_j = exp(2 pi i t), t = the forward strength phase in turns
            const double t = ((x * x + y * y) * ip.pa + (x * ip.px + y * ip.py)) + ip.pc;
            const double f = t - rint(t);
            double sn, c;
            sincospi(2.0 * f, &sn, &c);
            const double Gr = c * t0r - sn * t0i, Gi = sn * t0r + c * t0i;
            const double Hxr = c * t1r - sn * t1i;
            const double Hyr = c * t2r - sn * t2i;
            const double fac = 2.0 * kPi * ip.w[j] / (lz * lz);
            ow = Gi / lz;
            ox = fac * (x * Gr - Hxr);
            oy = fac * (y * Gr - Hyr);
        }
        if (ACC) {
            gx[j] += ox;
            gy[j] += oy;
            gw[j] += ow;
        } else {
            gx[j] = ox;
            gy[j] = oy;
            gw[j] = ow;
        }
    }
}

// LDS bytes of the gather's window, or 0 when it does not fit the budget.
inline size_t adj_window_lds(int rows, int span1, size_t rs)
{
    const size_t b = 3 * 2 * rs * (size_t)rows * span1;
    return b <= kLdsBudget ? b : 0;
}

// Nodes per wavefront: 64, halved (down to one gather trip's worth) while
// that leaves fewer than about 4 wavefronts per CU.
template <class R>
fh_status launch_gather(fh_ctx* c, int W, const R* F1, const InstParams& ip, const GridGeom& gg, double beta,
                        const void* poly, double lz, bool acc, int col0, int span1, double* gx, double* gy,
                        double* gw)
{
    const size_t wl = span1 > 0 ? adj_window_lds(gg.rows, span1, sizeof(R)) : 0;
    if (wl > 0) {
        // a block per window copy: as many as keep every CU busy, each
        // walking its share of the nodes
        const unsigned g = (unsigned)std::max<int64_t>(
            1, std::min<int64_t>((ip.N + 255) / 256, (int64_t)c->cu_count * (int64_t)(kCuLds / wl)));
        switch (W) {
#define FH_GATHER_LDS_CASE(w)                                                                                    \
    case w:                                                                                                     \
        if (acc)                                                                                                \
            hipLaunchKernelGGL((k_adj_gather_lds<R, w, true>), dim3(g), dim3(256), wl, c->stream, F1, ip, gg,    \
                               (R)beta, (const R*)poly, lz, col0, span1, gx, gy, gw);                           \
        else                                                                                                    \
            hipLaunchKernelGGL((k_adj_gather_lds<R, w, false>), dim3(g), dim3(256), wl, c->stream, F1, ip, gg,   \
                               (R)beta, (const R*)poly, lz, col0, span1, gx, gy, gw);                           \
        break;
            FH_GATHER_LDS_CASE(2) FH_GATHER_LDS_CASE(3) FH_GATHER_LDS_CASE(4) FH_GATHER_LDS_CASE(5)
            FH_GATHER_LDS_CASE(6) FH_GATHER_LDS_CASE(7) FH_GATHER_LDS_CASE(8) FH_GATHER_LDS_CASE(9)
            FH_GATHER_LDS_CASE(10) FH_GATHER_LDS_CASE(11) FH_GATHER_LDS_CASE(12) FH_GATHER_LDS_CASE(13)
            FH_GATHER_LDS_CASE(14) FH_GATHER_LDS_CASE(15) FH_GATHER_LDS_CASE(16) FH_GATHER_LDS_CASE(17)
            FH_GATHER_LDS_CASE(18) FH_GATHER_LDS_CASE(19) FH_GATHER_LDS_CASE(20)
#undef FH_GATHER_LDS_CASE
        default: set_error("kernel width %d unsupported", W); return FH_ERR_UNSUPPORTED;
        }
        FH_HIP(hipGetLastError());
        return FH_OK;
    }
    const int per_trip = W <= 8 ? 8 : (W <= 16 ? 4 : 2);
    int tpw = 64;
    while (tpw > per_trip && ip.N / tpw < (int64_t)c->cu_count * 4) tpw /= 2;
    const unsigned g = (unsigned)std::min<int64_t>((ip.N + tpw - 1) / tpw, 1 << 20);
    switch (W) {
#define FH_GATHER_CASE(w)                                                                                        \
    case w:                                                                                                     \
        if (acc)                                                                                                \
            hipLaunchKernelGGL((k_adj_gather<R, w, true>), dim3(g), dim3(64), 0, c->stream, F1, ip, gg, (R)beta, \
                               (const R*)poly, lz, tpw, gx, gy, gw);                                            \
        else                                                                                                    \
            hipLaunchKernelGGL((k_adj_gather<R, w, false>), dim3(g), dim3(64), 0, c->stream, F1, ip, gg,         \
                               (R)beta, (const R*)poly, lz, tpw, gx, gy, gw);                                   \
        break;
        FH_GATHER_CASE(2) FH_GATHER_CASE(3) FH_GATHER_CASE(4) FH_GATHER_CASE(5) FH_GATHER_CASE(6)
        FH_GATHER_CASE(7) FH_GATHER_CASE(8) FH_GATHER_CASE(9) FH_GATHER_CASE(10) FH_GATHER_CASE(11)
        FH_GATHER_CASE(12) FH_GATHER_CASE(13) FH_GATHER_CASE(14) FH_GATHER_CASE(15) FH_GATHER_CASE(16)
        FH_GATHER_CASE(17) FH_GATHER_CASE(18) FH_GATHER_CASE(19) FH_GATHER_CASE(20)
#undef FH_GATHER_CASE
    default: set_error("kernel width %d unsupported", W); return FH_ERR_UNSUPPORTED;
    }
    FH_HIP(hipGetLastError());
    return FH_OK;
}

__global__ void k_zero_doubles(double* __restrict__ p, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// Node gradients of one grid field's cotangent g_u, written to (acc: added
// to) g_x, g_y, g_w.
template <class R>
fh_status grid_vjp_impl(fh_ctx* c, const fh_quad* q, double lambda, double z, int n1, int n2, double h1, double h2,
                        double xc, double yc, int occ, const void* g_u, double* g_x, double* g_y, double* g_w,
                        bool acc = false)
{
    const size_t rs = sizeof(R);
    const double lz = lambda * z;
    const int64_t N = q->N;
    c->timing_kind = 2;
    if (N == 0) return FH_OK;
    T1Plan pl = plan_t1(c, n1, n2, N);
    FH_ARG(!pl.k.clamped, FH_ERR_UNSUPPORTED, "tolerance %g needs a kernel wider than %d at sigma %g", c->tol,
           kMaxWidth, pl.k.sigma);
    GridGeom gg = pl.gg;
    InstParams ip = inst_t1(q, lambda, z, h1, h2, xc, yc, gg);
    double bb[4];
    FH_TRY(quad_bbox(c, q, bb));
    int lo, span;
    window_rows(bb, ip.s2, gg.W, lo, span);
    const int rows = (span + gg.T - 1) / gg.T * gg.T;
    if (rows + gg.T < gg.nf2 && span > 0) {
        gg.rows = rows;
        gg.wrap_y = 0;
        ip.sh2 = lo;
    } else {
        gg.rows = gg.nf2;
        gg.wrap_y = 1;
        ip.sh2 = 0;
    }
    gg.nty = (gg.rows + gg.T - 1) / gg.T;
    gg.pady = gg.nty * gg.T - gg.rows;
    const double* ip1 = nullptr;
    const double* ip2 = nullptr;
    FH_TRY(iphi_table(c, pl.k, n1, gg.nf1, &ip1));
    FH_TRY(iphi_table(c, pl.k, n2, gg.nf2, &ip2));
    FftPlan* fa = nullptr;
    FftPlan* fb = nullptr;
    FH_TRY(fft_plan(c, gg.nf2, 0, 3 * n1, &fa));
    FH_TRY(fft_plan(c, gg.nf1, 0, 3 * gg.rows, &fb));
    const size_t Z_count = 2 * (size_t)3 * n1 * gg.nf2;
    const size_t F_count = 2 * (size_t)3 * gg.rows * gg.nf1;
    FH_TRY(arena_reserve(c, aligned_bytes(rs * Z_count) + aligned_bytes(rs * F_count)));
    R* Zt = c->arena.take<R>(Z_count);
    R* F1 = c->arena.take<R>(F_count);

    AdjParams ap{n1, n2, gg.nf1, gg.nf2, gg.rows, ip.sh2, h1, h2, xc, yc, 0.5 / lz, occ ? -1.0 : 1.0, ip1, ip2};
    timing_mark(c, 0);
    hipLaunchKernelGGL((k_adj_prep<R>), dim3(nblocks(n1, 32), nblocks(gg.nf2, 32)), dim3(256), 0, c->stream,
                       static_cast<const R*>(g_u), Zt, ap);
    FH_HIP(hipGetLastError());
    timing_mark(c, 1);
    timing_mark(c, 2);
    FH_TRY(fft_exec(c, fa, Zt));
    hipLaunchKernelGGL((k_adj_transpose<R>), dim3(nblocks(gg.nf1, 32), nblocks(gg.rows, 32), 3), dim3(256), 0,
                       c->stream, Zt, F1, ap);
    FH_HIP(hipGetLastError());
    FH_TRY(fft_exec(c, fb, F1));
    timing_mark(c, 3);
    // the columns the nodes reach: their box's cells with a cell of margin
    // (as the row window), when the rows are windowed too
    int col0 = 0, span1 = 0;
    if (!gg.wrap_y) {
        const double a0 = std::ceil(bb[0] * ip.s1 - 0.5 * gg.W) - 1.0;
        const double a1 = std::ceil(bb[1] * ip.s1 - 0.5 * gg.W) + gg.W + 1.0;
        if (a1 - a0 < gg.nf1 && std::fabs(a0) < 1e9) {
            col0 = (int)a0;
            span1 = (int)(a1 - a0);
        }
    }
    FH_TRY(launch_gather<R>(c, gg.W, F1, ip, gg, pl.k.beta, pl.k.poly, lz, acc, col0, span1, g_x, g_y, g_w));
    timing_mark(c, 4);
    timing_mark(c, 5);
    return FH_OK;
}

// ---------------------------------------------------- starshade chain rule
struct SsParams {
    int Np, m, np, K;
    double a, R, b, p;
    int64_t off;   // first petal node
    int chunk;     // petal nodes per block
    int nchunks;
};

constexpr int kCoefGroup = 16;

// Partial sums of dL/dc+-_{k,s} over one chunk of petal k's nodes, for the
// coefficient group s in [s0, s0 + kCoefGroup).  With s_s(r) = sin(s pi
// (r-a)/(R-a)): dphi/dc+_s = s_s (1 + tau)/(2r), dphi/dc-_s = s_s (tau - 1)/(2r),
// dw/dc+-_s = w_r w_t s_s / 2, d(x, y)/dphi = (-y, x).
__global__ void __launch_bounds__(128) k_ss_vjp_partial(SsParams sp, int s0, const double* __restrict__ glm,
                                                        const double* __restrict__ gln,
                                                        const double* __restrict__ coef,
                                                        const double* __restrict__ gx, const double* __restrict__ gy,
                                                        const double* __restrict__ gw, double* __restrict__ part)
{
    const int k = blockIdx.y, ch = blockIdx.x;
    const int per = sp.np * sp.m;
    const int t0 = ch * sp.chunk, t1 = min(per, t0 + sp.chunk);
    const int ns = min(kCoefGroup, sp.K - s0);
    double accp[kCoefGroup], accm[kCoefGroup];
#pragma unroll
    for (int s = 0; s < kCoefGroup; ++s) accp[s] = accm[s] = 0.0;
    const double L = sp.R - sp.a;
    const double* cp = coef + 2 * (int64_t)k * sp.K;
    for (int t = t0 + (int)threadIdx.x; t < t1; t += blockDim.x) {
        const int i = t / sp.m, l = t - i * sp.m;
        const double r = sp.a + 0.5 * L * (1.0 + glm[l]);
        const double wr = 0.5 * L * glm[sp.m + l];
        const double tau = gln[i], wt = gln[sp.np + i];
        const double A = exp(-pow((r - sp.a) / sp.b, sp.p));
        // sin(s theta), s = 1..K, by the three-term recurrence
        // sin((s+1) theta) = 2 cos(theta) sin(s theta) - sin((s-1) theta), as
        // the rule kernel evaluates them
        const double u = (r - sp.a) / L;
        double s1, c1;
        sincospi(u, &s1, &c1);
        double dp = 0.0, dm = 0.0;
        {
            double sm = 0.0, sk = s1;
            for (int s = 1; s <= sp.K; ++s) {
                dp += cp[s - 1] * sk;
                dm += cp[sp.K + s - 1] * sk;
                const double sn = 2.0 * c1 * sk - sm;
                sm = sk;
                sk = sn;
            }
        }
        // the group's sin((s0 + q + 1) theta), q < kCoefGroup, by the same
        // recurrence from sin(s0 theta)
        double sg[kCoefGroup];
        {
            double sa, ca;
            sincospi(s0 * u, &sa, &ca);
            double prev = sa, cur = sa * c1 + ca * s1;
#pragma unroll
            for (int q = 0; q < kCoefGroup; ++q) {
                sg[q] = cur;
                const double nx = 2.0 * c1 * cur - prev;
                prev = cur;
                cur = nx;
            }
        }
        const double mid = (dp - dm) / (2.0 * r);
        const double half = kPi * A / sp.Np + (dp + dm) / (2.0 * r);
        const double phi = 2.0 * kPi * k / sp.Np + mid + half * tau;
        double sn, cs;
        sincos(phi, &sn, &cs);
        const double x = r * cs, y = r * sn;
        const int64_t j = sp.off + (int64_t)k * per + t;
        const double dphi = gx[j] * (-y) + gy[j] * x;
        const double dwc = gw[j] * wr * wt * 0.5;
        const double up = dphi * (1.0 + tau) / (2.0 * r), um = dphi * (tau - 1.0) / (2.0 * r);
#pragma unroll
        for (int s = 0; s < kCoefGroup; ++s) {
            if (s < ns) {
                accp[s] += up * sg[s] + dwc * sg[s];
                accm[s] += um * sg[s] + dwc * sg[s];
            }
        }
    }
    // block reduction of the 2 kCoefGroup sums (fixed order)
    __shared__ double red[2 * kCoefGroup][128];
#pragma unroll
    for (int s = 0; s < kCoefGroup; ++s) {
        red[s][threadIdx.x] = accp[s];
        red[kCoefGroup + s][threadIdx.x] = accm[s];
    }
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int q = 0; q < 2 * kCoefGroup; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + o];
        __syncthreads();
    }
    if ((int)threadIdx.x < 2 * ns) {
        const int q = threadIdx.x;
        const int s = q < ns ? q : q - ns;
        const int sign = q < ns ? 0 : 1;  // 0: c+, 1: c-
        const double v = red[sign ? kCoefGroup + s : s][0];
        part[((int64_t)k * sp.nchunks + ch) * 2 * sp.K + sign * sp.K + s0 + s] = v;
    }
}

// g_coef[2 k K + j] = sum over chunks (fixed order).
__global__ void k_ss_vjp_final(SsParams sp, const double* __restrict__ part, double* __restrict__ gcoef)
{
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= sp.Np * 2 * sp.K) return;
    const int k = o / (2 * sp.K), jj = o - k * 2 * sp.K;
    double acc = 0.0;
    for (int ch = 0; ch < sp.nchunks; ++ch) acc += part[((int64_t)k * sp.nchunks + ch) * 2 * sp.K + jj];
    gcoef[o] = acc;
}

}  // namespace
}  // namespace fh

using namespace fh;

extern "C" {

fh_status fh_field_grid_vjp(fh_ctx* c, const fh_quad* q, double lambda, double z, int32_t n1, int32_t n2, double h1,
                            double h2, double xc, double yc, int32_t occulter, const void* g_u, double* g_x,
                            double* g_y, double* g_w)
{
    try {
        FH_ARG(c && q, FH_ERR_INVALID_ARG, "NULL argument");
        FH_ARG(q->ctx->device == c->device, FH_ERR_INVALID_ARG, "quadrature lives on another device");
        FH_ARG(q->N == 0 || (g_u && g_x && g_y && g_w), FH_ERR_INVALID_ARG, "NULL array");
        FH_TRY(check_lz(lambda, z));
        FH_TRY(check_grid(n1, n2, h1, h2, xc, yc));
        FH_ARG(q->N < ((int64_t)1 << 31), FH_ERR_UNSUPPORTED, "at most 2^31 - 1 nodes per call");
        FH_ARG(!q->src && !(q->D > 0.0), FH_ERR_UNSUPPORTED,
               "the adjoint covers plane-wave illumination without source terms");
        FH_HIP(hipSetDevice(c->device));
        if (c->prec == FH_FP64)
            return grid_vjp_impl<double>(c, q, lambda, z, n1, n2, h1, h2, xc, yc, occulter, g_u, g_x, g_y, g_w);
        return grid_vjp_impl<float>(c, q, lambda, z, n1, n2, h1, h2, xc, yc, occulter, g_u, g_x, g_y, g_w);
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_field_grid_vjp_sum(fh_ctx* c, const fh_quad* q, int32_t L, const double* lambda, const double* z,
                                int32_t n1, int32_t n2, double h1, double h2, double xc, double yc, int32_t occulter,
                                const void* g_u, double* g_x, double* g_y, double* g_w)
{
    try {
        FH_ARG(c && q && lambda && z, FH_ERR_INVALID_ARG, "NULL argument");
        FH_ARG(L >= 1, FH_ERR_INVALID_ARG, "L must be >= 1");
        FH_ARG(q->ctx->device == c->device, FH_ERR_INVALID_ARG, "quadrature lives on another device");
        FH_ARG(q->N == 0 || (g_u && g_x && g_y && g_w), FH_ERR_INVALID_ARG, "NULL array");
        for (int l = 0; l < L; ++l) FH_TRY(check_lz(lambda[l], z[l]));
        FH_TRY(check_grid(n1, n2, h1, h2, xc, yc));
        FH_ARG(q->N < ((int64_t)1 << 31), FH_ERR_UNSUPPORTED, "at most 2^31 - 1 nodes per call");
        FH_ARG(!q->src && !(q->D > 0.0), FH_ERR_UNSUPPORTED,
               "the adjoint covers plane-wave illumination without source terms");
        FH_HIP(hipSetDevice(c->device));
        const size_t plane = (c->prec == FH_FP64 ? 16 : 8) * (size_t)n1 * n2;
        for (int l = 0; l < L; ++l) {
            const void* gl = static_cast<const char*>(g_u) + plane * l;
            if (c->prec == FH_FP64)
                FH_TRY(grid_vjp_impl<double>(c, q, lambda[l], z[l], n1, n2, h1, h2, xc, yc, occulter, gl, g_x, g_y,
                                             g_w, l > 0));
            else
                FH_TRY(grid_vjp_impl<float>(c, q, lambda[l], z[l], n1, n2, h1, h2, xc, yc, occulter, gl, g_x, g_y,
                                            g_w, l > 0));
        }
        return FH_OK;
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_starshade_vjp(fh_ctx* c, int32_t Np, double a, double R, double b, double p, int32_t m, int32_t np,
                           int32_t nd, int32_t md, const double* coef, int32_t K, const double* g_x,
                           const double* g_y, const double* g_w, double* g_coef)
{
    try {
        FH_ARG(c && coef && g_x && g_y && g_w && g_coef, FH_ERR_INVALID_ARG, "NULL argument");
        FH_ARG(Np >= 1 && m >= 1 && np >= 1 && nd >= 0 && md >= 1, FH_ERR_INVALID_ARG,
               "need Np, m, np, md >= 1 and nd >= 0");
        FH_ARG(K >= 1 && K <= kMaxFourier, FH_ERR_INVALID_ARG, "K must be in [1, %d]", kMaxFourier);
        FH_ARG(std::isfinite(a) && std::isfinite(R) && std::isfinite(b) && std::isfinite(p), FH_ERR_NONFINITE,
               "starshade scalar not finite");
        FH_ARG(a >= 0 && R > a && b > 0 && p > 0, FH_ERR_INVALID_ARG, "need 0 <= a < R, b > 0, p > 0");
        FH_HIP(hipSetDevice(c->device));
        const double* glm = nullptr;
        const double* gln = nullptr;
        FH_TRY(gl_table(c, m, &glm));
        FH_TRY(gl_table(c, np, &gln));
        SsParams sp;
        sp.Np = Np;
        sp.m = m;
        sp.np = np;
        sp.K = K;
        sp.a = a;
        sp.R = R;
        sp.b = b;
        sp.p = p;
        sp.off = (int64_t)nd * md;
        sp.chunk = 1024;
        sp.nchunks = (np * m + sp.chunk - 1) / sp.chunk;
        const size_t npart = (size_t)Np * sp.nchunks * 2 * K;
        FH_TRY(arena_reserve(c, aligned_bytes(sizeof(double) * npart)));
        double* part = c->arena.take<double>(npart);
        for (int s0 = 0; s0 < K; s0 += kCoefGroup)
            hipLaunchKernelGGL(k_ss_vjp_partial, dim3(sp.nchunks, Np), dim3(128), 0, c->stream, sp, s0, glm, gln,
                               coef, g_x, g_y, g_w, part);
        hipLaunchKernelGGL(k_ss_vjp_final, dim3(nblocks((int64_t)Np * 2 * K, 256)), dim3(256), 0, c->stream, sp, part,
                           g_coef);
        FH_HIP(hipGetLastError());
        return FH_OK;
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

}  // extern "C"

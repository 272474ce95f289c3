// fh_fft.hpp -- FFTs of short sequences held in LDS, with the type-1 and
// type-3 steps around them fused in.
//
// A workgroup transforms several sequences of one length n (a product of
// 2, 3, 5 and 7, with all sequences together at most kLdsFftBytes) in place
// in LDS: self-sorting (Stockham) radix passes of 16, 8, 4, 2, 3, 5 and 7, each
// pass gathering its butterflies' inputs into registers, one barrier, and
// scattering the outputs, so that the result is in natural order.  A
// butterfly's twiddles are powers of one root of unity, read from a table of
// every pass's roots that the block builds in LDS with sincospi first.
// The forward transform is X[q] = sum_j x[j] exp(-2 pi i j q/n).
//
// Kernels:
//   k_t1_cols   type 1, second pass: the band of fine-grid rows the nodes
//               reach, n1 needed columns; per column, zero-pad to nf2, FFT,
//               then the epilogue (deconvolution, window shift, target chirp,
//               1/(i lambda z), Babinet) straight to the output.
//   k_t3_rows   type 3: precorrect the spread grid by 1/Phi, embed it in the
//               upsampled grid and FFT its rows.
//   k_t3_cols   type 3: FFT the columns of the upsampled grid in place.
#pragma once

#include "fh_common.hpp"

namespace fh {

constexpr size_t kLdsFftBytes = 64 * 1024;
constexpr int kLdsFftMaxStages = 24;
// Two block shapes: up to 2048 entries per block with 256 threads (small
// register arrays, several blocks per CU), or the whole 64 KB budget with
// 512 threads.
constexpr int kLdsFftSmall = 2048;

struct LdsFftPlan {
    int n = 0;
    int nst = 0;
    int radix[kLdsFftMaxStages] = {};
    int ntw = 0;               // twiddle table entries: sum over passes of Ns
    const void* tw = nullptr;  // the table in device memory (complex, the kernel's precision), or
                               // null: each workgroup computes it
};

// Radix passes for n (7s, 5s and 3s first, then the power of two in passes
// of at most 16, as even as they go); false if n has another prime factor.  A pass with Ns = 1 writes each thread's R outputs
// side by side, so neighbouring lanes write R elements apart: with R a power
// of two every lane of a write instruction lands in the same LDS banks,
// with R odd they spread over all of them; the later passes (Ns > 1) write
// runs of Ns consecutive elements.  Odd radices first also keep the twiddle
// table (the sum of Ns over the passes) small.
inline bool lds_fft_plan(int n, LdsFftPlan& p)
{
    p = LdsFftPlan{};
    p.n = n;
    if (n < 1) return false;
    int m = n;
    auto take = [&](int r) {
        while (m % r == 0 && p.nst < kLdsFftMaxStages) {
            p.radix[p.nst++] = r;
            m /= r;
        }
    };
    take(7);
    take(5);
    take(3);
    // the power of two 2^k left: ceil(k / 4) passes of radix 16 at most,
    // the k bits spread as evenly as they go (1024 = 8 8 16, not 16 16 4),
    // so that every pass gives each thread about the same work
    int k = 0;
    while ((1 << (k + 1)) <= m && m % (1 << (k + 1)) == 0) ++k;
    if (k > 0 && (1 << k) == m) {
        const int np = (k + 3) / 4;
        for (int i = 0; i < np && p.nst < kLdsFftMaxStages; ++i) {
            const int bits = k / np + (i >= np - k % np ? 1 : 0);
            p.radix[p.nst++] = 1 << bits;
            m >>= bits;
        }
    }
    take(16);
    take(8);
    take(4);
    take(2);
    int Ns = 1;
    for (int i = 0; i < p.nst; ++i) {
        p.ntw += Ns;
        Ns *= p.radix[i];
    }
    return m == 1;
}

template <class C2>
__device__ __forceinline__ C2 cmul(C2 a, C2 b)
{
    C2 r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

template <class C2>
__device__ __forceinline__ C2 cadd(C2 a, C2 b)
{
    C2 r;
    r.x = a.x + b.x;
    r.y = a.y + b.y;
    return r;
}

template <class C2>
__device__ __forceinline__ C2 csub(C2 a, C2 b)
{
    C2 r;
    r.x = a.x - b.x;
    r.y = a.y - b.y;
    return r;
}

// -i z
template <class C2>
__device__ __forceinline__ C2 cmul_negi(C2 a)
{
    C2 r;
    r.x = a.y;
    r.y = -a.x;
    return r;
}

template <class C2>
__device__ __forceinline__ void dft4(C2 a, C2 b, C2 c, C2 d, C2& X0, C2& X1, C2& X2, C2& X3)
{
    const C2 s0 = cadd(a, c), d0 = csub(a, c), s1 = cadd(b, d), d1 = cmul_negi(csub(b, d));
    X0 = cadd(s0, s1);
    X2 = csub(s0, s1);
    X1 = cadd(d0, d1);
    X3 = csub(d0, d1);
}

// Length-R DFT of t (forward) into X.
template <int R, class C2>
__device__ __forceinline__ void dft_small(const C2* t, C2* X)
{
    using Rl = decltype(t[0].x);
    if constexpr (R == 2) {
        X[0] = cadd(t[0], t[1]);
        X[1] = csub(t[0], t[1]);
    } else if constexpr (R == 4) {
        dft4(t[0], t[1], t[2], t[3], X[0], X[1], X[2], X[3]);
    } else if constexpr (R == 8) {
        // two length-4 DFTs of the even and odd entries, joined with
        // exp(-2 pi i q/8)
        C2 e[4], o[4];
        dft4(t[0], t[2], t[4], t[6], e[0], e[1], e[2], e[3]);
        dft4(t[1], t[3], t[5], t[7], o[0], o[1], o[2], o[3]);
        const Rl h = (Rl)0.70710678118654752440;
        C2 w1, w3;
        w1.x = h * (o[1].x + o[1].y);
        w1.y = h * (o[1].y - o[1].x);
        const C2 w2 = cmul_negi(o[2]);
        w3.x = h * (o[3].y - o[3].x);
        w3.y = -h * (o[3].x + o[3].y);
        X[0] = cadd(e[0], o[0]);
        X[4] = csub(e[0], o[0]);
        X[1] = cadd(e[1], w1);
        X[5] = csub(e[1], w1);
        X[2] = cadd(e[2], w2);
        X[6] = csub(e[2], w2);
        X[3] = cadd(e[3], w3);
        X[7] = csub(e[3], w3);
    } else if constexpr (R == 16) {
        // four length-4 DFTs of the entries r = 4 j + m, twiddled by
        // exp(-2 pi i m q/16), then length-4 DFTs across m
        C2 y[4][4];
#pragma unroll
        for (int m = 0; m < 4; ++m) dft4(t[m], t[m + 4], t[m + 8], t[m + 12], y[m][0], y[m][1], y[m][2], y[m][3]);
        const Rl c1 = (Rl)0.92387953251128675613, s1 = (Rl)0.38268343236508977173;
        const Rl h = (Rl)0.70710678118654752440;
        // y[m][q] *= exp(-2 pi i m q/16), m, q = 1..3
        auto rot = [&](C2 v, Rl c, Rl sn) {  // v exp(-i theta), cos c, sin sn
            C2 o;
            o.x = v.x * c + v.y * sn;
            o.y = v.y * c - v.x * sn;
            return o;
        };
        y[1][1] = rot(y[1][1], c1, s1);
        y[1][2] = rot(y[1][2], h, h);
        y[1][3] = rot(y[1][3], s1, c1);
        y[2][1] = rot(y[2][1], h, h);
        y[2][2] = cmul_negi(y[2][2]);
        y[2][3] = rot(y[2][3], -h, h);
        y[3][1] = rot(y[3][1], s1, c1);
        y[3][2] = rot(y[3][2], -h, h);
        y[3][3] = rot(y[3][3], -c1, -s1);
#pragma unroll
        for (int q = 0; q < 4; ++q) dft4(y[0][q], y[1][q], y[2][q], y[3][q], X[q], X[q + 4], X[q + 8], X[q + 12]);
    } else if constexpr (R == 3) {
        // X1, X2 = x0 - (x1 + x2)/2 -/+ i (sqrt(3)/2)(x1 - x2)
        const Rl s3 = (Rl)0.86602540378443864676;
        const C2 sum = cadd(t[1], t[2]), dif = csub(t[1], t[2]);
        C2 a, d;
        a.x = t[0].x - (Rl)0.5 * sum.x;
        a.y = t[0].y - (Rl)0.5 * sum.y;
        d.x = s3 * dif.x;
        d.y = s3 * dif.y;
        X[0] = cadd(t[0], sum);
        X[1] = cadd(a, cmul_negi(d));
        X[2] = csub(a, cmul_negi(d));
    } else if constexpr (R == 5) {
        // with c1, s1 = cos, sin(2 pi/5), c2, s2 = cos, sin(4 pi/5):
        // X1, X4 = x0 + c1 (x1 + x4) + c2 (x2 + x3) -/+ i (s1 (x1 - x4) + s2 (x2 - x3))
        // X2, X3 = x0 + c2 (x1 + x4) + c1 (x2 + x3) -/+ i (s2 (x1 - x4) - s1 (x2 - x3))
        const Rl c1 = (Rl)0.30901699437494742410, c2 = (Rl)-0.80901699437494742410;
        const Rl s1 = (Rl)0.95105651629515357212, s2 = (Rl)0.58778525229247312917;
        const C2 t1 = cadd(t[1], t[4]), t2 = cadd(t[2], t[3]), t3 = csub(t[1], t[4]), t4 = csub(t[2], t[3]);
        C2 a, b, d, e;
        a.x = t[0].x + c1 * t1.x + c2 * t2.x;
        a.y = t[0].y + c1 * t1.y + c2 * t2.y;
        b.x = t[0].x + c2 * t1.x + c1 * t2.x;
        b.y = t[0].y + c2 * t1.y + c1 * t2.y;
        d.x = s1 * t3.x + s2 * t4.x;
        d.y = s1 * t3.y + s2 * t4.y;
        e.x = s2 * t3.x - s1 * t4.x;
        e.y = s2 * t3.y - s1 * t4.y;
        X[0] = cadd(t[0], cadd(t1, t2));
        X[1] = cadd(a, cmul_negi(d));
        X[4] = csub(a, cmul_negi(d));
        X[2] = cadd(b, cmul_negi(e));
        X[3] = csub(b, cmul_negi(e));
    } else {
        // cos and sin of 2 pi m/R, m = 0..R-1
        constexpr double c3[3] = {1.0, -0.5, -0.5};
        constexpr double s3[3] = {0.0, 0.86602540378443864676, -0.86602540378443864676};
        constexpr double c5[5] = {1.0, 0.30901699437494742410, -0.80901699437494742410, -0.80901699437494742410,
                                  0.30901699437494742410};
        constexpr double s5[5] = {0.0, 0.95105651629515357212, 0.58778525229247312917, -0.58778525229247312917,
                                  -0.95105651629515357212};
        constexpr double c7[7] = {1.0,
                                  0.62348980185873353053,
                                  -0.22252093395631440429,
                                  -0.90096886790241912624,
                                  -0.90096886790241912624,
                                  -0.22252093395631440429,
                                  0.62348980185873353053};
        constexpr double s7[7] = {0.0,
                                  0.78183148246802980871,
                                  0.97492791218182360702,
                                  0.43388373911755812048,
                                  -0.43388373911755812048,
                                  -0.97492791218182360702,
                                  -0.78183148246802980871};
        static_assert(R == 3 || R == 5 || R == 7, "radix");
        const double* cs = R == 3 ? c3 : (R == 5 ? c5 : c7);
        const double* sn = R == 3 ? s3 : (R == 5 ? s5 : s7);
#pragma unroll
        for (int q = 0; q < R; ++q) {
            C2 acc = t[0];
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const int m = (r * q) % R;
                // t[r] exp(-2 pi i m/R)
                const Rl c = (Rl)cs[m], s = (Rl)sn[m];
                acc.x += t[r].x * c + t[r].y * s;
                acc.y += t[r].y * c - t[r].x * s;
            }
            X[q] = acc;
        }
    }
}

// Quotient by a divisor that is uniform across the block, by a multiply
// with the rounded-up reciprocal: exact while x d < 2^32 (here x, d < 2^13).
struct FastDiv {
    unsigned d, m;
};
__device__ __forceinline__ FastDiv fast_div(unsigned d) { return FastDiv{d, d > 1 ? 0xffffffffu / d + 1u : 0u}; }
__device__ __forceinline__ unsigned fdiv(unsigned x, const FastDiv& f) { return f.d > 1 ? __umulhi(x, f.m) : x; }

// exp(-2 pi i k/L) in the precision of C2, from the reduced fraction k/L
__device__ __forceinline__ double2 unit_root(double2*, int k, int L)
{
    double s, c;
    sincospi(-2.0 * (double)k / (double)L, &s, &c);
    return make_double2(c, s);
}
__device__ __forceinline__ float2 unit_root(float2*, int k, int L)
{
    float s, c;
    sincospif(-2.0f * (float)k / (float)L, &s, &c);
    return make_float2(c, s);
}

// LDS layout of a block's transforms: element i = s n + j (sequence s, index
// j) sits at lds_pad(i), one spare slot after every 16 elements.  Without it
// the first pass of a power-of-two length writes each thread's R outputs side
// by side, R elements apart across the lanes, and every lane of the write
// lands in the same banks; padded, 16 complex elements span 17 and the lanes
// spread over all banks.  lds_span: elements that nseq sequences occupy.
__host__ __device__ __forceinline__ int lds_pad(int i) { return i + (i >> 4); }
__host__ __device__ inline size_t lds_span(int n, int nseq)
{
    const size_t e = (size_t)n * nseq;
    return e + (e >> 4);
}

// One radix-R pass over nseq sequences of length n at lds_pad(s n), Ns =
// product of the radices already applied.  The twiddles exp(-2 pi i k r/(Ns R)) of a
// butterfly are the powers of its root tw[k] = exp(-2 pi i k/(Ns R)).
template <int R, int MAXE, int NT, class C2>
__device__ __forceinline__ void lds_fft_pass(C2* buf, int n, int nseq, int Ns, const C2* tw)
{
    constexpr int KB = (MAXE / R + NT - 1) / NT;
    const int nb = n / R;
    const int total = nb * nseq;
    const FastDiv dnb = fast_div((unsigned)nb), dns = fast_div((unsigned)Ns);
    // A butterfly reads R elements nb apart and writes R elements Ns apart.
    // Padded, such a run stays evenly spaced when its stride is a multiple
    // of 16 (stride s becomes s + s/16) or when the R writes fill part of
    // one aligned run of 16 (Ns R divides 16); else each address is padded.
    const int rstr = (nb & 15) == 0 ? nb + (nb >> 4) : 0;
    const int wstr = (Ns & 15) == 0 ? Ns + (Ns >> 4) : (16 % (Ns * R) == 0 ? Ns : 0);
    C2 v[KB][R];
#pragma unroll
    for (int i = 0; i < KB; ++i) {
        const int g = threadIdx.x + i * NT;
        if (g < total) {
            const int s = (int)fdiv((unsigned)g, dnb), j = g - s * nb;
            const int base = s * n + j;
            const int k = j - (int)fdiv((unsigned)j, dns) * Ns;
            C2 t[R];
            if (rstr) {
                const C2* src = buf + lds_pad(base);
#pragma unroll
                for (int r = 0; r < R; ++r) t[r] = src[r * rstr];
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) t[r] = buf[lds_pad(base + r * nb)];
            }
            if (k != 0) {
                const C2 w1 = tw[k];
                C2 w = w1;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    t[r] = cmul(t[r], w);
                    if (r + 1 < R) w = cmul(w, w1);
                }
            }
            dft_small<R>(t, v[i]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < KB; ++i) {
        const int g = threadIdx.x + i * NT;
        if (g < total) {
            const int s = (int)fdiv((unsigned)g, dnb), j = g - s * nb;
            const int q = (int)fdiv((unsigned)j, dns), k = j - q * Ns;
            const int base = s * n + q * Ns * R + k;
            if (wstr) {
                C2* dst = buf + lds_pad(base);
#pragma unroll
                for (int r = 0; r < R; ++r) dst[r * wstr] = v[i][r];
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) buf[lds_pad(base + r * Ns)] = v[i][r];
            }
        }
    }
    __syncthreads();
}

// Whole-block forward FFT of nseq sequences (n nseq <= MAXE) in LDS, laid
// out by lds_pad; the caller synchronises before (data written) and may read
// right after.
// twl: LDS room for p.ntw entries, filled here with every pass's roots
// (copied from p.tw when the plan has a precomputed table).
// R7: the radix-7 pass is compiled in.  Its pass holds two 7-point
// butterflies per thread, and in double precision a kernel with it needs 152
// registers per lane (three waves per SIMD) where the other passes need 90,
// so kernels are built with and without it and the plan picks (lds_has7).
template <int MAXE, int NT, bool R7, class C2>
__device__ void lds_fft(C2* buf, const LdsFftPlan& p, int nseq, C2* twl)
{
    if (p.tw) {
        const C2* tg = static_cast<const C2*>(p.tw);
        for (int k = threadIdx.x; k < p.ntw; k += NT) twl[k] = tg[k];
    } else {
        int off = 0, Ns = 1;
        for (int st = 0; st < p.nst; ++st) {
            const int L = Ns * p.radix[st];
            for (int k = threadIdx.x; k < Ns; k += NT) twl[off + k] = unit_root((C2*)nullptr, k, L);
            off += Ns;
            Ns = L;
        }
    }
    __syncthreads();
    int Ns = 1;
    const C2* tw = twl;
    for (int st = 0; st < p.nst; ++st) {
        const int R = p.radix[st];
        switch (R) {
        case 16: lds_fft_pass<16, MAXE, NT>(buf, p.n, nseq, Ns, tw); break;
        case 8: lds_fft_pass<8, MAXE, NT>(buf, p.n, nseq, Ns, tw); break;
        case 4: lds_fft_pass<4, MAXE, NT>(buf, p.n, nseq, Ns, tw); break;
        case 2: lds_fft_pass<2, MAXE, NT>(buf, p.n, nseq, Ns, tw); break;
        case 3: lds_fft_pass<3, MAXE, NT>(buf, p.n, nseq, Ns, tw); break;
        case 5: lds_fft_pass<5, MAXE, NT>(buf, p.n, nseq, Ns, tw); break;
        default:
            if constexpr (R7) lds_fft_pass<7, MAXE, NT>(buf, p.n, nseq, Ns, tw);
            break;
        }
        tw += Ns;
        Ns *= R;
    }
}

// Whether a plan has a radix-7 pass (its kernels must be built with R7).
inline bool lds_has7(const LdsFftPlan& p)
{
    for (int i = 0; i < p.nst; ++i)
        if (p.radix[i] == 7) return true;
    return false;
}

// Workgroup b of a launch over `groups` column groups, with consecutive
// groups on one XCD (workgroups are dealt to the 8 XCDs in turn), so that
// the partial output lines of neighbouring groups meet in one L2.
__device__ __forceinline__ int xcd_group(int groups)
{
    const int per = (groups + 7) / 8;
    return (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
}
inline unsigned xcd_blocks(int groups) { return 8u * (unsigned)((groups + 7) / 8); }

}  // namespace fh

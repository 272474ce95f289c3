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
//        spread:  exponential-of-semicircle (ES) kernel into a (T+W-1)^2 LDS
//                 tile per work item, written out as one slot per work item,
//        reduce:  every fine-grid cell sums the slots that cover it (no
//                 global atomics; a fixed order of slots, though the
//                 binning's atomic counters may order a tile's points
//                 differently from call to call),
//        FFT:     in LDS where a row or column fits, else rocFFT,
//        finish:  deconvolution by the kernel's Fourier transform (type 1), or
//                 precorrection, a second FFT and kernel interpolation at the
//                 targets (type 3);
//   3. the target chirp exp(i pi |xi_k|^2/(lambda z))/(i lambda z), and
//      u_oc = 1 - u_ap for occulters (eq. bab).
//
// Type 1 holds only the fine-grid rows the nodes can reach (a window found
// from the rule's bounding box): the first FFT pass runs over those rows, and
// the second pass and the epilogue work on the n1 needed columns only.  When
// a row and a column fit in LDS, the first pass is fused with the reduce (the
// fine grid is never stored) and the second with the epilogue; otherwise
// rocFFT transforms the stored rows, and a transpose pads the needed columns
// back to full length for a second rocFFT pass.
#include "fh_kernels.hpp"

#include <hipcub/device/device_radix_sort.hpp>

namespace fh {

size_t tile_sort_bytes(int64_t n)
{
    size_t temp = 0;
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, temp, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                           (const int*)nullptr, (int*)nullptr, (int)n, 0, 32) != hipSuccess)
        temp = 0;
    return std::max<size_t>(temp, 1);
}

// Stable sort of n (tile key, node index) pairs by the low key_bits of the
// key: least-significant-digit radix passes keep equal keys in input order.
fh_status tile_sort(fh_ctx* c, const uint32_t* key, uint32_t* key_sorted, const int* vals, int* vals_sorted,
                    int64_t n, int key_bits, void* tmp, size_t tmp_bytes)
{
    size_t temp = tmp_bytes;
    FH_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, temp, key, key_sorted, vals, vals_sorted, (int)n, 0, key_bits,
                                              c->stream));
    return FH_OK;
}

// Sequences per workgroup for an LDS FFT of length n over `count`
// sequences: as many as give 64 bytes of contiguous output per row segment
// (or `min_c` sequences), more while there are over two workgroups per CU,
// fewer while there are under two, within the LDS budget and the
// 16-sequence limit of the column kernel.  C = 0 when one sequence does not fit or n has a prime
// factor above 7.
struct LdsCols {
    int C = 0;
    size_t lds = 0;
    bool small = false;  // C n <= kLdsFftSmall: the 256-thread shape
    LdsFftPlan plan;
};

// The LDS FFT twiddle table of plan p (every pass's roots exp(-2 pi i k/L),
// k < Ns, L = Ns R, in pass order) in device memory, computed on the host
// in long double once per context, length and precision: otherwise every
// workgroup of an FFT launch evaluates the same sincospi values.  Null when
// the allocation or copy fails (the kernels then compute the table).
const void* lds_twiddles(fh_ctx* c, const LdsFftPlan& p, size_t rs)
{
    const auto key = std::make_pair(p.n, (int)rs);
    auto it = c->lds_tw_cache.find(key);
    if (it != c->lds_tw_cache.end()) return it->second;
    const long double two_pi = 6.283185307179586476925286766559005768L;
    std::vector<double> t(2 * (size_t)p.ntw);
    int off = 0, Ns = 1;
    for (int st = 0; st < p.nst; ++st) {
        const int L = Ns * p.radix[st];
        for (int k = 0; k < Ns; ++k) {
            const long double a = two_pi * (long double)k / (long double)L;
            t[2 * (size_t)(off + k)] = (double)cosl(a);
            t[2 * (size_t)(off + k) + 1] = (double)-sinl(a);
        }
        off += Ns;
        Ns = L;
    }
    void* dev = nullptr;
    if (dev_alloc(c, rs * t.size(), &dev) == FH_OK) {
        hipError_t e;
        if (rs == sizeof(double)) {
            e = hipMemcpy(dev, t.data(), rs * t.size(), hipMemcpyHostToDevice);
        } else {
            std::vector<float> tf(t.begin(), t.end());
            e = hipMemcpy(dev, tf.data(), rs * tf.size(), hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) {
            dev_free(c, dev);
            dev = nullptr;
        }
    }
    c->lds_tw_cache[key] = dev;
    return dev;
}

LdsCols lds_cols_plan(fh_ctx* c, int n, int64_t count, size_t rs, int min_c = 0)
{
    LdsCols r;
    // FH_FFT=rocfft in the environment keeps every transform on rocFFT
    static const bool force_rocfft = [] {
        const char* e = std::getenv("FH_FFT");
        return e && std::strcmp(e, "rocfft") == 0;
    }();
    if (force_rocfft) return r;
    const size_t cb = 2 * rs;
    if (!lds_fft_plan(n, r.plan)) return r;
    // data of C sequences and the twiddle table in one block's LDS
    int cap = 0;
    while (cap < 16 && cb * (lds_span(n, cap + 1) + (size_t)r.plan.ntw) + 512 <= kLdsFftBytes) ++cap;
    if (cap < 1) return r;
    int C = min_c > 0 ? min_c : std::max(1, (int)(64 / cb));
    const int64_t want = std::max<int64_t>(1, count / (2 * (int64_t)c->cu_count));
    C = (int)std::max<int64_t>(C, std::min<int64_t>(want, 16));
    C = std::min({C, cap, 16});
    // but keep at least two workgroups per CU where the count allows
    while (C > 1 && count / C < 2 * (int64_t)c->cu_count) C /= 2;
    // rather fewer sequences per block than the 512-thread shape: as many as
    // the 256-thread shape holds
    if (n <= kLdsFftSmall && n * C > kLdsFftSmall) C = kLdsFftSmall / n;
    r.C = C;
    r.plan.tw = lds_twiddles(c, r.plan, rs);
    r.lds = cb * (lds_span(n, C) + r.plan.ntw);
    r.small = n * C <= kLdsFftSmall;
    return r;
}

// Launch one of the LDS FFT kernels in the block shape that `lc` picked.
#define FH_LDS_LAUNCH_R7(KERNEL, R, R7, lc, grid, stream, ...)                                                \
    do {                                                                                                         \
        if ((lc).small)                                                                                          \
            hipLaunchKernelGGL((KERNEL<R, kLdsFftSmall, 256, R7>), grid, dim3(256), (lc).lds, stream,            \
                               __VA_ARGS__);                                                                     \
        else                                                                                                     \
            hipLaunchKernelGGL((KERNEL<R, (int)(kLdsFftBytes / (2 * sizeof(R))), 512, R7>), grid, dim3(512),     \
                               (lc).lds, stream, __VA_ARGS__);                                                   \
    } while (0)
#define FH_LDS_LAUNCH(KERNEL, R, lc, grid, stream, ...)                                                        \
    do {                                                                                                         \
        if (lds_has7((lc).plan))                                                                                 \
            FH_LDS_LAUNCH_R7(KERNEL, R, true, lc, grid, stream, __VA_ARGS__);                                    \
        else                                                                                                     \
            FH_LDS_LAUNCH_R7(KERNEL, R, false, lc, grid, stream, __VA_ARGS__);                                   \
    } while (0)

// LDS bytes of a k_t1_rows block: the rows and twiddles of the FFT, then the
// heads of the covering tile rows.
inline size_t t1_rows_lds(const LdsCols& lr, const GridGeom& gg, int reach, size_t rs)
{
    return t1_rows_table_offset(lr.C, lr.plan.n, lr.plan.ntw, 2 * rs) +
           sizeof(int4) * (size_t)t1_rows_table_rows(lr.C, gg.T, reach) * gg.ntx;
}

// The fused tile reduce and first FFT pass (k_t1_rows) in the block shape
// that lr picked, for a padded tile reaching one tile on.
template <class R>
fh_status launch_t1_rows(fh_ctx* c, const LdsCols& lr, int reach, int B, int groups, const GridGeom& gg,
                         const SpreadBufs& sb, int n1, R* G)
{
    using C2 = typename V2<R>::T;
    const int tpi = gg.ntx * gg.nty;
    const dim3 grid(xcd_blocks(groups), B);
    const size_t lds = t1_rows_lds(lr, gg, reach, sizeof(R));
#define FH_ROWS(RE, R7)                                                                                          \
    do {                                                                                                         \
        if (lr.small)                                                                                            \
            hipLaunchKernelGGL((k_t1_rows<R, kLdsFftSmall, 256, R7, RE>), grid, dim3(256), lds, c->stream,       \
                               (const C2*)sb.slots, sb.tsub, gg, tpi, lr.C, groups, lr.plan, n1, G, sb.cnt);     \
        else                                                                                                     \
            hipLaunchKernelGGL((k_t1_rows<R, (int)(kLdsFftBytes / (2 * sizeof(R))), 512, R7, RE>), grid,          \
                               dim3(512), lds, c->stream, (const C2*)sb.slots, sb.tsub, gg, tpi, lr.C, groups,    \
                               lr.plan, n1, G, sb.cnt);                                                          \
    } while (0)
    FH_ARG(reach == 1, FH_ERR_UNSUPPORTED, "the fused row pass needs a padded tile reaching one tile on");
    if (lds_has7(lr.plan)) FH_ROWS(1, true);
    else FH_ROWS(1, false);
#undef FH_ROWS
    FH_HIP(hipGetLastError());
    return FH_OK;
}

// The type-1 pipeline for B instances sharing one grid geometry; u is device
// memory (B x n2 x n1).  With `capture`, the launch sequence is recorded into
// a hipGraph keyed by everything baked into it and replayed.  With
// `rebuild`, every rule's kernels run again first (inside the graph).
template <class R>
fh_status t1_pipeline(fh_ctx* c, int B, const fh_quad* const* qs, const double* lambda, const double* z, int n1,
                      int n2, double h1, double h2, double xc, double yc, const int32_t* occ, R* u, bool capture,
                      size_t extra_bytes, void** extra, bool rebuild = false)
{
    const size_t rs = sizeof(R);
    int64_t Nall = 0;
    for (int b = 0; b < B; ++b) Nall += qs[b]->N;
    T1Plan pl = plan_t1(c, n1, n2, Nall);
    FH_ARG(!pl.k.clamped, FH_ERR_UNSUPPORTED, "tolerance %g needs a kernel wider than %d at sigma %g", c->tol,
           kMaxWidth, pl.k.sigma);
    GridGeom gg = pl.gg;
    std::vector<InstParams> inst(B);
    std::vector<EpiInst> epi(B);
    int64_t Ntot = 0;
    int max_span = 0;
    std::vector<int> spans(B, 0);
    for (int b = 0; b < B; ++b) {
        inst[b] = inst_t1(qs[b], lambda[b], z[b], h1, h2, xc, yc, gg);
        inst[b].node_off = Ntot;
        Ntot += qs[b]->N;
        const double lz = lambda[b] * z[b];
        epi[b] = EpiInst{0.5 / lz, 1.0 / lz, occ[b] ? 1 : 0, 0, 0, 0};
        if (qs[b]->N > 0) {
            double bb[4];
            FH_TRY(quad_bbox(c, qs[b], bb));
            int lo, span;
            window_rows(bb, inst[b].s2, gg.W, lo, span);
            inst[b].sh2 = lo;
            spans[b] = span;
            max_span = std::max(max_span, span);
        }
    }
    FH_ARG(Ntot < ((int64_t)1 << 31), FH_ERR_UNSUPPORTED, "%lld nodes in one call; at most 2^31 - 1",
           (long long)Ntot);
    size_items(c, gg, Ntot);
    // hold only the reachable rows unless they cover most of the period
    const int rows = (max_span + gg.T - 1) / gg.T * gg.T;
    if (rows + gg.T < gg.nf2 && max_span > 0) {
        gg.rows = rows;
        gg.wrap_y = 0;
    } else {
        gg.rows = gg.nf2;
        gg.wrap_y = 1;
        for (auto& ip : inst) ip.sh2 = 0;
    }
    gg.nty = (gg.rows + gg.T - 1) / gg.T;
    gg.pady = gg.nty * gg.T - gg.rows;
    const int tpi = gg.ntx * gg.nty;
    for (int b = 0; b < B; ++b) {
        inst[b].tile_off = b * tpi;
        epi[b].sh2 = inst[b].sh2;
        epi[b].rows = gg.rows;
        epi[b].roff = b * gg.rows;
    }
    FH_ARG((int64_t)tpi * B < ((int64_t)1 << 31), FH_ERR_UNSUPPORTED, "too many tiles");
    const double* ip1 = nullptr;
    const double* ip2 = nullptr;
    FH_TRY(iphi_table(c, pl.k, n1, gg.nf1, &ip1));
    FH_TRY(iphi_table(c, pl.k, n2, gg.nf2, &ip2));
    FftPlan* fa = nullptr;
    FftPlan* fb = nullptr;
    // second pass: in LDS, fused with the epilogue, when a column fits
    LdsCols lc = lds_cols_plan(c, gg.nf2, (int64_t)n1 * B, rs);
    // first pass: in LDS as well, fused with the tile reduce, when a row fits
    // too, a padded tile reaches one tile on (nine covering tiles per cell
    // cost more than the stored grid's list reduce) and there are rows
    // enough for 16 workgroups per CU (one row per workgroup: with fewer,
    // rocFFT's row pass and the tile reduce fill the chip better); the fine
    // grid is then never stored, only the n1 needed columns of its
    // transformed rows (F holds B x rows x n1 values)
    const int reach = tile_reach(gg);
    LdsCols lr;
    if (lc.C > 0 && reach == 1 && (int64_t)gg.rows * B >= 16 * (int64_t)c->cu_count)
        lr = lds_cols_plan(c, gg.nf1, (int64_t)gg.rows * B, rs, 1);
    const bool fused = lr.C > 0 && t1_rows_lds(lr, gg, reach, rs) <= kLdsFftBytes;
    // A batch of windowed instances on the stored grid holds each instance's
    // own rows (its span rounded up to whole tiles), one after another: the
    // zero fill, the row transforms and the column pass's loads then cover
    // only those; the tiles stay those of the tallest window.
    const bool ragged = B > 1 && !gg.wrap_y && !fused && lc.C > 0;
    std::vector<int2> rwin;
    int64_t total_rows = (int64_t)B * gg.rows;
    if (ragged) {
        rwin.resize(B);
        total_rows = 0;
        for (int b = 0; b < B; ++b) {
            const int rb = std::min(gg.rows, (spans[b] + gg.T - 1) / gg.T * gg.T);
            rwin[b] = make_int2(rb, (int)total_rows);
            epi[b].rows = rb;
            epi[b].roff = (int)total_rows;
            total_rows += rb;
        }
        FH_ARG(total_rows * gg.nf1 < ((int64_t)1 << 40), FH_ERR_UNSUPPORTED, "fine grid too large");
    }
    if (!fused) FH_TRY(fft_plan(c, gg.nf1, 0, (int)std::max<int64_t>(total_rows, 1), &fa));
    if (lc.C == 0) FH_TRY(fft_plan(c, gg.nf2, 0, n1 * B, &fb));

    FH_TRY(counters_ready(c, (int64_t)tpi * B));
    const size_t F_count = 2 * (size_t)std::max<int64_t>(total_rows, 1) * (fused ? n1 : gg.nf1);
    const size_t Z_count = lc.C > 0 ? 0 : 2 * (size_t)B * n1 * gg.nf2;
    const size_t E2_bytes = lc.C > 0 ? aligned_bytes(sizeof(double2) * (size_t)B * n2) : 0;
    size_t need = aligned_bytes(rs * F_count) + aligned_bytes(rs * Z_count) + E2_bytes +
                  spread_bytes(c, Ntot, gg, tpi * B, rs) + aligned_bytes(sizeof(InstParams) * B) +
                  aligned_bytes(sizeof(EpiInst) * B) + aligned_bytes(sizeof(int2) * B) +
                  aligned_bytes(extra_bytes);
    FH_TRY(arena_reserve(c, need));
    R* F = c->arena.take<R>(F_count);
    R* Z = c->arena.take<R>(Z_count);
    double2* E2 = lc.C > 0 ? c->arena.take<double2>((size_t)B * n2) : nullptr;
    SpreadBufs sb = spread_carve(c, Ntot, gg, tpi * B, rs);
    InstParams* dinst = c->arena.take<InstParams>(B);
    EpiInst* depi = c->arena.take<EpiInst>(B);
    int2* drwin = c->arena.take<int2>(B);
    if (extra) *extra = c->arena.take<char>(extra_bytes);
    if (!u) u = static_cast<R*>(*extra);
    const bool batched = B > 1;
    if (batched) {
        FH_HIP(hipMemcpyAsync(dinst, inst.data(), sizeof(InstParams) * B, hipMemcpyHostToDevice, c->stream));
        FH_HIP(hipMemcpyAsync(depi, epi.data(), sizeof(EpiInst) * B, hipMemcpyHostToDevice, c->stream));
        if (ragged)
            FH_HIP(hipMemcpyAsync(drwin, rwin.data(), sizeof(int2) * B, hipMemcpyHostToDevice, c->stream));
    }

    auto run = [&]() -> fh_status {
        timing_mark(c, 0);
        if (rebuild)
            for (int b = 0; b < B; ++b) FH_TRY(qs[b]->rebuild());
        if (fused) {
            FH_TRY(spread_items<R>(c, inst[0], batched ? dinst : nullptr, B, Ntot, gg, sb, pl.k.beta, pl.k.poly));
            FH_TRY(launch_t1_rows<R>(c, lr, reach, B, (gg.rows + lr.C - 1) / lr.C, gg, sb, n1, F));
            c->tile_cnt_dirty = false;
        } else {
            FH_TRY(run_spread<R>(c, inst[0], batched ? dinst : nullptr, B, Ntot, gg, sb, F, pl.k.beta, pl.k.poly,
                                 ragged ? (const int2*)drwin : nullptr, total_rows));
            if (total_rows > 0) FH_TRY(fft_exec(c, fa, F));
        }
        EpiParams ep{n1, n2, gg.nf1, gg.nf2, h1, h2, xc, yc, ip1, ip2};
        if (lc.C > 0) {
            hipLaunchKernelGGL(k_t1_rowfactors, dim3(nblocks(n2, 256), B), dim3(256), 0, c->stream, ep, epi[0],
                               batched ? (const EpiInst*)depi : nullptr, E2);
            timing_mark(c, 3);
            const int groups = (n1 + lc.C - 1) / lc.C;
            FH_LDS_LAUNCH(k_t1_cols, R, lc, dim3(xcd_blocks(groups), B), c->stream, F, u, gg.rows,
                          fused ? n1 : gg.nf1, fused ? 1 : 0, lc.C, groups,
                          lc.plan, ep, epi[0], batched ? (const EpiInst*)depi : nullptr, (const double2*)E2);
            FH_HIP(hipGetLastError());
            timing_mark(c, 4);
        } else {
            hipLaunchKernelGGL((k_transpose_pad<R>), dim3(nblocks(n1, 32), nblocks(gg.nf2, 32), B), dim3(256), 0,
                               c->stream, F, Z, n1, gg.nf1, gg.nf2, gg.rows);
            FH_HIP(hipGetLastError());
            FH_TRY(fft_exec(c, fb, Z));
            timing_mark(c, 3);
            hipLaunchKernelGGL((k_epilogue_t1<R>), dim3(nblocks(n1, 32), nblocks(n2, 32), B), dim3(256), 0,
                               c->stream, Z, u, ep, epi[0], batched ? (const EpiInst*)depi : nullptr);
            FH_HIP(hipGetLastError());
            timing_mark(c, 4);
        }
        timing_mark(c, 5);
        return FH_OK;
    };
    // A single instance passes its parameters to the kernels by value (no
    // device table), so a graph would bake in this call's quadrature and
    // wavelength: it runs eagerly, exactly as fh_field_grid does.
    // The stable binning's radix sort is a library call that may record
    // memory fills, which replay wrongly from a graph: it runs eagerly too.
    if (!capture || B == 1 || c->timing || c->opt.deterministic || std::getenv("FH_NO_GRAPH")) return run();

    // graph key: every pointer and size baked into the launches
    char key[512];
    snprintf(key, sizeof(key), "%p|%zu|%d|%lld|%d|%d|%d|%d|%d|%d|%a|%a|%a|%a|%d|%d|%d|%p|%p|%d|%lld",
             (void*)c->arena.base, c->arena.cap, B, (long long)Ntot, n1, n2, gg.nf1, gg.nf2, gg.W, gg.rows, h1, h2,
             xc, yc, gg.T, gg.P, gg.method, (void*)u, (void*)c->tile_cnt, rebuild ? 1 : 0, (long long)total_rows);
    std::string k2(key);
    for (int b = 0; b < B; ++b) k2 += "|" + std::to_string(qs[b]->N);
    // Graphs are captured and replayed on a private stream (the caller's may
    // be the null stream, which cannot be captured), ordered after the
    // caller's prior work and before its later work by events.
    if (!c->gstream) {
        FH_HIP(hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
        FH_HIP(hipEventCreateWithFlags(&c->gev_in, hipEventDisableTiming));
        FH_HIP(hipEventCreateWithFlags(&c->gev_out, hipEventDisableTiming));
    }
    hipStream_t user = c->stream;
    FH_HIP(hipEventRecord(c->gev_in, user));
    FH_HIP(hipStreamWaitEvent(c->gstream, c->gev_in, 0));
    auto it = c->graph_cache.find(k2);
    if (it == c->graph_cache.end()) {
        GraphEntry ge;
        c->stream = c->gstream;
        hipError_t eb = (c->inject & kInjectCapture)
                            ? hipErrorStreamCaptureUnsupported
                            : hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal);
        fh_status s = FH_OK;
        hipGraph_t g = nullptr;
        hipError_t e = hipSuccess;
        if (eb == hipSuccess) {
            s = run();
            e = hipStreamEndCapture(c->gstream, &g);
        }
        c->stream = user;
        if (eb != hipSuccess || e != hipSuccess || !g || s != FH_OK) {
            // capture refused (or a call failed inside it): run eagerly
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            return run();
        }
        ge.graph = g;
        FH_HIP(hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0));
        it = c->graph_cache.emplace(k2, ge).first;
    }
    FH_HIP(hipGraphLaunch(it->second.exec, c->gstream));
    FH_HIP(hipEventRecord(c->gev_out, c->gstream));
    FH_HIP(hipStreamWaitEvent(user, c->gev_out, 0));
    return FH_OK;
}

namespace {

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
fh_status field_grid_impl(fh_ctx* c, const fh_quad* q, double lambda, double z, int n1, int n2, double h1,
                          double h2, double xc, double yc, int occ, void* u, fh_memspace mem)
{
    const int64_t M = (int64_t)n1 * n2;
    const size_t out_bytes = 2 * sizeof(R) * (size_t)M;
    c->timing_kind = 0;
    if (q->N == 0) {
        FH_TRY(arena_reserve(c, mem == FH_MEM_HOST ? aligned_bytes(out_bytes) : 0));
        R* dout = mem == FH_MEM_HOST ? c->arena.take<R>(2 * M) : static_cast<R*>(u);
        timing_mark(c, 0);
        hipLaunchKernelGGL((k_fill_field<R>), dim3(nblocks(M, 256)), dim3(256), 0, c->stream, dout, M,
                           (R)(occ ? 1.0 : 0.0));
        FH_HIP(hipGetLastError());
        for (int i = 1; i <= 5; ++i) timing_mark(c, i);
        if (mem == FH_MEM_HOST) {
            FH_HIP(hipMemcpyAsync(u, dout, out_bytes, hipMemcpyDeviceToHost, c->stream));
            FH_HIP(hipStreamSynchronize(c->stream));
        }
        return FH_OK;
    }
    const int32_t o = occ ? 1 : 0;
    void* staging = nullptr;
    R* dout = mem == FH_MEM_HOST ? nullptr : static_cast<R*>(u);
    FH_TRY(t1_pipeline<R>(c, 1, &q, &lambda, &z, n1, n2, h1, h2, xc, yc, &o, dout, false,
                          mem == FH_MEM_HOST ? out_bytes : 0, mem == FH_MEM_HOST ? &staging : nullptr));
    if (mem == FH_MEM_HOST) {
        FH_HIP(hipMemcpyAsync(u, staging, out_bytes, hipMemcpyDeviceToHost, c->stream));
        FH_HIP(hipStreamSynchronize(c->stream));
    }
    return FH_OK;
}

// Type-3 evaluation at targets (xi_t, eta_t), t < M, all inside the box tb
// (xmin, xmax, ymin, ymax) the grids are planned from; the value of target t
// goes to dout[t].  With `host`, xi and eta are
// host arrays copied into the arena; with `host` or `stage_out` the field is
// written to arena staging returned in *staged, for the caller to copy back.
template <class R>
fh_status t3_core(fh_ctx* c, const fh_quad* q, double lambda, double z, int64_t M, const double* xi,
                  const double* eta, const double* tb, int occ, R* dout, bool host,
                  bool stage_out, R** staged, const int* perm = nullptr)
{
    stage_out = stage_out || host;
    const size_t rs = sizeof(R);
    const double lz = lambda * z;
    const int64_t N = q->N;
    const size_t cbytes = aligned_bytes(sizeof(double) * M);
    const size_t obytes = aligned_bytes(2 * rs * M);
    c->timing_kind = 1;
    if (N == 0) {
        FH_TRY(arena_reserve(c, stage_out ? obytes : 0));
        if (stage_out) *staged = dout = c->arena.take<R>(2 * M);
        timing_mark(c, 0);
        hipLaunchKernelGGL((k_fill_field<R>), dim3(nblocks(M, 256)), dim3(256), 0, c->stream, dout, M,
                           (R)(occ ? 1.0 : 0.0));
        FH_HIP(hipGetLastError());
        for (int i = 1; i <= 5; ++i) timing_mark(c, i);
        return FH_OK;
    }
    double sb[4];
    FH_TRY(quad_bbox(c, q, sb));
    EsKernel k = choose_kernel(c, 0);
    FH_ARG(!k.clamped, FH_ERR_UNSUPPORTED, "tolerance %g needs a kernel wider than %d at sigma %g", c->tol, kMaxWidth,
           k.sigma);
    es_poly_attach(c, k);
    const int T0 = c->opt.tile > 0 ? std::min(c->opt.tile, 32) : 16;
    T3Dim d1 = plan_t3_dim(sb[0], sb[1], tb[0], tb[1], lz, k, T0);
    T3Dim d2 = plan_t3_dim(sb[2], sb[3], tb[2], tb[3], lz, k, T0);
    FH_ARG((int64_t)d1.m * d2.m <= (int64_t)1 << 31, FH_ERR_UNSUPPORTED,
           "type-3 fine grid %d x %d too large (space-bandwidth product too big)", d1.m, d2.m);
    FH_ARG(d1.nf <= 65535 && d2.nf <= 65535 && d1.m <= 65535 && d2.m <= 65535, FH_ERR_UNSUPPORTED,
           "type-3 grid side above 65535");
    GridGeom gg;
    gg.T = T0;
    gg.W = k.w;
    gg.L = T0 + k.w - 1;
    gg.nf1 = d1.nf;
    gg.nf2 = d2.nf;
    gg.ntx = d1.nf / T0;
    gg.nty = d2.nf / T0;
    gg.rows = d2.nf;
    gg.wrap_y = 1;
    gg.padx = gg.pady = 0;  // the type-3 grids are multiples of the tile
    spread_defaults(c, gg);
    size_items(c, gg, N);
    const int ntiles = gg.ntx * gg.nty;

    const double* ip1 = nullptr;
    const double* ip2 = nullptr;
    FH_TRY(iphi_table(c, k, d1.nf, d1.m, &ip1));
    FH_TRY(iphi_table(c, k, d2.nf, d2.m, &ip2));
    FftPlan* fp = nullptr;
    // upsampled 2D FFT: rows (with the precorrection) and columns in LDS
    // when a row and a column fit, else rocFFT
    LdsCols lr = lds_cols_plan(c, d1.m, d2.m, rs, 1);
    LdsCols lcol = lds_cols_plan(c, d2.m, d1.m, rs);
    const bool lds2d = lr.C > 0 && lcol.C > 0;
    if (!lds2d) FH_TRY(fft_plan(c, d1.m, d2.m, 1, &fp));
    FH_TRY(counters_ready(c, ntiles));
    const size_t fine_count = 2 * (size_t)d1.nf * d2.nf;
    const size_t up_count = 2 * (size_t)d1.m * d2.m;
    const size_t need = aligned_bytes(rs * fine_count) + aligned_bytes(rs * up_count) +
                        spread_bytes(c, N, gg, ntiles, rs) + (host ? 2 * cbytes : 0) +
                        (stage_out ? obytes : 0);
    FH_TRY(arena_reserve(c, need));
    R* fine = c->arena.take<R>(fine_count);
    R* up = c->arena.take<R>(up_count);
    SpreadBufs sbuf = spread_carve(c, N, gg, ntiles, rs);
    const double* dxi = xi;
    const double* deta = eta;
    if (host) {
        double* a = c->arena.take<double>(M);
        double* b = c->arena.take<double>(M);
        FH_HIP(hipMemcpyAsync(a, xi, sizeof(double) * M, hipMemcpyHostToDevice, c->stream));
        FH_HIP(hipMemcpyAsync(b, eta, sizeof(double) * M, hipMemcpyHostToDevice, c->stream));
        dxi = a;
        deta = b;
    }
    if (stage_out) *staged = dout = c->arena.take<R>(2 * M);

    InstParams ip{};
    ip.x = q->x;
    ip.y = q->y;
    ip.w = q->w;
    ip.N = N;
    // chirp and pre-phase exp(-i D.(x - C)), D = 2 pi (target centre)/(lambda z),
    // and the incident wave of a point source at the rule's distance
    ip.pa = 0.5 / lz + (q->D > 0.0 ? 0.5 / (lambda * q->D) : 0.0);
    ip.src = q->src;
    ip.px = -d1.ctr / lz;
    ip.py = -d2.ctr / lz;
    ip.pc = (d1.ctr * d1.C + d2.ctr * d2.C) / lz;
    ip.cx = d1.C;
    ip.cy = d2.C;
    ip.s1 = d1.s;
    ip.s2 = d2.s;
    ip.sh2 = 0;

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
    for (int i = 0; i < 4; ++i) tp.box[i] = tb[i];
    tp.occ = occ ? 1 : 0;
    tp.ch1 = inv_phi_cheb_cached(c, k, d1.theta_max);
    tp.ch2 = inv_phi_cheb_cached(c, k, d2.theta_max);

    timing_mark(c, 0);
    FH_TRY(run_spread<R>(c, ip, nullptr, 1, N, gg, sbuf, fine, k.beta, k.poly));
    if (lds2d) {
        const int gr = (d2.m + lr.C - 1) / lr.C, gc = (d1.m + lcol.C - 1) / lcol.C;
        FH_LDS_LAUNCH(k_t3_rows, R, lr, dim3(xcd_blocks(gr)), c->stream, fine, d1.nf, d2.nf, up, d1.m, d2.m, lr.C,
                      gr, lr.plan, ip1, ip2);
        FH_LDS_LAUNCH(k_t3_cols, R, lcol, dim3(xcd_blocks(gc)), c->stream, up, d1.m, d2.m, lcol.C, gc, lcol.plan);
        FH_HIP(hipGetLastError());
    } else {
        hipLaunchKernelGGL((k_t3_precorrect<R>), dim3(nblocks(d1.m, 256), d2.m), dim3(256), 0, c->stream, fine,
                           d1.nf, d2.nf, up, d1.m, d2.m, ip1, ip2);
        FH_HIP(hipGetLastError());
        FH_TRY(fft_exec(c, fp, up));
    }
    timing_mark(c, 3);
    FH_TRY(launch_interp<R>(c, k.w, up, dxi, deta, M, k.beta, k.poly, tp, dout, perm));
    timing_mark(c, 4);
    timing_mark(c, 5);
    return FH_OK;
}

template <class R>
fh_status field_points_impl(fh_ctx* c, const fh_quad* q, double lambda, double z, int64_t M, const double* xi,
                            const double* eta, int occ, void* u, fh_memspace mem)
{
    const size_t rs = sizeof(R);
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
    if (mem == FH_MEM_DEVICE)
        return t3_core<R>(c, q, lambda, z, M, xi, eta, tb, occ, static_cast<R*>(u), false, false,
                          nullptr);
    R* staged = nullptr;
    FH_TRY(t3_core<R>(c, q, lambda, z, M, xi, eta, tb, occ, nullptr, true, true, &staged));
    FH_HIP(hipMemcpyAsync(u, staged, 2 * rs * M, hipMemcpyDeviceToHost, c->stream));
    FH_HIP(hipStreamSynchronize(c->stream));
    return FH_OK;
}

// Morton key of each target inside the set's box (16 bits per axis, clamped;
// non-finite coordinates key to 0) and its index.
__global__ void k_target_keys(const double* __restrict__ xs, const double* __restrict__ ys, int64_t M, double x0,
                              double sx, double y0, double sy, uint32_t* __restrict__ keys, int* __restrict__ idx)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= M) return;
    double fx = (xs[i] - x0) * sx, fy = (ys[i] - y0) * sy;
    fx = fx >= 0.0 ? fmin(fx, 65535.0) : 0.0;  // also maps NaN to 0
    fy = fy >= 0.0 ? fmin(fy, 65535.0) : 0.0;
    uint32_t qx = (uint32_t)fx, qy = (uint32_t)fy, key = 0;
    for (int b = 0; b < 16; ++b) key |= (((qx >> b) & 1u) << (2 * b)) | (((qy >> b) & 1u) << (2 * b + 1));
    keys[i] = key;
    idx[i] = (int)i;
}

__global__ void k_target_gather(const double* __restrict__ xs, const double* __restrict__ ys,
                                const int* __restrict__ perm, int64_t M, double* __restrict__ ox,
                                double* __restrict__ oy)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= M) return;
    const int k = perm[i];
    ox[i] = xs[k];
    oy[i] = ys[k];
}

// Field at a target set; no host synchronisation unless the output is host
// memory.
template <class R>
fh_status field_targets_impl(fh_ctx* c, const fh_quad* q, double lambda, double z, const fh_targets* t, int occ,
                             void* u, fh_memspace mem)
{
    const int64_t M = t->M;
    if (M == 0) return FH_OK;
    if (mem == FH_MEM_DEVICE)
        return t3_core<R>(c, q, lambda, z, M, t->xs, t->ys, t->box, occ, static_cast<R*>(u), false,
                          false, nullptr, t->perm);
    R* staged = nullptr;
    FH_TRY(t3_core<R>(c, q, lambda, z, M, t->xs, t->ys, t->box, occ, nullptr, false, true, &staged, t->perm));
    FH_HIP(hipMemcpyAsync(u, staged, 2 * sizeof(R) * M, hipMemcpyDeviceToHost, c->stream));
    FH_HIP(hipStreamSynchronize(c->stream));
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

fh_status counters_ready(fh_ctx* c, int64_t n)
{
    n = std::max<int64_t>(n, 1);
    if (n > c->tile_cnt_cap) {
        if (c->tile_cnt) {
            FH_HIP(hipStreamSynchronize(c->stream));
            FH_TRY(dev_free(c, c->tile_cnt));
            c->tile_cnt = nullptr;
            c->tile_cnt_cap = 0;
        }
        const int64_t cap = std::max<int64_t>(n + n / 4, 4096);
        void* p = nullptr;
        FH_TRY(dev_alloc(c, sizeof(int) * (size_t)cap, &p));
        c->tile_cnt = static_cast<int*>(p);
        c->tile_cnt_cap = cap;
        c->tile_cnt_dirty = true;
    }
    if (c->tile_cnt_dirty) {
        FH_TRY(launch_zero(c, c->tile_cnt, sizeof(int) * (size_t)c->tile_cnt_cap));
        c->tile_cnt_dirty = false;
    }
    return FH_OK;
}

// Bounding boxes of one or two point sets with a single readback.
fh_status device_bbox2(fh_ctx* c, const double* x1, const double* y1, int64_t n1, double* bb1, const double* x2,
                       const double* y2, int64_t n2, double* bb2)
{
    const int parts = 512;
    if (!c->bbox_dev) {
        void* p = nullptr;
        FH_TRY(dev_alloc(c, sizeof(double) * (10 * parts + 16), &p));
        c->bbox_dev = static_cast<double*>(p);
    }
    if (!c->bbox_host) {
        void* h = nullptr;
        FH_HIP(hipHostMalloc(&h, sizeof(double) * 16, 0));
        c->bbox_host = static_cast<double*>(h);
    }
    double* dv = c->bbox_dev;
    double* hv = c->bbox_host;
    const double* xs[2] = {x1, x2};
    const double* ys[2] = {y1, y2};
    const int64_t ns[2] = {n1, bb2 ? n2 : 0};
    double* outs[2] = {bb1, bb2};
    bool any = false;
    for (int s = 0; s < 2; ++s) {
        if (ns[s] <= 0) continue;
        any = true;
        const unsigned g = (unsigned)std::min<int64_t>(parts, (ns[s] + 255) / 256);
        hipLaunchKernelGGL(k_bbox_partial, dim3(g), dim3(256), 0, c->stream, xs[s], ys[s], ns[s], dv + 5 * parts * s);
        hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(256), 0, c->stream, dv + 5 * parts * s, (int)g,
                           dv + 10 * parts + 8 * s);
    }
    if (any) {
        FH_HIP(hipGetLastError());
        FH_HIP(hipMemcpyAsync(hv, dv + 10 * parts, sizeof(double) * 16, hipMemcpyDeviceToHost, c->stream));
        FH_HIP(hipStreamSynchronize(c->stream));
    }
    for (int s = 0; s < 2; ++s) {
        if (!outs[s]) continue;
        if (ns[s] <= 0) {
            outs[s][0] = outs[s][1] = outs[s][2] = outs[s][3] = 0.0;
            continue;
        }
        for (int q = 0; q < 4; ++q) outs[s][q] = hv[8 * s + q];
        FH_ARG(hv[8 * s + 4] == 0.0, FH_ERR_NONFINITE, "non-finite coordinate among %lld points", (long long)ns[s]);
    }
    return FH_OK;
}

fh_status device_bbox(fh_ctx* c, const double* x, const double* y, int64_t n, double* bb)
{
    return device_bbox2(c, x, y, n, bb, nullptr, nullptr, 0, nullptr);
}

}  // namespace fh

using namespace fh;

extern "C" {

fh_status fh_field_grid(fh_ctx* c, const fh_quad* q, double lambda, double z, int32_t n1, int32_t n2, double h1,
                        double h2, double xc, double yc, int32_t occulter, void* u, fh_memspace mem)
{
    try {
        FH_ARG(c && q && u, FH_ERR_INVALID_ARG, "NULL argument");
        FH_ARG(q->ctx->device == c->device, FH_ERR_INVALID_ARG, "quadrature lives on another device");
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
        FH_ARG(q->ctx->device == c->device, FH_ERR_INVALID_ARG, "quadrature lives on another device");
        FH_ARG(M >= 0, FH_ERR_INVALID_ARG, "M must be >= 0");
        FH_ARG(M == 0 || (xi && eta && u), FH_ERR_INVALID_ARG, "NULL target or output array");
        FH_ARG(mem == FH_MEM_HOST || mem == FH_MEM_DEVICE, FH_ERR_INVALID_ARG, "bad memspace");
        FH_TRY(check_lz(lambda, z));
        FH_ARG(q->N < ((int64_t)1 << 31), FH_ERR_UNSUPPORTED, "at most 2^31 - 1 nodes per call");
        FH_HIP(hipSetDevice(c->device));
        if (c->prec == FH_FP64) return field_points_impl<double>(c, q, lambda, z, M, xi, eta, occulter, u, mem);
        return field_points_impl<float>(c, q, lambda, z, M, xi, eta, occulter, u, mem);
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_targets_create(fh_ctx* c, int64_t M, const double* xi, const double* eta, const double* box,
                            fh_memspace mem, fh_targets** out)
{
    try {
        FH_ARG(c && out, FH_ERR_INVALID_ARG, "NULL argument");
        *out = nullptr;
        FH_ARG(M >= 0 && M < ((int64_t)1 << 31), FH_ERR_INVALID_ARG, "M must be in [0, 2^31)");
        FH_ARG(M == 0 || (xi && eta), FH_ERR_INVALID_ARG, "NULL target array");
        FH_ARG(mem == FH_MEM_HOST || mem == FH_MEM_DEVICE, FH_ERR_INVALID_ARG, "bad memspace");
        if (box) {
            for (int i = 0; i < 4; ++i) FH_ARG(std::isfinite(box[i]), FH_ERR_NONFINITE, "box not finite");
            FH_ARG(box[0] <= box[1] && box[2] <= box[3], FH_ERR_INVALID_ARG, "box needs xmin <= xmax, ymin <= ymax");
        }
        FH_HIP(hipSetDevice(c->device));
        std::unique_ptr<fh_targets> t(new fh_targets());
        t->ctx = c;
        t->M = M;
        double tb[4] = {0.0, 0.0, 0.0, 0.0};
        if (box) {
            for (int i = 0; i < 4; ++i) tb[i] = box[i];
        } else if (M > 0 && mem == FH_MEM_HOST) {
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
        } else if (M > 0) {
            FH_TRY(device_bbox(c, xi, eta, M, tb));
        }
        for (int i = 0; i < 4; ++i) t->box[i] = tb[i];
        if (mem == FH_MEM_DEVICE || M == 0) {
            // device arrays are used in place
            t->xs = xi;
            t->ys = eta;
            *out = t.release();
            return FH_OK;
        }
        // host arrays: a library copy (the caller may release them on return)
        const size_t cb = aligned_bytes(sizeof(double) * (size_t)M);
        t->buf_bytes = 2 * cb;
        auto it = c->pool.find(t->buf_bytes);
        void* p = nullptr;
        if (it != c->pool.end() && !it->second.empty()) {
            p = it->second.back();
            it->second.pop_back();
        } else {
            FH_TRY(dev_alloc(c, t->buf_bytes, &p));
        }
        t->buf = p;
        double* dx = static_cast<double*>(p);
        double* dy = reinterpret_cast<double*>(static_cast<char*>(p) + cb);
        hipError_t e1 = hipMemcpyAsync(dx, xi, sizeof(double) * M, hipMemcpyHostToDevice, c->stream);
        hipError_t e2 = hipMemcpyAsync(dy, eta, sizeof(double) * M, hipMemcpyHostToDevice, c->stream);
        hipError_t e3 = hipStreamSynchronize(c->stream);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
            c->pool[t->buf_bytes].push_back(p);
            (void)hipGetLastError();
            set_error("copying the targets to the device failed");
            return FH_ERR_HIP;
        }
        t->xs = dx;
        t->ys = dy;
        *out = t.release();
        return FH_OK;
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_targets_size(const fh_targets* t, int64_t* M)
{
    FH_ARG(t && M, FH_ERR_INVALID_ARG, "NULL argument");
    *M = t->M;
    return FH_OK;
}

fh_status fh_targets_box(const fh_targets* t, double* box)
{
    FH_ARG(t && box, FH_ERR_INVALID_ARG, "NULL argument");
    for (int i = 0; i < 4; ++i) box[i] = t->box[i];
    return FH_OK;
}

fh_status fh_targets_sort(fh_targets* t)
{
    try {
        FH_ARG(t, FH_ERR_INVALID_ARG, "NULL target set");
        const int64_t M = t->M;
        if (M < 2 || t->perm) return FH_OK;
        fh_ctx* c = t->ctx;
        FH_HIP(hipSetDevice(c->device));
        const double* box = t->box;
        const double sx = box[1] > box[0] ? 65535.0 / (box[1] - box[0]) : 0.0;
        const double sy = box[3] > box[2] ? 65535.0 / (box[3] - box[2]) : 0.0;
        // the sorted copy and the permutation live in one library buffer
        const size_t cb = aligned_bytes(sizeof(double) * (size_t)M);
        const size_t pb = aligned_bytes(sizeof(int) * (size_t)M);
        const size_t bytes = 2 * cb + pb;
        void* nb = nullptr;
        auto it = c->pool.find(bytes);
        if (it != c->pool.end() && !it->second.empty()) {
            nb = it->second.back();
            it->second.pop_back();
        } else {
            FH_TRY(dev_alloc(c, bytes, &nb));
        }
        double* ox = static_cast<double*>(nb);
        double* oy = reinterpret_cast<double*>(static_cast<char*>(nb) + cb);
        int* perm = reinterpret_cast<int*>(static_cast<char*>(nb) + 2 * cb);
        size_t temp = 0;
        FH_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, temp, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                                  (const int*)nullptr, (int*)nullptr, (int)M, 0, 32, c->stream));
        const size_t kb = aligned_bytes(sizeof(uint32_t) * (size_t)M);
        fh_status s = arena_reserve(c, 2 * kb + pb + aligned_bytes(std::max<size_t>(temp, 1)));
        if (s != FH_OK) {
            c->pool[bytes].push_back(nb);
            return s;
        }
        uint32_t* kin = c->arena.take<uint32_t>((size_t)M);
        uint32_t* kout = c->arena.take<uint32_t>((size_t)M);
        int* iin = c->arena.take<int>((size_t)M);
        void* tmp = c->arena.take<char>(std::max<size_t>(temp, 1));
        hipLaunchKernelGGL(k_target_keys, dim3(nblocks(M, 256)), dim3(256), 0, c->stream, t->xs, t->ys, M, box[0],
                           sx, box[2], sy, kin, iin);
        FH_HIP(hipGetLastError());
        FH_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, temp, kin, kout, iin, perm, (int)M, 0, 32, c->stream));
        hipLaunchKernelGGL(k_target_gather, dim3(nblocks(M, 256)), dim3(256), 0, c->stream, t->xs, t->ys, perm, M,
                           ox, oy);
        FH_HIP(hipGetLastError());
        // a previous library copy goes back to the pool (stream order keeps
        // the gather above before any reuse)
        if (t->buf) c->pool[t->buf_bytes].push_back(t->buf);
        t->buf = nb;
        t->buf_bytes = bytes;
        t->xs = ox;
        t->ys = oy;
        t->perm = perm;
        return FH_OK;
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_targets_destroy(fh_targets* t)
{
    if (!t) return FH_OK;
    if (t->buf) {
        try {
            t->ctx->pool[t->buf_bytes].push_back(t->buf);
        } catch (...) {
            (void)dev_free(t->ctx, t->buf);
        }
    }
    delete t;
    return FH_OK;
}

fh_status fh_field_targets(fh_ctx* c, const fh_quad* q, double lambda, double z, const fh_targets* t,
                           int32_t occulter, void* u, fh_memspace mem)
{
    try {
        FH_ARG(c && q && t, FH_ERR_INVALID_ARG, "NULL argument");
        FH_ARG(q->ctx->device == c->device, FH_ERR_INVALID_ARG, "quadrature lives on another device");
        FH_ARG(t->ctx->device == c->device, FH_ERR_INVALID_ARG, "target set lives on another device");
        FH_ARG(t->M == 0 || u, FH_ERR_INVALID_ARG, "NULL output array");
        FH_ARG(mem == FH_MEM_HOST || mem == FH_MEM_DEVICE, FH_ERR_INVALID_ARG, "bad memspace");
        FH_TRY(check_lz(lambda, z));
        FH_ARG(q->N < ((int64_t)1 << 31), FH_ERR_UNSUPPORTED, "at most 2^31 - 1 nodes per call");
        FH_HIP(hipSetDevice(c->device));
        if (c->prec == FH_FP64) return field_targets_impl<double>(c, q, lambda, z, t, occulter, u, mem);
        return field_targets_impl<float>(c, q, lambda, z, t, occulter, u, mem);
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_field_grid_batch(fh_ctx* c, int32_t B, const fh_quad* const* q, const double* lambda, const double* z,
                              int32_t n1, int32_t n2, double h1, double h2, double xc, double yc,
                              const int32_t* occulter, void* u)
{
    try {
        FH_ARG(c && q && lambda && z && occulter && u, FH_ERR_INVALID_ARG, "NULL argument");
        FH_ARG(B >= 1, FH_ERR_INVALID_ARG, "B must be >= 1");
        FH_TRY(check_grid(n1, n2, h1, h2, xc, yc));
        for (int b = 0; b < B; ++b) {
            FH_ARG(q[b] && q[b]->ctx->device == c->device, FH_ERR_INVALID_ARG, "quadrature %d NULL or on another device", b);
            FH_TRY(check_lz(lambda[b], z[b]));
        }
        FH_HIP(hipSetDevice(c->device));
        c->timing_kind = 3;
        if (c->prec == FH_FP64)
            return t1_pipeline<double>(c, B, q, lambda, z, n1, n2, h1, h2, xc, yc, occulter, static_cast<double*>(u),
                                       true, 0, nullptr);
        return t1_pipeline<float>(c, B, q, lambda, z, n1, n2, h1, h2, xc, yc, occulter, static_cast<float*>(u), true,
                                  0, nullptr);
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_field_grid_batch_rebuild(fh_ctx* c, int32_t B, fh_quad* const* q, const double* lambda,
                                      const double* z, int32_t n1, int32_t n2, double h1, double h2, double xc,
                                      double yc, const int32_t* occulter, void* u)
{
    try {
        FH_ARG(c && q && lambda && z && occulter && u, FH_ERR_INVALID_ARG, "NULL argument");
        FH_ARG(B >= 1, FH_ERR_INVALID_ARG, "B must be >= 1");
        FH_TRY(check_grid(n1, n2, h1, h2, xc, yc));
        for (int b = 0; b < B; ++b) {
            FH_ARG(q[b] && q[b]->ctx->device == c->device, FH_ERR_INVALID_ARG, "quadrature %d NULL or on another device", b);
            FH_ARG(static_cast<bool>(q[b]->rebuild), FH_ERR_UNSUPPORTED,
                   "quadrature %d cannot be rebuilt on the device (radial curves and polygons of up to %d vertices "
                   "can)",
                   b, kPolyByValue);
            FH_TRY(check_lz(lambda[b], z[b]));
        }
        FH_HIP(hipSetDevice(c->device));
        c->timing_kind = 3;
        const fh_quad* const* cq = q;
        if (c->prec == FH_FP64)
            return t1_pipeline<double>(c, B, cq, lambda, z, n1, n2, h1, h2, xc, yc, occulter,
                                       static_cast<double*>(u), true, 0, nullptr, true);
        return t1_pipeline<float>(c, B, cq, lambda, z, n1, n2, h1, h2, xc, yc, occulter, static_cast<float*>(u),
                                  true, 0, nullptr, true);
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

}  // extern "C"

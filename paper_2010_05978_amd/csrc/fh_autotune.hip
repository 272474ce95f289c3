// fh_autotune.hip -- choice of spread method, work-item size, tile edge and
// upsampling factor by timing the grid field (one rule, or a batch as it
// replays from its graph) on the device.
//
// Every candidate meets the context's tolerance (the kernel width follows
// from sigma and the tolerance), so the search only trades spread work
// against FFT size and parallelism.  Results are cached per context and,
// optionally, in a JSON-lines file keyed by precision, tolerance, grid size
// and the node count's power-of-two class (for a batch: the instance count
// and the classes of the total and of the largest instance).
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "fh_common.hpp"

namespace fh {
namespace {

int size_class(int64_t N)
{
    int cls = 0;
    while (((int64_t)1 << cls) < std::max<int64_t>(N, 1)) ++cls;
    return cls;
}

std::string tune_key(const fh_ctx* c, int n1, int n2, int64_t N)
{
    char buf[160];
    snprintf(buf, sizeof(buf), "%s|%.3e|%d|%d|%d", c->prec == FH_FP64 ? "fp64" : "mixed", c->tol, n1, n2,
             size_class(N));
    return buf;
}

// A batch's signature: precision, tolerance, grid, instance count and the
// node-count classes of the whole batch and of its largest instance.
std::string batch_key(const fh_ctx* c, int B, int n1, int n2, int64_t Ntot, int64_t Nmax)
{
    char buf[200];
    snprintf(buf, sizeof(buf), "batch|%s|%.3e|%d|%d|%d|%d|%d", c->prec == FH_FP64 ? "fp64" : "mixed", c->tol, n1,
             n2, B, size_class(Ntot), size_class(Nmax));
    return buf;
}

bool cache_lookup(const char* path, const std::string& key, fh_options* o)
{
    if (!path) return false;
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        const std::string tag = "\"key\": \"" + key + "\"";
        if (line.find(tag) == std::string::npos) continue;
        fh_options t{};
        const char* p = std::strstr(line.c_str(), "\"sigma\":");
        if (!p || std::sscanf(p, "\"sigma\": %lf, \"tile\": %d, \"max_subproblem\": %d, \"spread_method\": %d",
                              &t.sigma, &t.tile, &t.max_subproblem, &t.spread_method) != 4)
            continue;
        *o = t;  // the last matching line wins
        found = true;
    }
    return found;
}

void cache_append(const char* path, const std::string& key, const fh_options& o, double ms)
{
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    if (!f) return;
    char buf[400];
    snprintf(buf, sizeof(buf),
             "{\"key\": \"%s\", \"sigma\": %.2f, \"tile\": %d, \"max_subproblem\": %d, \"spread_method\": %d, "
             "\"ms\": %.5f}\n",
             key.c_str(), o.sigma, o.tile, o.max_subproblem, o.spread_method, ms);
    f << buf;
}

}  // namespace
}  // namespace fh

using namespace fh;

namespace fh {
namespace {

// The tuned fields of t over the caller's other options (kernel width, beta
// and the deterministic flag are kept).
fh_options merged(const fh_options& saved, const fh_options& t)
{
    fh_options o = saved;
    o.sigma = t.sigma;
    o.kernel_width = 0;
    o.beta = 0.0;
    o.tile = t.tile;
    o.max_subproblem = t.max_subproblem;
    o.spread_method = t.spread_method;
    return o;
}

// Time `call` (which enqueues one field evaluation into u) for every
// candidate that meets the context's tolerance; keep the fastest in the
// context.  Each candidate runs twice untimed (for a batch: capture and a
// first replay), then `reps` times between events.
template <class Call>
fh_status tune(fh_ctx* c, int n, const std::vector<int>& methods, const std::vector<int>& tiles,
               const std::vector<int>& items, int reps, const std::string& key, const char* cache_path,
               fh_options* best, Call call)
{
    fh_options hit{};
    if (cache_lookup(cache_path, key, &hit)) {
        c->opt = merged(c->opt, hit);
        *best = c->opt;
        return FH_OK;
    }
    const fh_options saved = c->opt;
    hipEvent_t e0, e1;
    FH_HIP(hipEventCreate(&e0));
    FH_HIP(hipEventCreate(&e1));
    const bool timing = c->timing;
    c->timing = false;
    double best_ms = 1e300;
    fh_options best_o = saved;
    fh_status st = FH_OK;
    // In FP32 the deconvolution at sigma = 1.25 lifts the rounding of
    // the spread and FFT near the band edge by about 1/Phi(pi/sigma)
    // over 1/Phi(0) (~150 at tolerance 1e-5), which leaves the field
    // near 1e-5 relative: mixed contexts tune over sigma = 2 only unless
    // the tolerance is looser than 1e-4.
    const bool try_125 = c->prec == FH_FP64 || c->tol >= 1e-4;
    for (double sigma : {2.0, 1.25})
        for (int method : methods)
            for (int tile : tiles)  // 0: the method's own choice (16 but for method 5)
                for (int P : items) {  // 0: sized from the node count
                    if (sigma == 1.25 && !try_125) continue;
                    if (tile == 0 && method != 5) continue;
                    fh_options o = saved;
                    o.sigma = sigma;
                    o.kernel_width = 0;
                    o.beta = 0.0;
                    o.tile = tile;
                    o.max_subproblem = P;
                    o.spread_method = method;
                    c->opt = o;
                    // the kernel must fit at this sigma without widening
                    const EsKernel k = choose_kernel(c, n);
                    if (k.sigma != sigma || k.clamped) continue;
                    fh_status s = FH_OK;
                    for (int w = 0; w < 2 && s == FH_OK; ++w) s = call();
                    if (s == FH_ERR_UNSUPPORTED) continue;  // e.g. tile too large for the LDS budget
                    if (s != FH_OK) {
                        st = s;
                        break;
                    }
                    FH_HIP(hipEventRecord(e0, c->stream));
                    for (int r = 0; r < reps && s == FH_OK; ++r) s = call();
                    FH_HIP(hipEventRecord(e1, c->stream));
                    FH_HIP(hipEventSynchronize(e1));
                    float ms = 0;
                    FH_HIP(hipEventElapsedTime(&ms, e0, e1));
                    if (s != FH_OK) {
                        st = s;
                        break;
                    }
                    if (ms / reps < best_ms) {
                        best_ms = ms / reps;
                        best_o = o;
                    }
                }
    c->timing = timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != FH_OK) {
        c->opt = saved;
        return st;
    }
    c->opt = best_o;
    *best = best_o;
    cache_append(cache_path, key, best_o, best_ms);
    return FH_OK;
}

}  // namespace
}  // namespace fh

extern "C" {

fh_status fh_autotune_grid(fh_ctx* c, const fh_quad* q, double lambda, double z, int32_t n1, int32_t n2, double h1,
                           double h2, const char* cache_path, fh_options* best)
{
    try {
        FH_ARG(c && q && best, FH_ERR_INVALID_ARG, "NULL argument");
        FH_ARG(q->ctx->device == c->device, FH_ERR_INVALID_ARG, "quadrature lives on another device");
        FH_ARG(n1 > 0 && n2 > 0 && n1 % 2 == 0 && n2 % 2 == 0, FH_ERR_ODD_GRID, "grid sizes must be even");
        FH_HIP(hipSetDevice(c->device));
        const size_t ubytes = (c->prec == FH_FP64 ? 16 : 8) * (size_t)n1 * n2;
        void* u = nullptr;
        FH_TRY(dev_alloc(c, ubytes, &u));
        const fh_status st =
            tune(c, std::max(n1, n2), {2, 5, 4, 3, 1}, {0, 16, 32}, {0, 64, 256, 1024, 4096}, 5,
                 tune_key(c, n1, n2, q->N), cache_path, best, [&]() {
                     return fh_field_grid(c, q, lambda, z, n1, n2, h1, h2, 0.0, 0.0, 0, u, FH_MEM_DEVICE);
                 });
        (void)dev_free(c, u);
        return st;
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_autotune_batch(fh_ctx* c, int32_t B, const fh_quad* const* q, const double* lambda, const double* z,
                            int32_t n1, int32_t n2, double h1, double h2, const char* cache_path, fh_options* best)
{
    try {
        FH_ARG(c && q && lambda && z && best && B > 0, FH_ERR_INVALID_ARG, "NULL argument or B <= 0");
        FH_ARG(n1 > 0 && n2 > 0 && n1 % 2 == 0 && n2 % 2 == 0, FH_ERR_ODD_GRID, "grid sizes must be even");
        int64_t Ntot = 0, Nmax = 0;
        for (int b = 0; b < B; ++b) {
            FH_ARG(q[b], FH_ERR_INVALID_ARG, "quadrature %d is NULL", b);
            FH_ARG(q[b]->ctx->device == c->device, FH_ERR_INVALID_ARG, "quadrature %d lives on another device", b);
            Ntot += q[b]->N;
            Nmax = std::max<int64_t>(Nmax, q[b]->N);
        }
        FH_HIP(hipSetDevice(c->device));
        const size_t ubytes = (c->prec == FH_FP64 ? 16 : 8) * (size_t)B * n1 * n2;
        void* u = nullptr;
        FH_TRY(dev_alloc(c, ubytes, &u));
        const std::vector<int32_t> occ(B, 0);
        // the batched call as it runs: captured into a graph, then replayed
        const fh_status st =
            tune(c, std::max(n1, n2), {5, 2, 4}, {0, 16, 32}, {0, 256, 512, 1024, 2048}, 3, batch_key(c, B, n1, n2, Ntot, Nmax),
                 cache_path, best, [&]() {
                     return fh_field_grid_batch(c, B, q, lambda, z, n1, n2, h1, h2, 0.0, 0.0, occ.data(), u);
                 });
        (void)dev_free(c, u);
        return st;
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

}  // extern "C"

// fh_common.hpp -- internal declarations of libfresnel_hip (not installed).
//
// Shared between the host-side control code and the HIP kernels: the context
// and quadrature objects, workspace arena, error reporting, kernel-parameter
// structs and the small helpers that several translation units need.
#pragma once

#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <array>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "fresnel_hip.h"

namespace fh {

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));

#define FH_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            ::fh::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),    \
                            __FILE__, __LINE__);                                      \
            return (e_ == hipErrorOutOfMemory) ? FH_ERR_ALLOC : FH_ERR_HIP;           \
        }                                                                             \
    } while (0)

#define FH_TRY(call)                        \
    do {                                    \
        fh_status s_ = (call);              \
        if (s_ != FH_OK) return s_;         \
    } while (0)

#define FH_ARG(cond, code, ...)             \
    do {                                    \
        if (!(cond)) {                      \
            ::fh::set_error(__VA_ARGS__);   \
            return code;                    \
        }                                   \
    } while (0)

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr unsigned kInjectFftPlan = 1u;
constexpr unsigned kInjectCapture = 2u;
constexpr int kMaxWidth = 20;
constexpr int kMaxFourier = 64;

// ------------------------------------------------------------ ES kernel
// phi(z) = exp(beta (sqrt(1 - z^2) - 1)), |z| <= 1, spanning `w` cells.
struct EsKernel {
    int w = 0;
    double beta = 0;
    double sigma = 2.0;
    bool clamped = false;        // the tolerance needs a wider kernel than supported
    const void* poly = nullptr;  // device polynomial table (es_poly_attach) or null
};

// The kernel on one stencil is evaluated as w polynomials of degree
// poly_np(w) - 1 in t = 2 d + w - 1, d in [-w/2, -w/2 + 1) the offset of
// the first stencil cell: poly[j * w + a] is the coefficient of t^(deg - j)
// for stencil index a, in the working precision.
// poly_np(w) is the fewest coefficients whose Chebyshev interpolants come
// within a quarter of the error floor that the square-root branch point of
// phi at the stencil edges puts under every degree (near e^-beta / 2): more
// only cost arithmetic.  From width 14 on the floor is rounding.
__host__ __device__ constexpr int poly_np(int w)
{
    return w <= 3 ? 6 : w <= 5 ? 7 : w <= 8 ? w + 2 : w <= 11 ? 11 : w == 12 ? 13 : w + 2;
}

// The pieces mirror each other: the piece of stencil cell w - 1 - a at t is
// that of cell a at -t (phi is even).  The matrix-core spread evaluates each
// such pair from one piece split into even and odd parts in s = t^2,
// P_a(t) = E(s) + t O(s) and P_{w-1-a}(t) = E(s) - t O(s), for half the
// multiply-adds.  Its table follows the plain one in the same allocation:
// for pair p < poly_npair(w), E's poly_ne(w) coefficients (highest power
// first), then O's poly_no(w), at eo[j * npair + p].
__host__ __device__ constexpr int poly_npair(int w) { return (w + 1) / 2; }
__host__ __device__ constexpr int poly_ne(int w) { return (poly_np(w) - 1) / 2 + 1; }
__host__ __device__ constexpr int poly_no(int w) { return poly_np(w) / 2; }

// Wavefront spread staging: per point its 2w kernel values and its strength
// (2 reals), for 64 points, and the kernel arguments of 64 points for each of
// up to two wavefronts.
inline size_t spread_staging_bytes(int w, size_t rsize)
{
    return rsize * ((size_t)64 * (2 * (size_t)w + 2) + 128);
}

// 1/Phi(theta) for |theta| <= theta_max as a Chebyshev series in
// s = 2 (theta/theta_max)^2 - 1 (Phi is even and entire).
constexpr int kMaxCheb = 96;
struct InvPhiCheb {
    double theta_max = 0;
    int deg = 0;
    double c[kMaxCheb + 1];
};

// ----------------------------------------------- per-instance prep params
// Source-side parameters of one (quadrature, lambda, z) instance.
//   phase in turns: t = (x^2 + y^2) pa + x px + y py + pc
//   fine-grid coordinate: g1 = (x - cx) s1, g2 = (y - cy) s2 - sh2, where the
//   integer sh2 is the first fine-grid row of the instance's window
//   src: the rule's source term per node (N interleaved complex), or null
struct InstParams {
    const double* x;
    const double* y;
    const double* w;
    int64_t N;
    int64_t node_off;  // first slot of this instance in the concatenated node range
    int32_t tile_off;  // first tile id of this instance
    int32_t sh2;
    double pa, px, py, pc;
    double cx, cy, s1, s2;
    const double* src;
};

// Tiles need not divide the grid: the last tile of a row (of a column)
// covers the cells left, ntx T - nf1 (nty T - rows) fewer than T, and a padded
// tile that wraps around the period lands that many cells earlier.
struct GridGeom {
    int nf1, nf2;  // fine grid period (x fastest)
    int T;         // tile edge
    int ntx, nty;  // tiles per dimension (nty covers the held rows), rounded up
    int W;         // kernel width
    int L;         // padded tile edge T + W - 1
    int P;         // min points per spread work item
    int method;    // 1: thread per point, 2: wavefront per point, ...
    int rows;      // fine-grid rows held per instance (nf2 unless windowed)
    int wrap_y;    // 1 when the held rows are the whole period
    int padx, pady;  // ntx T - nf1 and nty T - rows (0 when T divides them)
};

struct Sub {
    int tile;
    int start;
    int end;
};

// ---------------------------------------------------------- rocFFT plans
struct FftPlan {
    rocfft_plan plan = nullptr;
    rocfft_execution_info info = nullptr;
    void* work = nullptr;
    size_t work_bytes = 0;
};

// ------------------------------------------------------------- workspace
// One stream-ordered bump arena per context.  A call first sums what it
// needs, grows the arena if necessary (synchronising), then carves buffers.
struct Arena {
    char* base = nullptr;
    size_t cap = 0;
    size_t used = 0;
    void reset() { used = 0; }
    template <class T>
    T* take(size_t count) {
        size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
        T* p = reinterpret_cast<T*>(base + used);
        used += bytes;
        return p;
    }
};
inline size_t aligned_bytes(size_t b) { return (b + 255) & ~size_t(255); }

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

}  // namespace fh

// ---------------------------------------------------------------- objects
struct fh_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    fh_precision prec = FH_FP64;
    double tol = 1e-9;
    fh_options opt{};
    int cu_count = 256;
    // Stage timing: every timed call records 6 events on the context stream
    // (start, after bin, after spread, after FFT, after finish, end); the
    // sets are read back only when the caller asks, so timing adds no sync.
    // Calls are tallied per kind: 0 grid, 1 points, 2 adjoint, 3 batch.
    bool timing = false;
    int timing_kind = 0;
    std::vector<std::pair<int, std::array<hipEvent_t, 6>>> ev_sets;  // recorded, not yet read
    std::vector<std::array<hipEvent_t, 6>> ev_free;                   // reusable
    std::array<hipEvent_t, 6> ev_cur{};
    bool ev_open = false;
    double last_ms[5]{};
    double sum_ms[4][5]{};
    int64_t timed_calls[4]{};

    fh::Arena arena;
    size_t alloc_cap = 0;  // optional cap on device bytes (testing)
    size_t alloc_total = 0;
    // Failures forced from the host for tests (FH_INJECT_FAULT at creation):
    // kInjectFftPlan makes every new rocFFT plan fail, kInjectCapture makes
    // every graph capture be refused.
    unsigned inject = 0;

    std::map<int, double*> gl_cache;  // device GL tables: x[q], w[q]
    std::map<std::tuple<int, int, int, long long>, double*> iphi_cache;
    std::map<std::tuple<int, int, int, int>, fh::FftPlan> fft_cache;
    std::map<size_t, std::vector<void*>> pool;  // freed quadrature buffers by size
    std::map<std::string, fh::GraphEntry> graph_cache;
    hipStream_t gstream = nullptr;  // private stream for graph capture/replay
    hipEvent_t gev_in = nullptr, gev_out = nullptr;
    std::map<std::tuple<int, long long, long long>, fh::InvPhiCheb> cheb_cache;
    std::map<std::tuple<int, long long, int>, void*> poly_cache;  // (w, beta bits, precision)
    std::map<std::pair<int, int>, void*> lds_tw_cache;             // (LDS FFT length, real size)
    std::map<void*, size_t> owned;  // every hipMalloc'd block and its size
    double* bbox_dev = nullptr;      // bounding-box reduction scratch
    double* bbox_host = nullptr;     // pinned readback of the box
    // Binning counters kept at zero between calls: the tile counts of the
    // spread, zeroed again by the reduce that ends each spread.  A call that
    // stops between the count and the reset leaves them dirty, and the next
    // call clears them first.
    int* tile_cnt = nullptr;
    int64_t tile_cnt_cap = 0;
    bool tile_cnt_dirty = false;
    uint64_t* order_sig = nullptr;   // fh_order_after: counter written by this stream
    uint64_t order_seq = 0;          // last value enqueued for it
};

namespace fh {
// Polygons of up to this many vertices pass them to the rule kernel by value.
constexpr int kPolyByValue = 128;

// The stable binning's sort of n (tile key, node index) pairs by the low
// key_bits of the key, on the context stream, and its scratch bytes
// (fh_field.hip).
size_t tile_sort_bytes(int64_t n);
fh_status tile_sort(fh_ctx* c, const uint32_t* key, uint32_t* key_sorted, const int* vals, int* vals_sorted,
                    int64_t n, int key_bits, void* tmp, size_t tmp_bytes);
}  // namespace fh

struct fh_quad {
    fh_ctx* ctx = nullptr;
    int64_t N = 0;
    double* buf = nullptr;  // 3 N doubles: x, y, w
    size_t buf_bytes = 0;
    double* x = nullptr;
    double* y = nullptr;
    double* w = nullptr;
    // Illumination (fh_quad_set_illumination): a source term per node (N
    // interleaved complex in its own allocation, never pooled) or null, and
    // the distance D of a point source (0: plane wave).
    double* src = nullptr;
    double D = 0.0;
    bool bbox_valid = false;
    double bbox[4] = {0, 0, 0, 0};  // xmin, xmax, ymin, ymax
    // Enqueues the rule kernels again, in place, from the boundary parameters
    // the rule was made from (rules built by one launch with their
    // parameters by value: radial curves and small polygons); empty for the
    // others.
    std::function<fh_status()> rebuild;
    // Computes the bounding box on the host when a call first needs it
    // (generated rules whose box comes from their boundary parameters);
    // empty: a device reduction over the nodes.
    std::function<void(double*)> host_box;
};

// A scattered-target set: the device coordinates (the caller's arrays, or a
// library copy of host arrays) and the box the type-3 grids are planned from.
struct fh_targets {
    fh_ctx* ctx = nullptr;
    int64_t M = 0;
    void* buf = nullptr;  // library copy (host input, or sorted): xs[M], ys[M] (and perm[M] if sorted)
    size_t buf_bytes = 0;
    const double* xs = nullptr;
    const double* ys = nullptr;
    const int* perm = nullptr;     // after fh_targets_sort: caller index of each (sorted) target
    double box[4] = {0, 0, 0, 0};  // xmin, xmax, ymin, ymax
};

namespace fh {
// context services (fh_context.cpp)
fh_status dev_alloc(fh_ctx* c, size_t bytes, void** p);
fh_status dev_free(fh_ctx* c, void* p);
fh_status arena_reserve(fh_ctx* c, size_t bytes);
fh_status gl_table(fh_ctx* c, int q, const double** dev);  // x[q] then w[q]
void gl_host(int q, std::vector<double>& x, std::vector<double>& w);
EsKernel choose_kernel(const fh_ctx* c, int n_hint);
void es_poly_attach(fh_ctx* c, EsKernel& k);
constexpr int64_t kMfmaMinNodes = (int64_t)1 << 18;  // nodes per call before the matrix-core spread pays
int pick_tile(const fh_ctx* c, int nf, int w, int64_t N);
int t1_method(const fh_ctx* c, int w, int64_t N);
int next_fft_size(int n, int multiple);
double phi_hat(const EsKernel& k, double theta);
fh_status iphi_table(fh_ctx* c, const EsKernel& k, int n, int nf, const double** dev);
void inv_phi_cheb(const EsKernel& k, double theta_max, InvPhiCheb* out);
const InvPhiCheb& inv_phi_cheb_cached(fh_ctx* c, const EsKernel& k, double theta_max);
// 2D transforms of nf1 x nf2 grids (nf1 fastest), or batched 1D transforms
// of length nf1 when nf2 == 0; forward, in place, contiguous batches.
fh_status fft_plan(fh_ctx* c, int nf1, int nf2, int batch, FftPlan** out);
fh_status fft_exec(fh_ctx* c, FftPlan* p, void* data);
fh_status quad_alloc(fh_ctx* c, int64_t N, fh_quad** out);
fh_status quad_bbox(fh_ctx* c, const fh_quad* q, double* bb);
fh_status device_bbox(fh_ctx* c, const double* x, const double* y, int64_t n, double* bb);
fh_status device_bbox2(fh_ctx* c, const double* x1, const double* y1, int64_t n1, double* bb1, const double* x2,
                       const double* y2, int64_t n2, double* bb2);
void timing_mark(fh_ctx* c, int i);
void timing_finish(fh_ctx* c);

// kernel launchers shared across translation units (fh_field.hip)
fh_status launch_zero(fh_ctx* c, void* p, size_t bytes);
// Make the persistent tile counters hold n zeros (grow, or clear if dirty);
// call before carving a spread and outside any stream capture.
fh_status counters_ready(fh_ctx* c, int64_t n);
}  // namespace fh

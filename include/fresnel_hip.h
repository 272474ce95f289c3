/*
 * fresnel_hip.h -- C ABI of libfresnel_hip.so: fast scalar Fresnel diffraction
 * from binary planar apertures and occulters on AMD Instinct MI355X (gfx950).
 *
 * Method (Barnett, arXiv:2010.05978):
 *   The field of an aperture Omega at target (xi, eta) is the Fresnel integral
 *     u_ap = 1/(i lambda z) iint_Omega exp(i pi |(xi,eta)-(x,y)|^2/(lambda z)) dx dy
 *   (eq. fres; the plane propagation phase exp(2 pi i z/lambda) is dropped, as in
 *   sec. 2).  For an occulter, Babinet gives u_oc = 1 - u_ap (eq. bab).
 *   An areal quadrature (x_j, y_j, w_j) of Omega (eq. aq) turns the integral
 *   into the sum of eq. faq, which factorises (eq. split) into a source chirp
 *   c_j = exp(i pi |x_j|^2/(lambda z)) w_j, a 2D nonuniform FFT (type 3 for
 *   scattered targets, eq. nufft3 / sec. 2.1; type 1 for a uniform target grid,
 *   sec. 2.2), and a target chirp exp(i pi |xi_k|^2/(lambda z))/(i lambda z).
 *
 * Conventions used by every call:
 *   - Every call returns an fh_status; FH_OK is 0.  No C++ exception crosses
 *     the ABI.  On failure a message is available from fh_last_error() (thread
 *     local, valid until the next failing call on the same thread).
 *   - Lengths are metres (any consistent unit works; only lambda*z enters).
 *   - Complex arrays are interleaved (re, im).  In FH_FP64 contexts complex
 *     values are double (complex128); in FH_MIXED contexts the fields and
 *     field cotangents are float (complex64).  Node coordinates and weights
 *     are always double.
 *   - fh_memspace says where a caller pointer lives: FH_MEM_HOST (pageable
 *     or pinned host memory; the call copies and synchronises) or
 *     FH_MEM_DEVICE (device memory on the context's device; work is
 *     enqueued on the context's stream and the call returns without
 *     synchronising, except where noted).
 *   - Caller buffers are owned by the caller.  fh_ctx and fh_quad objects are
 *     owned by the library and released with fh_destroy / fh_quad_destroy.
 *   - One context per host thread and stream; calls on one context are
 *     serialised on its stream.
 *   - Empty inputs: a quadrature with N = 0 nodes gives u_ap = 0 (u_oc = 1);
 *     M = 0 targets is a no-op.  Nodes outside Omega and negative weights are
 *     legal (sec. 3.1 allows them for non-star-shaped domains).
 */
#ifndef FRESNEL_HIP_H
#define FRESNEL_HIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fh_status {
    FH_OK = 0,
    FH_ERR_INVALID_ARG = 1,    /* null pointer, negative size, bad option   */
    FH_ERR_ODD_GRID = 2,       /* target grid sizes must be even (sec. 2.2)  */
    FH_ERR_NONPOSITIVE_LZ = 3, /* lambda * z must be > 0                     */
    FH_ERR_NONFINITE = 4,      /* NaN or Inf scalar argument                 */
    FH_ERR_ALLOC = 5,          /* device memory exhausted (or capped)        */
    FH_ERR_HIP = 6,            /* HIP runtime error                          */
    FH_ERR_FFT = 7,            /* rocFFT plan or execution error             */
    FH_ERR_UNSUPPORTED = 8     /* valid request outside the implemented range */
} fh_status;

typedef enum fh_precision {
    FH_FP64 = 0,  /* spreading, FFT and outputs in double                    */
    FH_MIXED = 1  /* spreading and FFT in float with float accumulation;     */
                  /* chirp phases and node rescaling in double               */
} fh_precision;

typedef enum fh_memspace { FH_MEM_HOST = 0, FH_MEM_DEVICE = 1 } fh_memspace;

typedef struct fh_ctx fh_ctx;
typedef struct fh_quad fh_quad;
typedef struct fh_targets fh_targets;

/* NUFFT and spreading options.  Zero in any field means "choose
 * automatically".  The exponential-of-semicircle kernel
 * phi(z) = exp(beta (sqrt(1 - z^2) - 1)) on |z| <= 1 spans kernel_width
 * fine-grid cells; sigma is the fine-grid upsampling factor (2 or 1.25, the
 * two factors the paper reports for its FFTs, sec. 3.1). */
typedef struct fh_options {
    double sigma;           /* 2.0 or 1.25 (in FH_MIXED, 1.25 amplifies the  *
                             * FP32 rounding near the band edge and suits    *
                             * tolerances of 1e-4 and looser)                */
    int32_t kernel_width;   /* 2..20 cells                                   */
    double beta;            /* kernel shape parameter                        */
    int32_t tile;           /* spread tile edge in cells, 4..32 (the tile    *
                             * reduce needs T + W - 2 < 3 T: a padded tile   *
                             * may reach two tiles on, else the call is      *
                             * FH_ERR_UNSUPPORTED); 0: 16, or for method 5   *
                             * 17 - W when W <= 11 (a 16-cell padded tile)   */
    int32_t max_subproblem; /* nonuniform points per spread work item (a     *
                             * tile with more than 2048 items' worth gets    *
                             * larger items); 0: about 96 items per CU,      *
                             * at least 64 points each                       */
    int32_t spread_method;  /* 1: thread per point, shared LDS tile with     *
                             * atomics; 2: one or two wavefronts per work    *
                             * item, lanes over the stencil, a private LDS   *
                             * tile each, runs of points with one first cell *
                             * summed in registers and added to the tile     *
                             * (read when the run starts, written when it    *
                             * ends); 3: as 2, runs added by LDS atomics;    *
                             * 4: four wavefronts per work item, each with   *
                             * the padded tile in registers (lane per column *
                             * and row bank), tiles 8 or 16 only (else 2);   *
                             * 5: one wavefront per work item holding its    *
                             * padded tile (at most 32 x 32 cells) in        *
                             * matrix-core accumulators, four points per     *
                             * 16 x 16 x 4 product (every point costs the    *
                             * same; method 2 wins where points crowd);      *
                             * 2 to 5 sum a work item's points in a fixed    *
                             * order (the point order within a tile comes    *
                             * from atomic counters in the binning)          */
    int32_t deterministic;  /* 1: stable binning -- the nodes of each tile   *
                             * in node order (a stable radix sort of the     *
                             * tile keys instead of atomic ranks), method 1  *
                             * replaced by 2, and batched calls run eagerly  *
                             * (no graph): a call repeated with the same     *
                             * inputs and options on the same device gives   *
                             * bitwise the same field.  0: atomic ranks,     *
                             * equal to rounding only.                       */
} fh_options;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device` with precision `prec` and target
 * accuracy `tol` (the relative L2 error of the field against the exact
 * quadrature sum; e.g. 1e-9 for FH_FP64, 1e-5 for FH_MIXED).  `opt` may be
 * NULL.  The context owns a stream-ordered workspace, cached FFT plans and
 * kernel tables; it starts on the device's null stream. */
fh_status fh_create(fh_ctx** out, int device, fh_precision prec, double tol,
                    const fh_options* opt);
fh_status fh_destroy(fh_ctx* ctx);
/* Bind the context to a HIP stream (hipStream_t passed as void*).  The
 * previous stream is synchronised first. */
fh_status fh_set_stream(fh_ctx* ctx, void* hip_stream);
/* Block until all work enqueued by the context has finished. */
fh_status fh_synchronize(fh_ctx* ctx);
/* Make work enqueued later on `after` wait for all work enqueued so far on
 * `before` (same device), with no host synchronisation: before's stream
 * writes the next value of a counter in signal memory, after's stream waits
 * for it.  This orders calls that share a rule or a target set across two
 * contexts' streams.  Not for use inside a stream capture. */
fh_status fh_order_after(fh_ctx* after, fh_ctx* before);
/* Replace the NUFFT/spread options (NULL restores automatic choices). */
fh_status fh_set_options(fh_ctx* ctx, const fh_options* opt);
/* Report the kernel parameters a type-1 call with an n-point grid would
 * use: kernel width, beta, sigma and fine-grid size. */
fh_status fh_query_params(const fh_ctx* ctx, int32_t n, int32_t* width, double* beta,
                          double* sigma, int32_t* nf);
const char* fh_status_string(fh_status s);
const char* fh_last_error(void);

/* ------------------------------------------------------------- quadrature
 * Each generator runs on the device and returns a library-owned areal rule
 * (x_j, y_j, w_j), j = 0..N-1, in double. */

/* Dilation rule (sec. 3.1, eqs. aqnod/aqwei) from a caller-supplied vector
 * line-integral rule (eq. vliq) on the boundary: nodes (X_i, Y_i) and vector
 * weights (W_i, V_i), i = 0..n-1, counter-clockwise.  m radial
 * Gauss-Legendre nodes on (0,1); node j = l + i m, N = n m. */
fh_status fh_quad_from_boundary(fh_ctx* ctx, const double* X, const double* Y,
                                const double* W, const double* V, int64_t n, int32_t m,
                                fh_memspace mem, fh_quad** out);

/* Star-shaped curve x(t) = r(t)(cos t, sin t), r(t) = r0 + sum_{k=1}^{K}
 * a[k-1] cos kt + b[k-1] sin kt (host arrays; a or b may be NULL for zeros;
 * K <= 64).  Boundary rule: `panels` equal panels in t with q Gauss-Legendre
 * nodes each (eq. vliq1 with Gauss-Legendre in place of the trapezoid rule);
 * panels = 0 selects the periodic trapezoid rule of eq. ptr with q nodes.
 * Then the dilation rule with m radial nodes.  N = panels q m (or q m). */
fh_status fh_quad_radial(fh_ctx* ctx, double r0, const double* a, const double* b,
                         int32_t K, int32_t panels, int32_t q, int32_t m, fh_quad** out);

/* General smooth closed CCW curve X(t) = sum_{k=0}^{K} ax[k] cos kt +
 * bx[k] sin kt, Y(t) = sum ay[k] cos kt + by[k] sin kt (host arrays of K + 1
 * doubles, K <= 64; bx and by may be NULL for zeros; bx[0], by[0] are
 * ignored), e.g. the kite of sec. 3.1 (ax = {0, 0.5, 0.5}, by = {0, 1, 0}).
 * Boundary rule as for fh_quad_radial (panels = 0: the trapezoid rule of
 * eq. ptr with q nodes), then the dilation rule about the origin with m
 * radial nodes (sec. 3.1; the weights may be negative where the curve is
 * not star-shaped about the origin).  N = panels q m (or q m). */
fh_status fh_quad_fourier(fh_ctx* ctx, int32_t K, const double* ax, const double* bx, const double* ay,
                          const double* by, int32_t panels, int32_t q, int32_t m, fh_quad** out);

/* Koch snowflake of sec. 4.4, level L <= 15: the equilateral triangle of
 * side sqrt 3 inscribed in the unit circle (vertices at 90, 210 and 330
 * degrees) plus, at each level k = 1..L, the outward triangles on the middle
 * thirds of the previous outline's edges (1 + 3 (4^L - 1)/3 triangles).
 * Every level-k triangle gets the p[k] x p[k] rule of the paper: one vertex
 * moved to the origin and the dilation rule applied to the p[k]-node
 * Gauss-Legendre line rule on the opposite edge.  p: host array of L + 1
 * orders in [1, 1024].  N = sum_k ntri_k p[k]^2 (level 13 with p = 1 from
 * level 10 on is the paper's ~69 million nodes).  Node order: level by
 * level, triangles in the order of the previous outline's edges starting
 * from the 90-degree vertex, edge index outer, radial index inner. */
fh_status fh_quad_koch(fh_ctx* ctx, int32_t L, const int32_t* p, fh_quad** out);

/* Polygon with nv >= 3 CCW vertices (host arrays), q Gauss-Legendre nodes
 * per edge, m radial nodes.  N = nv q m. */
fh_status fh_quad_polygon(fh_ctx* ctx, const double* vx, const double* vy, int32_t nv,
                          int32_t q, int32_t m, fh_quad** out);

/* Starshade disc + petal rule (sec. 3.2, eq. Omega): Np petals, disc radius
 * a, tip radius R, apodisation A(r) = exp(-((r-a)/b)^p) on (a, R).  Disc:
 * periodic trapezoid rule with nd boundary nodes and md radial nodes.
 * Petal k (centre angle 2 pi k/Np): m Gauss-Legendre radii on (a, R) times
 * np Gauss-Legendre angles across the petal width 2 pi A(r)/Np, weight
 * r w_r (pi A(r)/Np) w_t.  N = nd md + Np np m; disc nodes first, then
 * petals, angular index outer and radial index inner.
 * Optional edge perturbation: coef (2 Np K doubles, in memory `coef_mem`, or
 * NULL) moves petal k's upper edge outward by the arc length
 * d+(r) = sum_s coef[2kK+s-1] sin(s pi (r-a)/(R-a)) and its lower edge by
 * d-(r) = sum_s coef[2kK+K+s-1] sin(s pi (r-a)/(R-a)), s = 1..K <= 64. */
fh_status fh_quad_starshade(fh_ctx* ctx, int32_t Np, double a, double R, double b, double p,
                            int32_t m, int32_t np, int32_t nd, int32_t md,
                            const double* coef, int32_t K, fh_memspace coef_mem,
                            fh_quad** out);

/* Ribbon form of the perturbed starshade (sec. 5, the third construction):
 * the unperturbed rule of fh_quad_starshade (same parameters), followed by,
 * for each petal k, the signed ribbon between its upper edge and that edge
 * moved outward by the arc length d+(r) and then the ribbon of its lower
 * edge for d-(r) (coef and K as for fh_quad_starshade, required here).  The
 * ribbon of an edge with ideal angle phi_e(r) covers the angles between
 * phi_e(r) and phi_e(r) +- d(r)/r (+ for the upper edge); it gets the
 * petal's m Gauss-Legendre radii times mr Gauss-Legendre nodes tau in (0, 1)
 * across, node r (cos phi, sin phi) with phi = phi_e +- tau d/r and weight
 * w_r d(r) w_tau (negative where the edge moved inward), across index outer
 * and radial index inner.  mr = 0 gives the paper's line integral on the
 * ideal boundary: one node on the edge with weight w_r d(r), whose error is
 * second order in the ribbon's width.  The ideal part does not depend on
 * the perturbation, so perturbation studies change only the ribbon nodes.
 * N = nd md + Np np m + 2 Np m max(mr, 1). */
fh_status fh_quad_starshade_ribbon(fh_ctx* ctx, int32_t Np, double a, double R, double b, double p,
                                   int32_t m, int32_t np, int32_t nd, int32_t md, const double* coef,
                                   int32_t K, fh_memspace coef_mem, int32_t mr, fh_quad** out);

/* As fh_quad_starshade with a tabulated apodisation instead of the HG family
 * (the paper's NI2 design is given as samples of A(r), interpolated to the
 * radial Gauss nodes, sec. 4.2): A holds m host doubles, A[l] = A(r_l) at
 * r_l = a + (R - a)(1 + x_l)/2, x_l the m-node Gauss-Legendre nodes on
 * [-1, 1] ascending.  fh_starshade_vjp covers the HG family only. */
fh_status fh_quad_starshade_tab(fh_ctx* ctx, int32_t Np, double a, double R, const double* A, int32_t m,
                                int32_t np, int32_t nd, int32_t md, const double* coef, int32_t K,
                                fh_memspace coef_mem, fh_quad** out);

/* Starshade with misaligned rigid petals (sec. 5): the unperturbed rule of
 * fh_quad_starshade (same parameters, no edge perturbation), then petal k's
 * nodes move by x -> Rot(d_k) x + (tx_k, ty_k) (rotation about the centre,
 * then translation) with unchanged weights, and the signed region between
 * the petal's root arc on the disc (r = a, angles theta_k +- pi/Np) and its
 * moved image is covered by the map X(tau, t) = P(tau) + t (M(tau) - P(tau))
 * with nb Gauss-Legendre nodes along the arc and mb across: positive weights
 * where the petal moved outward, negative where it moved into the disc.
 * motion: 3 Np host doubles (d_k, tx_k, ty_k), Np <= 64.
 * N = nd md + Np np m + Np nb mb (disc, moved petals, then the bridges). */
fh_status fh_quad_starshade_rigid(fh_ctx* ctx, int32_t Np, double a, double R, double b, double p,
                                  int32_t m, int32_t np, int32_t nd, int32_t md, const double* motion,
                                  int32_t nb, int32_t mb, fh_quad** out);

/* Raw areal rule (eq. aq): N nodes and weights, copied into a new object. */
fh_status fh_quad_from_nodes(fh_ctx* ctx, const double* x, const double* y, const double* w,
                             int64_t N, fh_memspace mem, fh_quad** out);

/* Illumination of a rule (sec. 1 and sec. 5's source-plane extension):
 *   src: a complex source term s_j per node multiplying its weight (a smooth
 *     amplitude and phase over the source plane), N interleaved complex in
 *     `mem`, or NULL for s_j = 1;
 *   D: distance of a point source before the aperture (D > 0), whose
 *     spherical incident wave exp(i pi |x|^2/(lambda D)) multiplies the
 *     source chirp (z^-1 becomes z^-1 + D^-1 there, sec. 1); 0 for a plane
 *     wave.
 * Every later field call with the rule (grid, points, target sets, batches)
 * evaluates u_ap = 1/(i lambda z) sum_j w_j s_j exp(i pi |x_j|^2/(lambda D))
 * exp(i pi |xi - x_j|^2/(lambda z)); fh_field_grid_vjp refuses a rule with
 * either (FH_ERR_UNSUPPORTED).  The call waits for all device work first
 * (earlier calls may still read the old terms), copies src into library
 * memory owned by the rule (released by fh_quad_destroy or a NULL src) and
 * returns with the copy done; src may be released on return.  A non-finite
 * host term is FH_ERR_NONFINITE; D < 0 is FH_ERR_INVALID_ARG. */
fh_status fh_quad_set_illumination(fh_ctx* ctx, fh_quad* q, const double* src, double D, fh_memspace mem);

fh_status fh_quad_size(const fh_quad* q, int64_t* N);
/* Copy the rule out (x, y, w each N doubles; any may be NULL). */
fh_status fh_quad_export(const fh_quad* q, double* x, double* y, double* w, fh_memspace mem);
/* Device pointers of the rule's arrays (owned by the object). */
fh_status fh_quad_device_ptrs(const fh_quad* q, const double** x, const double** y,
                              const double** w);
/* A rule may be passed to any context on the same device.  Its arrays are
 * written on the stream of the context that made it; a call on another
 * stream must be ordered after that (e.g. with an event), and
 * fh_quad_destroy (which hands the memory back to the making context, to be
 * reused on its stream) must come after every call reading the rule has been
 * ordered before that stream's later work. */
fh_status fh_quad_destroy(fh_quad* q);

/* ------------------------------------------------------------------ fields */

/* Field on the uniform grid (sec. 2.2, type-1 NUFFT): targets
 * (xc + h1 k1, yc + h2 k2), -n1/2 <= k1 < n1/2, -n2/2 <= k2 < n2/2, n1 and
 * n2 even.  A translated grid (xc, yc != 0) is handled by pre-phasing the
 * strengths.  Output u[(k2 + n2/2) n1 + (k1 + n1/2)] (k1 fastest), complex
 * in the context's precision.  occulter != 0 returns u_oc = 1 - u_ap. */
fh_status fh_field_grid(fh_ctx* ctx, const fh_quad* q, double lambda, double z,
                        int32_t n1, int32_t n2, double h1, double h2, double xc, double yc,
                        int32_t occulter, void* u, fh_memspace mem);

/* Field at M scattered targets (xi_k, eta_k) (sec. 2.1, type-3 NUFFT).  xi,
 * eta and u are all in `mem`.  This call reads the target bounding box back
 * to the host to size the fine grid, so it synchronises the stream once. */
fh_status fh_field_points(fh_ctx* ctx, const fh_quad* q, double lambda, double z, int64_t M,
                          const double* xi, const double* eta, int32_t occulter, void* u,
                          fh_memspace mem);

/* Scattered-target set for repeated type-3 evaluation (sec. 2.1's targets;
 * the paper's sweeps evaluate many wavelengths and shapes at one fixed set of
 * pupil points, sec. 4.3): the M targets (xi, eta in `mem`) and the box the
 * type-3 grids are planned for.
 *   Device arrays are used in place: they must stay allocated and unchanged
 *   while the set is in use (stream order as for any input).  Host arrays
 *   are copied to library memory (one synchronisation) and may be released
 *   on return.
 *   box (host, 4 doubles xmin, xmax, ymin, ymax, or NULL): with a box the
 *     call does no device work and no synchronisation, and targets outside
 *     it, or with a non-finite coordinate, get NaN from fh_field_targets.
 *     With NULL the bounding box is computed (device arrays: one readback,
 *     which synchronises the stream) and a non-finite target is
 *     FH_ERR_NONFINITE.
 *   M must be below 2^31; M = 0 gives an empty set.  fh_targets_destroy
 *   hands any copy back to the making context's memory pool (stream order
 *   as for rules). */
fh_status fh_targets_create(fh_ctx* ctx, int64_t M, const double* xi, const double* eta,
                            const double* box, fh_memspace mem, fh_targets** out);
/* Evaluate the set's targets in spatial (Morton) order within its box from
 * now on, for cache locality on large type-3 grids; fh_field_targets still
 * writes u in the order the targets were given.  Enqueues the sort on the
 * making context's stream (no synchronisation) and keeps a sorted copy in
 * library memory, so the caller's device arrays are no longer read after
 * the call's work has run.  A one-time cost for sets evaluated many times;
 * M < 2, or a sorted set, is a no-op. */
fh_status fh_targets_sort(fh_targets* t);
fh_status fh_targets_size(const fh_targets* t, int64_t* M);
/* The planning box (declared or computed), 4 doubles. */
fh_status fh_targets_box(const fh_targets* t, double* box);
fh_status fh_targets_destroy(fh_targets* t);

/* Field at a target set (sec. 2.1, type-3 NUFFT), as fh_field_points but
 * without a host synchronisation for device output: u (M complex in `mem`,
 * in the order the targets were given to fh_targets_create) is written on
 * the context stream.  Host output copies back and synchronises. */
fh_status fh_field_targets(fh_ctx* ctx, const fh_quad* q, double lambda, double z,
                           const fh_targets* t, int32_t occulter, void* u, fh_memspace mem);

/* B grid fields in one batched pass: instance b uses rule q[b], lambda[b],
 * z[b] and occulter[b] (host arrays of length B), all on the same grid
 * parameters.  u (device, B n1 n2 complex) is written instance-major.  All
 * instances share one fine-grid size; the spread runs as one persistent
 * launch over every instance's work items, the FFT is one batched rocFFT
 * call, and for B > 1 the sequence is captured once into a hipGraph keyed by
 * the batch signature and replayed on later calls with the same signature
 * (B = 1 runs eagerly, as fh_field_grid). */
fh_status fh_field_grid_batch(fh_ctx* ctx, int32_t B, const fh_quad* const* q,
                              const double* lambda, const double* z, int32_t n1, int32_t n2,
                              double h1, double h2, double xc, double yc,
                              const int32_t* occulter, void* u);

/* As fh_field_grid_batch, with the quadrature generation (sec. 3) inside the
 * call: every rule's nodes and weights are first computed again on the
 * device, in place, from the boundary parameters it was made with, and for
 * B > 1 those rule kernels are captured into the same hipGraph as the field
 * (the paper's wavelength sweep counts quadrature generation, sec. 4.3).
 * Only rules built by one launch from parameters held by value can be
 * rebuilt: fh_quad_radial rules and fh_quad_polygon rules of up to 128
 * vertices; any other rule gives FH_ERR_UNSUPPORTED before anything is
 * enqueued.  The rules' contents afterwards are what their constructors
 * wrote. */
fh_status fh_field_grid_batch_rebuild(fh_ctx* ctx, int32_t B, fh_quad* const* q,
                                      const double* lambda, const double* z, int32_t n1,
                                      int32_t n2, double h1, double h2, double xc, double yc,
                                      const int32_t* occulter, void* u);

/* ----------------------------------------------------------------- adjoint */

/* Vector-Jacobian product of fh_field_grid with respect to the rule's nodes
 * and weights.  g_u (device, same layout and precision as the field) holds
 * dL/dRe(u) + i dL/dIm(u) for a real loss L.  Outputs (device doubles, N
 * each): dL/dx_j, dL/dy_j, dL/dw_j.  Derivation: du_k/dw_j =
 * E_kj/(i lambda z), du_k/dx_j = (w_j/(i lambda z)) E_kj (2 pi i/(lambda z))
 * (x_j - xi_k) with E_kj the Fresnel kernel of eq. faq; the sums over k are
 * evaluated as three type-2 NUFFTs sharing one set of kernel weights. */
fh_status fh_field_grid_vjp(fh_ctx* ctx, const fh_quad* q, double lambda, double z,
                            int32_t n1, int32_t n2, double h1, double h2, double xc, double yc,
                            int32_t occulter, const void* g_u, double* g_x, double* g_y,
                            double* g_w);

/* The node gradients of a loss summed over L wavelengths (the paper's
 * sweep of one rule over wavelengths, sec. 4.3): as fh_field_grid_vjp for
 * each (lambda[l], z[l]) with cotangent plane l of g_u (device, L x n2 x n1
 * complex in the context's precision), the L results added in order into
 * g_x, g_y, g_w (device, N doubles each, overwritten).  The chain rule
 * through the rule's construction is linear, so it then runs once on the
 * sums (fh_starshade_vjp).  lambda and z are host arrays of L entries. */
fh_status fh_field_grid_vjp_sum(fh_ctx* ctx, const fh_quad* q, int32_t L, const double* lambda,
                                const double* z, int32_t n1, int32_t n2, double h1, double h2,
                                double xc, double yc, int32_t occulter, const void* g_u,
                                double* g_x, double* g_y, double* g_w);

/* Chain (dL/dx, dL/dy, dL/dw) of a perturbed starshade rule (same
 * parameters as fh_quad_starshade; all arrays on the device) to dL/dcoef
 * (2 Np K doubles). */
fh_status fh_starshade_vjp(fh_ctx* ctx, int32_t Np, double a, double R, double b, double p,
                           int32_t m, int32_t np, int32_t nd, int32_t md, const double* coef,
                           int32_t K, const double* g_x, const double* g_y, const double* g_w,
                           double* g_coef);

/* ----------------------------------------------------------- edge integral
 * The non-singular line integral of the appendix (eq. nsli): an O(n M) direct
 * method from a boundary rule alone, accurate for targets inside, outside and
 * on the boundary; the paper's reference for its error tables. */

/* Boundary vector line-integral rules (eq. vliq), written to caller arrays
 * X, Y, W, V (n doubles each, in `mem`; host output synchronises):
 *   fh_boundary_radial: the star-shaped curve of fh_quad_radial (same
 *     parameters without m), n = panels q (or q with panels = 0);
 *   fh_boundary_fourier: the curve of fh_quad_fourier (same parameters
 *     without m), n = panels q (or q with panels = 0);
 *   fh_boundary_polygon: q Gauss-Legendre nodes per edge of the CCW polygon
 *     (host vertex arrays), n = nv q;
 *   fh_boundary_starshade: the outline of fh_quad_starshade's petal shape
 *     (sec. 3.2; unperturbed): per petal, in this order, the lower edge
 *     theta_k - pi A(r)/Np for r from a to R (m Gauss-Legendre radii), the
 *     tip arc at r = R (ntip Gauss-Legendre angles), the upper edge
 *     theta_k + pi A(r)/Np from R back to a, and the arc at r = a to the next
 *     petal (ngap nodes; zero weights for this profile, whose A(a) = 1);
 *     n = Np (2 m + ntip + ngap).  The paper's HG outline is m = 60,
 *     ntip = ngap = 4 (n = 2048 for 16 petals). */
fh_status fh_boundary_radial(fh_ctx* ctx, double r0, const double* a, const double* b, int32_t K,
                             int32_t panels, int32_t q, double* X, double* Y, double* W, double* V,
                             fh_memspace mem);
fh_status fh_boundary_fourier(fh_ctx* ctx, int32_t K, const double* ax, const double* bx,
                              const double* ay, const double* by, int32_t panels, int32_t q, double* X,
                              double* Y, double* W, double* V, fh_memspace mem);
fh_status fh_boundary_polygon(fh_ctx* ctx, const double* vx, const double* vy, int32_t nv, int32_t q,
                              double* X, double* Y, double* W, double* V, fh_memspace mem);
fh_status fh_boundary_starshade(fh_ctx* ctx, int32_t Np, double a, double R, double b, double p,
                                int32_t m, int32_t ntip, int32_t ngap, double* X, double* Y, double* W,
                                double* V, fh_memspace mem);

/* Field at M targets by the edge integral (appendix, eq. nsli) over a CCW
 * boundary rule (X_i, Y_i) with vector weights (W_i, V_i), i < n:
 *   u_ap = (1/2pi) sum_i (1 - exp(i pi r_i^2/(lambda z))) (r_i x ds_i)/r_i^2,
 *   r_i = (X_i - xi, Y_i - eta), r x ds = r_x V_i - r_y W_i,
 * a term being 0 when r_i = 0 (a target on a node).  far > 0 selects, for
 * targets at least `far` from every node, the form of eq. li with the exact
 * geometric term (the nearest integer to the rule's winding number), which
 * removes a low-order rule's error from that term in deep shadow (the
 * appendix's remark); far = 0 uses eq. nsli everywhere.  All arrays are in
 * `mem`; u gets M complex values in the context's precision (u_oc = 1 - u_ap
 * if occulter).  The arithmetic is FP64 in both precisions.  n = 0 gives
 * u_ap = 0; M = 0 is a no-op.  Device memory: enqueued on the context stream
 * without synchronising; host memory: copies and synchronises. */
fh_status fh_field_nsli(fh_ctx* ctx, const double* X, const double* Y, const double* W, const double* V,
                        int64_t n, double lambda, double z, int64_t M, const double* xi,
                        const double* eta, double far, int32_t occulter, void* u, fh_memspace mem);

/* Allocation-free form of fh_field_nsli, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc.  Same arguments and result as fh_field_nsli with
 * every array in device memory (X, Y, W, V: n doubles each; xi, eta: M
 * doubles; u: M complex in the context's precision), enqueued on the context
 * stream without synchronising.  It calls no allocator: when the targets are
 * few enough that the nodes are split into groups, the groups' partial sums
 * (4 x groups x M doubles) go to a 32 MiB device array that the library holds
 * on each device until the process ends, shared by every call on that
 * device, so calls that overlap on one device (two streams, two threads)
 * race and must be ordered by the caller.  With fh_field_nsli's choice of
 * node groups the partial sums stay below 32 MiB on devices of up to 320 CUs
 * (MI355X has 256); a call whose partial sums would exceed it returns
 * FH_ERR_UNSUPPORTED without enqueuing anything. */
fh_status fh_field_nsli_noalloc(fh_ctx* ctx, const double* X, const double* Y, const double* W,
                                const double* V, int64_t n, double lambda, double z, int64_t M,
                                const double* xi, const double* eta, double far, int32_t occulter,
                                void* u);

/* --------------------------------------------------------------- autotuner */

/* Time fh_field_grid for this rule and grid over a set of tile sizes,
 * subproblem sizes, spread methods and upsampling factors that all meet the
 * context's tolerance; keep the fastest in the context and return it in
 * *best.  If cache_path is not NULL the result is read from / appended to
 * that JSON-lines file, keyed by precision, tolerance, grid size and node
 * count class. */
fh_status fh_autotune_grid(fh_ctx* ctx, const fh_quad* q, double lambda, double z, int32_t n1,
                           int32_t n2, double h1, double h2, const char* cache_path,
                           fh_options* best);

/* The same for a batch (sec. 4.3's many shapes and wavelengths): time
 * fh_field_grid_batch with these B rules, wavelengths and distances as it
 * runs (captured into a graph, then replayed) over spread methods 5, 2 and
 * 4, tile edges, work-item sizes and upsampling factors that meet the
 * context's tolerance, and keep the fastest in the context (the caller's
 * kernel width, beta and deterministic flag are kept).  The cache key is the
 * batch's signature: precision, tolerance, grid size, B, and the node-count
 * classes (powers of two) of the whole batch and of its largest rule.
 * Arguments as fh_field_grid_batch (plane grids centred on the axis, no
 * occulter); q, lambda and z are host arrays of B entries.  Allocates a
 * B x n2 x n1 output for the trials. */
fh_status fh_autotune_batch(fh_ctx* ctx, int32_t B, const fh_quad* const* q, const double* lambda,
                            const double* z, int32_t n1, int32_t n2, double h1, double h2,
                            const char* cache_path, fh_options* best);

/* Stage timing.  While enabled (fh_set_timing, or FH_TIMING=1 in the
 * environment at fh_create) every fh_field_grid / fh_field_points /
 * fh_field_grid_vjp call records HIP events on the context stream around
 * its stages, without synchronising.  Stages: [0] strengths + binning,
 * [1] the spread kernel alone (for the adjoint: empty), [2] slot merge and
 * reduce + FFT (for the adjoint: its FFTs), [3] finish
 * (deconvolution epilogue, type-3 interpolation, or adjoint node
 * gradients), [4] whole call.  While timing is on, batched calls run
 * eagerly instead of as a hipGraph so that their stages can be timed.
 * fh_last_timing returns the most recent call's stage times in
 * milliseconds; fh_timing_totals returns, for one kind of call (0 grid,
 * 1 points, 2 adjoint, 3 batch), the sums over all timed calls since its
 * last reset and their count.  Both synchronise. */
fh_status fh_set_timing(fh_ctx* ctx, int32_t enable);
fh_status fh_last_timing(fh_ctx* ctx, double* ms5);
fh_status fh_timing_totals(fh_ctx* ctx, int32_t kind, double* ms5, int64_t* ncalls, int32_t reset);

/* ------------------------------------------------------------ diagnostics */

/* Measured ceilings of the device the context runs on, for roofline
 * fractions (not part of any field computation).  out (host, 7 doubles):
 *   out[0] HBM bandwidth of a device-to-device copy of 1 GiB (the faster of
 *          a plain and a four-loads-in-flight copy), in GB/s of bytes read
 *          plus bytes written;
 *   out[1] LDS atomic adds of float (non-returning, conflict-free cells,
 *          every CU), in GB/s of operands;
 *   out[2] the same for double;
 *   out[3] LDS read-modify-write of complex doubles (16-byte cells), in GB/s
 *          of bytes read plus written;
 *   out[4] the same for complex floats (8-byte cells);
 *   out[5] matrix-core rate of 16 x 16 x 4 double products (TFLOP/s, eight
 *          independent accumulators per wavefront);
 *   out[6] the same for float products.
 * Each is the best of five timed launches.  Allocates 2 GiB of device memory
 * for the duration of the call (FH_ERR_ALLOC if that fails) and synchronises
 * the context stream. */
fh_status fh_probe_ceilings(fh_ctx* ctx, double* out);

#ifdef __cplusplus
}
#endif
#endif /* FRESNEL_HIP_H */

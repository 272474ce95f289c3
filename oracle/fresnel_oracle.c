/*
 * fresnel_oracle.c -- plain, slow FP64 reference for areal-quadrature Fresnel
 * diffraction (Barnett, "Efficient high-order accurate Fresnel diffraction via
 * areal quadrature and the nonuniform FFT", arXiv:2010.05978).
 *
 * THIS IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no source with the GPU library.
 *
 * Everything here follows the paper's definitions literally:
 *   - 1D Gauss-Legendre rules (used throughout sec. 3),
 *   - vector line-integral rules on the boundary (eq. vliq; eq. ptr for the
 *     periodic trapezoid variant, Gauss-Legendre panels otherwise),
 *   - the "dilation" areal rule (eqs. aqnod / aqwei, sec. 3.1),
 *   - the starshade disc + petal rule (sec. 3.2, with the weight's A(r) taken
 *     at the radial node, i.e. the Jacobian of theta = A(r) t), also with
 *     misaligned rigid petals and the signed bridges to the disc (sec. 5),
 *   - the direct areal-quadrature sum (eq. faq), un-factorised, phase carried
 *     in turns and reduced before cos/sin, pairwise summation over nodes,
 *   - the Babinet complement u_oc = 1 - u_ap (eq. bab),
 *   - the same sum with a source term per node and a spherical incident
 *     wave (secs. 1 and 5),
 *   - the ribbon construction of sec. 5 (the ideal starshade plus signed
 *     ribbons between each petal's ideal and displaced edges, with Gauss-
 *     Legendre nodes across, or the line integral on the ideal edge),
 *   - the Koch snowflake rule of sec. 4.4 (a p x p dilation rule per
 *     triangle of the level-L construction),
 *   - the non-singular line integral over a boundary rule (appendix, eq.
 *     nsli), with the deep-shadow option of eq. li, and the starshade
 *     outline rule it is fed with,
 *   - the exact gradient of the quadrature sum with respect to node
 *     coordinates and weights, and its chain rule through the perturbed
 *     starshade construction.
 * No blocking, fusion or factorisation beyond what those definitions state.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846264338327950288

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre rule on [-1,1]: q nodes ascending, weights.               */
/* Newton iteration on the Legendre polynomial P_q, evaluated with the      */
/* three-term recurrence k P_k = (2k-1) x P_{k-1} - (k-1) P_{k-2}.          */
/* ------------------------------------------------------------------------ */
static void legendre_eval(int q, double x, double* p, double* dp)
{
    double p0 = 1.0, p1 = x;
    if (q == 0) { *p = 1.0; *dp = 0.0; return; }
    for (int k = 2; k <= q; k++) {
        double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
    }
    *p = p1;
    /* derivative from P_q and P_{q-1}: (x^2-1) P_q' = q (x P_q - P_{q-1}) */
    *dp = q * (x * p1 - p0) / (x * x - 1.0);
}

int orc_gauss_legendre(int q, double* x, double* w)
{
    if (q < 1) return 1;
    for (int i = 0; i < q; i++) {
        /* i-th largest root: classical Chebyshev-like initial guess */
        double t = cos(ORC_PI * (i + 0.75) / (q + 0.5));
        double p, dp;
        for (int it = 0; it < 100; it++) {
            legendre_eval(q, t, &p, &dp);
            double dt = p / dp;
            t -= dt;
            if (fabs(dt) < 1e-16) break;
        }
        legendre_eval(q, t, &p, &dp);
        /* store ascending */
        x[q - 1 - i] = t;
        w[q - 1 - i] = 2.0 / ((1.0 - t * t) * dp * dp);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Boundary (vector line-integral) rules, eq. vliq:                         */
/*   int_{dOmega} f . ds  ~=  sum_i f(X_i,Y_i) . (W_i,V_i),  CCW.           */
/* ------------------------------------------------------------------------ */

/* radial Fourier curve r(t) = r0 + sum_{k=1}^K a_k cos kt + b_k sin kt,     */
/* x(t) = r(t) (cos t, sin t).  Returns position and derivative at t.      */
static void radial_curve(double r0, const double* a, const double* b, int K,
                         double t, double* X, double* Y, double* dX, double* dY)
{
    double r = r0, dr = 0.0;
    for (int k = 1; k <= K; k++) {
        double ak = a ? a[k - 1] : 0.0, bk = b ? b[k - 1] : 0.0;
        r += ak * cos(k * t) + bk * sin(k * t);
        dr += k * (-ak * sin(k * t) + bk * cos(k * t));
    }
    double c = cos(t), s = sin(t);
    *X = r * c;
    *Y = r * s;
    *dX = dr * c - r * s;
    *dY = dr * s + r * c;
}

/* Gauss-Legendre panels in the angle t: P equal panels of [0,2pi), q nodes
 * each; n = P q boundary nodes.  Panel p node i sits at
 * t = (2pi/P)(p + (1+x_i)/2) with line weight (pi/P) w_i, and
 * (W,V) = weight * x'(t)  (eq. vliq1 with the GL rule replacing the PTR). */
int orc_bdry_radial_gl(double r0, const double* a, const double* b, int K,
                       int P, int q, double* X, double* Y, double* W, double* V)
{
    if (P < 1 || q < 1) return 1;
    double* gx = (double*)malloc(sizeof(double) * q);
    double* gw = (double*)malloc(sizeof(double) * q);
    orc_gauss_legendre(q, gx, gw);
    for (int p = 0; p < P; p++)
        for (int i = 0; i < q; i++) {
            double t = (2.0 * ORC_PI / P) * (p + 0.5 * (1.0 + gx[i]));
            double om = (ORC_PI / P) * gw[i];
            double x, y, dx, dy;
            radial_curve(r0, a, b, K, t, &x, &y, &dx, &dy);
            int64_t ii = (int64_t)p * q + i;
            X[ii] = x; Y[ii] = y; W[ii] = om * dx; V[ii] = om * dy;
        }
    free(gx); free(gw);
    return 0;
}

/* Periodic trapezoid rule, eq. ptr: t_i = 2 pi i / n, weight 2 pi / n,     */
/* i = 1..n (stored at index i-1).                                          */
int orc_bdry_radial_ptr(double r0, const double* a, const double* b, int K,
                        int n, double* X, double* Y, double* W, double* V)
{
    if (n < 1) return 1;
    for (int i = 1; i <= n; i++) {
        double t = 2.0 * ORC_PI * i / n, om = 2.0 * ORC_PI / n;
        double x, y, dx, dy;
        radial_curve(r0, a, b, K, t, &x, &y, &dx, &dy);
        X[i - 1] = x; Y[i - 1] = y; W[i - 1] = om * dx; V[i - 1] = om * dy;
    }
    return 0;
}

/* Polygon with nv vertices (CCW), q GL nodes per straight edge:            */
/* node v_e + (1+x_i)/2 (v_{e+1}-v_e), vector weight (v_{e+1}-v_e) w_i / 2. */
int orc_bdry_polygon(const double* vx, const double* vy, int nv, int q,
                     double* X, double* Y, double* W, double* V)
{
    if (nv < 3 || q < 1) return 1;
    double* gx = (double*)malloc(sizeof(double) * q);
    double* gw = (double*)malloc(sizeof(double) * q);
    orc_gauss_legendre(q, gx, gw);
    for (int e = 0; e < nv; e++) {
        int f = (e + 1) % nv;
        double ex = vx[f] - vx[e], ey = vy[f] - vy[e];
        for (int i = 0; i < q; i++) {
            double s = 0.5 * (1.0 + gx[i]);
            int64_t ii = (int64_t)e * q + i;
            X[ii] = vx[e] + s * ex;
            Y[ii] = vy[e] + s * ey;
            W[ii] = 0.5 * gw[i] * ex;
            V[ii] = 0.5 * gw[i] * ey;
        }
    }
    free(gx); free(gw);
    return 0;
}

/* General smooth closed curve given by its Fourier series, eq. vliq1:      */
/*   X(t) = sum_{k=0}^K ax_k cos kt + bx_k sin kt,  Y(t) likewise (ay, by), */
/* CCW in t.  P > 0: P Gauss-Legendre panels of q nodes in t (as for the    */
/* radial curve); P = 0: the periodic trapezoid rule of eq. ptr with q      */
/* nodes t_i = 2 pi i/q, i = 1..q.  (W, V) = weight * x'(t).                */
static void fourier_curve(const double* ax, const double* bx, const double* ay, const double* by,
                          int K, double t, double* X, double* Y, double* dX, double* dY)
{
    double x = 0.0, y = 0.0, dx = 0.0, dy = 0.0;
    for (int k = 0; k <= K; k++) {
        double c = cos(k * t), s = sin(k * t);
        x += ax[k] * c + bx[k] * s;
        y += ay[k] * c + by[k] * s;
        dx += k * (-ax[k] * s + bx[k] * c);
        dy += k * (-ay[k] * s + by[k] * c);
    }
    *X = x; *Y = y; *dX = dx; *dY = dy;
}

int orc_bdry_fourier(const double* ax, const double* bx, const double* ay, const double* by, int K,
                     int P, int q, double* X, double* Y, double* W, double* V)
{
    if (K < 0 || P < 0 || q < 1) return 1;
    if (P == 0) {
        for (int i = 1; i <= q; i++) {
            double t = 2.0 * ORC_PI * i / q, om = 2.0 * ORC_PI / q;
            double x, y, dx, dy;
            fourier_curve(ax, bx, ay, by, K, t, &x, &y, &dx, &dy);
            X[i - 1] = x; Y[i - 1] = y; W[i - 1] = om * dx; V[i - 1] = om * dy;
        }
        return 0;
    }
    double* gx = (double*)malloc(sizeof(double) * q);
    double* gw = (double*)malloc(sizeof(double) * q);
    orc_gauss_legendre(q, gx, gw);
    for (int p = 0; p < P; p++)
        for (int i = 0; i < q; i++) {
            double t = (2.0 * ORC_PI / P) * (p + 0.5 * (1.0 + gx[i]));
            double om = (ORC_PI / P) * gw[i];
            double x, y, dx, dy;
            fourier_curve(ax, bx, ay, by, K, t, &x, &y, &dx, &dy);
            int64_t ii = (int64_t)p * q + i;
            X[ii] = x; Y[ii] = y; W[ii] = om * dx; V[ii] = om * dy;
        }
    free(gx); free(gw);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Dilation areal rule, eqs. aqnod / aqwei (sec. 3.1):                      */
/*   alpha_l, wt_l = m-node GL on (0,1);                                    */
/*   node j = l + i m  (0-based, radial index l inner):                     */
/*   (x_j, y_j) = alpha_l (X_i, Y_i),  w_j = alpha_l wt_l (X_i V_i - Y_i W_i) */
/* ------------------------------------------------------------------------ */
int orc_dilation(const double* X, const double* Y, const double* W, const double* V,
                 int64_t n, int m, double* x, double* y, double* w)
{
    if (m < 1 || n < 0) return 1;
    double* gx = (double*)malloc(sizeof(double) * m);
    double* gw = (double*)malloc(sizeof(double) * m);
    orc_gauss_legendre(m, gx, gw);
    for (int64_t i = 0; i < n; i++) {
        double cross = X[i] * V[i] - Y[i] * W[i];
        for (int l = 0; l < m; l++) {
            double al = 0.5 * (1.0 + gx[l]);
            double wl = 0.5 * gw[l];
            int64_t j = (int64_t)l + i * m;
            x[j] = al * X[i];
            y[j] = al * Y[i];
            w[j] = al * wl * cross;
        }
    }
    free(gx); free(gw);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Starshade rule (sec. 3.2, eq. Omega).                                     */
/* Apodisation A(r) = 1 for r < a, exp(-((r-a)/b)^p) for a <= r <= R (the   */
/* offset hyper-Gaussian family).                                           */
/* Disc of radius a: PTR boundary rule with nd nodes (eq. ptr), dilation    */
/* with md radial nodes.  Petal k = 0..Np-1 centred at theta_k = 2 pi k/Np:  */
/* r_l, wr_l = GL on (a,R) (m nodes); tau_i, om_i = GL on [-1,1] (np nodes); */
/* half-width angle h(r) = pi A(r)/Np, node r_l (cos phi, sin phi) with     */
/* phi = theta_k + h(r_l) tau_i, weight r_l wr_l h(r_l) om_i.  (This equals */
/* the printed petal rule with angular nodes t_i = (pi/Np) tau_i, with the  */
/* apodisation in the weight evaluated at the radial node r_l.)             */
/*                                                                          */
/* Optional lateral edge perturbation, K sine modes per edge:               */
/*   d+(r) = sum_k c+_k sin(k pi (r-a)/(R-a)),  likewise d-(r);             */
/* the upper edge moves outward by d+ (arc length), the lower edge by d-:   */
/*   mid(r) = (d+ - d-)/(2r),  h(r) = pi A/Np + (d+ + d-)/(2r),              */
/*   phi = theta_k + mid + h tau.                                           */
/* coef layout: petal k: c+ at [2kK, 2kK+K), c- at [2kK+K, 2kK+2K).          */
/* Node order: disc first (i outer, l inner), then petals k, i outer, l     */
/* inner.  N = nd md + Np np m.                                             */
/* ------------------------------------------------------------------------ */
static double hg_profile(double r, double a, double b, double p)
{
    if (r < a) return 1.0;
    return exp(-pow((r - a) / b, p));
}

int64_t orc_starshade_size(int Np, int m, int np, int nd, int md)
{
    return (int64_t)nd * md + (int64_t)Np * np * m;
}

/* The rule with the apodisation given either by the HG family (Atab NULL) */
/* or as a table Atab[l] = A(r_l) at the m GL radii r_l on (a, R).          */
static int starshade_impl(int Np, double a, double R, double b, double p, const double* Atab,
                          int m, int np, int nd, int md, const double* coef, int K,
                          double* x, double* y, double* w)
{
    if (Np < 1 || m < 1 || np < 1 || nd < 0 || md < 1 || !(R > a) || !(a >= 0)) return 1;
    /* disc */
    if (nd > 0) {
        double* X = (double*)malloc(sizeof(double) * nd * 4);
        orc_bdry_radial_ptr(a, NULL, NULL, 0, nd, X, X + nd, X + 2 * nd, X + 3 * nd);
        orc_dilation(X, X + nd, X + 2 * nd, X + 3 * nd, nd, md, x, y, w);
        free(X);
    }
    int64_t off = (int64_t)nd * md;
    double* rx = (double*)malloc(sizeof(double) * m);
    double* rw = (double*)malloc(sizeof(double) * m);
    double* tx = (double*)malloc(sizeof(double) * np);
    double* tw = (double*)malloc(sizeof(double) * np);
    orc_gauss_legendre(m, rx, rw);
    orc_gauss_legendre(np, tx, tw);
    for (int k = 0; k < Np; k++) {
        double thk = 2.0 * ORC_PI * k / Np;
        for (int i = 0; i < np; i++)
            for (int l = 0; l < m; l++) {
                double r = a + 0.5 * (R - a) * (1.0 + rx[l]);
                double wr = 0.5 * (R - a) * rw[l];
                double dp = 0.0, dm = 0.0;
                if (coef && K > 0)
                    for (int s = 1; s <= K; s++) {
                        double sk = sin(s * ORC_PI * (r - a) / (R - a));
                        dp += coef[2 * k * K + (s - 1)] * sk;
                        dm += coef[2 * k * K + K + (s - 1)] * sk;
                    }
                double mid = (dp - dm) / (2.0 * r);
                double A = Atab ? Atab[l] : hg_profile(r, a, b, p);
                double half = ORC_PI * A / Np + (dp + dm) / (2.0 * r);
                double phi = thk + mid + half * tx[i];
                int64_t j = off + (int64_t)k * np * m + (int64_t)i * m + l;
                x[j] = r * cos(phi);
                y[j] = r * sin(phi);
                w[j] = r * wr * half * tw[i];
            }
    }
    free(rx); free(rw); free(tx); free(tw);
    return 0;
}

int orc_starshade(int Np, double a, double R, double b, double p,
                  int m, int np, int nd, int md, const double* coef, int K,
                  double* x, double* y, double* w)
{
    if (!(b > 0) || !(p > 0)) return 1;
    return starshade_impl(Np, a, R, b, p, NULL, m, np, nd, md, coef, K, x, y, w);
}

/* Tabulated apodisation (the paper's NI2 design comes as samples of A(r),  */
/* interpolated to the m radial Gauss nodes, sec. 4.2): Atab[l] = A(r_l).   */
int orc_starshade_tab(int Np, double a, double R, const double* Atab, int m, int np, int nd, int md,
                      const double* coef, int K, double* x, double* y, double* w)
{
    if (!Atab) return 1;
    return starshade_impl(Np, a, R, 1.0, 1.0, Atab, m, np, nd, md, coef, K, x, y, w);
}

/* ------------------------------------------------------------------------ */
/* Ribbon quadrature (sec. 5, the third construction): a perturbed shape is  */
/* the ideal shape plus a narrow signed "ribbon" along its boundary.  For    */
/* the starshade with the lateral edge displacements of orc_starshade (the   */
/* upper edge of petal k moves outward by the arc length d+(r), the lower   */
/* by d-(r)), the ribbon of the upper edge is the set of angles between the  */
/* ideal edge theta_k + pi A(r)/Np and that angle plus d+(r)/r, the lower   */
/* edge's between theta_k - pi A(r)/Np - d-(r)/r and the ideal edge.  The    */
/* area element is r dr dphi, so with the petal's m Gauss-Legendre radii     */
/* (weights wr_l) and mr Gauss-Legendre nodes tau_j on (0, 1) (weights v_j)  */
/* across the ribbon: node r_l (cos phi, sin phi), phi = ideal edge angle   */
/* +- tau_j d(r_l)/r_l, weight wr_l d(r_l) v_j, negative where the edge     */
/* moved inward.  mr = 0 is the paper's line integral on the ideal boundary: */
/* one node on the edge (tau = 0) with weight wr_l d(r_l), first order in    */
/* the ribbon's width.  Rule: the unperturbed starshade (orc_starshade with  */
/* no coefficients), then per petal the upper edge's ribbon and the lower    */
/* edge's, each with the radial index inner and the across index outer.     */
/* N = nd md + Np np m + 2 Np m max(mr, 1).                                 */
/* ------------------------------------------------------------------------ */
int64_t orc_starshade_ribbon_size(int Np, int m, int np, int nd, int md, int mr)
{
    return (int64_t)nd * md + (int64_t)Np * np * m + 2 * (int64_t)Np * m * (mr > 0 ? mr : 1);
}

int orc_starshade_ribbon(int Np, double a, double R, double b, double p, int m, int np, int nd, int md,
                         const double* coef, int K, int mr, double* x, double* y, double* w)
{
    if (mr < 0 || !coef || K < 1) return 1;
    int rc = orc_starshade(Np, a, R, b, p, m, np, nd, md, NULL, 0, x, y, w);
    if (rc) return rc;
    int nt = mr > 0 ? mr : 1;
    double* rx = (double*)malloc(sizeof(double) * m);
    double* rw = (double*)malloc(sizeof(double) * m);
    double* tx = (double*)malloc(sizeof(double) * nt);
    double* tw = (double*)malloc(sizeof(double) * nt);
    orc_gauss_legendre(m, rx, rw);
    if (mr > 0) {
        orc_gauss_legendre(mr, tx, tw);
        for (int j = 0; j < mr; j++) {  /* map [-1, 1] to (0, 1) */
            tx[j] = 0.5 * (1.0 + tx[j]);
            tw[j] = 0.5 * tw[j];
        }
    } else {
        tx[0] = 0.0;  /* the node on the ideal edge */
        tw[0] = 1.0;
    }
    int64_t j = (int64_t)nd * md + (int64_t)Np * np * m;
    for (int k = 0; k < Np; k++) {
        double thk = 2.0 * ORC_PI * k / Np;
        for (int e = 0; e < 2; e++) {            /* 0: upper edge, 1: lower edge */
            double sg = e == 0 ? 1.0 : -1.0;     /* outward is +phi above, -phi below */
            for (int i = 0; i < nt; i++)
                for (int l = 0; l < m; l++) {
                    double r = a + 0.5 * (R - a) * (1.0 + rx[l]);
                    double wr = 0.5 * (R - a) * rw[l];
                    double d = 0.0;
                    for (int s = 1; s <= K; s++)
                        d += coef[2 * k * K + e * K + (s - 1)] * sin(s * ORC_PI * (r - a) / (R - a));
                    double edge = thk + sg * ORC_PI * hg_profile(r, a, b, p) / Np;
                    double phi = edge + sg * tx[i] * d / r;
                    x[j] = r * cos(phi);
                    y[j] = r * sin(phi);
                    w[j] = wr * d * tw[i];
                    j++;
                }
        }
    }
    free(rx); free(rw); free(tx); free(tw);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Direct sum, eq. faq, and Babinet, eq. bab:                               */
/*  u_ap(k) = 1/(i lambda z) sum_j exp(i pi |xi_k - x_j|^2/(lambda z)) w_j   */
/*  u_oc(k) = 1 - u_ap(k)                                                   */
/* The phase is kept in turns, t = |xi-x|^2/(2 lambda z), reduced to         */
/* f = t - rint(t) (exact in FP64) before cos/sin(2 pi f).  The sum over j  */
/* is pairwise.  Output u is interleaved (re, im).                          */
/* ------------------------------------------------------------------------ */
typedef struct { double re, im; } cplx;

static cplx pairwise_terms(const double* x, const double* y, const double* w,
                           int64_t j0, int64_t j1, double xi, double eta, double inv2lz)
{
    cplx s = {0.0, 0.0};
    if (j1 - j0 <= 16) {
        for (int64_t j = j0; j < j1; j++) {
            double dx = xi - x[j], dy = eta - y[j];
            double t = (dx * dx + dy * dy) * inv2lz;
            double f = t - rint(t);
            double ang = 2.0 * ORC_PI * f;
            s.re += cos(ang) * w[j];
            s.im += sin(ang) * w[j];
        }
        return s;
    }
    int64_t jm = j0 + (j1 - j0) / 2;
    cplx a = pairwise_terms(x, y, w, j0, jm, xi, eta, inv2lz);
    cplx b = pairwise_terms(x, y, w, jm, j1, xi, eta, inv2lz);
    s.re = a.re + b.re;
    s.im = a.im + b.im;
    return s;
}

int orc_fresnel_direct(const double* x, const double* y, const double* w, int64_t N,
                       double lambda, double z, const double* xi, const double* eta,
                       int64_t M, int occulter, double* u)
{
    double lz = lambda * z;
    if (!(lz > 0.0)) return 2;
    double inv2lz = 1.0 / (2.0 * lz);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < M; k++) {
        cplx s = {0.0, 0.0};
        if (N > 0) s = pairwise_terms(x, y, w, 0, N, xi[k], eta[k], inv2lz);
        /* multiply by 1/(i lz) = -i/lz */
        double re = s.im / lz, im = -s.re / lz;
        if (occulter) { re = 1.0 - re; im = -im; }
        u[2 * k] = re;
        u[2 * k + 1] = im;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Source-plane variations (sec. 5: a smooth source amplitude/phase enters  */
/* by multiplying each areal weight by the source term at its node) and a  */
/* spherical incident wave from a point source at distance D before the     */
/* aperture (sec. 1: z^-1 becomes z^-1 + D^-1; in the Fresnel approximation */
/* the incident wave at the aperture is exp(i pi |x|^2/(lambda D))):        */
/*  u_ap(k) = 1/(i lambda z) sum_j w_j s_j exp(i pi |x_j|^2/(lambda D))     */
/*                                      exp(i pi |xi_k - x_j|^2/(lambda z)) */
/* src: N interleaved complex s_j, or NULL for s_j = 1; D <= 0 or infinite: */
/* plane wave.  Phase in turns t = |xi-x|^2/(2 lambda z) + |x|^2/(2 lambda D) */
/* reduced by rint; pairwise sum over j.                                    */
/* ------------------------------------------------------------------------ */
static cplx pairwise_src(const double* x, const double* y, const double* w, const double* src,
                         int64_t j0, int64_t j1, double xi, double eta, double inv2lz, double inv2lD)
{
    cplx s = {0.0, 0.0};
    if (j1 - j0 <= 16) {
        for (int64_t j = j0; j < j1; j++) {
            double dx = xi - x[j], dy = eta - y[j];
            double t = (dx * dx + dy * dy) * inv2lz + (x[j] * x[j] + y[j] * y[j]) * inv2lD;
            double f = t - rint(t);
            double c = cos(2.0 * ORC_PI * f), sn = sin(2.0 * ORC_PI * f);
            double ar = w[j], ai = 0.0;
            if (src) { ar = w[j] * src[2 * j]; ai = w[j] * src[2 * j + 1]; }
            s.re += c * ar - sn * ai;
            s.im += sn * ar + c * ai;
        }
        return s;
    }
    int64_t jm = j0 + (j1 - j0) / 2;
    cplx a = pairwise_src(x, y, w, src, j0, jm, xi, eta, inv2lz, inv2lD);
    cplx b = pairwise_src(x, y, w, src, jm, j1, xi, eta, inv2lz, inv2lD);
    s.re = a.re + b.re;
    s.im = a.im + b.im;
    return s;
}

int orc_fresnel_direct_src(const double* x, const double* y, const double* w, const double* src, int64_t N,
                           double lambda, double z, double D, const double* xi, const double* eta, int64_t M,
                           int occulter, double* u)
{
    double lz = lambda * z;
    if (!(lz > 0.0)) return 2;
    double inv2lz = 1.0 / (2.0 * lz);
    double inv2lD = (D > 0.0 && isfinite(D)) ? 1.0 / (2.0 * lambda * D) : 0.0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < M; k++) {
        cplx s = {0.0, 0.0};
        if (N > 0) s = pairwise_src(x, y, w, src, 0, N, xi[k], eta[k], inv2lz, inv2lD);
        double re = s.im / lz, im = -s.re / lz;
        if (occulter) { re = 1.0 - re; im = -im; }
        u[2 * k] = re;
        u[2 * k + 1] = im;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Misaligned rigid petals (sec. 5): petal k's nodes undergo the rigid      */
/* motion x -> Rot(d_k) x + (tx_k, ty_k) (rotation about the origin, then   */
/* translation), weights unchanged; motion = 3 Np doubles (d_k, tx_k, ty_k). */
/* The signed region between the petal's root arc on the disc,              */
/* P(tau) = a (cos phi, sin phi), phi = theta_k + (pi/Np) tau, tau in       */
/* [-1, 1] (the petals meet the disc along the whole circle, A(a) = 1), and */
/* its moved image M(tau) is covered by the map                              */
/* X(tau, t) = P(tau) + t (M(tau) - P(tau)), t in [0, 1], with nb GL nodes  */
/* in tau and mb on (0, 1) in t and weight                                  */
/* omega_tau v_t (dX/dt x dX/dtau): positive where the petal moved outward  */
/* (area added), negative where it moved into the disc (area counted twice). */
/* Node order: the unperturbed starshade rule (disc, then petals), then the */
/* bridges, petal k outer, tau index, then t index inner.                   */
/* N = nd md + Np np m + Np nb mb.                                          */
/* ------------------------------------------------------------------------ */
int orc_starshade_rigid(int Np, double a, double R, double b, double p, int m, int np, int nd, int md,
                        const double* motion, int nb, int mb, double* x, double* y, double* w)
{
    if (nb < 1 || mb < 1) return 1;
    int rc = orc_starshade(Np, a, R, b, p, m, np, nd, md, NULL, 0, x, y, w);
    if (rc) return rc;
    int64_t off = (int64_t)nd * md;
    for (int k = 0; k < Np; k++) {
        double c = cos(motion[3 * k]), sn = sin(motion[3 * k]);
        double tx = motion[3 * k + 1], ty = motion[3 * k + 2];
        for (int64_t j = off + (int64_t)k * np * m; j < off + (int64_t)(k + 1) * np * m; j++) {
            double xx = x[j], yy = y[j];
            x[j] = c * xx - sn * yy + tx;
            y[j] = sn * xx + c * yy + ty;
        }
    }
    double* tg = (double*)malloc(sizeof(double) * nb);
    double* tw = (double*)malloc(sizeof(double) * nb);
    double* ug = (double*)malloc(sizeof(double) * mb);
    double* uw = (double*)malloc(sizeof(double) * mb);
    orc_gauss_legendre(nb, tg, tw);
    orc_gauss_legendre(mb, ug, uw);
    int64_t j = off + (int64_t)Np * np * m;
    for (int k = 0; k < Np; k++) {
        double c = cos(motion[3 * k]), sn = sin(motion[3 * k]);
        double tx = motion[3 * k + 1], ty = motion[3 * k + 2];
        double thk = 2.0 * ORC_PI * k / Np, h = ORC_PI / Np;
        for (int i = 0; i < nb; i++) {
            double phi = thk + h * tg[i];
            double Px = a * cos(phi), Py = a * sin(phi);
            double dPx = -a * h * sin(phi), dPy = a * h * cos(phi);  /* dP/dtau */
            double Mx = c * Px - sn * Py + tx, My = sn * Px + c * Py + ty;
            double dMx = c * dPx - sn * dPy, dMy = sn * dPx + c * dPy;
            for (int l = 0; l < mb; l++) {
                double t = 0.5 * (1.0 + ug[l]), vt = 0.5 * uw[l];
                double Xt = Mx - Px, Yt = My - Py;                  /* dX/dt */
                double Xs = dPx + t * (dMx - dPx), Ys = dPy + t * (dMy - dPy); /* dX/dtau */
                x[j] = Px + t * Xt;
                y[j] = Py + t * Yt;
                w[j] = tw[i] * vt * (Xt * Ys - Yt * Xs);
                j++;
            }
        }
    }
    free(tg); free(tw); free(ug); free(uw);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Gradient of a real loss L through the direct sum.                        */
/* g_k = dL/dRe(u_k) + i dL/dIm(u_k) (interleaved), so that                 */
/* dL = sum_k Re(conj(g_k) du_k).  With E_kj = exp(i pi|xi_k-x_j|^2/lz),     */
/* a_k = conj(g_k) (negated for an occulter, since u_oc = 1 - u_ap):        */
/*   G_j  = sum_k a_k E_kj,   Hx_j = sum_k a_k E_kj xi_k,  Hy_j likewise,    */
/*   dL/dw_j = Re[G_j / (i lz)],                                            */
/*   dL/dx_j = Re[(w_j/(i lz)) (2 pi i/lz) (x_j G_j - Hx_j)],  y likewise.  */
/* (du_k/dx_j = (w_j/(i lz)) E_kj (2 pi i / lz)(x_j - xi_k).)               */
/* ------------------------------------------------------------------------ */
int orc_fresnel_direct_vjp(const double* x, const double* y, const double* w, int64_t N,
                           double lambda, double z, const double* xi, const double* eta,
                           int64_t M, int occulter, const double* g,
                           double* gx, double* gy, double* gw)
{
    double lz = lambda * z;
    if (!(lz > 0.0)) return 2;
    double inv2lz = 1.0 / (2.0 * lz);
    double sgn = occulter ? -1.0 : 1.0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < N; j++) {
        double Gr = 0, Gi = 0, Hxr = 0, Hxi = 0, Hyr = 0, Hyi = 0;
        for (int64_t k = 0; k < M; k++) {
            double dx = xi[k] - x[j], dy = eta[k] - y[j];
            double t = (dx * dx + dy * dy) * inv2lz;
            double f = t - rint(t);
            double c = cos(2.0 * ORC_PI * f), s = sin(2.0 * ORC_PI * f);
            double ar = sgn * g[2 * k], ai = -sgn * g[2 * k + 1]; /* a = sgn conj(g) */
            double er = ar * c - ai * s, ei = ar * s + ai * c;     /* a E */
            Gr += er; Gi += ei;
            Hxr += er * xi[k]; Hxi += ei * xi[k];
            Hyr += er * eta[k]; Hyi += ei * eta[k];
        }
        /* G/(i lz) = (Gi - i Gr)/lz */
        gw[j] = Gi / lz;
        /* (w/(i lz)) (2 pi i/lz) = 2 pi w / lz^2 (real) */
        double fac = 2.0 * ORC_PI * w[j] / (lz * lz);
        gx[j] = fac * (x[j] * Gr - Hxr);
        gy[j] = fac * (y[j] * Gr - Hyr);
    }
    return 0;
}

/* Chain rule through the perturbed starshade construction (same parameters */
/* as orc_starshade).  Disc nodes do not depend on the coefficients.  For a  */
/* petal node, with s_k(r) = sin(k pi (r-a)/(R-a)):                          */
/*   dphi/dc+_k = s_k (1 + tau)/(2r),  dphi/dc-_k = s_k (tau - 1)/(2r),      */
/*   dw/dc+-_k  = wr om s_k / 2,  d(x,y)/dphi = (-y, x).                     */
int orc_starshade_vjp(int Np, double a, double R, double b, double p,
                      int m, int np, int nd, int md, const double* coef, int K,
                      const double* gx, const double* gy, const double* gw, double* gcoef)
{
    if (Np < 1 || m < 1 || np < 1 || K < 1) return 1;
    int64_t off = (int64_t)nd * md;
    double* x = (double*)malloc(sizeof(double) * orc_starshade_size(Np, m, np, nd, md) * 3);
    int64_t N = orc_starshade_size(Np, m, np, nd, md);
    double* y = x + N;
    double* w = y + N;
    orc_starshade(Np, a, R, b, p, m, np, nd, md, coef, K, x, y, w);
    double* rx = (double*)malloc(sizeof(double) * m);
    double* rw = (double*)malloc(sizeof(double) * m);
    double* tx = (double*)malloc(sizeof(double) * np);
    double* tw = (double*)malloc(sizeof(double) * np);
    orc_gauss_legendre(m, rx, rw);
    orc_gauss_legendre(np, tx, tw);
    for (int k = 0; k < Np; k++)
        for (int s = 1; s <= K; s++) {
            double accp = 0.0, accm = 0.0;
            for (int i = 0; i < np; i++)
                for (int l = 0; l < m; l++) {
                    double r = a + 0.5 * (R - a) * (1.0 + rx[l]);
                    double wr = 0.5 * (R - a) * rw[l];
                    double sk = sin(s * ORC_PI * (r - a) / (R - a));
                    int64_t j = off + (int64_t)k * np * m + (int64_t)i * m + l;
                    double dphi_term = gx[j] * (-y[j]) + gy[j] * x[j];
                    double dw = wr * tw[i] * sk / 2.0;
                    accp += dphi_term * sk * (1.0 + tx[i]) / (2.0 * r) + gw[j] * dw;
                    accm += dphi_term * sk * (tx[i] - 1.0) / (2.0 * r) + gw[j] * dw;
                }
            gcoef[2 * k * K + (s - 1)] = accp;
            gcoef[2 * k * K + K + (s - 1)] = accm;
        }
    free(rx); free(rw); free(tx); free(tw); free(x);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Koch snowflake (sec. 4.4): Omega_0 is the equilateral triangle inscribed */
/* in the unit circle, vertices at angles 90, 210, 330 degrees (CCW, side   */
/* sqrt 3, maximum radius 1); Omega_k adds, on the middle third of every    */
/* edge of Omega_{k-1}, the outward equilateral triangle.  Every triangle   */
/* (A, B, C), CCW, gets the p x p rule of the paper: translate A to the     */
/* origin and apply the dilation rule (eqs. aqnod/aqwei) to the p-node GL   */
/* vector line rule on the edge B -> C.  Node order: Omega_0's triangle,    */
/* then level 1's triangles in the order of Omega_0's edges, and so on;     */
/* within a triangle edge index outer, radial index inner.  p[k] is the     */
/* rule order at level k (k = 0..L).                                        */
/* The boundary vertices of Omega_k are kept as a CCW list and each edge    */
/* P -> Q is replaced by P, P + d, P + d + R(-60) d, P + 2d (d = (Q-P)/3);  */
/* for a CCW outline the outward side is to the right, hence R(-60).        */
/* ------------------------------------------------------------------------ */
static void koch_vertices0(double* vx, double* vy)
{
    for (int m = 0; m < 3; m++) {
        double a = 0.5 * ORC_PI + 2.0 * ORC_PI * m / 3.0;
        vx[m] = cos(a);
        vy[m] = sin(a);
    }
}

int64_t orc_koch_size(int L, const int* p)
{
    if (L < 0) return -1;
    int64_t N = 0, ntri = 1;
    for (int k = 0; k <= L; k++) {
        if (p[k] < 1) return -1;
        N += ntri * (int64_t)p[k] * p[k];
        ntri = (k == 0) ? 3 : ntri * 4;
    }
    return N;
}

static int64_t koch_triangle(double ax, double ay, double bx, double by, double cx, double cy, int p,
                             const double* gx, const double* gw, double* x, double* y, double* w, int64_t j)
{
    double ex = cx - bx, ey = cy - by;
    for (int i = 0; i < p; i++) {
        double t = 0.5 * (1.0 + gx[i]);
        double X = bx + t * ex - ax, Y = by + t * ey - ay;
        double W = 0.5 * gw[i] * ex, V = 0.5 * gw[i] * ey;
        double cross = X * V - Y * W;
        for (int l = 0; l < p; l++) {
            double al = 0.5 * (1.0 + gx[l]);
            double wl = 0.5 * gw[l];
            x[j] = ax + al * X;
            y[j] = ay + al * Y;
            w[j] = al * wl * cross;
            j++;
        }
    }
    return j;
}

/* Vertices of Omega_L's outline (3 4^L of them, CCW) into vx, vy. */
int orc_koch_outline(int L, double* vx, double* vy)
{
    if (L < 0) return 1;
    int64_t nv = 3;
    koch_vertices0(vx, vy);
    const double c60 = 0.5, s60 = 0.86602540378443864676;
    double* tx = (double*)malloc(sizeof(double) * 3 * ((int64_t)1 << (2 * L)));
    double* ty = (double*)malloc(sizeof(double) * 3 * ((int64_t)1 << (2 * L)));
    for (int k = 1; k <= L; k++) {
        int64_t o = 0;
        for (int64_t e = 0; e < nv; e++) {
            double px = vx[e], py = vy[e];
            double qx = vx[(e + 1) % nv], qy = vy[(e + 1) % nv];
            double dx = (qx - px) / 3.0, dy = (qy - py) / 3.0;
            tx[o] = px; ty[o] = py; o++;
            tx[o] = px + dx; ty[o] = py + dy; o++;
            tx[o] = px + dx + (c60 * dx + s60 * dy); ty[o] = py + dy + (-s60 * dx + c60 * dy); o++;
            tx[o] = px + 2.0 * dx; ty[o] = py + 2.0 * dy; o++;
        }
        memcpy(vx, tx, sizeof(double) * o);
        memcpy(vy, ty, sizeof(double) * o);
        nv = o;
    }
    free(tx); free(ty);
    return 0;
}

int orc_koch(int L, const int* p, double* x, double* y, double* w)
{
    if (orc_koch_size(L, p) < 0) return 1;
    int pmax = 1;
    for (int k = 0; k <= L; k++) if (p[k] > pmax) pmax = p[k];
    double* gx = (double*)malloc(sizeof(double) * pmax);
    double* gw = (double*)malloc(sizeof(double) * pmax);
    int64_t cap = 3 * ((int64_t)1 << (2 * (L > 0 ? L - 1 : 0)));
    double* vx = (double*)malloc(sizeof(double) * cap);
    double* vy = (double*)malloc(sizeof(double) * cap);
    const double c60 = 0.5, s60 = 0.86602540378443864676;
    koch_vertices0(vx, vy);
    orc_gauss_legendre(p[0], gx, gw);
    int64_t j = koch_triangle(vx[0], vy[0], vx[1], vy[1], vx[2], vy[2], p[0], gx, gw, x, y, w, 0);
    for (int k = 1; k <= L; k++) {
        /* the outline of Omega_{k-1}: its edges carry level k's triangles */
        orc_koch_outline(k - 1, vx, vy);
        int64_t nv = 3 * ((int64_t)1 << (2 * (k - 1)));
        orc_gauss_legendre(p[k], gx, gw);
        for (int64_t e = 0; e < nv; e++) {
            double px = vx[e], py = vy[e];
            double qx = vx[(e + 1) % nv], qy = vy[(e + 1) % nv];
            double dx = (qx - px) / 3.0, dy = (qy - py) / 3.0;
            double ax = px + dx, ay = py + dy;
            double bx = ax + (c60 * dx + s60 * dy), by = ay + (-s60 * dx + c60 * dy);
            double cx = px + 2.0 * dx, cy = py + 2.0 * dy;
            j = koch_triangle(ax, ay, bx, by, cx, cy, p[k], gx, gw, x, y, w, j);
        }
    }
    free(gx); free(gw); free(vx); free(vy);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Starshade boundary rule for the edge integral (eq. vliq on the outline   */
/* of sec. 3.2's petal shape, A(r) = exp(-((r-a)/b)^p) on (a, R)).          */
/* Petal k (centre theta_k = 2 pi k/Np), half-width angle h(r) = pi A(r)/Np: */
/*   lower edge  phi = theta_k - h(r), r from a to R, m GL nodes in r;      */
/*   tip arc     r = R, phi from theta_k - h(R) to theta_k + h(R), ntip GL; */
/*   upper edge  phi = theta_k + h(r), r from R to a, m GL nodes in r;      */
/*   gap arc     r = a, phi from theta_k + h(a) to theta_{k+1} - h(a),      */
/*               ngap GL nodes (zero width, so zero weights, when A(a) = 1, */
/*               as for this profile family).                               */
/* An edge point is P(r) = r (cos phi, sin phi) with                        */
/* P'(r) = (cos phi, sin phi) + r phi'(r) (-sin phi, cos phi),              */
/* phi' = -+ pi A'(r)/Np, A'(r) = -(p/b) ((r-a)/b)^(p-1) A(r); the vector   */
/* weight is P'(r) times the GL weight in r, negated on the upper edge      */
/* (traversed inward), so the outline is counter-clockwise.                 */
/* Node order per petal: lower, tip, upper (outward-to-inward), gap;        */
/* n = Np (2 m + ntip + ngap).                                              */
/* ------------------------------------------------------------------------ */
static double hg_profile_deriv(double r, double a, double b, double p)
{
    if (r <= a) return 0.0;
    double s = (r - a) / b;
    return -(p / b) * pow(s, p - 1.0) * exp(-pow(s, p));
}

static void arc_nodes(double rad, double phi0, double phi1, int nq, const double* gx,
                      const double* gw, double* X, double* Y, double* W, double* V)
{
    double half = 0.5 * (phi1 - phi0);
    for (int i = 0; i < nq; i++) {
        double phi = phi0 + half * (1.0 + gx[i]);
        double om = half * gw[i];
        X[i] = rad * cos(phi);
        Y[i] = rad * sin(phi);
        W[i] = -om * rad * sin(phi);
        V[i] = om * rad * cos(phi);
    }
}

int orc_bdry_starshade(int Np, double a, double R, double b, double p, int m, int ntip,
                       int ngap, double* X, double* Y, double* W, double* V)
{
    if (Np < 1 || m < 1 || ntip < 0 || ngap < 0 || !(R > a) || !(a >= 0)) return 1;
    int nmax = m > ntip ? m : ntip;
    if (ngap > nmax) nmax = ngap;
    double* gx = (double*)malloc(sizeof(double) * nmax);
    double* gw = (double*)malloc(sizeof(double) * nmax);
    int64_t per = 2 * (int64_t)m + ntip + ngap;
    for (int k = 0; k < Np; k++) {
        double thk = 2.0 * ORC_PI * k / Np;
        int64_t o = (int64_t)k * per;
        orc_gauss_legendre(m, gx, gw);
        for (int l = 0; l < m; l++) {
            double r = a + 0.5 * (R - a) * (1.0 + gx[l]);
            double wr = 0.5 * (R - a) * gw[l];
            double h = ORC_PI * hg_profile(r, a, b, p) / Np;
            double dh = ORC_PI * hg_profile_deriv(r, a, b, p) / Np;
            /* lower edge, outward: phi = thk - h, phi' = -dh */
            double pl = thk - h;
            X[o + l] = r * cos(pl);
            Y[o + l] = r * sin(pl);
            W[o + l] = wr * (cos(pl) + r * dh * sin(pl));
            V[o + l] = wr * (sin(pl) - r * dh * cos(pl));
            /* upper edge, inward: phi = thk + h, phi' = dh, node order R -> a */
            double pu = thk + h;
            int64_t iu = o + m + ntip + (m - 1 - l);
            X[iu] = r * cos(pu);
            Y[iu] = r * sin(pu);
            W[iu] = -wr * (cos(pu) - r * dh * sin(pu));
            V[iu] = -wr * (sin(pu) + r * dh * cos(pu));
        }
        if (ntip > 0) {
            orc_gauss_legendre(ntip, gx, gw);
            double hR = ORC_PI * hg_profile(R, a, b, p) / Np;
            arc_nodes(R, thk - hR, thk + hR, ntip, gx, gw, X + o + m, Y + o + m, W + o + m, V + o + m);
        }
        if (ngap > 0) {
            orc_gauss_legendre(ngap, gx, gw);
            double ha = ORC_PI * hg_profile(a, a, b, p) / Np;
            double thn = 2.0 * ORC_PI * (k + 1) / Np;
            int64_t og = o + 2 * (int64_t)m + ntip;
            arc_nodes(a, thk + ha, thn - ha, ngap, gx, gw, X + og, Y + og, W + og, V + og);
        }
    }
    free(gx); free(gw);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Non-singular line integral (appendix, eq. nsli): with r_i = (X_i - xi,   */
/* Y_i - eta) and ds_i = (W_i, V_i) a CCW vector line rule on the boundary, */
/*   u_ap = (1/2pi) sum_i (1 - exp(i pi r_i^2/(lambda z))) (r_i x ds_i)/r_i^2 */
/* with r x ds = r_x V - r_y W and the term taken as 0 when r_i^2 = 0 (the  */
/* cross product vanishes there too).  With t = r^2/(2 lambda z) turns and  */
/* f = t - rint(t), 1 - exp(2 pi i f) = 2 sin(pi f) (sin(pi f) - i cos(pi f)) */
/* (the half-angle identities), which has no cancellation as r -> 0.        */
/* Shadow option (the appendix's remark on deep shadows, with eq. li): when */
/* far > 0 and every node is at distance >= far from the target,            */
/*   u_ap = u_geom - (1/2pi) sum_i exp(i pi r_i^2/(lambda z)) (r_i x ds_i)/r_i^2, */
/* u_geom = 1 inside, 0 outside, taken as the nearest integer to the        */
/* winding number (1/2pi) sum_i (r_i x ds_i)/r_i^2 (u_geom as the integral   */
/* of d theta over 2pi, evaluated with the same rule).                      */
/* Sums over i are pairwise.  u_oc = 1 - u_ap.                              */
/* ------------------------------------------------------------------------ */
typedef struct { double s_re, s_im, e_re, e_im, wind, d2min; } nsli_acc;

static nsli_acc nsli_terms(const double* X, const double* Y, const double* W, const double* V,
                           int64_t i0, int64_t i1, double xi, double eta, double inv2lz)
{
    nsli_acc s = {0.0, 0.0, 0.0, 0.0, 0.0, INFINITY};
    if (i1 - i0 <= 16) {
        for (int64_t i = i0; i < i1; i++) {
            double rx = X[i] - xi, ry = Y[i] - eta;
            double r2 = rx * rx + ry * ry;
            if (r2 < s.d2min) s.d2min = r2;
            if (r2 == 0.0) continue;
            double c = (rx * V[i] - ry * W[i]) / r2;
            double t = r2 * inv2lz;
            double f = t - rint(t);
            double sn = sin(ORC_PI * f), cs = cos(ORC_PI * f);
            s.s_re += 2.0 * sn * sn * c;
            s.s_im += -2.0 * sn * cs * c;
            s.e_re += cos(2.0 * ORC_PI * f) * c;
            s.e_im += sin(2.0 * ORC_PI * f) * c;
            s.wind += c;
        }
        return s;
    }
    int64_t im = i0 + (i1 - i0) / 2;
    nsli_acc a = nsli_terms(X, Y, W, V, i0, im, xi, eta, inv2lz);
    nsli_acc b = nsli_terms(X, Y, W, V, im, i1, xi, eta, inv2lz);
    s.s_re = a.s_re + b.s_re;
    s.s_im = a.s_im + b.s_im;
    s.e_re = a.e_re + b.e_re;
    s.e_im = a.e_im + b.e_im;
    s.wind = a.wind + b.wind;
    s.d2min = a.d2min < b.d2min ? a.d2min : b.d2min;
    return s;
}

int orc_nsli(const double* X, const double* Y, const double* W, const double* V, int64_t n,
             double lambda, double z, const double* xi, const double* eta, int64_t M,
             double far, int occulter, double* u)
{
    double lz = lambda * z;
    if (!(lz > 0.0)) return 2;
    double inv2lz = 1.0 / (2.0 * lz);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < M; k++) {
        double re = 0.0, im = 0.0;
        if (n > 0) {
            nsli_acc s = nsli_terms(X, Y, W, V, 0, n, xi[k], eta[k], inv2lz);
            if (far > 0.0 && s.d2min >= far * far) {
                double geom = rint(s.wind / (2.0 * ORC_PI));
                re = geom - s.e_re / (2.0 * ORC_PI);
                im = -s.e_im / (2.0 * ORC_PI);
            } else {
                re = s.s_re / (2.0 * ORC_PI);
                im = s.s_im / (2.0 * ORC_PI);
            }
        }
        if (occulter) { re = 1.0 - re; im = -im; }
        u[2 * k] = re;
        u[2 * k + 1] = im;
    }
    return 0;
}

/* Number of OpenMP threads the direct sum will use (1 without OpenMP). */
int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Use n threads from now on (n >= 1; ignored without OpenMP). */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
    return 0;
}

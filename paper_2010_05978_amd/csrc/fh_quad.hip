// fh_quad.hip -- areal quadrature generation on the device.
//
// Boundary vector line-integral rules (eq. vliq): Gauss-Legendre panels in
// angle for star-shaped curves (eq. vliq1 with Gauss-Legendre in place of the
// trapezoid rule), the periodic trapezoid rule (eq. ptr), and Gauss-Legendre
// nodes along polygon edges.  The dilation areal rule (eqs. aqnod/aqwei,
// sec. 3.1) and the starshade disc + petal rule (sec. 3.2) turn them into
// areal nodes and weights.  Generated rules run as one kernel, a block of
// areal nodes evaluating the boundary nodes it needs into LDS first; every
// coordinate is double.
#include <algorithm>
#include <cstring>

#include "fh_common.hpp"

namespace fh {
namespace {

struct RadialParams {
    double r0;
    int K;
    int panels;  // 0: periodic trapezoid rule with q nodes
    int q;
    double a[kMaxFourier];
    double b[kMaxFourier];
};

// Boundary node i of the star-shaped curve r(t)(cos t, sin t) and its
// vector weight (W, V) = x'(t) omega.
__device__ __forceinline__ void radial_node(const RadialParams& rp, const double* __restrict__ gl, int64_t n,
                                            int64_t i, double& X, double& Y, double& W, double& V)
{
    double t, om;
    if (rp.panels > 0) {
        const int p = (int)(i / rp.q), k = (int)(i % rp.q);
        t = (2.0 * kPi / rp.panels) * (p + 0.5 * (1.0 + gl[k]));
        om = (kPi / rp.panels) * gl[rp.q + k];
    } else {
        t = 2.0 * kPi * (double)(i + 1) / (double)n;
        om = 2.0 * kPi / (double)n;
    }
    double r = rp.r0, dr = 0.0;
    for (int k = 1; k <= rp.K; ++k) {
        double s, c;
        sincos(k * t, &s, &c);
        r += rp.a[k - 1] * c + rp.b[k - 1] * s;
        dr += k * (rp.b[k - 1] * c - rp.a[k - 1] * s);
    }
    double st, ct;
    sincos(t, &st, &ct);
    X = r * ct;
    Y = r * st;
    W = om * (dr * ct - r * st);
    V = om * (dr * st + r * ct);
}

// General closed curve X(t) = sum_{k=0}^{K} ax_k cos kt + bx_k sin kt, Y(t)
// likewise (the kite of sec. 3.1 is X = 0.5 cos t + 0.5 cos 2t, Y = sin t),
// with the same panel or trapezoid rule in t as the star-shaped curve.
struct FourierParams {
    int K;
    int panels;  // 0: periodic trapezoid rule with q nodes
    int q;
    double ax[kMaxFourier + 1];
    double bx[kMaxFourier + 1];
    double ay[kMaxFourier + 1];
    double by[kMaxFourier + 1];
};

__device__ __forceinline__ void bdry_node(const RadialParams& rp, const double* __restrict__ gl, int64_t n,
                                          int64_t i, double& X, double& Y, double& W, double& V)
{
    radial_node(rp, gl, n, i, X, Y, W, V);
}

__device__ __forceinline__ void bdry_node(const FourierParams& fp, const double* __restrict__ gl, int64_t n,
                                          int64_t i, double& X, double& Y, double& W, double& V)
{
    double t, om;
    if (fp.panels > 0) {
        const int p = (int)(i / fp.q), k = (int)(i % fp.q);
        t = (2.0 * kPi / fp.panels) * (p + 0.5 * (1.0 + gl[k]));
        om = (kPi / fp.panels) * gl[fp.q + k];
    } else {
        t = 2.0 * kPi * (double)(i + 1) / (double)n;
        om = 2.0 * kPi / (double)n;
    }
    double x = 0.0, y = 0.0, dx = 0.0, dy = 0.0;
    for (int k = 0; k <= fp.K; ++k) {
        double s, c;
        sincos(k * t, &s, &c);
        x += fp.ax[k] * c + fp.bx[k] * s;
        y += fp.ay[k] * c + fp.by[k] * s;
        dx += k * (fp.bx[k] * c - fp.ax[k] * s);
        dy += k * (fp.by[k] * c - fp.ay[k] * s);
    }
    X = x;
    Y = y;
    W = om * dx;
    V = om * dy;
}

// Boundary rule and dilation in one pass: a block of 256 areal nodes
// j = l + i m first evaluates the boundary nodes i it touches (one thread
// each, through LDS), then every thread dilates its own node.
template <class P>
__device__ __forceinline__ void curve_rule(const P& rp, const double* __restrict__ glq, int64_t n, int m,
                                           const double* __restrict__ glm, double* __restrict__ x,
                                           double* __restrict__ y, double* __restrict__ w)
{
    __shared__ double sb[4][256];
    const int64_t j0 = blockIdx.x * (int64_t)blockDim.x;
    const int64_t i0 = j0 / m;
    const int64_t jl = min(j0 + (int64_t)blockDim.x, n * m) - 1;
    const int nb = (int)(jl / m - i0) + 1;  // at most 256 boundary nodes
    if ((int)threadIdx.x < nb) {
        double X, Y, W, V;
        bdry_node(rp, glq, n, i0 + threadIdx.x, X, Y, W, V);
        sb[0][threadIdx.x] = X;
        sb[1][threadIdx.x] = Y;
        sb[2][threadIdx.x] = W;
        sb[3][threadIdx.x] = V;
    }
    __syncthreads();
    const int64_t j = j0 + threadIdx.x;
    if (j >= n * m) return;
    const int64_t i = j / m;
    const int l = (int)(j - i * m);
    const int bi = (int)(i - i0);
    const double al = 0.5 * (1.0 + glm[l]);
    const double wl = 0.5 * glm[m + l];
    const double Xi = sb[0][bi], Yi = sb[1][bi];
    x[j] = al * Xi;
    y[j] = al * Yi;
    w[j] = al * wl * (Xi * sb[3][bi] - Yi * sb[2][bi]);
}

__global__ void __launch_bounds__(256) k_radial_rule(RadialParams rp, const double* __restrict__ glq, int64_t n,
                                                     int m, const double* __restrict__ glm, double* __restrict__ x,
                                                     double* __restrict__ y, double* __restrict__ w)
{
    curve_rule(rp, glq, n, m, glm, x, y, w);
}

__global__ void __launch_bounds__(256) k_fourier_rule(FourierParams fp, const double* __restrict__ glq, int64_t n,
                                                      int m, const double* __restrict__ glm, double* __restrict__ x,
                                                      double* __restrict__ y, double* __restrict__ w)
{
    curve_rule(fp, glq, n, m, glm, x, y, w);
}

// Koch snowflake (sec. 4.4): Omega_0 is the equilateral triangle inscribed in
// the unit circle (vertices at 90, 210, 330 degrees, CCW); level k >= 1 adds
// the outward equilateral triangle on the middle third of every edge of
// Omega_{k-1}.  Each triangle (A, B, C) gets the p_k x p_k rule obtained by
// translating A to the origin and dilating the p_k-node GL line rule on the
// edge B -> C (eqs. aqnod/aqwei).  One thread per node: the level from the
// node offsets, the triangle from its edge index, whose base-4 digits (most
// significant first) walk the construction down from one of the three
// sides: digit 0 keeps the first third, 1 turns -60 degrees after it, 2 turns
// +60 degrees after the bump's apex, 3 takes the last third.
constexpr int kKochMaxLevel = 15;
struct KochParams {
    int L;
    int p[kKochMaxLevel + 1];
    int64_t off[kKochMaxLevel + 2];        // first node of each level, off[L + 1] = N
    const double* gl[kKochMaxLevel + 1];   // GL rule of order p[k]: x then w
};

__device__ __forceinline__ void rot60(double x, double y, double sg, double& rx, double& ry)
{
    constexpr double c = 0.5, s = 0.86602540378443864676;  // cos, sin of 60 degrees
    rx = c * x - sg * s * y;
    ry = sg * s * x + c * y;
}

__global__ void __launch_bounds__(256) k_koch_rule(KochParams kp, double* __restrict__ x, double* __restrict__ y,
                                                   double* __restrict__ w)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= kp.off[kp.L + 1]) return;
    int k = 0;
    while (j >= kp.off[k + 1]) ++k;
    const int pk = kp.p[k];
    const int64_t local = j - kp.off[k];
    const int64_t pp = (int64_t)pk * pk;
    const int64_t tri = local / pp;
    const int r = (int)(local - tri * pp);
    const int i = r / pk, l = r - i * pk;
    double V[3][2];
    for (int m = 0; m < 3; ++m) sincos(0.5 * kPi + 2.0 * kPi * m / 3.0, &V[m][1], &V[m][0]);
    double ax, ay, bx, by, cx, cy;
    if (k == 0) {
        ax = V[0][0]; ay = V[0][1];
        bx = V[1][0]; by = V[1][1];
        cx = V[2][0]; cy = V[2][1];
    } else {
        // edge `tri` of Omega_{k-1}: side b, then k - 1 base-4 digits
        int64_t nb = (int64_t)1 << (2 * (k - 1));
        const int b = (int)(tri / nb);
        int64_t rem = tri - (int64_t)b * nb;
        double px = V[b][0], py = V[b][1];
        double dx = V[(b + 1) % 3][0] - px, dy = V[(b + 1) % 3][1] - py;
        for (int t = k - 2; t >= 0; --t) {
            nb >>= 2;
            const int d = (int)(rem / nb);
            rem -= (int64_t)d * nb;
            dx /= 3.0;
            dy /= 3.0;
            double rx, ry;
            if (d == 1) {
                px += dx; py += dy;
                rot60(dx, dy, -1.0, rx, ry);
                dx = rx; dy = ry;
            } else if (d == 2) {
                rot60(dx, dy, -1.0, rx, ry);
                px += dx + rx; py += dy + ry;
                rot60(dx, dy, 1.0, rx, ry);
                dx = rx; dy = ry;
            } else if (d == 3) {
                px += 2.0 * dx; py += 2.0 * dy;
            }
        }
        // the outward triangle on the middle third of the edge (P, P + D)
        dx /= 3.0;
        dy /= 3.0;
        double rx, ry;
        rot60(dx, dy, -1.0, rx, ry);
        ax = px + dx; ay = py + dy;
        bx = ax + rx; by = ay + ry;
        cx = px + 2.0 * dx; cy = py + 2.0 * dy;
    }
    const double* g = kp.gl[k];
    const double ex = cx - bx, ey = cy - by;
    const double t = 0.5 * (1.0 + g[i]);
    const double X = bx + t * ex - ax, Y = by + t * ey - ay;
    const double cross = X * (0.5 * g[pk + i] * ey) - Y * (0.5 * g[pk + i] * ex);
    const double al = 0.5 * (1.0 + g[l]);
    x[j] = ax + al * X;
    y[j] = ay + al * Y;
    w[j] = al * (0.5 * g[pk + l]) * cross;
}

// Gauss-Legendre nodes along each straight edge of a CCW polygon.
__global__ void k_bdry_polygon(const double* __restrict__ vx, const double* __restrict__ vy, int nv,
                               int q, const double* __restrict__ gl, double* __restrict__ X,
                               double* __restrict__ Y, double* __restrict__ Wv,
                               double* __restrict__ Vv)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)nv * q) return;
    const int e = (int)(i / q), k = (int)(i % q);
    const int f = (e + 1 == nv) ? 0 : e + 1;
    const double ex = vx[f] - vx[e], ey = vy[f] - vy[e];
    const double s = 0.5 * (1.0 + gl[k]);
    const double hw = 0.5 * gl[q + k];
    X[i] = vx[e] + s * ex;
    Y[i] = vy[e] + s * ey;
    Wv[i] = hw * ex;
    Vv[i] = hw * ey;
}

// Polygons of up to this many vertices travel in the kernel arguments.
struct PolyParams {
    int nv, q;
    double vx[kPolyByValue];
    double vy[kPolyByValue];
};

// Polygon edge rule and dilation in one pass (as k_radial_rule).
__global__ void __launch_bounds__(256) k_polygon_rule(PolyParams pp, const double* __restrict__ glq, int m,
                                                      const double* __restrict__ glm, double* __restrict__ x,
                                                      double* __restrict__ y, double* __restrict__ w)
{
    __shared__ double sb[4][256];
    const int64_t n = (int64_t)pp.nv * pp.q;
    const int64_t j0 = blockIdx.x * (int64_t)blockDim.x;
    const int64_t i0 = j0 / m;
    const int64_t jl = min(j0 + (int64_t)blockDim.x, n * m) - 1;
    const int nb = (int)(jl / m - i0) + 1;
    if ((int)threadIdx.x < nb) {
        const int64_t i = i0 + threadIdx.x;
        const int e = (int)(i / pp.q), k = (int)(i % pp.q);
        const int f = (e + 1 == pp.nv) ? 0 : e + 1;
        const double ex = pp.vx[f] - pp.vx[e], ey = pp.vy[f] - pp.vy[e];
        const double sg = 0.5 * (1.0 + glq[k]);
        const double hw = 0.5 * glq[pp.q + k];
        sb[0][threadIdx.x] = pp.vx[e] + sg * ex;
        sb[1][threadIdx.x] = pp.vy[e] + sg * ey;
        sb[2][threadIdx.x] = hw * ex;
        sb[3][threadIdx.x] = hw * ey;
    }
    __syncthreads();
    const int64_t j = j0 + threadIdx.x;
    if (j >= n * m) return;
    const int64_t i = j / m;
    const int l = (int)(j - i * m);
    const int bi = (int)(i - i0);
    const double al = 0.5 * (1.0 + glm[l]);
    const double wl = 0.5 * glm[m + l];
    const double Xi = sb[0][bi], Yi = sb[1][bi];
    x[j] = al * Xi;
    y[j] = al * Yi;
    w[j] = al * wl * (Xi * sb[3][bi] - Yi * sb[2][bi]);
}

// Dilation rule: node j = l + i m takes alpha_l (X_i, Y_i) with weight
// alpha_l wt_l (X_i V_i - Y_i W_i); alpha, wt = m-node GL on (0,1).
__global__ void k_dilation(const double* __restrict__ X, const double* __restrict__ Y,
                           const double* __restrict__ Wv, const double* __restrict__ Vv, int64_t n,
                           int m, const double* __restrict__ gl, double* __restrict__ x,
                           double* __restrict__ y, double* __restrict__ w)
{
    int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n * m) return;
    const int64_t i = j / m;
    const int l = (int)(j - i * m);
    const double al = 0.5 * (1.0 + gl[l]);
    const double wl = 0.5 * gl[m + l];
    const double Xi = X[i], Yi = Y[i];
    x[j] = al * Xi;
    y[j] = al * Yi;
    w[j] = al * wl * (Xi * Vv[i] - Yi * Wv[i]);
}

struct PetalParams {
    int Np, m, np, K;
    double a, R, b, p;
    int64_t off;  // first petal node
};

// Petal node j = off + k np m + i m + l.
// The apodisation is the HG family A(r) = exp(-((r-a)/b)^p), or, with
// Atab, the table Atab[l] = A(r_l) at the radial nodes.
__global__ void k_petals(PetalParams pp, const double* __restrict__ glm, const double* __restrict__ gln,
                         const double* __restrict__ coef, const double* __restrict__ Atab, double* __restrict__ x,
                         double* __restrict__ y, double* __restrict__ w)
{
    const int64_t per = (int64_t)pp.np * pp.m;
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= per * pp.Np) return;
    const int k = (int)(t / per);
    const int64_t rem = t - k * per;
    const int i = (int)(rem / pp.m);
    const int l = (int)(rem - (int64_t)i * pp.m);
    const double L = pp.R - pp.a;
    const double r = pp.a + 0.5 * L * (1.0 + glm[l]);
    const double wr = 0.5 * L * glm[pp.m + l];
    const double tau = gln[i], wt = gln[pp.np + i];
    const double A = Atab ? Atab[l] : exp(-pow((r - pp.a) / pp.b, pp.p));
    double dp = 0.0, dm = 0.0;
    if (coef) {
        // sin(s theta), s = 1..K, by the three-term recurrence
        // sin((s+1) theta) = 2 cos(theta) sin(s theta) - sin((s-1) theta)
        const double* cp = coef + 2 * (int64_t)k * pp.K;
        double s1, c1;
        sincospi((r - pp.a) / L, &s1, &c1);
        double sm = 0.0, sk = s1;
        for (int s = 1; s <= pp.K; ++s) {
            dp += cp[s - 1] * sk;
            dm += cp[pp.K + s - 1] * sk;
            const double sn = 2.0 * c1 * sk - sm;
            sm = sk;
            sk = sn;
        }
    }
    const double mid = (dp - dm) / (2.0 * r);
    const double half = kPi * A / pp.Np + (dp + dm) / (2.0 * r);
    const double phi = 2.0 * kPi * k / pp.Np + mid + half * tau;
    double sp, cp;
    sincos(phi, &sp, &cp);
    const int64_t j = pp.off + t;
    x[j] = r * cp;
    y[j] = r * sp;
    w[j] = r * wr * half * wt;
}

// Ribbon quadrature (sec. 5): the signed strip between each petal edge of the
// ideal starshade and the same edge displaced outward by the arc length
// d(r) = sum_s coef[s - 1] sin(s pi (r - a)/(R - a)) (the upper edge's
// coefficients, then the lower edge's, per petal).  Node t = ((2 k + e) nt +
// i) m + l of the ribbon part: petal k, edge e (0 upper, 1 lower), across
// index i, radial index l; phi = ideal edge angle +- tau_i d(r_l)/r_l (+ for
// the upper edge, - for the lower: outward), weight wr_l d(r_l) v_i.  glt
// holds the nt across nodes tau in (0, 1) and their weights v (or the single
// node tau = 0 with v = 1: the line integral on the ideal edge).
struct RibbonParams {
    int Np, m, nt, K;
    double a, R, b, p;
    int64_t off;  // first ribbon node
};

__global__ void k_ribbons(RibbonParams rp, const double* __restrict__ glm, const double* __restrict__ glt,
                          const double* __restrict__ coef, double* __restrict__ x, double* __restrict__ y,
                          double* __restrict__ w)
{
    const int64_t per_edge = (int64_t)rp.nt * rp.m;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= 2 * per_edge * rp.Np) return;
    const int ke = (int)(t / per_edge);  // 2 k + e
    const int k = ke >> 1, e = ke & 1;
    const int64_t rem = t - (int64_t)ke * per_edge;
    const int i = (int)(rem / rp.m);
    const int l = (int)(rem - (int64_t)i * rp.m);
    const double L = rp.R - rp.a;
    const double r = rp.a + 0.5 * L * (1.0 + glm[l]);
    const double wr = 0.5 * L * glm[rp.m + l];
    const double* cp = coef + (2 * (int64_t)k + e) * rp.K;
    double d = 0.0;
    {
        // sin(s theta) by the three-term recurrence, as in k_petals
        double s1, c1;
        sincospi((r - rp.a) / L, &s1, &c1);
        double sm = 0.0, sk = s1;
        for (int s = 1; s <= rp.K; ++s) {
            d += cp[s - 1] * sk;
            const double sn = 2.0 * c1 * sk - sm;
            sm = sk;
            sk = sn;
        }
    }
    const double sg = e == 0 ? 1.0 : -1.0;
    const double A = exp(-pow((r - rp.a) / rp.b, rp.p));
    const double phi = 2.0 * kPi * k / rp.Np + sg * (kPi * A / rp.Np + glt[i] * d / r);
    double sp, cph;
    sincos(phi, &sp, &cph);
    const int64_t j = rp.off + t;
    x[j] = r * cph;
    y[j] = r * sp;
    w[j] = wr * d * glt[rp.nt + i];
}

// Boundary rule alone (for the edge integral): one thread per node.
__global__ void k_bdry_radial(RadialParams rp, const double* __restrict__ glq, int64_t n, double* __restrict__ X,
                              double* __restrict__ Y, double* __restrict__ Wv, double* __restrict__ Vv)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x, y, w, v;
    radial_node(rp, glq, n, i, x, y, w, v);
    X[i] = x;
    Y[i] = y;
    Wv[i] = w;
    Vv[i] = v;
}

__global__ void k_bdry_fourier(FourierParams fp, const double* __restrict__ glq, int64_t n, double* __restrict__ X,
                               double* __restrict__ Y, double* __restrict__ Wv, double* __restrict__ Vv)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x, y, w, v;
    bdry_node(fp, glq, n, i, x, y, w, v);
    X[i] = x;
    Y[i] = y;
    Wv[i] = w;
    Vv[i] = v;
}

// Starshade outline (sec. 3.2's petal shape): per petal k, with half-width
// angle h(r) = pi A(r)/Np about theta_k = 2 pi k/Np, the lower edge
// theta_k - h(r) for r from a to R (m GL radii), the tip arc at r = R
// (ntip GL angles), the upper edge theta_k + h(r) from R back to a, and the
// arc at r = a to the next petal (ngap GL angles; of zero width when
// A(a) = 1).  Edge weights are P'(r) w_r with P(r) = r (cos phi, sin phi)
// and phi'(r) = -+ pi A'(r)/Np, negated on the inward upper edge.
struct OutlineParams {
    int Np, m, ntip, ngap;
    double a, R, b, p;
};

__device__ __forceinline__ void arc_node(double rad, double phi0, double phi1, double x, double wq, double& X,
                                         double& Y, double& W, double& V)
{
    const double half = 0.5 * (phi1 - phi0);
    double s, c;
    sincos(phi0 + half * (1.0 + x), &s, &c);
    X = rad * c;
    Y = rad * s;
    W = -half * wq * rad * s;
    V = half * wq * rad * c;
}

__global__ void k_bdry_starshade(OutlineParams op, const double* __restrict__ glm, const double* __restrict__ glt,
                                 const double* __restrict__ glg, double* __restrict__ X, double* __restrict__ Y,
                                 double* __restrict__ Wv, double* __restrict__ Vv)
{
    const int per = 2 * op.m + op.ntip + op.ngap;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)per * op.Np) return;
    const int k = (int)(i / per);
    const int j = (int)(i - (int64_t)k * per);
    const double thk = 2.0 * kPi * k / op.Np;
    double x, y, w, v;
    if (j < op.m || (j >= op.m + op.ntip && j < 2 * op.m + op.ntip)) {
        const bool lower = j < op.m;
        const int l = lower ? j : 2 * op.m + op.ntip - 1 - j;
        const double L = op.R - op.a;
        const double r = op.a + 0.5 * L * (1.0 + glm[l]);
        const double wr = 0.5 * L * glm[op.m + l];
        const double sr = (r - op.a) / op.b;
        const double A = exp(-pow(sr, op.p));
        const double dA = r > op.a ? -(op.p / op.b) * pow(sr, op.p - 1.0) * A : 0.0;
        const double sg = lower ? -1.0 : 1.0;  // phi = thk + sg h(r)
        const double phi = thk + sg * kPi * A / op.Np;
        const double dphi = sg * kPi * dA / op.Np;
        double s, c;
        sincos(phi, &s, &c);
        const double ww = lower ? wr : -wr;
        x = r * c;
        y = r * s;
        w = ww * (c - r * dphi * s);
        v = ww * (s + r * dphi * c);
    } else if (j < op.m + op.ntip) {
        const int t = j - op.m;
        const double h = kPi * exp(-pow((op.R - op.a) / op.b, op.p)) / op.Np;
        arc_node(op.R, thk - h, thk + h, glt[t], glt[op.ntip + t], x, y, w, v);
    } else {
        const int t = j - 2 * op.m - op.ntip;
        const double h = kPi / op.Np;  // A(a) = 1
        arc_node(op.a, thk + h, thk + 2.0 * kPi / op.Np - h, glg[t], glg[op.ngap + t], x, y, w, v);
    }
    X[i] = x;
    Y[i] = y;
    Wv[i] = w;
    Vv[i] = v;
}

// Misaligned rigid petals (sec. 5): petal k's nodes move by
// x -> Rot(d_k) x + (tx_k, ty_k), weights unchanged, and the signed region
// between its root arc P(tau) = a (cos phi, sin phi), phi = theta_k +
// (pi/Np) tau, and the moved arc M(tau) is covered by
// X(tau, t) = P + t (M - P) with weight w_tau v_t (dX/dt x dX/dtau).
constexpr int kRigidMaxPetals = 64;
struct RigidParams {
    int Np, np, m, nb, mb;
    double a;
    int64_t petal_off;   // first petal node
    int64_t bridge_off;  // first bridge node
    double motion[3 * kRigidMaxPetals];  // per petal: angle, tx, ty
};

__global__ void k_rigid_move(RigidParams rp, double* __restrict__ x, double* __restrict__ y)
{
    const int64_t per = (int64_t)rp.np * rp.m;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= per * rp.Np) return;
    const int k = (int)(t / per);
    const int64_t j = rp.petal_off + t;
    double s, c;
    sincos(rp.motion[3 * k], &s, &c);
    const double xx = x[j], yy = y[j];
    x[j] = c * xx - s * yy + rp.motion[3 * k + 1];
    y[j] = s * xx + c * yy + rp.motion[3 * k + 2];
}

__global__ void k_rigid_bridges(RigidParams rp, const double* __restrict__ glb, const double* __restrict__ glt,
                                double* __restrict__ x, double* __restrict__ y, double* __restrict__ w)
{
    const int64_t per = (int64_t)rp.nb * rp.mb;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= per * rp.Np) return;
    const int k = (int)(t / per);
    const int r = (int)(t - (int64_t)k * per);
    const int i = r / rp.mb, l = r - i * rp.mb;
    double s, c;
    sincos(rp.motion[3 * k], &s, &c);
    const double h = kPi / rp.Np;
    const double phi = 2.0 * kPi * k / rp.Np + h * glb[i];
    double sp, cp;
    sincos(phi, &sp, &cp);
    const double px = rp.a * cp, py = rp.a * sp;
    const double dpx = -rp.a * h * sp, dpy = rp.a * h * cp;
    const double mx = c * px - s * py + rp.motion[3 * k + 1], my = s * px + c * py + rp.motion[3 * k + 2];
    const double dmx = c * dpx - s * dpy, dmy = s * dpx + c * dpy;
    const double tt = 0.5 * (1.0 + glt[l]);
    const double xt = mx - px, yt = my - py;
    const double xs = dpx + tt * (dmx - dpx), ys = dpy + tt * (dmy - dpy);
    const int64_t j = rp.bridge_off + t;
    x[j] = px + tt * xt;
    y[j] = py + tt * yt;
    w[j] = glb[rp.nb + i] * (0.5 * glt[rp.mb + l]) * (xt * ys - yt * xs);
}

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)std::max<int64_t>(1, (n + bs - 1) / bs); }

// A box that contains every node (used to size fine grids and row windows).
void set_bbox(fh_quad* q, double x0, double x1, double y0, double y1)
{
    q->bbox[0] = x0;
    q->bbox[1] = x1;
    q->bbox[2] = y0;
    q->bbox[3] = y1;
    q->bbox_valid = true;
}

// A box holding every node of a dilation rule: each node is alpha (X_i, Y_i)
// with 0 < alpha < 1, so the box of the boundary nodes and the origin holds
// them all.  The boundary nodes are evaluated on the host at the rule's own
// parameters t_i (Gauss-Legendre panels, or the trapezoid rule when panels is
// 0), curve(cos t, sin t, X, Y) giving the point; the box is widened by a
// relative 1e-9 for the rounding of either side.  A tight box keeps the
// type-1 row window (and with it the FFT and the column pass) as small as the
// shape allows.  cos t and sin t come from angle-addition recurrences (one
// sincos per panel and per Gauss node offset, or a rotation by 2 pi/n per
// trapezoid node, re-anchored every 1024 nodes), whose rounding the widening
// covers: a rule is
// built per call, and a sincos per boundary node would cost tens of
// microseconds of host time for a few hundred nodes.
template <class Curve>
void boundary_box(int64_t n, int panels, int q, Curve curve, double* box)
{
    double b[4] = {0.0, 0.0, 0.0, 0.0};
    auto take = [&](double ct, double st) {
        double X, Y;
        curve(ct, st, X, Y);
        b[0] = std::min(b[0], X);
        b[1] = std::max(b[1], X);
        b[2] = std::min(b[2], Y);
        b[3] = std::max(b[3], Y);
    };
    if (panels > 0) {
        std::vector<double> gx, gw, cd(q), sd(q);
        gl_host(q, gx, gw);
        const double hp = 2.0 * kPi / panels;
        for (int k = 0; k < q; ++k) {
            cd[k] = std::cos(0.5 * hp * (1.0 + gx[k]));
            sd[k] = std::sin(0.5 * hp * (1.0 + gx[k]));
        }
        for (int p = 0; p < panels; ++p) {
            const double cp = std::cos(hp * p), sp = std::sin(hp * p);
            for (int k = 0; k < q; ++k) take(cp * cd[k] - sp * sd[k], sp * cd[k] + cp * sd[k]);
        }
    } else {
        const double cs = std::cos(2.0 * kPi / (double)n), sn = std::sin(2.0 * kPi / (double)n);
        double ct = cs, st = sn;  // t_0 = 2 pi/n
        for (int64_t i = 0; i < n; ++i) {
            take(ct, st);
            if ((i & 1023) == 1023) {
                // re-anchored every 1024 nodes: the drift stays ~1e-13
                const double t = 2.0 * kPi * (double)(i + 2) / (double)n;
                ct = std::cos(t);
                st = std::sin(t);
                continue;
            }
            const double cn = ct * cs - st * sn;
            st = st * cs + ct * sn;
            ct = cn;
        }
    }
    const double pad = 1e-9 * (std::max({-b[0], b[1], -b[2], b[3]}) + 1.0);
    box[0] = b[0] - pad;
    box[1] = b[1] + pad;
    box[2] = b[2] - pad;
    box[3] = b[3] + pad;
}

// cos k t and sin k t for k = 1..K from c1 = cos t, s1 = sin t.
inline void harmonics(double c1, double s1, int K, double* c, double* s)
{
    double ck = 1.0, sk = 0.0;
    for (int k = 1; k <= K; ++k) {
        const double cn = ck * c1 - sk * s1;
        sk = sk * c1 + ck * s1;
        ck = cn;
        c[k] = ck;
        s[k] = sk;
    }
}

void radial_box(const RadialParams& rp, int64_t n, double* box)
{
    boundary_box(n, rp.panels, rp.q, [&](double ct, double st, double& X, double& Y) {
        double c[kMaxFourier + 1], s[kMaxFourier + 1];
        harmonics(ct, st, rp.K, c, s);
        double r = rp.r0;
        for (int k = 1; k <= rp.K; ++k) r += rp.a[k - 1] * c[k] + rp.b[k - 1] * s[k];
        X = r * ct;
        Y = r * st;
    }, box);
}

void fourier_box(const FourierParams& fp, int64_t n, double* box)
{
    boundary_box(n, fp.panels, fp.q, [&](double ct, double st, double& X, double& Y) {
        double c[kMaxFourier + 1], s[kMaxFourier + 1];
        harmonics(ct, st, fp.K, c, s);
        X = fp.ax[0];
        Y = fp.ay[0];
        for (int k = 1; k <= fp.K; ++k) {
            X += fp.ax[k] * c[k] + fp.bx[k] * s[k];
            Y += fp.ay[k] * c[k] + fp.by[k] * s[k];
        }
    }, box);
}

fh_status radial_into(fh_ctx* c, const RadialParams& rp, int64_t n, int m, double* x, double* y,
                      double* w)
{
    const double* glq = nullptr;
    const double* glm = nullptr;
    if (rp.panels > 0) FH_TRY(gl_table(c, rp.q, &glq));
    FH_TRY(gl_table(c, m, &glm));
    hipLaunchKernelGGL(k_radial_rule, dim3(nblocks(n * m, 256)), dim3(256), 0, c->stream, rp, glq, n, m, glm, x, y,
                       w);
    FH_HIP(hipGetLastError());
    return FH_OK;
}

// Fourier-curve parameters from host coefficient arrays (K + 1 each; bx[0],
// by[0] multiply sin 0 and are ignored); also returns a box holding the curve
// and the origin (the dilation nodes lie on segments from the origin).
fh_status fourier_params(const double* ax, const double* bx, const double* ay, const double* by, int K, int panels,
                         int q, FourierParams* fp, double* box)
{
    FH_ARG(ax && ay, FH_ERR_INVALID_ARG, "NULL coefficient array");
    FH_ARG(K >= 0 && K <= kMaxFourier, FH_ERR_INVALID_ARG, "K must be in [0, %d]", kMaxFourier);
    FH_ARG(panels >= 0 && q >= 1, FH_ERR_INVALID_ARG, "need panels >= 0, q >= 1");
    *fp = FourierParams{};
    fp->K = K;
    fp->panels = panels;
    fp->q = q;
    double ex = 0.0, ey = 0.0;
    for (int k = 0; k <= K; ++k) {
        fp->ax[k] = ax[k];
        fp->bx[k] = (bx && k > 0) ? bx[k] : 0.0;
        fp->ay[k] = ay[k];
        fp->by[k] = (by && k > 0) ? by[k] : 0.0;
        FH_ARG(std::isfinite(fp->ax[k]) && std::isfinite(fp->bx[k]) && std::isfinite(fp->ay[k]) &&
                   std::isfinite(fp->by[k]),
               FH_ERR_NONFINITE, "Fourier coefficient %d not finite", k);
        if (k > 0) {
            ex += std::fabs(fp->ax[k]) + std::fabs(fp->bx[k]);
            ey += std::fabs(fp->ay[k]) + std::fabs(fp->by[k]);
        }
    }
    box[0] = std::min(0.0, fp->ax[0] - ex);
    box[1] = std::max(0.0, fp->ax[0] + ex);
    box[2] = std::min(0.0, fp->ay[0] - ey);
    box[3] = std::max(0.0, fp->ay[0] + ey);
    return FH_OK;
}

// Boundary-rule outputs: device arrays are written in place; host arrays go
// through the arena and are copied back (one synchronisation).  The arena is
// reserved once for those and for `extra` bytes the caller takes afterwards.
struct BdryOut {
    double* d[4];
};

fh_status bdry_begin(fh_ctx* c, int64_t n, double* X, double* Y, double* W, double* V, fh_memspace mem,
                     size_t extra, BdryOut* o)
{
    const size_t nb = aligned_bytes(sizeof(double) * std::max<int64_t>(n, 1));
    FH_TRY(arena_reserve(c, (mem == FH_MEM_HOST ? 4 * nb : 0) + extra));
    if (mem == FH_MEM_DEVICE) {
        o->d[0] = X; o->d[1] = Y; o->d[2] = W; o->d[3] = V;
        return FH_OK;
    }
    for (int k = 0; k < 4; ++k) o->d[k] = c->arena.take<double>(std::max<int64_t>(n, 1));
    return FH_OK;
}

fh_status bdry_end(fh_ctx* c, int64_t n, double* X, double* Y, double* W, double* V, fh_memspace mem,
                   const BdryOut& o)
{
    FH_HIP(hipGetLastError());
    if (mem == FH_MEM_HOST) {
        double* h[4] = {X, Y, W, V};
        for (int k = 0; k < 4; ++k)
            FH_HIP(hipMemcpyAsync(h[k], o.d[k], sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
        FH_HIP(hipStreamSynchronize(c->stream));
    }
    return FH_OK;
}

}  // namespace
}  // namespace fh

namespace fh {
namespace {

// The disc + petal rule; Atab (m host values at the radial nodes) replaces
// the HG family when not null.
// The starshade rule: disc, then petals.  mr < 0: the coefficients (if any)
// deform the petals.  mr >= 0: the petals stay ideal and the coefficients
// give the signed ribbons of sec. 5 after them (mr nodes across each, or the
// line integral on the ideal edge for mr = 0).
fh_status starshade_build(fh_ctx* c, int32_t Np, double a, double R, double b, double p, const double* Atab,
                          int32_t m, int32_t np, int32_t nd, int32_t md, const double* coef, int32_t K,
                          fh_memspace coef_mem, fh_quad** out, int32_t mr = -1)
{
    FH_ARG(c && out, FH_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    FH_ARG(Np >= 1 && m >= 1 && np >= 1 && nd >= 0 && md >= 1, FH_ERR_INVALID_ARG,
           "need Np, m, np, md >= 1 and nd >= 0");
    FH_ARG(std::isfinite(a) && std::isfinite(R) && std::isfinite(b) && std::isfinite(p), FH_ERR_NONFINITE,
           "starshade scalar not finite");
    FH_ARG(a >= 0 && R > a && b > 0 && p > 0, FH_ERR_INVALID_ARG, "need 0 <= a < R, b > 0, p > 0");
    FH_ARG(!coef || (K >= 1 && K <= kMaxFourier), FH_ERR_INVALID_ARG, "K must be in [1, %d]", kMaxFourier);
    FH_ARG(coef_mem == FH_MEM_HOST || coef_mem == FH_MEM_DEVICE, FH_ERR_INVALID_ARG, "bad memspace");
    if (Atab)
        for (int l = 0; l < m; ++l)
            FH_ARG(std::isfinite(Atab[l]), FH_ERR_NONFINITE, "apodisation value %d not finite", l);
    FH_HIP(hipSetDevice(c->device));
    const double* glm = nullptr;
    const double* gln = nullptr;
    const double* glmd = nullptr;
    FH_TRY(gl_table(c, m, &glm));
    FH_TRY(gl_table(c, np, &gln));
    FH_TRY(gl_table(c, md, &glmd));
    FH_ARG(mr < 0 || (coef && !Atab), FH_ERR_INVALID_ARG, "a ribbon rule needs coefficients and the HG profile");
    FH_ARG(mr <= 1024, FH_ERR_INVALID_ARG, "at most 1024 nodes across a ribbon");
    const int nt = mr > 0 ? mr : 1;  // nodes across each ribbon
    const int64_t Nd = (int64_t)nd * md;
    const int64_t Npet = Nd + (int64_t)Np * np * m;
    const int64_t N = Npet + (mr >= 0 ? 2 * (int64_t)Np * nt * m : 0);
    // the across rule on (0, 1): Gauss-Legendre mapped from [-1, 1], or the
    // single node on the ideal edge
    std::vector<double> tab;
    if (mr >= 0) {
        tab.assign(2 * (size_t)nt, 0.0);
        if (mr > 0) {
            std::vector<double> gx, gw;
            gl_host(mr, gx, gw);
            for (int i = 0; i < mr; ++i) {
                tab[i] = 0.5 * (1.0 + gx[i]);
                tab[nt + i] = 0.5 * gw[i];
            }
        } else {
            tab[0] = 0.0;
            tab[1] = 1.0;
        }
    }
    fh_quad* qd = nullptr;
    FH_TRY(quad_alloc(c, N, &qd));
    const size_t ncoef = coef ? (size_t)2 * Np * K : 0;
    fh_status s = arena_reserve(c, aligned_bytes(sizeof(double) * std::max<size_t>(ncoef, 1)) +
                                       aligned_bytes(sizeof(double) * (Atab ? (size_t)m : 1)) +
                                       aligned_bytes(sizeof(double) * std::max<size_t>(tab.size(), 1)));
    if (s != FH_OK) {
        fh_quad_destroy(qd);
        return s;
    }
    const double* dcoef = coef;
    if (coef && coef_mem == FH_MEM_HOST) {
        double* dc = c->arena.take<double>(ncoef);
        FH_HIP(hipMemcpyAsync(dc, coef, sizeof(double) * ncoef, hipMemcpyHostToDevice, c->stream));
        dcoef = dc;
    }
    const double* dA = nullptr;
    if (Atab) {
        double* da = c->arena.take<double>((size_t)m);
        FH_HIP(hipMemcpyAsync(da, Atab, sizeof(double) * m, hipMemcpyHostToDevice, c->stream));
        dA = da;
    }
    if (nd > 0) {
        // disc of radius a: trapezoid boundary rule (eq. ptr) + dilation
        RadialParams rp{};
        rp.r0 = a;
        rp.K = 0;
        rp.panels = 0;
        rp.q = nd;
        hipLaunchKernelGGL(k_radial_rule, dim3(nblocks(Nd, 256)), dim3(256), 0, c->stream, rp,
                           (const double*)nullptr, (int64_t)nd, md, glmd, qd->x, qd->y, qd->w);
    }
    const bool deform = coef && mr < 0;
    PetalParams pp{Np, m, np, deform ? K : 0, a, R, b, p, Nd};
    hipLaunchKernelGGL(k_petals, dim3(nblocks((int64_t)Np * np * m, 256)), dim3(256), 0, c->stream, pp, glm, gln,
                       deform ? dcoef : nullptr, dA, qd->x, qd->y, qd->w);
    FH_HIP(hipGetLastError());
    if (mr >= 0) {
        double* dt = c->arena.take<double>(tab.size());
        FH_HIP(hipMemcpyAsync(dt, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice, c->stream));
        RibbonParams rp{Np, m, nt, K, a, R, b, p, Npet};
        hipLaunchKernelGGL(k_ribbons, dim3(nblocks(2 * (int64_t)Np * nt * m, 256)), dim3(256), 0, c->stream, rp,
                           glm, (const double*)dt, dcoef, qd->x, qd->y, qd->w);
        FH_HIP(hipGetLastError());
    }
    // host inputs (and the across table) may be released on return
    if ((coef && coef_mem == FH_MEM_HOST) || Atab || mr >= 0) FH_HIP(hipStreamSynchronize(c->stream));
    // every node radius is at most R (edge perturbations move angles only)
    set_bbox(qd, -R, R, -R, R);
    *out = qd;
    return FH_OK;
}

}  // namespace
}  // namespace fh

using namespace fh;

extern "C" {

fh_status fh_quad_radial(fh_ctx* c, double r0, const double* a, const double* b, int32_t K,
                         int32_t panels, int32_t q, int32_t m, fh_quad** out)
{
    try {
        FH_ARG(c && out, FH_ERR_INVALID_ARG, "NULL argument");
        *out = nullptr;
        FH_ARG(K >= 0 && K <= kMaxFourier, FH_ERR_INVALID_ARG, "K must be in [0, %d]", kMaxFourier);
        FH_ARG(panels >= 0 && q >= 1 && m >= 1, FH_ERR_INVALID_ARG, "need panels >= 0, q >= 1, m >= 1");
        FH_ARG(std::isfinite(r0), FH_ERR_NONFINITE, "r0 not finite");
        RadialParams rp{};
        rp.r0 = r0;
        rp.K = K;
        rp.panels = panels;
        rp.q = q;
        for (int k = 0; k < K; ++k) {
            rp.a[k] = a ? a[k] : 0.0;
            rp.b[k] = b ? b[k] : 0.0;
            FH_ARG(std::isfinite(rp.a[k]) && std::isfinite(rp.b[k]), FH_ERR_NONFINITE,
                   "Fourier coefficient %d not finite", k + 1);
        }
        const int64_t n = panels > 0 ? (int64_t)panels * q : q;
        FH_HIP(hipSetDevice(c->device));
        fh_quad* qd = nullptr;
        FH_TRY(quad_alloc(c, n * m, &qd));
        fh_status s = radial_into(c, rp, n, m, qd->x, qd->y, qd->w);
        if (s != FH_OK) {
            fh_quad_destroy(qd);
            return s;
        }
        qd->rebuild = [c, rp, n, m, qd]() { return radial_into(c, rp, n, m, qd->x, qd->y, qd->w); };
        // the box waits for a call that needs it (a type-1 row window)
        qd->host_box = [rp, n](double* box) { radial_box(rp, n, box); };
        *out = qd;
        return FH_OK;
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_quad_polygon(fh_ctx* c, const double* vx, const double* vy, int32_t nv, int32_t q,
                          int32_t m, fh_quad** out)
{
    try {
        FH_ARG(c && out && vx && vy, FH_ERR_INVALID_ARG, "NULL argument");
        *out = nullptr;
        FH_ARG(nv >= 3 && q >= 1 && m >= 1, FH_ERR_INVALID_ARG, "need nv >= 3, q >= 1, m >= 1");
        for (int i = 0; i < nv; ++i)
            FH_ARG(std::isfinite(vx[i]) && std::isfinite(vy[i]), FH_ERR_NONFINITE, "vertex %d not finite", i);
        FH_HIP(hipSetDevice(c->device));
        const double* glq = nullptr;
        const double* glm = nullptr;
        FH_TRY(gl_table(c, q, &glq));
        FH_TRY(gl_table(c, m, &glm));
        const int64_t n = (int64_t)nv * q;
        fh_quad* qd = nullptr;
        FH_TRY(quad_alloc(c, n * m, &qd));
        // nodes lie on segments from the origin to the boundary
        double bb[4] = {0.0, 0.0, 0.0, 0.0};
        for (int i = 0; i < nv; ++i) {
            bb[0] = std::min(bb[0], vx[i]);
            bb[1] = std::max(bb[1], vx[i]);
            bb[2] = std::min(bb[2], vy[i]);
            bb[3] = std::max(bb[3], vy[i]);
        }
        if (nv <= kPolyByValue) {
            // vertices in the kernel arguments: no copy, no synchronisation
            PolyParams pp{};
            pp.nv = nv;
            pp.q = q;
            for (int i = 0; i < nv; ++i) {
                pp.vx[i] = vx[i];
                pp.vy[i] = vy[i];
            }
            hipLaunchKernelGGL(k_polygon_rule, dim3(nblocks(n * m, 256)), dim3(256), 0, c->stream, pp, glq, m, glm,
                               qd->x, qd->y, qd->w);
            FH_HIP(hipGetLastError());
            qd->rebuild = [c, pp, glq, m, glm, n, qd]() -> fh_status {
                hipLaunchKernelGGL(k_polygon_rule, dim3(nblocks(n * m, 256)), dim3(256), 0, c->stream, pp, glq, m,
                                   glm, qd->x, qd->y, qd->w);
                FH_HIP(hipGetLastError());
                return FH_OK;
            };
            set_bbox(qd, bb[0], bb[1], bb[2], bb[3]);
            *out = qd;
            return FH_OK;
        }
        fh_status s = arena_reserve(c, 4 * aligned_bytes(sizeof(double) * n) +
                                           2 * aligned_bytes(sizeof(double) * nv));
        if (s != FH_OK) {
            fh_quad_destroy(qd);
            return s;
        }
        double* X = c->arena.take<double>(n);
        double* Y = c->arena.take<double>(n);
        double* Wv = c->arena.take<double>(n);
        double* Vv = c->arena.take<double>(n);
        double* dvx = c->arena.take<double>(nv);
        double* dvy = c->arena.take<double>(nv);
        FH_HIP(hipMemcpyAsync(dvx, vx, sizeof(double) * nv, hipMemcpyHostToDevice, c->stream));
        FH_HIP(hipMemcpyAsync(dvy, vy, sizeof(double) * nv, hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL(k_bdry_polygon, dim3(nblocks(n, 256)), dim3(256), 0, c->stream, dvx, dvy,
                           nv, q, glq, X, Y, Wv, Vv);
        hipLaunchKernelGGL(k_dilation, dim3(nblocks(n * m, 256)), dim3(256), 0, c->stream, X, Y, Wv,
                           Vv, n, m, glm, qd->x, qd->y, qd->w);
        FH_HIP(hipGetLastError());
        // the host vertex arrays may be released by the caller on return
        FH_HIP(hipStreamSynchronize(c->stream));
        set_bbox(qd, bb[0], bb[1], bb[2], bb[3]);
        *out = qd;
        return FH_OK;
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_quad_from_boundary(fh_ctx* c, const double* X, const double* Y, const double* W,
                                const double* V, int64_t n, int32_t m, fh_memspace mem,
                                fh_quad** out)
{
    try {
        FH_ARG(c && out, FH_ERR_INVALID_ARG, "NULL argument");
        *out = nullptr;
        FH_ARG(n >= 0 && m >= 1, FH_ERR_INVALID_ARG, "need n >= 0, m >= 1");
        FH_ARG(n == 0 || (X && Y && W && V), FH_ERR_INVALID_ARG, "NULL boundary array");
        FH_ARG(mem == FH_MEM_HOST || mem == FH_MEM_DEVICE, FH_ERR_INVALID_ARG, "bad memspace");
        FH_HIP(hipSetDevice(c->device));
        const double* glm = nullptr;
        FH_TRY(gl_table(c, m, &glm));
        fh_quad* qd = nullptr;
        FH_TRY(quad_alloc(c, n * m, &qd));
        if (n == 0) {
            set_bbox(qd, 0.0, 0.0, 0.0, 0.0);
            *out = qd;
            return FH_OK;
        }
        // nodes lie on segments from the origin to the boundary nodes
        double bb[4] = {0.0, 0.0, 0.0, 0.0};
        if (mem == FH_MEM_HOST) {
            for (int64_t i = 0; i < n; ++i) {
                if (!(std::isfinite(X[i]) && std::isfinite(Y[i]) && std::isfinite(W[i]) && std::isfinite(V[i]))) {
                    fh_quad_destroy(qd);
                    set_error("boundary node %lld not finite", (long long)i);
                    return FH_ERR_NONFINITE;
                }
                bb[0] = std::min(bb[0], X[i]);
                bb[1] = std::max(bb[1], X[i]);
                bb[2] = std::min(bb[2], Y[i]);
                bb[3] = std::max(bb[3], Y[i]);
            }
        } else {
            double d[4];
            fh_status s = device_bbox(c, X, Y, n, d);
            if (s != FH_OK) {
                fh_quad_destroy(qd);
                return s;
            }
            bb[0] = std::min(0.0, d[0]);
            bb[1] = std::max(0.0, d[1]);
            bb[2] = std::min(0.0, d[2]);
            bb[3] = std::max(0.0, d[3]);
        }
        set_bbox(qd, bb[0], bb[1], bb[2], bb[3]);
        const double *dX = X, *dY = Y, *dW = W, *dV = V;
        if (mem == FH_MEM_HOST) {
            fh_status s = arena_reserve(c, 4 * aligned_bytes(sizeof(double) * n));
            if (s != FH_OK) {
                fh_quad_destroy(qd);
                return s;
            }
            double* b[4];
            const double* h[4] = {X, Y, W, V};
            for (int k = 0; k < 4; ++k) {
                b[k] = c->arena.take<double>(n);
                FH_HIP(hipMemcpyAsync(b[k], h[k], sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
            }
            dX = b[0]; dY = b[1]; dW = b[2]; dV = b[3];
        }
        hipLaunchKernelGGL(k_dilation, dim3(nblocks(n * m, 256)), dim3(256), 0, c->stream, dX, dY, dW,
                           dV, n, m, glm, qd->x, qd->y, qd->w);
        FH_HIP(hipGetLastError());
        if (mem == FH_MEM_HOST) FH_HIP(hipStreamSynchronize(c->stream));
        *out = qd;
        return FH_OK;
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}


fh_status fh_quad_starshade(fh_ctx* c, int32_t Np, double a, double R, double b, double p, int32_t m,
                            int32_t np, int32_t nd, int32_t md, const double* coef, int32_t K,
                            fh_memspace coef_mem, fh_quad** out)
{
    try {
        return starshade_build(c, Np, a, R, b, p, nullptr, m, np, nd, md, coef, K, coef_mem, out);
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_quad_starshade_ribbon(fh_ctx* c, int32_t Np, double a, double R, double b, double p, int32_t m,
                                   int32_t np, int32_t nd, int32_t md, const double* coef, int32_t K,
                                   fh_memspace coef_mem, int32_t mr, fh_quad** out)
{
    try {
        FH_ARG(coef, FH_ERR_INVALID_ARG, "a ribbon rule needs its edge coefficients");
        FH_ARG(mr >= 0, FH_ERR_INVALID_ARG, "mr must be >= 0");
        return starshade_build(c, Np, a, R, b, p, nullptr, m, np, nd, md, coef, K, coef_mem, out, mr);
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_quad_starshade_tab(fh_ctx* c, int32_t Np, double a, double R, const double* A, int32_t m,
                                int32_t np, int32_t nd, int32_t md, const double* coef, int32_t K,
                                fh_memspace coef_mem, fh_quad** out)
{
    try {
        FH_ARG(A, FH_ERR_INVALID_ARG, "NULL apodisation table");
        return starshade_build(c, Np, a, R, 1.0, 1.0, A, m, np, nd, md, coef, K, coef_mem, out);
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_quad_starshade_rigid(fh_ctx* c, int32_t Np, double a, double R, double b, double p, int32_t m,
                                  int32_t np, int32_t nd, int32_t md, const double* motion, int32_t nb, int32_t mb,
                                  fh_quad** out)
{
    try {
        FH_ARG(c && out && motion, FH_ERR_INVALID_ARG, "NULL argument");
        *out = nullptr;
        FH_ARG(Np >= 1 && Np <= kRigidMaxPetals, FH_ERR_INVALID_ARG, "Np must be in [1, %d]", kRigidMaxPetals);
        FH_ARG(m >= 1 && np >= 1 && nd >= 0 && md >= 1 && nb >= 1 && mb >= 1, FH_ERR_INVALID_ARG,
               "need Np, m, np, md, nb, mb >= 1 and nd >= 0");
        FH_ARG(std::isfinite(a) && std::isfinite(R) && std::isfinite(b) && std::isfinite(p), FH_ERR_NONFINITE,
               "starshade scalar not finite");
        FH_ARG(a > 0 && R > a && b > 0 && p > 0, FH_ERR_INVALID_ARG, "need 0 < a < R, b > 0, p > 0");
        RigidParams rp{};
        double shift = 0.0;
        for (int k = 0; k < 3 * Np; ++k) {
            FH_ARG(std::isfinite(motion[k]), FH_ERR_NONFINITE, "motion entry %d not finite", k);
            rp.motion[k] = motion[k];
        }
        for (int k = 0; k < Np; ++k) shift = std::max(shift, std::hypot(motion[3 * k + 1], motion[3 * k + 2]));
        FH_HIP(hipSetDevice(c->device));
        const double *glm = nullptr, *gln = nullptr, *glmd = nullptr, *glb = nullptr, *glt = nullptr;
        FH_TRY(gl_table(c, m, &glm));
        FH_TRY(gl_table(c, np, &gln));
        FH_TRY(gl_table(c, md, &glmd));
        FH_TRY(gl_table(c, nb, &glb));
        FH_TRY(gl_table(c, mb, &glt));
        const int64_t Nd = (int64_t)nd * md, Npet = (int64_t)Np * np * m, Nb = (int64_t)Np * nb * mb;
        fh_quad* qd = nullptr;
        FH_TRY(quad_alloc(c, Nd + Npet + Nb, &qd));
        if (nd > 0) {
            RadialParams dp{};
            dp.r0 = a;
            dp.q = nd;
            hipLaunchKernelGGL(k_radial_rule, dim3(nblocks(Nd, 256)), dim3(256), 0, c->stream, dp,
                               (const double*)nullptr, (int64_t)nd, md, glmd, qd->x, qd->y, qd->w);
        }
        PetalParams pp{Np, m, np, 0, a, R, b, p, Nd};
        hipLaunchKernelGGL(k_petals, dim3(nblocks(Npet, 256)), dim3(256), 0, c->stream, pp, glm, gln,
                           (const double*)nullptr, (const double*)nullptr, qd->x, qd->y, qd->w);
        rp.Np = Np;
        rp.np = np;
        rp.m = m;
        rp.nb = nb;
        rp.mb = mb;
        rp.a = a;
        rp.petal_off = Nd;
        rp.bridge_off = Nd + Npet;
        hipLaunchKernelGGL(k_rigid_move, dim3(nblocks(Npet, 256)), dim3(256), 0, c->stream, rp, qd->x, qd->y);
        hipLaunchKernelGGL(k_rigid_bridges, dim3(nblocks(Nb, 256)), dim3(256), 0, c->stream, rp, glb, glt, qd->x,
                           qd->y, qd->w);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            fh_quad_destroy(qd);
            set_error("rigid-petal rule launch failed: %s", hipGetErrorString(e));
            return FH_ERR_HIP;
        }
        // rotations about the centre keep radii; translations add at most `shift`
        set_bbox(qd, -R - shift, R + shift, -R - shift, R + shift);
        *out = qd;
        return FH_OK;
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_quad_from_nodes(fh_ctx* c, const double* x, const double* y, const double* w, int64_t N,
                             fh_memspace mem, fh_quad** out)
{
    try {
        FH_ARG(c && out, FH_ERR_INVALID_ARG, "NULL argument");
        *out = nullptr;
        FH_ARG(N >= 0, FH_ERR_INVALID_ARG, "N must be >= 0");
        FH_ARG(N == 0 || (x && y && w), FH_ERR_INVALID_ARG, "NULL node array");
        FH_ARG(mem == FH_MEM_HOST || mem == FH_MEM_DEVICE, FH_ERR_INVALID_ARG, "bad memspace");
        FH_HIP(hipSetDevice(c->device));
        fh_quad* qd = nullptr;
        FH_TRY(quad_alloc(c, N, &qd));
        if (N > 0) {
            hipMemcpyKind kind = mem == FH_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
            FH_HIP(hipMemcpyAsync(qd->x, x, sizeof(double) * N, kind, c->stream));
            FH_HIP(hipMemcpyAsync(qd->y, y, sizeof(double) * N, kind, c->stream));
            FH_HIP(hipMemcpyAsync(qd->w, w, sizeof(double) * N, kind, c->stream));
            if (mem == FH_MEM_HOST) FH_HIP(hipStreamSynchronize(c->stream));
            double bb[4];
            fh_status s = device_bbox(c, qd->x, qd->y, N, bb);
            if (s != FH_OK) {
                fh_quad_destroy(qd);
                return s;
            }
            set_bbox(qd, bb[0], bb[1], bb[2], bb[3]);
        } else {
            set_bbox(qd, 0.0, 0.0, 0.0, 0.0);
        }
        *out = qd;
        return FH_OK;
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_quad_koch(fh_ctx* c, int32_t L, const int32_t* p, fh_quad** out)
{
    try {
        FH_ARG(c && out && p, FH_ERR_INVALID_ARG, "NULL argument");
        *out = nullptr;
        FH_ARG(L >= 0 && L <= kKochMaxLevel, FH_ERR_INVALID_ARG, "L must be in [0, %d]", kKochMaxLevel);
        KochParams kp{};
        kp.L = L;
        int64_t N = 0, ntri = 1;
        FH_HIP(hipSetDevice(c->device));
        for (int k = 0; k <= L; ++k) {
            FH_ARG(p[k] >= 1 && p[k] <= 1024, FH_ERR_INVALID_ARG, "p[%d] must be in [1, 1024]", k);
            kp.p[k] = p[k];
            kp.off[k] = N;
            N += ntri * (int64_t)p[k] * p[k];
            ntri = k == 0 ? 3 : ntri * 4;
            FH_TRY(gl_table(c, p[k], &kp.gl[k]));
        }
        kp.off[L + 1] = N;
        fh_quad* qd = nullptr;
        FH_TRY(quad_alloc(c, N, &qd));
        hipLaunchKernelGGL(k_koch_rule, dim3(nblocks(N, 256)), dim3(256), 0, c->stream, kp, qd->x, qd->y, qd->w);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            fh_quad_destroy(qd);
            set_error("k_koch_rule launch failed: %s", hipGetErrorString(e));
            return FH_ERR_HIP;
        }
        // the snowflake lies in the unit disc
        set_bbox(qd, -1.0, 1.0, -1.0, 1.0);
        *out = qd;
        return FH_OK;
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_quad_fourier(fh_ctx* c, int32_t K, const double* ax, const double* bx, const double* ay,
                          const double* by, int32_t panels, int32_t q, int32_t m, fh_quad** out)
{
    try {
        FH_ARG(c && out, FH_ERR_INVALID_ARG, "NULL argument");
        *out = nullptr;
        FH_ARG(m >= 1, FH_ERR_INVALID_ARG, "need m >= 1");
        FourierParams fp;
        double box[4];
        FH_TRY(fourier_params(ax, bx, ay, by, K, panels, q, &fp, box));
        const int64_t n = panels > 0 ? (int64_t)panels * q : q;
        fourier_box(fp, n, box);
        FH_HIP(hipSetDevice(c->device));
        const double* glq = nullptr;
        const double* glm = nullptr;
        if (panels > 0) FH_TRY(gl_table(c, q, &glq));
        FH_TRY(gl_table(c, m, &glm));
        fh_quad* qd = nullptr;
        FH_TRY(quad_alloc(c, n * m, &qd));
        hipLaunchKernelGGL(k_fourier_rule, dim3(nblocks(n * m, 256)), dim3(256), 0, c->stream, fp, glq, n, m, glm,
                           qd->x, qd->y, qd->w);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            fh_quad_destroy(qd);
            set_error("k_fourier_rule launch failed: %s", hipGetErrorString(e));
            return FH_ERR_HIP;
        }
        set_bbox(qd, box[0], box[1], box[2], box[3]);
        *out = qd;
        return FH_OK;
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_boundary_fourier(fh_ctx* c, int32_t K, const double* ax, const double* bx, const double* ay,
                              const double* by, int32_t panels, int32_t q, double* X, double* Y, double* W, double* V,
                              fh_memspace mem)
{
    try {
        FH_ARG(c && X && Y && W && V, FH_ERR_INVALID_ARG, "NULL argument");
        FH_ARG(mem == FH_MEM_HOST || mem == FH_MEM_DEVICE, FH_ERR_INVALID_ARG, "bad memspace");
        FourierParams fp;
        double box[4];
        FH_TRY(fourier_params(ax, bx, ay, by, K, panels, q, &fp, box));
        const int64_t n = panels > 0 ? (int64_t)panels * q : q;
        FH_HIP(hipSetDevice(c->device));
        const double* glq = nullptr;
        if (panels > 0) FH_TRY(gl_table(c, q, &glq));
        BdryOut o;
        FH_TRY(bdry_begin(c, n, X, Y, W, V, mem, 0, &o));
        hipLaunchKernelGGL(k_bdry_fourier, dim3(nblocks(n, 256)), dim3(256), 0, c->stream, fp, glq, n, o.d[0], o.d[1],
                           o.d[2], o.d[3]);
        return bdry_end(c, n, X, Y, W, V, mem, o);
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_boundary_radial(fh_ctx* c, double r0, const double* a, const double* b, int32_t K,
                             int32_t panels, int32_t q, double* X, double* Y, double* W, double* V,
                             fh_memspace mem)
{
    try {
        FH_ARG(c && X && Y && W && V, FH_ERR_INVALID_ARG, "NULL argument");
        FH_ARG(K >= 0 && K <= kMaxFourier, FH_ERR_INVALID_ARG, "K must be in [0, %d]", kMaxFourier);
        FH_ARG(panels >= 0 && q >= 1, FH_ERR_INVALID_ARG, "need panels >= 0, q >= 1");
        FH_ARG(mem == FH_MEM_HOST || mem == FH_MEM_DEVICE, FH_ERR_INVALID_ARG, "bad memspace");
        FH_ARG(std::isfinite(r0), FH_ERR_NONFINITE, "r0 not finite");
        RadialParams rp{};
        rp.r0 = r0;
        rp.K = K;
        rp.panels = panels;
        rp.q = q;
        for (int k = 0; k < K; ++k) {
            rp.a[k] = a ? a[k] : 0.0;
            rp.b[k] = b ? b[k] : 0.0;
            FH_ARG(std::isfinite(rp.a[k]) && std::isfinite(rp.b[k]), FH_ERR_NONFINITE,
                   "Fourier coefficient %d not finite", k + 1);
        }
        const int64_t n = panels > 0 ? (int64_t)panels * q : q;
        FH_HIP(hipSetDevice(c->device));
        const double* glq = nullptr;
        if (panels > 0) FH_TRY(gl_table(c, q, &glq));
        BdryOut o;
        FH_TRY(bdry_begin(c, n, X, Y, W, V, mem, 0, &o));
        hipLaunchKernelGGL(k_bdry_radial, dim3(nblocks(n, 256)), dim3(256), 0, c->stream, rp, glq, n, o.d[0], o.d[1],
                           o.d[2], o.d[3]);
        return bdry_end(c, n, X, Y, W, V, mem, o);
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_boundary_polygon(fh_ctx* c, const double* vx, const double* vy, int32_t nv, int32_t q, double* X,
                              double* Y, double* W, double* V, fh_memspace mem)
{
    try {
        FH_ARG(c && vx && vy && X && Y && W && V, FH_ERR_INVALID_ARG, "NULL argument");
        FH_ARG(nv >= 3 && q >= 1, FH_ERR_INVALID_ARG, "need nv >= 3, q >= 1");
        FH_ARG(mem == FH_MEM_HOST || mem == FH_MEM_DEVICE, FH_ERR_INVALID_ARG, "bad memspace");
        for (int i = 0; i < nv; ++i)
            FH_ARG(std::isfinite(vx[i]) && std::isfinite(vy[i]), FH_ERR_NONFINITE, "vertex %d not finite", i);
        FH_HIP(hipSetDevice(c->device));
        const double* glq = nullptr;
        FH_TRY(gl_table(c, q, &glq));
        const int64_t n = (int64_t)nv * q;
        BdryOut o;
        FH_TRY(bdry_begin(c, n, X, Y, W, V, mem, 2 * aligned_bytes(sizeof(double) * nv), &o));
        double* dvx = c->arena.take<double>(nv);
        double* dvy = c->arena.take<double>(nv);
        FH_HIP(hipMemcpyAsync(dvx, vx, sizeof(double) * nv, hipMemcpyHostToDevice, c->stream));
        FH_HIP(hipMemcpyAsync(dvy, vy, sizeof(double) * nv, hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL(k_bdry_polygon, dim3(nblocks(n, 256)), dim3(256), 0, c->stream, dvx, dvy, nv, q, glq,
                           o.d[0], o.d[1], o.d[2], o.d[3]);
        fh_status s = bdry_end(c, n, X, Y, W, V, mem, o);
        // the host vertex arrays may be released by the caller on return
        if (s == FH_OK && mem == FH_MEM_DEVICE) FH_HIP(hipStreamSynchronize(c->stream));
        return s;
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_boundary_starshade(fh_ctx* c, int32_t Np, double a, double R, double b, double p, int32_t m,
                                int32_t ntip, int32_t ngap, double* X, double* Y, double* W, double* V,
                                fh_memspace mem)
{
    try {
        FH_ARG(c && X && Y && W && V, FH_ERR_INVALID_ARG, "NULL argument");
        FH_ARG(Np >= 1 && m >= 1 && ntip >= 0 && ngap >= 0, FH_ERR_INVALID_ARG,
               "need Np, m >= 1 and ntip, ngap >= 0");
        FH_ARG(std::isfinite(a) && std::isfinite(R) && std::isfinite(b) && std::isfinite(p),
               FH_ERR_NONFINITE, "starshade scalar not finite");
        FH_ARG(a >= 0 && R > a && b > 0 && p > 0, FH_ERR_INVALID_ARG, "need 0 <= a < R, b > 0, p > 0");
        FH_ARG(mem == FH_MEM_HOST || mem == FH_MEM_DEVICE, FH_ERR_INVALID_ARG, "bad memspace");
        FH_HIP(hipSetDevice(c->device));
        const double* glm = nullptr;
        const double* glt = nullptr;
        const double* glg = nullptr;
        FH_TRY(gl_table(c, m, &glm));
        if (ntip > 0) FH_TRY(gl_table(c, ntip, &glt));
        if (ngap > 0) FH_TRY(gl_table(c, ngap, &glg));
        const int64_t n = (int64_t)Np * (2 * (int64_t)m + ntip + ngap);
        BdryOut o;
        FH_TRY(bdry_begin(c, n, X, Y, W, V, mem, 0, &o));
        OutlineParams op{Np, m, ntip, ngap, a, R, b, p};
        hipLaunchKernelGGL(k_bdry_starshade, dim3(nblocks(n, 256)), dim3(256), 0, c->stream, op, glm, glt, glg,
                           o.d[0], o.d[1], o.d[2], o.d[3]);
        return bdry_end(c, n, X, Y, W, V, mem, o);
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_quad_size(const fh_quad* q, int64_t* N)
{
    FH_ARG(q && N, FH_ERR_INVALID_ARG, "NULL argument");
    *N = q->N;
    return FH_OK;
}

fh_status fh_quad_export(const fh_quad* q, double* x, double* y, double* w, fh_memspace mem)
{
    FH_ARG(q, FH_ERR_INVALID_ARG, "NULL quadrature");
    FH_ARG(mem == FH_MEM_HOST || mem == FH_MEM_DEVICE, FH_ERR_INVALID_ARG, "bad memspace");
    fh_ctx* c = q->ctx;
    FH_HIP(hipSetDevice(c->device));
    hipMemcpyKind kind = mem == FH_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    const size_t bytes = sizeof(double) * q->N;
    if (q->N > 0) {
        if (x) FH_HIP(hipMemcpyAsync(x, q->x, bytes, kind, c->stream));
        if (y) FH_HIP(hipMemcpyAsync(y, q->y, bytes, kind, c->stream));
        if (w) FH_HIP(hipMemcpyAsync(w, q->w, bytes, kind, c->stream));
    }
    if (mem == FH_MEM_HOST) FH_HIP(hipStreamSynchronize(c->stream));
    return FH_OK;
}

fh_status fh_quad_device_ptrs(const fh_quad* q, const double** x, const double** y, const double** w)
{
    FH_ARG(q, FH_ERR_INVALID_ARG, "NULL quadrature");
    if (x) *x = q->x;
    if (y) *y = q->y;
    if (w) *w = q->w;
    return FH_OK;
}

fh_status fh_quad_set_illumination(fh_ctx* c, fh_quad* q, const double* src, double D, fh_memspace mem)
{
    try {
        FH_ARG(c && q, FH_ERR_INVALID_ARG, "NULL argument");
        FH_ARG(q->ctx->device == c->device, FH_ERR_INVALID_ARG, "quadrature lives on another device");
        FH_ARG(mem == FH_MEM_HOST || mem == FH_MEM_DEVICE, FH_ERR_INVALID_ARG, "bad memspace");
        FH_ARG(std::isfinite(D), FH_ERR_NONFINITE, "D not finite");
        FH_ARG(D >= 0.0, FH_ERR_INVALID_ARG, "D must be >= 0 (0: plane wave)");
        FH_HIP(hipSetDevice(c->device));
        const size_t bytes = 2 * sizeof(double) * (size_t)q->N;
        if (src && mem == FH_MEM_HOST) {
            for (int64_t j = 0; j < 2 * q->N; ++j)
                FH_ARG(std::isfinite(src[j]), FH_ERR_NONFINITE, "source term %lld not finite", (long long)(j / 2));
        }
        // Every call that may read the old terms, on any stream, has finished
        // before they are replaced or released; the copy below is synchronous.
        FH_HIP(hipDeviceSynchronize());
        if (q->src && (!src || q->N == 0)) {
            FH_TRY(dev_free(q->ctx, q->src));
            q->src = nullptr;
        }
        if (src && q->N > 0) {
            if (!q->src) {
                void* p = nullptr;
                FH_TRY(dev_alloc(q->ctx, bytes, &p));
                q->src = static_cast<double*>(p);
            }
            FH_HIP(hipMemcpy(q->src, src, bytes, mem == FH_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice));
        }
        q->D = D;
        return FH_OK;
    } catch (...) {
        set_error("host allocation failed");
        return FH_ERR_ALLOC;
    }
}

fh_status fh_quad_destroy(fh_quad* q)
{
    if (!q) return FH_OK;
    if (q->src) {
        // the source terms are released at once (not pooled): every call
        // that may still read them finishes first
        (void)hipSetDevice(q->ctx->device);
        (void)hipDeviceSynchronize();
        (void)dev_free(q->ctx, q->src);
        q->src = nullptr;
    }
    try {
        // keep the buffer for the next rule of the same size: work already
        // enqueued on the context stream that reads it stays ordered before
        // any later writer on the same stream.
        q->ctx->pool[q->buf_bytes].push_back(q->buf);
    } catch (...) {
        (void)dev_free(q->ctx, q->buf);
    }
    delete q;
    return FH_OK;
}

}  // extern "C"

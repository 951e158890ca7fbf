/*
 * FP64 CPU oracle for dense RGB-D alignment in inverse-depth parametrisation
 * and inverse-depth keyframe fusion (Gutierrez-Gomez & Guerrero, RGBiD-SLAM).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the HIP path is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or constant with the HIP library.
 *
 * Everything is double precision and plain loops, in the paper's order:
 *   pyramid + gradients        (sec. 6.2, "Iterative optimisation")
 *   inverse geometric warp     (sec. 5.3, eq. for W_{B*})
 *   residuals and Jacobians    (sec. 6.2, eq:res_int, eq:res_depth, eq:DeltaX)
 *   lambda_n                   (sec. 6.2, normal-vector weight)
 *   location / scale / nu      (sec. 6.3, eq:logLikelihood_St, eq:robustnessValue)
 *   normal equations, update   (sec. 6.2, H xi = b and the inverse-exp update)
 *   decoupled SE(3) exp / log  (sec. 3)
 *   keyframe fusion            (sec. 7.2, with the covisibility test of sec. 6.4)
 *
 * Readings where the paper is silent or garbled are stated at each function.
 * Image layout: row-major, width w, height h, index v*w + u.  Inverse depth
 * W <= 0 or non-finite marks a hole.  Pose T = (R row-major, t) is the pose of
 * B in A: X_A = R X_B + t.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int w, h;
    double fx, fy, cx, cy;
} or_cam;

enum { OR_WEIGHT_STUDENT_T = 0, OR_WEIGHT_HUBER = 1 };
enum { OR_WARP_FULLRES = 0, OR_WARP_PER_LEVEL = 1 };
enum { OR_STORE_F64 = 0, OR_STORE_F32 = 1, OR_STORE_F16 = 2 };
enum { OR_OK = 0, OR_DEGENERATE = -5, OR_ARG = -1 };

typedef struct {
    int levels;
    int iters[8];
    int weight;          /* OR_WEIGHT_* */
    double huber_k;      /* 1.345 */
    int estimate_nu;     /* Student-t only */
    int sample_max;      /* 19200 (sec. 6.3) */
    int scale_iters;     /* fixed-point iterations for mu, sigma */
    int warp;            /* OR_WARP_* */
    double stop_eps_t, stop_eps_r;
    int storage;         /* rounding applied to every stored pyramid level */
    int scale_warm;      /* 1: warm-started fixed point with the convergence stop */
} or_params;

/* Where the mu, sigma fixed point of the next linearisation at a level
   starts: the last estimate of each channel and its sample size (0: none
   yet, start cold). */
typedef struct {
    double mu[2], sigma[2];
    int n[2];
} or_scale_state;

/* Convergence stop of the warm-started fixed point: a step that moves mu and
   sigma by at most this fraction of sigma is the last. */
#define OR_SCALE_TOL 1.52587890625e-5   /* 2^-16 */

typedef struct {
    double H[36], g[6];
    double mu_I, sigma_I, nu_I, mu_W, sigma_W, nu_W, cost;
    long long n_valid_I, n_valid_W;
    int iters_done[8];
    int status;
} or_stats;

static int valid_w(double w) { return w > 0.0 && isfinite(w); }

/* ---------------------------------------------------------------- rounding */

/* Round to the nearest binary16 value (ties to even), returned as double.
   Quantum is 2^(e-10) for |x| in [2^e, 2^(e+1)), e >= -14, 2^-24 below. */
double or_round_f16(double x)
{
    if (!isfinite(x) || x == 0.0) return x;
    double ax = fabs(x);
    int e;
    frexp(ax, &e);          /* ax in [2^(e-1), 2^e) */
    e -= 1;
    if (e < -14) e = -14;
    double q = ldexp(1.0, e - 10);
    double r = nearbyint(ax / q) * q;
    if (r > 65504.0) r = INFINITY;
    return x < 0 ? -r : r;
}

static double store_round(double x, int storage)
{
    if (storage == OR_STORE_F32) return (double)(float)x;
    if (storage == OR_STORE_F16) return or_round_f16(x);
    return x;
}

/* ---------------------------------------------------------------- camera */

/* Level-l intrinsics for 2x2 block averaging with pixel centres at integers:
   f_l = f / 2^l, c_l = (c + 0.5) / 2^l - 0.5.  (The paper does not state the
   convention; this one makes the block mean of a field linear in pixel
   coordinates equal to that field at the block centre.) */
void or_camera_level(const or_cam* c0, int l, or_cam* cl)
{
    double s = ldexp(1.0, -l);
    int w = c0->w, h = c0->h;
    for (int i = 0; i < l; ++i) { w /= 2; h /= 2; }
    cl->w = w;
    cl->h = h;
    cl->fx = c0->fx * s;
    cl->fy = c0->fy * s;
    cl->cx = (c0->cx + 0.5) * s - 0.5;
    cl->cy = (c0->cy + 0.5) * s - 0.5;
}

/* ---------------------------------------------------------------- pyramid */

/* One pyramid step (sec. 6.2: {I_A, W_A} are downsampled at every level).
   I: mean of the 2x2 children in the order (0,0),(1,0),(0,1),(1,1).
   W: mean of the valid children in the same order; hole if none is valid.
   Output size floor(w/2) x floor(h/2). */
void or_downsample(const double* I, const double* W, int w, int h,
                   double* I2, double* W2, int storage)
{
    int w2 = w / 2, h2 = h / 2;
    for (int v = 0; v < h2; ++v)
        for (int u = 0; u < w2; ++u) {
            const int idx[4] = {(2 * v) * w + 2 * u, (2 * v) * w + 2 * u + 1,
                                (2 * v + 1) * w + 2 * u, (2 * v + 1) * w + 2 * u + 1};
            double si = 0.0, sw = 0.0;
            int nw = 0;
            for (int k = 0; k < 4; ++k) {
                si += I[idx[k]];
                if (valid_w(W[idx[k]])) { sw += W[idx[k]]; ++nw; }
            }
            I2[v * w2 + u] = store_round(si / 4.0, storage);
            W2[v * w2 + u] = nw ? store_round(sw / nw, storage) : 0.0;
        }
}

/* ---------------------------------------------------------------- SO(3), SE(3) */

static void skew(const double a[3], double S[9])
{
    S[0] = 0;     S[1] = -a[2]; S[2] = a[1];
    S[3] = a[2];  S[4] = 0;     S[5] = -a[0];
    S[6] = -a[1]; S[7] = a[0];  S[8] = 0;
}

static void matmul3(const double A[9], const double B[9], double C[9])
{
    double T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
            T[3 * i + j] = s;
        }
    memcpy(C, T, sizeof T);
}

/* Rodrigues' formula (sec. 3): R = I + sin|th|/|th| [th]x
   + (1 - cos|th|)/|th|^2 [th]x^2.  The paper prints |th| in the last
   denominator; |th|^2 is the rotation.  Second-order Taylor for |th| < 1e-8. */
void or_exp_so3(const double th[3], double R[9])
{
    double n = sqrt(th[0] * th[0] + th[1] * th[1] + th[2] * th[2]);
    double S[9], S2[9];
    skew(th, S);
    matmul3(S, S, S2);
    double a, b;
    if (n < 1e-8) { a = 1.0; b = 0.5; }
    else { a = sin(n) / n; b = (1.0 - cos(n)) / (n * n); }
    for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0 ? 1.0 : 0.0) + a * S[i] + b * S2[i];
}

/* Logarithm of SO(3) (sec. 3): |th| = acos((tr R - 1)/2),
   [th]x = |th| (R - R^T) / (2 sin|th|). */
void or_log_so3(const double R[9], double th[3])
{
    double c = (R[0] + R[4] + R[8] - 1.0) / 2.0;
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    double n = acos(c);
    double f = (n < 1e-8) ? 0.5 : n / (2.0 * sin(n));
    th[0] = f * (R[7] - R[5]);
    th[1] = f * (R[2] - R[6]);
    th[2] = f * (R[3] - R[1]);
}

/* Pose update of sec. 6.2: T <- exp(xi)^-1 T with the decoupled exponential of
   sec. 3, exp(xi) = [Rod(theta), v; 0, 1], xi = (v, theta).
   exp(xi)^-1 T = (Rod^T R, Rod^T (t - v)). */
void or_update(double R[9], double t[3], const double xi[6])
{
    double E[9], Et[9], Rn[9];
    or_exp_so3(xi + 3, E);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Et[3 * i + j] = E[3 * j + i];
    matmul3(Et, R, Rn);
    double d[3] = {t[0] - xi[0], t[1] - xi[1], t[2] - xi[2]};
    for (int i = 0; i < 3; ++i) t[i] = Et[3 * i] * d[0] + Et[3 * i + 1] * d[1] + Et[3 * i + 2] * d[2];
    memcpy(R, Rn, sizeof Rn);
}

/* ---------------------------------------------------------------- warp */

/* Bilinear sample with the bounds rule -0.5 <= x < w-0.5 (same in y) and taps
   clamped to the image; returns 0 when out of bounds or (need_valid) when any
   of the four taps is a hole. */
static int bilinear(const double* img, int w, int h, double x, double y,
                    int need_valid, double* out)
{
    if (!(x >= -0.5 && x < w - 0.5 && y >= -0.5 && y < h - 0.5)) return 0;
    double fx0 = floor(x), fy0 = floor(y);
    double a = x - fx0, b = y - fy0;
    int x0 = (int)fx0, y0 = (int)fy0, x1 = x0 + 1, y1 = y0 + 1;
    if (x0 < 0) x0 = 0;
    if (y0 < 0) y0 = 0;
    if (x1 > w - 1) x1 = w - 1;
    if (y1 > h - 1) y1 = h - 1;
    double v00 = img[y0 * w + x0], v10 = img[y0 * w + x1];
    double v01 = img[y1 * w + x0], v11 = img[y1 * w + x1];
    if (need_valid && !(valid_w(v00) && valid_w(v10) && valid_w(v01) && valid_w(v11)))
        return 0;
    *out = (1 - a) * (1 - b) * v00 + a * (1 - b) * v10 + (1 - a) * b * v01 + a * b * v11;
    return 1;
}

/* Inverse geometric warp of {I_B, W_B} towards A at pose (R, t) for every
   pixel of a w x h grid with camera c (sec. 5.3):
     X = K^-1 p / W_A(p),  Y = R^T (X - t),  p_B = K Y / Y_z,
     I_B*(p) = I_B(p_B),
     W_B*(p) = (R^T K^-1 p)_z W_B(p_B) / (1 + W_B(p_B) (R^T t)_z)
   (the printed formula with R~_BA = K R^T K^-1 and t~_B^A = -K R^T t).
   A pixel is warp-valid iff W_A(p) is valid, Y_z > 0, p_B is in bounds, the
   four W_B taps are valid and W_B* is positive and finite. */
void or_warp(const or_cam* c, const double* WA, const double* IB, const double* WB,
             const double R[9], const double t[3],
             double* Iw, double* Ww, uint8_t* valid)
{
    const int w = c->w, h = c->h;
    /* (R^T t) */
    double Rtt[3];
    for (int i = 0; i < 3; ++i) Rtt[i] = R[i] * t[0] + R[3 + i] * t[1] + R[6 + i] * t[2];
    for (int v = 0; v < h; ++v)
        for (int u = 0; u < w; ++u) {
            int i = v * w + u;
            valid[i] = 0;
            Iw[i] = 0.0;
            Ww[i] = 0.0;
            double wa = WA[i];
            if (!valid_w(wa)) continue;
            double ray[3] = {(u - c->cx) / c->fx, (v - c->cy) / c->fy, 1.0};
            double X[3] = {ray[0] / wa - t[0], ray[1] / wa - t[1], ray[2] / wa - t[2]};
            double Y[3], Rray[3];
            for (int k = 0; k < 3; ++k) {
                Y[k] = R[k] * X[0] + R[3 + k] * X[1] + R[6 + k] * X[2];
                Rray[k] = R[k] * ray[0] + R[3 + k] * ray[1] + R[6 + k] * ray[2];
            }
            if (!(Y[2] > 0.0)) continue;
            double ub = c->fx * Y[0] / Y[2] + c->cx;
            double vb = c->fy * Y[1] / Y[2] + c->cy;
            double ib, wb;
            if (!bilinear(WB, w, h, ub, vb, 1, &wb)) continue;
            bilinear(IB, w, h, ub, vb, 0, &ib);
            double ws = Rray[2] * wb / (1.0 + wb * Rtt[2]);
            if (!valid_w(ws)) continue;
            Iw[i] = ib;
            Ww[i] = ws;
            valid[i] = 1;
        }
}

/* Paper-literal warp of sec. 6.2: warp at full resolution, then downsample the
   warped images to level l by recursive 2x2 means (order (0,0),(1,0),(0,1),
   (1,1)).  A coarse pixel has warped values only if all its children have. */
void or_warp_fullres(const or_cam* c0, int level, const double* WA0,
                     const double* IB0, const double* WB0, const double R[9],
                     const double t[3], double* Iw, double* Ww, uint8_t* valid)
{
    int w = c0->w, h = c0->h;
    size_t n0 = (size_t)w * h;
    double* I = malloc(n0 * sizeof(double));
    double* W = malloc(n0 * sizeof(double));
    uint8_t* V = malloc(n0);
    or_warp(c0, WA0, IB0, WB0, R, t, I, W, V);
    for (int l = 0; l < level; ++l) {
        int w2 = w / 2, h2 = h / 2;
        for (int v = 0; v < h2; ++v)
            for (int u = 0; u < w2; ++u) {
                const int idx[4] = {(2 * v) * w + 2 * u, (2 * v) * w + 2 * u + 1,
                                    (2 * v + 1) * w + 2 * u, (2 * v + 1) * w + 2 * u + 1};
                int ok = V[idx[0]] && V[idx[1]] && V[idx[2]] && V[idx[3]];
                double si = 0, sw = 0;
                for (int k = 0; k < 4; ++k) { si += I[idx[k]]; sw += W[idx[k]]; }
                int o = v * w2 + u;     /* o <= every idx: in-place is safe */
                I[o] = ok ? si / 4.0 : 0.0;
                W[o] = ok ? sw / 4.0 : 0.0;
                V[o] = (uint8_t)ok;
            }
        w = w2;
        h = h2;
    }
    memcpy(Iw, I, (size_t)w * h * sizeof(double));
    memcpy(Ww, W, (size_t)w * h * sizeof(double));
    memcpy(valid, V, (size_t)w * h);
    free(I);
    free(W);
    free(V);
}

/* ---------------------------------------------------------------- residuals */

/* Residuals, Jacobians and lambda_n at one level (sec. 6.2).
   With Z = 1/W_A, x = K^-1 p, X = Z x and the central-difference gradients
   (interior pixels only; grad W needs W at p and its 4 neighbours valid):
     r_I = I_B* - I_A,      a_I = W_A grad(I_A) (K - p e_z^T),
     r_W = W_B* - W_A,      a_W = W_A (grad(W_A) (K - p e_z^T) + W_B* e_z^T),
     J = a M(p) with M = [I | -[X]x], i.e. J = (a, X x a)      (eq:DeltaX)
     n~ = Z grad(W_A)(K - p e_z^T) + e_z^T,  lambda_n = n~.x/(|n~||x|)
   The paper's "p/|p|" in lambda_n is read as the viewing ray x/|x|; since
   n~.x = 1 identically, lambda_n = 1/(|n~||x|).
   vI: r_I defined (W_A valid, interior, warped values exist).
   vW: vI and grad W defined. */
void or_residuals(const or_cam* c, const double* IA, const double* WA,
                  const double* Iw, const double* Ww, const uint8_t* wvalid,
                  double* rI, double* rW, double* JI, double* JW, double* lam,
                  uint8_t* vI, uint8_t* vW)
{
    const int w = c->w, h = c->h;
    for (int v = 0; v < h; ++v)
        for (int u = 0; u < w; ++u) {
            int i = v * w + u;
            vI[i] = vW[i] = 0;
            rI[i] = rW[i] = lam[i] = 0.0;
            for (int k = 0; k < 6; ++k) JI[6 * i + k] = JW[6 * i + k] = 0.0;
            if (u < 1 || u > w - 2 || v < 1 || v > h - 2) continue;
            double wa = WA[i];
            if (!valid_w(wa) || !wvalid[i]) continue;
            double Z = 1.0 / wa;
            double x[3] = {(u - c->cx) / c->fx, (v - c->cy) / c->fy, 1.0};
            double X[3] = {Z * x[0], Z * x[1], Z * x[2]};
            double gu = (IA[i + 1] - IA[i - 1]) / 2.0;
            double gv = (IA[i + w] - IA[i - w]) / 2.0;
            double a[3] = {wa * gu * c->fx, wa * gv * c->fy,
                           wa * (gu * (c->cx - u) + gv * (c->cy - v))};
            JI[6 * i + 0] = a[0];
            JI[6 * i + 1] = a[1];
            JI[6 * i + 2] = a[2];
            JI[6 * i + 3] = X[1] * a[2] - X[2] * a[1];
            JI[6 * i + 4] = X[2] * a[0] - X[0] * a[2];
            JI[6 * i + 5] = X[0] * a[1] - X[1] * a[0];
            rI[i] = Iw[i] - IA[i];
            vI[i] = 1;
            if (!(valid_w(WA[i + 1]) && valid_w(WA[i - 1]) && valid_w(WA[i + w]) &&
                  valid_w(WA[i - w])))
                continue;
            double wu = (WA[i + 1] - WA[i - 1]) / 2.0;
            double wv = (WA[i + w] - WA[i - w]) / 2.0;
            double gk[3] = {wu * c->fx, wv * c->fy, wu * (c->cx - u) + wv * (c->cy - v)};
            double b[3] = {wa * gk[0], wa * gk[1], wa * (gk[2] + Ww[i])};
            JW[6 * i + 0] = b[0];
            JW[6 * i + 1] = b[1];
            JW[6 * i + 2] = b[2];
            JW[6 * i + 3] = X[1] * b[2] - X[2] * b[1];
            JW[6 * i + 4] = X[2] * b[0] - X[0] * b[2];
            JW[6 * i + 5] = X[0] * b[1] - X[1] * b[0];
            rW[i] = Ww[i] - wa;
            double n[3] = {Z * gk[0], Z * gk[1], Z * gk[2] + 1.0};
            double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
            double xn = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
            lam[i] = (n[0] * x[0] + n[1] * x[1] + n[2] * x[2]) / (nn * xn);
            vW[i] = 1;
        }
}

/* ---------------------------------------------------------------- robust scale */

/* Weight functions.  Student-t (sec. 6.3): w = (1/x) d rho/dx with
   rho = (nu+1)/2 ln(nu + x^2), i.e. w = (nu+1)/(nu + x^2).
   Huber: w = min(1, k/|x|). */
double or_omega(int kind, double x, double nu, double k)
{
    if (kind == OR_WEIGHT_HUBER) {
        double ax = fabs(x);
        return ax <= k ? 1.0 : k / ax;
    }
    return (nu + 1.0) / (nu + x * x);
}

/* Digamma for x > 0: recurrence psi(x) = psi(x+1) - 1/x up to x >= 10, then
   the asymptotic series through the z^-14 term (Abramowitz & Stegun 6.3.5,
   6.3.18); truncation error below 1e-15 there. */
double or_digamma(double x)
{
    double acc = 0.0;
    while (x < 10.0) { acc -= 1.0 / x; x += 1.0; }
    double x2 = 1.0 / (x * x);
    double s = log(x) - 0.5 / x -
               x2 * (1.0 / 12 - x2 * (1.0 / 120 - x2 * (1.0 / 252 - x2 * (1.0 / 240 -
               x2 * (1.0 / 132 - x2 * (691.0 / 32760 - x2 * (1.0 / 12)))))));
    return acc + s;
}

/* Location and scale by the fixed point of the two stationarity equations of
   sec. 6.3 (sum w (r - mu) = 0, sum (1 - w (r-mu)^2/sigma^2) = 0), updating
   the weights from the previous estimate before each step:
     mu <- sum w r / sum w,   sigma^2 <- sum w (r - mu)^2 / n.
   Start: start = {mu0, sigma0}, or mu = 0, sigma^2 = mean r^2 when start is
   NULL.  At most iters steps; the step after which both |mu' - mu| and
   |sigma' - sigma| are at most tol sigma' is the last (tol = 0: only a step
   that changes nothing, after which every further step would repeat it).
   sigma is floored at sigma_floor.  n == 0 returns mu = 0, sigma =
   sigma_floor (the caller disables the channel). */
void or_scale(const double* r, int n, int kind, double nu, double k, int iters,
              double sigma_floor, const double* start, double tol, double* mu_out,
              double* sigma_out)
{
    double mu = 0.0, sigma;
    if (n == 0) { *mu_out = 0.0; *sigma_out = sigma_floor; return; }
    if (start) {
        mu = start[0];
        sigma = start[1];
    } else {
        double s2 = 0.0;
        for (int i = 0; i < n; ++i) s2 += r[i] * r[i];
        sigma = sqrt(s2 / n);
    }
    if (sigma < sigma_floor) sigma = sigma_floor;
    for (int it = 0; it < iters; ++it) {
        double sw = 0.0, swr = 0.0;
        double* wts = malloc((size_t)n * sizeof(double));
        for (int i = 0; i < n; ++i) {
            wts[i] = or_omega(kind, (r[i] - mu) / sigma, nu, k);
            sw += wts[i];
            swr += wts[i] * r[i];
        }
        double mu_new = swr / sw;
        double sv = 0.0;
        for (int i = 0; i < n; ++i) sv += wts[i] * (r[i] - mu_new) * (r[i] - mu_new);
        free(wts);
        double sigma_new = sqrt(sv / n);
        if (sigma_new < sigma_floor) sigma_new = sigma_floor;
        int last = fabs(mu_new - mu) <= tol * sigma_new && fabs(sigma_new - sigma) <= tol * sigma_new;
        mu = mu_new;
        sigma = sigma_new;
        if (last) break;
    }
    *mu_out = mu;
    *sigma_out = sigma;
}

/* Left side of eq:robustnessValue with x_i = (r_i - mu)/sigma frozen:
   f(nu) = n [-psi(nu/2) + ln(nu/2) + psi((nu+1)/2) - ln((nu+1)/2)]
           + sum (1 + ln w_i(nu) - w_i(nu)). */
double or_nu_equation(const double* r, int n, double mu, double sigma, double nu)
{
    double c = -or_digamma(nu / 2) + log(nu / 2) + or_digamma((nu + 1) / 2) - log((nu + 1) / 2);
    double s = n * c;
    for (int i = 0; i < n; ++i) {
        double x = (r[i] - mu) / sigma;
        double wi = (nu + 1.0) / (nu + x * x);
        s += 1.0 + log(wi) - wi;
    }
    return s;
}

/* nu by bisection on [2, 10] (sec. 6.3): clamp to 10 if f(10) > 0, to 2 if
   f(2) < 0, else 30 halvings (f(mid) > 0 moves the lower end) and the mid. */
double or_estimate_nu(const double* r, int n, double mu, double sigma)
{
    if (n == 0) return 5.0;
    if (or_nu_equation(r, n, mu, sigma, 10.0) > 0) return 10.0;
    if (or_nu_equation(r, n, mu, sigma, 2.0) < 0) return 2.0;
    double lo = 2.0, hi = 10.0;
    for (int it = 0; it < 30; ++it) {
        double mid = 0.5 * (lo + hi);
        if (or_nu_equation(r, n, mu, sigma, mid) > 0) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Systematic sample (sec. 6.3, "a sample with a maximum size of N"): the
   pixels with u = v = 0 (mod s), with s the smallest stride >= 1 whose sample
   grid ceil(w/s) x ceil(h/s) holds at most N pixels. */
int or_sample_stride(int w, int h, int nmax)
{
    int s = 1;
    while ((long long)((w + s - 1) / s) * ((h + s - 1) / s) > nmax) ++s;
    return s;
}

/* ---------------------------------------------------------------- solve */

/* Cholesky solve of H xi = -g (6x6).  A pivot <= 1e-12 max(diag H) is
   reported as degenerate. */
int or_solve(const double H[36], const double g[6], double xi[6])
{
    double L[36] = {0};
    double dmax = 0.0;
    for (int i = 0; i < 6; ++i) if (H[7 * i] > dmax) dmax = H[7 * i];
    if (!(dmax > 0.0)) return OR_DEGENERATE;
    for (int j = 0; j < 6; ++j) {
        double d = H[6 * j + j];
        for (int k = 0; k < j; ++k) d -= L[6 * j + k] * L[6 * j + k];
        if (!(d > 1e-12 * dmax)) return OR_DEGENERATE;
        L[6 * j + j] = sqrt(d);
        for (int i = j + 1; i < 6; ++i) {
            double s = H[6 * i + j];
            for (int k = 0; k < j; ++k) s -= L[6 * i + k] * L[6 * j + k];
            L[6 * i + j] = s / L[6 * j + j];
        }
    }
    double y[6];
    for (int i = 0; i < 6; ++i) {
        double s = -g[i];
        for (int k = 0; k < i; ++k) s -= L[6 * i + k] * y[k];
        y[i] = s / L[6 * i + i];
    }
    for (int i = 5; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < 6; ++k) s -= L[6 * k + i] * xi[k];
        xi[i] = s / L[6 * i + i];
    }
    return OR_OK;
}

/* ---------------------------------------------------------------- one iteration */

typedef struct {
    or_cam c;             /* level camera */
    const double *IA, *WA;/* level-l reference */
} or_level_ref;

/* Builds H, g (sec. 6.2, the IRLS objective 2eq:minimisationIRLS) at one level
   for the warped images.  Per channel the sample residuals give mu, sigma
   (with nu = 5 for Student-t); then nu by bisection and nu_I = max(nu_I, nu_W);
   per-pixel weights
     w_I = omega((r_I - mu_I)/sigma_I; nu_I) / sigma_I^2,
     w_W = lambda_n omega((r_W - mu_W)/sigma_W; nu_W) / sigma_W^2,
   H = sum w J J^T, g = sum w J r (uncentred r), cost = sum w r^2. */
void or_normal_equations(const or_cam* c, const double* IA, const double* WA,
                         const double* Iw, const double* Ww, const uint8_t* wvalid,
                         const or_params* P, or_scale_state* ss, or_stats* st)
{
    const int w = c->w, h = c->h;
    size_t n = (size_t)w * h;
    double* rI = malloc(n * sizeof(double));
    double* rW = malloc(n * sizeof(double));
    double* JI = malloc(6 * n * sizeof(double));
    double* JW = malloc(6 * n * sizeof(double));
    double* lam = malloc(n * sizeof(double));
    uint8_t* vI = malloc(n);
    uint8_t* vW = malloc(n);
    or_residuals(c, IA, WA, Iw, Ww, wvalid, rI, rW, JI, JW, lam, vI, vW);

    int s = or_sample_stride(w, h, P->sample_max);
    double* sI = malloc(n * sizeof(double));
    double* sW = malloc(n * sizeof(double));
    int nI = 0, nW = 0;
    for (int v = 0; v < h; v += s)
        for (int u = 0; u < w; u += s) {
            int i = v * w + u;
            if (vI[i]) sI[nI++] = rI[i];
            if (vW[i]) sW[nW++] = rW[i];
        }
    double nu0 = 5.0;
    /* warm start (scale_warm): from the last estimate at this level of a
       channel whose sample was not empty, ending at the convergence stop */
    const int warm = P->scale_warm && ss;
    const double tol = P->scale_warm ? OR_SCALE_TOL : 0.0;
    double s0I[2], s0W[2];
    const double* startI = NULL;
    const double* startW = NULL;
    if (warm && ss->n[0] > 0) { s0I[0] = ss->mu[0]; s0I[1] = ss->sigma[0]; startI = s0I; }
    if (warm && ss->n[1] > 0) { s0W[0] = ss->mu[1]; s0W[1] = ss->sigma[1]; startW = s0W; }
    or_scale(sI, nI, P->weight, nu0, P->huber_k, P->scale_iters, 1e-3, startI, tol, &st->mu_I,
             &st->sigma_I);
    or_scale(sW, nW, P->weight, nu0, P->huber_k, P->scale_iters, 1e-6, startW, tol, &st->mu_W,
             &st->sigma_W);
    if (ss) {
        ss->mu[0] = st->mu_I;
        ss->sigma[0] = st->sigma_I;
        ss->n[0] = nI;
        ss->mu[1] = st->mu_W;
        ss->sigma[1] = st->sigma_W;
        ss->n[1] = nW;
    }
    st->nu_I = st->nu_W = nu0;
    if (P->weight == OR_WEIGHT_STUDENT_T && P->estimate_nu) {
        st->nu_I = or_estimate_nu(sI, nI, st->mu_I, st->sigma_I);
        st->nu_W = or_estimate_nu(sW, nW, st->mu_W, st->sigma_W);
        if (st->nu_W > st->nu_I) st->nu_I = st->nu_W;
    }
    free(sI);
    free(sW);

    memset(st->H, 0, sizeof st->H);
    memset(st->g, 0, sizeof st->g);
    st->cost = 0.0;
    st->n_valid_I = st->n_valid_W = 0;
    for (size_t i = 0; i < n; ++i) {
        if (vI[i] && nI > 0) {
            double x = (rI[i] - st->mu_I) / st->sigma_I;
            double wt = or_omega(P->weight, x, st->nu_I, P->huber_k) / (st->sigma_I * st->sigma_I);
            const double* J = JI + 6 * i;
            for (int a = 0; a < 6; ++a) {
                for (int b = 0; b < 6; ++b) st->H[6 * a + b] += wt * J[a] * J[b];
                st->g[a] += wt * J[a] * rI[i];
            }
            st->cost += wt * rI[i] * rI[i];
            st->n_valid_I++;
        }
        if (vW[i] && nW > 0) {
            double x = (rW[i] - st->mu_W) / st->sigma_W;
            double wt = lam[i] * or_omega(P->weight, x, st->nu_W, P->huber_k) /
                        (st->sigma_W * st->sigma_W);
            const double* J = JW + 6 * i;
            for (int a = 0; a < 6; ++a) {
                for (int b = 0; b < 6; ++b) st->H[6 * a + b] += wt * J[a] * J[b];
                st->g[a] += wt * J[a] * rW[i];
            }
            st->cost += wt * rW[i] * rW[i];
            st->n_valid_W++;
        }
    }
    free(rI); free(rW); free(JI); free(JW); free(lam); free(vI); free(vW);
}

/* ---------------------------------------------------------------- pyramids */

typedef struct {
    int levels;
    or_cam cam[8];
    double* I[8];
    double* W[8];
} or_pyr;

static void pyr_build(or_pyr* p, const or_cam* c0, int levels, const double* I0,
                      const double* W0, int storage)
{
    p->levels = levels;
    size_t n0 = (size_t)c0->w * c0->h;
    for (int l = 0; l < levels; ++l) {
        or_camera_level(c0, l, &p->cam[l]);
        size_t n = (size_t)p->cam[l].w * p->cam[l].h;
        p->I[l] = malloc((n ? n : 1) * sizeof(double));
        p->W[l] = malloc((n ? n : 1) * sizeof(double));
        if (l == 0) {
            for (size_t i = 0; i < n0; ++i) {
                p->I[0][i] = I0[i];
                p->W[0][i] = valid_w(W0[i]) ? W0[i] : 0.0;
            }
        } else {
            or_downsample(p->I[l - 1], p->W[l - 1], p->cam[l - 1].w, p->cam[l - 1].h,
                          p->I[l], p->W[l], storage);
        }
    }
}

static void pyr_free(or_pyr* p)
{
    for (int l = 0; l < p->levels; ++l) { free(p->I[l]); free(p->W[l]); }
}

/* Builds the pyramid into caller buffers laid out level after level. */
void or_pyramid(const or_cam* c0, int levels, const double* I0, const double* W0,
                int storage, double* I_out, double* W_out)
{
    or_pyr p;
    pyr_build(&p, c0, levels, I0, W0, storage);
    size_t off = 0;
    for (int l = 0; l < levels; ++l) {
        size_t n = (size_t)p.cam[l].w * p.cam[l].h;
        memcpy(I_out + off, p.I[l], n * sizeof(double));
        memcpy(W_out + off, p.W[l], n * sizeof(double));
        off += n;
    }
    pyr_free(&p);
}

/* One linearisation at a level: warp B at T (paper-literal full resolution or
   per level), then residuals, scale and normal equations. */
void or_linearise(const or_cam* c0, const or_pyr* A, const or_pyr* B, int level,
                  const double R[9], const double t[3], const or_params* P, or_scale_state* ss,
                  or_stats* st)
{
    const or_cam* cl = &A->cam[level];
    size_t n = (size_t)cl->w * cl->h;
    double* Iw = malloc((n ? n : 1) * sizeof(double));
    double* Ww = malloc((n ? n : 1) * sizeof(double));
    uint8_t* V = malloc(n ? n : 1);
    if (P->warp == OR_WARP_FULLRES)
        or_warp_fullres(c0, level, A->W[0], B->I[0], B->W[0], R, t, Iw, Ww, V);
    else
        or_warp(cl, A->W[level], B->I[level], B->W[level], R, t, Iw, Ww, V);
    or_normal_equations(cl, A->I[level], A->W[level], Iw, Ww, V, P, ss, st);
    free(Iw); free(Ww); free(V);
}

/* Normal equations of one linearisation from level-0 images (builds both
   pyramids first). */
void or_normal_equations_at(const or_cam* c0, int levels, const double* IA0,
                            const double* WA0, const double* IB0, const double* WB0,
                            int level, const double R[9], const double t[3],
                            const or_params* P, or_stats* st)
{
    or_pyr A, B;
    pyr_build(&A, c0, levels, IA0, WA0, P->storage);
    pyr_build(&B, c0, levels, IB0, WB0, P->storage);
    or_linearise(c0, &A, &B, level, R, t, P, NULL, st);
    pyr_free(&A);
    pyr_free(&B);
}

/* ---------------------------------------------------------------- align */

/* Coarse-to-fine Gauss-Newton / IRLS (sec. 6.2): levels L-1 .. 0, iters[l]
   iterations each; each iteration warps B at the current estimate, builds H, g,
   solves H xi = -g and applies T <- exp(xi)^-1 T.  Optional early stop per
   level when |v| < eps_t and |theta| < eps_r.  A degenerate system stops the
   alignment and keeps the last estimate.  With scale_warm, the mu, sigma
   fixed point of every iteration after the first at a level starts from the
   previous iteration's estimates (sec. 6.3: the weights of each step come from
   the previous estimates). */
int or_align(const or_cam* c0, const double* IA0, const double* WA0, const double* IB0,
             const double* WB0, const double* R_init, const double* t_init,
             const or_params* P, double R[9], double t[3], or_stats* st)
{
    if (P->levels < 1 || P->levels > 8) return OR_ARG;
    or_pyr A, B;
    pyr_build(&A, c0, P->levels, IA0, WA0, P->storage);
    pyr_build(&B, c0, P->levels, IB0, WB0, P->storage);
    if (R_init) memcpy(R, R_init, 9 * sizeof(double));
    else { memset(R, 0, 9 * sizeof(double)); R[0] = R[4] = R[8] = 1.0; }
    if (t_init) memcpy(t, t_init, 3 * sizeof(double));
    else memset(t, 0, 3 * sizeof(double));
    memset(st, 0, sizeof *st);
    st->status = OR_OK;
    for (int l = P->levels - 1; l >= 0 && st->status == OR_OK; --l) {
        or_scale_state ss;   /* no estimate yet at this level */
        memset(&ss, 0, sizeof ss);
        for (int it = 0; it < P->iters[l]; ++it) {
            or_stats cur;
            memset(&cur, 0, sizeof cur);
            or_linearise(c0, &A, &B, l, R, t, P, &ss, &cur);
            int done[8];
            memcpy(done, st->iters_done, sizeof done);
            double xi[6];
            int rc = (cur.n_valid_I + cur.n_valid_W < 6) ? OR_DEGENERATE
                                                          : or_solve(cur.H, cur.g, xi);
            *st = cur;
            memcpy(st->iters_done, done, sizeof done);
            if (rc != OR_OK) { st->status = rc; break; }
            or_update(R, t, xi);
            st->iters_done[l]++;
            if (P->stop_eps_t > 0 || P->stop_eps_r > 0) {
                double nv = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
                double nr = sqrt(xi[3] * xi[3] + xi[4] * xi[4] + xi[5] * xi[5]);
                if (nv < P->stop_eps_t && nr < P->stop_eps_r) break;
            }
        }
    }
    pyr_free(&A);
    pyr_free(&B);
    return st->status;
}

/* ---------------------------------------------------------------- fusion */

/* Keyframe fusion (sec. 7.2).  For every keyframe pixel with a valid W_kf:
   transfer it into frame k with T = (R, t), the pose of frame k in the
   keyframe (X_kf = R X_k + t): Y = R^T (K^-1 p / W_kf - t), require Y_z > 0,
   p_w = K Y / Y_z, w_k = 1 / Y_z; sample W_k bilinearly at p_w (four valid
   taps, same bounds rule as the warp).  The covisibility check of sec. 6.4:
   fuse iff |W_k(p_w) - w_k| < tol.  The fused value is the warped inverse depth
   W* = (R^T K^-1 p)_z w_b / (1 + w_b (R^T t)_z) with the variance weight
   C_k = ((1 + w_b (R^T t)_z)^2 / (R^T K^-1 p)_z)^2, and
   W_kf <- (W_kf C_kf + C_k W*) / (C_kf + C_k),  C_kf <- C_kf + C_k.
   Reading: the printed update uses W_k(p_w), which is in frame k's coordinates;
   the warped W* (keyframe coordinates, sec. 5.3) is used. */
long long or_fuse(const or_cam* c, double* Wkf, double* Ckf, const double* Wk,
                  const double R[9], const double t[3], double tol)
{
    const int w = c->w, h = c->h;
    double Rtt[3];
    for (int i = 0; i < 3; ++i) Rtt[i] = R[i] * t[0] + R[3 + i] * t[1] + R[6 + i] * t[2];
    long long nf = 0;
    for (int v = 0; v < h; ++v)
        for (int u = 0; u < w; ++u) {
            int i = v * w + u;
            double wkf = Wkf[i];
            if (!valid_w(wkf)) continue;
            double ray[3] = {(u - c->cx) / c->fx, (v - c->cy) / c->fy, 1.0};
            double X[3] = {ray[0] / wkf - t[0], ray[1] / wkf - t[1], ray[2] / wkf - t[2]};
            double Y[3], Rray[3];
            for (int k = 0; k < 3; ++k) {
                Y[k] = R[k] * X[0] + R[3 + k] * X[1] + R[6 + k] * X[2];
                Rray[k] = R[k] * ray[0] + R[3 + k] * ray[1] + R[6 + k] * ray[2];
            }
            if (!(Y[2] > 0.0)) continue;
            double ub = c->fx * Y[0] / Y[2] + c->cx;
            double vb = c->fy * Y[1] / Y[2] + c->cy;
            double wb;
            if (!bilinear(Wk, w, h, ub, vb, 1, &wb)) continue;
            double wk = 1.0 / Y[2];
            if (!(fabs(wb - wk) < tol)) continue;
            double den = 1.0 + wb * Rtt[2];
            double ws = Rray[2] * wb / den;
            double ck = (den * den / Rray[2]) * (den * den / Rray[2]);
            if (!valid_w(ws) || !(ck > 0.0) || !isfinite(ck)) continue;
            Wkf[i] = (wkf * Ckf[i] + ck * ws) / (Ckf[i] + ck);
            Ckf[i] += ck;
            ++nf;
        }
    return nf;
}

/* ---------------------------------------------------------------- covisibility */

/* Dense covisibility of sec. 6.4 in one direction: pixels of A with a valid
   W_A (S_H) are transferred into B with T = (R, t), the pose of B in A
   (Y = R^T (K^-1 p / W_A - t), p_B = K Y / Y_z, w_B = 1 / Y_z); a pixel is
   visible (S_V) when Y_z > 0, p_B lies in the image (the bilinear bounds rule)
   with four valid W_B taps, and |W_B(p_B) - w_B| < tol (tol = 3 sigma_W).
   Writes |S_H| and |S_V|. */
void or_covisibility(const or_cam* c, const double* WA, const double* WB, const double R[9],
                     const double t[3], double tol, long long* nH, long long* nV)
{
    const int w = c->w, h = c->h;
    long long h_ = 0, v_ = 0;
    for (int v = 0; v < h; ++v)
        for (int u = 0; u < w; ++u) {
            const double wa = WA[v * w + u];
            if (!valid_w(wa)) continue;
            ++h_;
            const double ray[3] = {(u - c->cx) / c->fx, (v - c->cy) / c->fy, 1.0};
            const double X[3] = {ray[0] / wa - t[0], ray[1] / wa - t[1], ray[2] / wa - t[2]};
            double Y[3];
            for (int k = 0; k < 3; ++k) Y[k] = R[k] * X[0] + R[3 + k] * X[1] + R[6 + k] * X[2];
            if (!(Y[2] > 0.0)) continue;
            const double ub = c->fx * Y[0] / Y[2] + c->cx, vb = c->fy * Y[1] / Y[2] + c->cy;
            double wb;
            if (!bilinear(WB, w, h, ub, vb, 1, &wb)) continue;
            if (fabs(wb - 1.0 / Y[2]) < tol) ++v_;
        }
    *nH = h_;
    *nV = v_;
}

/* ---------------------------------------------------------------- covariance */

/* Bilateral filter applied to {I_A, W_A} before the covariance iteration
   (sec. 6.2).  The paper gives no parameters; reading: window (2r+1)^2,
   spatial weight exp(-d^2 / (2 sigma_s^2)), range weight exp(-dI^2 /
   (2 sigma_I^2)) for intensity and exp(-(dW / (rel_W W(p)))^2 / 2) for inverse
   depth; W holes neither contribute nor receive a value; out-of-image
   neighbours are skipped. */
void or_bilateral(const double* I, const double* W, int w, int h, int radius, double sigma_s,
                  double sigma_I, double rel_W, double* Io, double* Wo)
{
    for (int v = 0; v < h; ++v)
        for (int u = 0; u < w; ++u) {
            const int i = v * w + u;
            double si = 0, swi = 0, sw = 0, sww = 0;
            const double w0 = W[i];
            const int wv = valid_w(w0);
            for (int dv = -radius; dv <= radius; ++dv)
                for (int du = -radius; du <= radius; ++du) {
                    const int x = u + du, y = v + dv;
                    if (x < 0 || y < 0 || x >= w || y >= h) continue;
                    const int j = y * w + x;
                    const double gs = exp(-(double)(du * du + dv * dv) / (2.0 * sigma_s * sigma_s));
                    const double di = (I[j] - I[i]) / sigma_I;
                    const double gi = gs * exp(-0.5 * di * di);
                    si += gi * I[j];
                    swi += gi;
                    if (wv && valid_w(W[j])) {
                        const double dw = (W[j] - w0) / (rel_W * w0);
                        const double gw = gs * exp(-0.5 * dw * dw);
                        sw += gw * W[j];
                        sww += gw;
                    }
                }
            Io[i] = si / swi;
            Wo[i] = wv ? sw / sww : 0.0;
        }
}

/* Pose covariance of sec. 6.2: one extra linearisation at level 0 and pose T
   without update, with {I_A, W_A} bilateral-filtered (then the pyramid and the
   gradients are computed from the filtered images); Sigma = H_filt^-1 (full
   6x6, row-major).  Returns OR_DEGENERATE if H_filt is not positive definite. */
int or_covariance(const or_cam* c0, int levels, const double* IA0, const double* WA0,
                  const double* IB0, const double* WB0, const double R[9], const double t[3],
                  const or_params* P, int radius, double sigma_s, double sigma_I, double rel_W,
                  double Sigma[36], or_stats* st)
{
    const size_t n = (size_t)c0->w * c0->h;
    double* If = malloc(n * sizeof(double));
    double* Wf = malloc(n * sizeof(double));
    or_bilateral(IA0, WA0, c0->w, c0->h, radius, sigma_s, sigma_I, rel_W, If, Wf);
    if (P->storage != OR_STORE_F64)
        for (size_t i = 0; i < n; ++i) {
            If[i] = store_round(If[i], P->storage);
            Wf[i] = store_round(Wf[i], P->storage);
        }
    memset(st, 0, sizeof *st);
    or_normal_equations_at(c0, levels, If, Wf, IB0, WB0, 0, R, t, P, st);
    free(If);
    free(Wf);
    /* inverse by solving H x = e_k with the Cholesky solver (xi = -H^-1 g) */
    for (int k = 0; k < 6; ++k) {
        double e[6] = {0}, x[6];
        e[k] = -1.0;
        if (or_solve(st->H, e, x) != OR_OK) return OR_DEGENERATE;
        for (int r = 0; r < 6; ++r) Sigma[6 * r + k] = x[r];
    }
    return OR_OK;
}

/* ---------------------------------------------------------------- sensor input path */

/* Brown distortion h of eq:proj_dist on the normalised plane, k = (k1..k5):
     r^2 = x^2 + y^2,  rad = k1 r^2 + k2 r^4 + k5 r^6,
     x_d = (1 + rad) x + 2 k3 x y + k4 (r^2 + 2 x^2),
     y_d = (1 + rad) y + 2 k4 x y + k3 (r^2 + 2 y^2),
   and the third coordinate stays 1. */
void or_distort(const double k[5], double x, double y, double* xd, double* yd)
{
    const double r2 = x * x + y * y;
    const double rad = k[0] * r2 + k[1] * r2 * r2 + k[4] * r2 * r2 * r2;
    *xd = (1.0 + rad) * x + 2.0 * k[2] * x * y + k[3] * (r2 + 2.0 * x * x);
    *yd = (1.0 + rad) * y + 2.0 * k[3] * x * y + k[2] * (r2 + 2.0 * y * y);
}

/* Inverse warping for undistortion (sec. 5.1): dst(p) = src(K h(K^-1 p)) by
   bilinear interpolation.  Reading: the bounds rule and clamped taps of the
   alignment's sampler; a depth image (is_depth) needs four valid taps, and an
   unmapped pixel is 0 (a hole for depth). */
void or_undistort(const or_cam* c, const double k[5], const double* src, int is_depth,
                  double* dst)
{
    for (int v = 0; v < c->h; ++v)
        for (int u = 0; u < c->w; ++u) {
            double xd, yd, val = 0.0;
            const double mx = (u - c->cx) / c->fx, my = (v - c->cy) / c->fy;
            or_distort(k, mx, my, &xd, &yd);
            /* K h(m) = p + f (h(m) - m): exact at zero distortion */
            const double x = u + c->fx * (xd - mx), y = v + c->fy * (yd - my);
            if (!bilinear(src, c->w, c->h, x, y, is_depth, &val)) val = 0.0;
            if (is_depth && !valid_w(val)) val = 0.0;
            dst[v * c->w + u] = val;
        }
}

/* Spatially varying factor / offset of eq:depth_spatial_correction at pixel
   (u, v): a polynomial in m = K^-1 p with nine coefficients q0..q8 (the text
   announces eight parameters but lists nine terms; all nine are used). */
static double depth_poly(const double q[9], double mx, double my)
{
    const double r2 = mx * mx + my * my;
    return q[0] + q[1] * r2 + q[2] * r2 * r2 + q[3] * r2 * r2 * r2 + q[4] * mx + q[5] * my +
           q[6] * mx * my + q[7] * mx * mx * my + q[8] * mx * my * my;
}

/* Depth correction of sec. 4.1 on the raw depth image Z_m (metres):
     W_d(p) = beta1 W_m(p - p0) + beta0,  W_m = 1 / Z_m   (eq:depth_linear_correction)
     W_u(p) = D1(p) W_d(p) + D0(p)                        (eq:depth_spatial_correction)
   Holes (Z_m <= 0 or non-finite, p - p0 outside the image, W_u <= 0) are 0. */
void or_depth_correct(const or_cam* c, const double* Zm, double beta0, double beta1, int p0x,
                      int p0y, int spatial, const double q0[9], const double q1[9], double* Wu)
{
    for (int v = 0; v < c->h; ++v)
        for (int u = 0; u < c->w; ++u) {
            const int us = u - p0x, vs = v - p0y;
            double out = 0.0;
            if (us >= 0 && us < c->w && vs >= 0 && vs < c->h) {
                const double Z = Zm[vs * c->w + us];
                if (Z > 0.0 && isfinite(Z)) {
                    double W = beta1 * (1.0 / Z) + beta0;
                    if (spatial) {
                        const double mx = (u - c->cx) / c->fx, my = (v - c->cy) / c->fy;
                        W = depth_poly(q1, mx, my) * W + depth_poly(q0, mx, my);
                    }
                    out = valid_w(W) ? W : 0.0;
                }
            }
            Wu[v * c->w + u] = out;
        }
}

/* Forward registration, step 1 (sec. 5.2, eq:register_trans): W_A of camera
   cA is moved by the translation t = t_A^B alone into the intermediate frame
   B_t (camera cA, same size).  With t~ = K_A t and den = 1 - W t~_z (> 0),
     w_t = W / den,  p_t = (p - W t~) / den,
   and the pixel's footprint, a square of side 1/den centred on p_t, is
   written to every pixel of B_t whose centre lies inside it (half-open on the
   high side, so that the identity maps each pixel to itself), keeping the
   greatest inverse depth.  Unwritten pixels are 0. */
void or_register_translate(const or_cam* cA, const double* WA, const double t[3], double* WBt)
{
    const int n = cA->w * cA->h;
    for (int i = 0; i < n; ++i) WBt[i] = 0.0;
    const double tx = cA->fx * t[0] + cA->cx * t[2];
    const double ty = cA->fy * t[1] + cA->cy * t[2];
    const double tz = t[2];
    for (int v = 0; v < cA->h; ++v)
        for (int u = 0; u < cA->w; ++u) {
            const double W = WA[v * cA->w + u];
            if (!valid_w(W)) continue;
            const double den = 1.0 - W * tz;
            if (!(den > 0.0)) continue;
            const double wt = W / den;
            const double x = (u - W * tx) / den, y = (v - W * ty) / den;
            const double half = 0.5 / den;
            const double qx0 = ceil(x - half), qx1 = ceil(x + half) - 1.0;
            const double qy0 = ceil(y - half), qy1 = ceil(y + half) - 1.0;
            for (double qy = fmax(qy0, 0.0); qy <= fmin(qy1, cA->h - 1.0); qy += 1.0)
                for (double qx = fmax(qx0, 0.0); qx <= fmin(qx1, cA->w - 1.0); qx += 1.0) {
                    double* d = &WBt[(int)qy * cA->w + (int)qx];
                    if (wt > *d) *d = wt;
                }
        }
}

/* Forward registration, step 2 (sec. 5.2): the remaining rotation as an
   inverse warp into camera cB.  With R~_AB = K_A R K_B^-1 (R = R_A^B),
   d = R~_AB p, p_t = (d_x, d_y) / d_z, W_Bt taken at the nearest pixel
   (floor(x + 0.5)), W_B(p) = W_Bt(p_t) d_z.  Holes: d_z <= 0, p_t outside
   the image, or a hole of W_Bt. */
void or_register_rotate(const or_cam* cA, const double* WBt, const or_cam* cB, const double R[9],
                        double* WB)
{
    for (int v = 0; v < cB->h; ++v)
        for (int u = 0; u < cB->w; ++u) {
            const double m[3] = {(u - cB->cx) / cB->fx, (v - cB->cy) / cB->fy, 1.0};
            double r[3];
            for (int i = 0; i < 3; ++i) r[i] = R[3 * i] * m[0] + R[3 * i + 1] * m[1] + R[3 * i + 2] * m[2];
            double out = 0.0;
            if (r[2] > 0.0) {
                const double x = (cA->fx * r[0] + cA->cx * r[2]) / r[2];
                const double y = (cA->fy * r[1] + cA->cy * r[2]) / r[2];
                const double qx = floor(x + 0.5), qy = floor(y + 0.5);
                if (qx >= 0 && qx <= cA->w - 1 && qy >= 0 && qy <= cA->h - 1) {
                    const double wt = WBt[(int)qy * cA->w + (int)qx];
                    if (valid_w(wt)) out = wt * r[2];
                }
            }
            WB[v * cB->w + u] = valid_w(out) ? out : 0.0;
        }
}

/* Input path of one RGB-D frame (sec. 4.1, 4.2, 5.1, 5.2) in the paper's
   order: depth correction and spatial correction on the raw depth grid,
   undistortion of the corrected inverse depth (depth lens) and of the
   intensity (colour lens), then forward registration of the inverse depth
   into the colour camera with T_D^C (pose of the colour camera in the depth
   camera).  Outputs are on the colour camera's grid. */
void or_preprocess(const or_cam* cc, const double kc[5], const or_cam* cd, const double kd[5],
                   double beta0, double beta1, int p0x, int p0y, int spatial, const double q0[9],
                   const double q1[9], const double R_dc[9], const double t_dc[3],
                   const double* I_raw, const double* Z_raw, double* I_out, double* W_out)
{
    const size_t nd = (size_t)cd->w * cd->h;
    double* Wu = malloc(nd * sizeof(double));
    double* Wund = malloc(nd * sizeof(double));
    double* Wt = malloc(nd * sizeof(double));
    or_depth_correct(cd, Z_raw, beta0, beta1, p0x, p0y, spatial, q0, q1, Wu);
    or_undistort(cd, kd, Wu, 1, Wund);
    or_register_translate(cd, Wund, t_dc, Wt);
    or_register_rotate(cd, Wt, cc, R_dc, W_out);
    or_undistort(cc, kc, I_raw, 0, I_out);
    free(Wu);
    free(Wund);
    free(Wt);
}

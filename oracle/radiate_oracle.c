/*
 * radiate_oracle.c -- plain FP64 CPU reference of the differentiable acoustic
 * radiation model of PA-SFM (Li, Gao et al., arxiv 2604.09643).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no code, header or table with the GPU
 * path.
 *
 * What it computes (all in double precision, SI units, row-major arrays):
 *
 *   Forward model.  Main text Eq. (1) states the measured pressure as a sum over
 *   the volume of the source intensity times a kernel of the source-sensor
 *   distance.  Appendix A ("GPU-Accelerated Forward Simulation Framework",
 *   the discretised far-field model Eq. (A13) with the Gaussian kernel K_G)
 *   fixes that kernel: a source of amplitude a at distance d from a detector
 *   contributes
 *        a * (d - c t) / (2 d) * exp(-(d - c t)^2 / (2 sigma^2))
 *   at time t.  The same expression is the far-field Gaussian pulse of
 *   Appendix A (Eq. (A12)), i.e. the outward half of the exact spherically
 *   symmetric Gaussian solution (Eq. (A8)).
 *
 *   Sampling and truncation (readings of what the paper leaves open):
 *   t_k = k / fs for k = 0..K-1, and a term is kept iff |d - c t_k| <= trunc*sigma
 *   (inclusive).
 *
 *   Adjoints.  The paper's engine differentiates with respect to the source
 *   intensity and the sensor coordinates (section "Differentiable Acoustic
 *   Radiation").  With r = dL/ds:
 *        dL/da_n   = sum_e sum_k r[e,k] * phi(u)/(2d)                (adjoint, A^T r)
 *        dL/dx_e   = sum_n a_n * sum_k r[e,k] * [phi'(u)/(2d) - phi(u)/(2d^2)] * (x_e - x_n)/d
 *   with u = d - c t_k, phi(u) = u exp(-u^2/2sigma^2),
 *   phi'(u) = (1 - u^2/sigma^2) exp(-u^2/2sigma^2).
 *
 *   Rigid array.  Stage 4 writes the element coordinates of a posed rigid
 *   array as X = R X_template + t; the per-frame pose gradient follows by the
 *   chain rule: dL/dt = sum_m dL/dx_m, dL/dR = sum_m dL/dx_m e_m^T.  For an
 *   axis-angle parameterisation R = exp([w]x) the vector-Jacobian product is
 *   taken through the product rule applied to the Rodrigues formula.
 *
 * Sums use Neumaier compensated summation so that identities such as
 * <A p, r> = <p, A^T r> hold to ~1e-15 relative in tests.
 *
 * OpenMP only splits independent outputs across threads; every output is
 * accumulated in the same order as the serial loop would.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double s, c; } nsum; /* Neumaier accumulator */

static void nadd(nsum* a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double nval(const nsum* a) { return a->s + a->c; }

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the parallel loops (harness control, no arithmetic). */
void or_set_threads(int n) {
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

/* Window of sample indices kept for a source-element distance d: the k in
 * [0, K) with |d - c k/fs| <= trunc*sigma.  Membership is decided by that
 * inequality itself; the bounds below only bracket the search. */
static void window_bracket(double d, double c, double fs, int K, double tsig, long* k0, long* k1) {
    long a = (long)ceil((d - tsig) * fs / c) - 1;
    long b = (long)floor((d + tsig) * fs / c) + 1;
    if (a < 0) a = 0;
    if (b > K - 1) b = K - 1;
    *k0 = a; *k1 = b;
}
static int in_window(double u, double tsig) { return fabs(u) <= tsig; }

/* Source profiles of Appendix A (analytical solutions for typical initial distributions):
 * under the far-field form p ~ (r - v t) p0(|r - v t|) / (2 r), each profile gives a kernel
 * K(x), x = |u|, here normalised to K(0) = 1 with width w (the sampling's sigma field):
 *   0 Gaussian       exp(-x^2 / (2 w^2))
 *   1 exponential    exp(-x / w)
 *   2 power law      (1 + x^2 / w^2)^(-nu)      (the profile A / (r^2 + a^2)^nu, a = w)
 *   3 uniform sphere 1 for x <= w                 (the window is then |u| <= w: trunc = 1)
 * phi(u) = u K(|u|) and phi'(u) = K(x) + x K'(x). */
enum { KER_GAUSS = 0, KER_EXP = 1, KER_POWER = 2, KER_UNIFORM = 3 };

static double kern(int type, double x, double w, double nu) {
    switch (type) {
        case KER_EXP: return exp(-x / w);
        case KER_POWER: return pow(1.0 + (x / w) * (x / w), -nu);
        case KER_UNIFORM: return 1.0;
        default: return exp(-x * x / (2.0 * w * w));
    }
}

/* d phi / du at u (x = |u|): K(x) + x K'(x). */
static double dphi(int type, double x, double w, double nu) {
    const double k = kern(type, x, w, nu);
    switch (type) {
        case KER_EXP: return k * (1.0 - x / w);
        case KER_POWER: return k * (1.0 - 2.0 * nu * x * x / (w * w + x * x));
        case KER_UNIFORM: return 1.0;
        default: return k * (1.0 - x * x / (w * w));
    }
}

/* One term of the sum: a * phi(u) / (2 d). */
static double kernel_term(double a, double u, double d, int type, double w, double nu) {
    double phi = u * kern(type, fabs(u), w, nu);
    return a * phi / (2.0 * d);
}

static double dist3(const double* x, const double* y, double* delta /* x - y, may be NULL */) {
    double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
    if (delta) { delta[0] = dx; delta[1] = dy; delta[2] = dz; }
    return sqrt(dx * dx + dy * dy + dz * dz);
}

/* Element positions of a posed rigid array: x[f,m] = R_f e_m + t_f (Stage 4).
 * poses: [F][12] = R (row-major 3x3) followed by t; elem: [M][3]; xe: [F][M][3]. */
void or_element_positions(int F, const double* poses, int M, const double* elem, double* xe) {
    for (int f = 0; f < F; ++f) {
        const double* R = poses + 12 * f;
        const double* t = R + 9;
        for (int m = 0; m < M; ++m) {
            const double* e = elem + 3 * m;
            double* x = xe + 3 * ((long)f * M + m);
            for (int i = 0; i < 3; ++i)
                x[i] = R[3 * i + 0] * e[0] + R[3 * i + 1] * e[1] + R[3 * i + 2] * e[2] + t[i];
        }
    }
}

/* Forward model, Eq. (1) with the kernel of Eq. (A13):
 * s[e,k] = sum_n amp[n] * phi(d - c t_k) / (2 d),  d = |src_n - xe_e|.
 * src: [N][3], amp: [N], xe: [E][3], s: [E][K] (overwritten). */
void or_forward(long N, const double* src, const double* amp, long E, const double* xe,
                double c, double fs, int K, double sigma, double trunc, int kernel, double nu, double* s) {
    const double tsig = trunc * sigma;
#pragma omp parallel for schedule(dynamic, 1)
    for (long e = 0; e < E; ++e) {
        nsum* acc = (nsum*)calloc((size_t)K, sizeof(nsum));
        for (long n = 0; n < N; ++n) {
            double d = dist3(src + 3 * n, xe + 3 * e, NULL);
            long k0, k1;
            window_bracket(d, c, fs, K, tsig, &k0, &k1);
            for (long k = k0; k <= k1; ++k) {
                double t = (double)k / fs;
                double u = d - c * t;
                if (!in_window(u, tsig)) continue;
                nadd(&acc[k], kernel_term(amp[n], u, d, kernel, sigma, nu));
            }
        }
        for (int k = 0; k < K; ++k) s[e * (long)K + k] = nval(&acc[k]);
        free(acc);
    }
}

/* Same model evaluated without the window bracket: every k in [0, K) is
 * visited and the truncation test alone decides membership.  Used to pin
 * the bracketing logic of or_forward. */
void or_forward_dense(long N, const double* src, const double* amp, long E, const double* xe,
                      double c, double fs, int K, double sigma, double trunc, int kernel, double nu, double* s) {
    const double tsig = trunc * sigma;
    for (long e = 0; e < E; ++e) {
        for (int k = 0; k < K; ++k) {
            nsum acc = {0.0, 0.0};
            for (long n = 0; n < N; ++n) {
                double d = dist3(src + 3 * n, xe + 3 * e, NULL);
                double t = (double)k / fs;
                double u = d - c * t;
                if (!in_window(u, tsig)) continue;
                nadd(&acc, kernel_term(amp[n], u, d, kernel, sigma, nu));
            }
            s[e * (long)K + k] = nval(&acc);
        }
    }
}

/* Adjoint with respect to the source amplitudes (back-projection along
 * spherical shells): g[n] = sum_e sum_k r[e,k] * phi(d - c t_k) / (2 d). */
void or_adjoint_amp(long N, const double* src, long E, const double* xe,
                    double c, double fs, int K, double sigma, double trunc, int kernel, double nu,
                    const double* r, double* g) {
    const double tsig = trunc * sigma;
#pragma omp parallel for schedule(dynamic, 64)
    for (long n = 0; n < N; ++n) {
        nsum acc = {0.0, 0.0};
        for (long e = 0; e < E; ++e) {
            double d = dist3(src + 3 * n, xe + 3 * e, NULL);
            long k0, k1;
            window_bracket(d, c, fs, K, tsig, &k0, &k1);
            for (long k = k0; k <= k1; ++k) {
                double t = (double)k / fs;
                double u = d - c * t;
                if (!in_window(u, tsig)) continue;
                nadd(&acc, kernel_term(r[e * (long)K + k], u, d, kernel, sigma, nu));
            }
        }
        g[n] = nval(&acc);
    }
}

/* Gradient with respect to the element (sensor) coordinates:
 * ge[e] = sum_n amp[n] * (B/(2d) - A/(2d^2)) * (xe_e - src_n)/d,
 * A = sum_k r phi(u), B = sum_k r phi'(u).  ge: [E][3]. */
void or_adjoint_elem(long N, const double* src, const double* amp, long E, const double* xe,
                     double c, double fs, int K, double sigma, double trunc, int kernel, double nu,
                     const double* r, double* ge) {
    const double tsig = trunc * sigma;
#pragma omp parallel for schedule(dynamic, 1)
    for (long e = 0; e < E; ++e) {
        nsum gx = {0, 0}, gy = {0, 0}, gz = {0, 0};
        for (long n = 0; n < N; ++n) {
            double delta[3];
            double d = dist3(xe + 3 * e, src + 3 * n, delta); /* delta = xe - src = d(d)/d(xe) * d */
            long k0, k1;
            window_bracket(d, c, fs, K, tsig, &k0, &k1);
            nsum A = {0, 0}, B = {0, 0};
            for (long k = k0; k <= k1; ++k) {
                double t = (double)k / fs;
                double u = d - c * t;
                if (!in_window(u, tsig)) continue;
                double rk = r[e * (long)K + k];
                nadd(&A, rk * u * kern(kernel, fabs(u), sigma, nu));
                nadd(&B, rk * dphi(kernel, fabs(u), sigma, nu));
            }
            double coef = amp[n] * (nval(&B) / (2.0 * d) - nval(&A) / (2.0 * d * d)) / d;
            nadd(&gx, coef * delta[0]);
            nadd(&gy, coef * delta[1]);
            nadd(&gz, coef * delta[2]);
        }
        ge[3 * e + 0] = nval(&gx);
        ge[3 * e + 1] = nval(&gy);
        ge[3 * e + 2] = nval(&gz);
    }
}

/* Exact count of in-window (source, element, sample) triples. */
long long or_count_updates(long N, const double* src, long E, const double* xe,
                           double c, double fs, int K, double sigma, double trunc, int kernel, double nu) {
    const double tsig = trunc * sigma;
    long long total = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
    for (long e = 0; e < E; ++e) {
        long long cnt = 0;
        for (long n = 0; n < N; ++n) {
            double d = dist3(src + 3 * n, xe + 3 * e, NULL);
            long k0, k1;
            window_bracket(d, c, fs, K, tsig, &k0, &k1);
            for (long k = k0; k <= k1; ++k) {
                double t = (double)k / fs;
                if (in_window(d - c * t, tsig)) ++cnt;
            }
        }
        total += cnt;
    }
    return total;
}

/* Loss of the reconstruction objective (Stage 1, lambda = 0):
 * L = sum (s - y)^2, and r = dL/ds = 2 (s - y).  Returns L. */
double or_loss_residual(long n, const double* s, const double* y, double* r) {
    nsum L = {0, 0};
    for (long i = 0; i < n; ++i) {
        double d = s[i] - y[i];
        nadd(&L, d * d);
        if (r) r[i] = 2.0 * d;
    }
    return nval(&L);
}

/* Chain rule from element gradients to the rigid pose of each frame:
 * gpose[f] = [dL/dR (row-major 3x3), dL/dt], dL/dR = sum_m ge[f,m] e_m^T,
 * dL/dt = sum_m ge[f,m].  ge: [F][M][3], elem: [M][3], gpose: [F][12]. */
void or_pose_grad(int F, int M, const double* elem, const double* ge, double* gpose) {
    for (int f = 0; f < F; ++f) {
        nsum acc[12];
        memset(acc, 0, sizeof(acc));
        for (int m = 0; m < M; ++m) {
            const double* g = ge + 3 * ((long)f * M + m);
            const double* e = elem + 3 * m;
            for (int i = 0; i < 3; ++i) {
                for (int j = 0; j < 3; ++j) nadd(&acc[3 * i + j], g[i] * e[j]);
                nadd(&acc[9 + i], g[i]);
            }
        }
        for (int q = 0; q < 12; ++q) gpose[12 * f + q] = nval(&acc[q]);
    }
}

/* ---- axis-angle rotations ------------------------------------------------
 * R(w) = I + a(th) [w]x + b(th) [w]x^2,  th = |w|,
 * a = sin(th)/th, b = (1 - cos(th))/th^2.
 * Near th = 0 the coefficients come from their Taylor series. */
static void skew(const double* w, double* S) {
    S[0] = 0;     S[1] = -w[2]; S[2] = w[1];
    S[3] = w[2];  S[4] = 0;     S[5] = -w[0];
    S[6] = -w[1]; S[7] = w[0];  S[8] = 0;
}
static void matmul3(const double* A, const double* B, double* C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}
/* a, b and the derivatives a'(th)/th, b'(th)/th. */
static void rodrigues_coefs(double th, double* a, double* b, double* da, double* db) {
    double t2 = th * th;
    if (th < 0.1) {
        *a = 1.0 - t2 / 6.0 + t2 * t2 / 120.0 - t2 * t2 * t2 / 5040.0 + t2 * t2 * t2 * t2 / 362880.0;
        *b = 0.5 - t2 / 24.0 + t2 * t2 / 720.0 - t2 * t2 * t2 / 40320.0 + t2 * t2 * t2 * t2 / 3628800.0;
        *da = -1.0 / 3.0 + t2 / 30.0 - t2 * t2 / 840.0 + t2 * t2 * t2 / 45360.0;
        *db = -1.0 / 12.0 + t2 / 180.0 - t2 * t2 / 6720.0 + t2 * t2 * t2 / 453600.0;
    } else {
        double s = sin(th), c = cos(th);
        *a = s / th;
        *b = (1.0 - c) / t2;
        *da = (th * c - s) / (t2 * th);
        *db = (th * s - 2.0 * (1.0 - c)) / (t2 * t2);
    }
}
void or_rodrigues(const double* w, double* R) {
    double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    double a, b, da, db, S[9], S2[9];
    rodrigues_coefs(th, &a, &b, &da, &db);
    skew(w, S);
    matmul3(S, S, S2);
    for (int i = 0; i < 9; ++i) R[i] = a * S[i] + b * S2[i];
    R[0] += 1.0; R[4] += 1.0; R[8] += 1.0;
}
/* gw[i] = <gR, dR/dw_i>_F with
 * dR/dw_i = a [e_i]x + b([e_i]x[w]x + [w]x[e_i]x) + (a'/th) w_i [w]x + (b'/th) w_i [w]x^2. */
void or_rodrigues_vjp(const double* w, const double* gR, double* gw) {
    double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    double a, b, da, db, S[9], S2[9];
    rodrigues_coefs(th, &a, &b, &da, &db);
    skew(w, S);
    matmul3(S, S, S2);
    for (int i = 0; i < 3; ++i) {
        double ei[3] = {0, 0, 0}, Ei[9], P[9], Q[9], D[9];
        ei[i] = 1.0;
        skew(ei, Ei);
        matmul3(Ei, S, P);
        matmul3(S, Ei, Q);
        for (int q = 0; q < 9; ++q)
            D[q] = a * Ei[q] + b * (P[q] + Q[q]) + da * w[i] * S[q] + db * w[i] * S2[q];
        nsum acc = {0, 0};
        for (int q = 0; q < 9; ++q) nadd(&acc, gR[q] * D[q]);
        gw[i] = nval(&acc);
    }
}

/* Calls every function of the C oracle on small inputs, including empty and clipped cases, for
 * every source profile.  Built with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_oracle_sanitize.py: a run that ends with status 0 and prints no sanitizer report
 * shows the oracle stays inside its buffers and free of undefined behaviour on these inputs. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int or_num_threads(void);
void or_set_threads(int n);
void or_element_positions(int F, const double* poses, int M, const double* elem, double* xe);
void or_forward(long N, const double* src, const double* amp, long E, const double* xe, double c, double fs,
                int K, double sigma, double trunc, int kernel, double nu, double* s);
void or_forward_dense(long N, const double* src, const double* amp, long E, const double* xe, double c,
                      double fs, int K, double sigma, double trunc, int kernel, double nu, double* s);
void or_adjoint_amp(long N, const double* src, long E, const double* xe, double c, double fs, int K,
                    double sigma, double trunc, int kernel, double nu, const double* r, double* g);
void or_adjoint_elem(long N, const double* src, const double* amp, long E, const double* xe, double c, double fs,
                     int K, double sigma, double trunc, int kernel, double nu, const double* r, double* ge);
long long or_count_updates(long N, const double* src, long E, const double* xe, double c, double fs, int K,
                           double sigma, double trunc, int kernel, double nu);
double or_loss_residual(long n, const double* s, const double* y, double* r);
void or_pose_grad(int F, int M, const double* elem, const double* ge, double* gpose);
void or_rodrigues(const double* w, double* R);
void or_rodrigues_vjp(const double* w, const double* gR, double* gw);

static unsigned long long state = 88172645463325252ULL;
static double urand(void) {           /* xorshift64, uniform in [0, 1) */
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0);
}

static double* alloc(long n) {
    double* p = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!p) exit(3);
    for (long i = 0; i < n; ++i) p[i] = 0.0;
    return p;
}

/* One configuration: N sources in a 2 mm cube 8 mm below E elements; records of K samples. */
static double run(long N, long E, int K, int kernel, double trunc, double nu) {
    const double c = 1540.0, fs = 40e6, sigma = 1e-4;
    double *src = alloc(3 * N), *amp = alloc(N), *xe = alloc(3 * E);
    for (long n = 0; n < N; ++n) {
        src[3 * n] = 2e-3 * (urand() - 0.5);
        src[3 * n + 1] = 2e-3 * (urand() - 0.5);
        src[3 * n + 2] = 8e-3 + 2e-3 * urand();
        amp[n] = urand() - 0.3;
    }
    for (long e = 0; e < E; ++e) {
        xe[3 * e] = 3e-4 * (double)e - 3e-3;
        xe[3 * e + 1] = 1e-4 * urand();
        xe[3 * e + 2] = 0.0;
    }
    double *s = alloc(E * K), *sd = alloc(E * K), *y = alloc(E * K), *r = alloc(E * K);
    double *g = alloc(N), *ge = alloc(3 * E);
    or_forward(N, src, amp, E, xe, c, fs, K, sigma, trunc, kernel, nu, s);
    or_forward_dense(N, src, amp, E, xe, c, fs, K, sigma, trunc, kernel, nu, sd);
    for (long i = 0; i < E * K; ++i) y[i] = 0.5 * s[i] + 1e-3 * urand();
    double L = or_loss_residual(E * K, s, y, r);
    or_adjoint_amp(N, src, E, xe, c, fs, K, sigma, trunc, kernel, nu, r, g);
    or_adjoint_elem(N, src, amp, E, xe, c, fs, K, sigma, trunc, kernel, nu, r, ge);
    long long cnt = or_count_updates(N, src, E, xe, c, fs, K, sigma, trunc, kernel, nu);
    double acc = L + (double)cnt;
    for (long i = 0; i < E * K; ++i) acc += fabs(s[i] - sd[i]);
    for (long n = 0; n < N; ++n) acc += g[n];
    for (long i = 0; i < 3 * E; ++i) acc += ge[i];
    free(src); free(amp); free(xe); free(s); free(sd); free(y); free(r); free(g); free(ge);
    return acc;
}

int main(void) {
    or_set_threads(2);
    double acc = (double)or_num_threads();
    const int kernels[4] = {0, 1, 2, 3};
    const double truncs[4] = {6.0, 12.0, 10.0, 1.0};
    for (int q = 0; q < 4; ++q) {
        acc += run(40, 7, 400, kernels[q], truncs[q], 1.5);   /* whole windows inside the record */
        acc += run(40, 7, 280, kernels[q], truncs[q], 2.0);   /* records ending inside the windows */
        acc += run(40, 3, 1, kernels[q], truncs[q], 2.0);     /* one sample: every window clipped */
        acc += run(0, 5, 300, kernels[q], truncs[q], 2.0);    /* no sources */
        acc += run(25, 0, 300, kernels[q], truncs[q], 2.0);   /* no elements */
    }
    /* poses and element positions, the pose gradient, Rodrigues and its VJP (small and zero angles) */
    const int F = 3, M = 4;
    double poses[3 * 12], elem[4 * 3], xe[3 * 4 * 3], ge[3 * 4 * 3], gpose[3 * 12];
    for (int f = 0; f < F; ++f) {
        double w[3] = {0.3 * urand(), f == 1 ? 0.0 : 1e-9 * urand(), 0.2 * urand() - 0.1}, R[9];
        if (f == 2) w[0] = w[1] = w[2] = 0.0;
        or_rodrigues(w, R);
        double gw[3];
        or_rodrigues_vjp(w, R, gw);
        for (int i = 0; i < 9; ++i) poses[12 * f + i] = R[i];
        for (int i = 0; i < 3; ++i) poses[12 * f + 9 + i] = 1e-3 * urand();
        acc += gw[0] + gw[1] + gw[2];
    }
    for (int i = 0; i < 3 * M; ++i) elem[i] = 1e-3 * urand();
    or_element_positions(F, poses, M, elem, xe);
    for (int i = 0; i < 3 * F * M; ++i) ge[i] = urand() - 0.5;
    or_pose_grad(F, M, elem, ge, gpose);
    for (int i = 0; i < 3 * F * M; ++i) acc += xe[i];
    for (int i = 0; i < 12 * F; ++i) acc += gpose[i];
    printf("oracle driver checksum %.17g\n", acc);
    return isfinite(acc) ? 0 : 4;
}

/*
 * Plain FP64 CPU oracle for non-gridding MEM imaging (Carcamo et al.,
 * "Multi-GPU maximum entropy image synthesis for radio astronomy").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code with the GPU path.
 *
 * Every function is a direct sum written straight from its definition:
 * no separable factorisation, no blocking, no recurrences.  All sums are
 * FP64 with Neumaier-compensated accumulation.  OpenMP splits the outer
 * loop only (each output element is summed by one thread, in index order),
 * so results do not depend on the thread count.
 *
 * Conventions (Sec. 2.1; Alg. 3 with x_c = y_c = N/2):
 *   image index p = N*i + j, row i <-> y, column j <-> x,
 *   x_j = (j - N/2) * cell, y_i = (i - N/2) * cell   (cell in radians),
 *   u, v in wavelengths.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TWO_PI 6.283185307179586476925286766559

/* Neumaier compensated summation. */
typedef struct { double s, c; } nsum;
static inline void nadd(nsum *a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static inline double nval(const nsum *a) { return a->s + a->c; }

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Angle 2*pi*theta evaluated as 2*pi*f with f = theta - rint(theta) in
 * [-1/2, 1/2]: the phase is reduced modulo one cycle in FP64 before the
 * trigonometric call (the exponent of Eq. fft is periodic in theta). */
static inline void cis(double theta, double *c, double *s) {
    double f = theta - nearbyint(theta);
    double a = TWO_PI * f;
    *c = cos(a);
    *s = sin(a);
}

/* Primary beam A_ij = exp(-4 ln2 (x_j^2 + y_i^2) / fwhm^2): a Gaussian of the
 * given FWHM centred on the phase centre (Sec. 2.4 item 1), so A = 1 at
 * pixel (N/2, N/2). */
void or_beam(int n, double cell, double fwhm, double *A) {
    const double k = 4.0 * log(2.0) / (fwhm * fwhm);
    for (int i = 0; i < n; ++i) {
        double y = (double)(i - n / 2) * cell;
        for (int j = 0; j < n; ++j) {
            double x = (double)(j - n / 2) * cell;
            A[(size_t)i * n + j] = exp(-k * (x * x + y * y));
        }
    }
}

/* Forward model, Eq. fft discretised at the measured (u, v):
 *   V_k = sum_{i,j} A_ij I_ij exp(-2 pi i (u_k x_j + v_k y_i)).
 * A may be NULL (A = 1).  V is interleaved complex [nvis][2]. */
void or_forward(int n, double cell, int64_t nvis, const double *u, const double *v,
                const double *A, const double *I, double *V) {
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nvis; ++k) {
        nsum re = {0, 0}, im = {0, 0};
        for (int i = 0; i < n; ++i) {
            double y = (double)(i - n / 2) * cell;
            for (int j = 0; j < n; ++j) {
                double x = (double)(j - n / 2) * cell;
                size_t p = (size_t)i * n + j;
                double b = (A ? A[p] : 1.0) * I[p];
                double c, s;
                cis(u[k] * x + v[k] * y, &c, &s);
                nadd(&re, b * c);
                nadd(&im, -b * s);
            }
        }
        V[2 * k] = nval(&re);
        V[2 * k + 1] = nval(&im);
    }
}

/* Adjoint of the forward model applied to complex weights c_k:
 *   G_ij = A_ij sum_k Re( c_k exp(+2 pi i (u_k x_j + v_k y_i)) )
 * With c_k = w_k R_k this is the chi^2 gradient, Eq. chi2gradient (and the
 * sum of Alg. 3), multiplied by the A_ij that the exact derivative of the
 * attenuated forward model carries (App. C drops it as an approximation).
 * Pixels are the outer loop.  npix_sel < 0 means every pixel (G is N*N);
 * otherwise only the listed linear pixel indices, written to G[0..npix_sel). */
void or_adjoint(int n, double cell, int64_t nvis, const double *u, const double *v,
                const double *A, const double *cw, int64_t npix_sel, const int64_t *pix,
                double *G) {
    int64_t np = npix_sel < 0 ? (int64_t)n * n : npix_sel;
    #pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < np; ++q) {
        int64_t p = npix_sel < 0 ? q : pix[q];
        int i = (int)(p / n), j = (int)(p % n);
        double x = (double)(j - n / 2) * cell;
        double y = (double)(i - n / 2) * cell;
        nsum g = {0, 0};
        for (int64_t k = 0; k < nvis; ++k) {
            double c, s;
            cis(u[k] * x + v[k] * y, &c, &s);
            nadd(&g, cw[2 * k] * c - cw[2 * k + 1] * s);
        }
        G[q] = (A ? A[p] : 1.0) * nval(&g);
    }
}

/* Forward model at a subset of visibilities only (sampled parity checks at
 * full size): V[q] = V_{idx[q]}. */
void or_forward_sel(int n, double cell, int64_t nsel, const int64_t *idx,
                    const double *u, const double *v, const double *A, const double *I,
                    double *V) {
    #pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < nsel; ++q) {
        int64_t k = idx[q];
        nsum re = {0, 0}, im = {0, 0};
        for (int i = 0; i < n; ++i) {
            double y = (double)(i - n / 2) * cell;
            for (int j = 0; j < n; ++j) {
                double x = (double)(j - n / 2) * cell;
                size_t p = (size_t)i * n + j;
                double b = (A ? A[p] : 1.0) * I[p];
                double c, s;
                cis(u[k] * x + v[k] * y, &c, &s);
                nadd(&re, b * c);
                nadd(&im, -b * s);
            }
        }
        V[2 * q] = nval(&re);
        V[2 * q + 1] = nval(&im);
    }
}

/* Forward model of an image that is zero except at the listed pixels
 * (Eq. fft with the sum restricted to its nonzero terms):
 *   V_k = sum_q A_{p_q} val_q exp(-2 pi i (u_k x_{j_q} + v_k y_{i_q})),
 * p_q = N i_q + j_q.  Used to evaluate the model at a one-pixel change of an
 * image by linearity, V(I + h e_p) = V(I) + h V(e_p). */
void or_forward_pix(int n, double cell, int64_t nvis, const double *u, const double *v,
                    const double *A, int64_t npix, const int64_t *pix, const double *val, double *V) {
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nvis; ++k) {
        nsum re = {0, 0}, im = {0, 0};
        for (int64_t q = 0; q < npix; ++q) {
            int64_t p = pix[q];
            int i = (int)(p / n), j = (int)(p % n);
            double x = (double)(j - n / 2) * cell;
            double y = (double)(i - n / 2) * cell;
            double b = (A ? A[p] : 1.0) * val[q];
            double c, s;
            cis(u[k] * x + v[k] * y, &c, &s);
            nadd(&re, b * c);
            nadd(&im, -b * s);
        }
        V[2 * k] = nval(&re);
        V[2 * k + 1] = nval(&im);
    }
}

/* chi^2 = 1/2 sum_k w_k |V_k - Vo_k|^2  (Eq. phi2; Alg. 2 gives the per-term
 * residual V^R = V^m - V^o).  R (may be NULL) receives the residuals. */
double or_chi2(int64_t nvis, const double *V, const double *Vo, const double *w, double *R) {
    nsum acc = {0, 0};
    for (int64_t k = 0; k < nvis; ++k) {
        double rr = V[2 * k] - Vo[2 * k];
        double ri = V[2 * k + 1] - Vo[2 * k + 1];
        if (R) { R[2 * k] = rr; R[2 * k + 1] = ri; }
        nadd(&acc, w[k] * (rr * rr + ri * ri));
    }
    return 0.5 * nval(&acc);
}

/* Entropy term S = sum_p I_p ln(I_p / M) and its gradient ln(I_p/M) + 1
 * (Eq. Sgradient; the objective's regulariser written with the gradient's
 * normalisation, M playing the role of G).  Returns NAN if any I_p <= 0. */
double or_entropy(int64_t npix, const double *I, double M, double *grad) {
    nsum acc = {0, 0};
    int bad = 0;
    for (int64_t p = 0; p < npix; ++p) {
        if (!(I[p] > 0.0)) { bad = 1; if (grad) grad[p] = NAN; continue; }
        double l = log(I[p] / M);
        nadd(&acc, I[p] * l);
        if (grad) grad[p] = l + 1.0;
    }
    return bad ? NAN : nval(&acc);
}

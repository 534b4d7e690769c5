/*
 * CPU oracle for FFT-based circular convolution (Venkovic & Anzt,
 * "Permutation-Avoiding FFT-Based Convolution", arXiv 2506.12718).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library, and it is deliberately
 * plain: no blocking, no fusion, no reordering beyond what the paper's
 * definitions state.  Complex arrays are interleaved (re, im) doubles,
 * row-major with the last index fastest (Sec. "Multi-dimensional problem",
 * definition of vec).
 *
 * Contents
 *   orc_conv_direct     the definition of circular convolution, summed
 *                       directly (Sec. "1D problem", eq. convolution; its
 *                       d-way form, eq. convolution-multi-dimensional),
 *                       accumulated in long double.
 *   orc_conv_direct_at  the same sum for selected output entries only.
 *   orc_perm_index      the index-reversal permutation P_rho built from its
 *                       definition as a product of modulo-r perfect shuffles
 *                       (Sec. "Mixed-radix framework"; for uniform radix it is
 *                       the product of modulo-r sorts, eq. r-ary-sorting).
 *   orc_fft             the paper's *standard* ordered FFT along every axis:
 *                       explicit permutation P_rho^T, then the butterfly
 *                       stages A_rho, q = 1..t (Alg. alg:forward-fft, FFT
 *                       branch, with the stage loop of
 *                       Alg. alg:butterfly-related-kernel and the butterfly
 *                       matrix of eq. 25); the inverse is conj(A_rho) P_rho^T/n
 *                       (Alg. alg:backward-fft).
 *   orc_conv_fft        standard FFT-based convolution, three permutations
 *                       per evaluation (Alg. alg:fft-based-convolution).
 *
 * Twiddles are evaluated inline from cosl/sinl of the integer-reduced angle;
 * no table is kept.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.141592653589793238462643383279502884L

/* omega_n^e = exp(-2 pi i e / n) (Sec. "1D problem"), e reduced mod n. */
static void orc_omega(int64_t n, int64_t e, long double *c, long double *s)
{
    int64_t r = e % n;
    if (r < 0) r += n;
    long double a = -2.0L * ORC_PI * (long double)r / (long double)n;
    *c = cosl(a);
    *s = sinl(a);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int64_t prod_dims(int ndim, const int64_t *dims)
{
    int64_t n = 1;
    for (int a = 0; a < ndim; ++a) n *= dims[a];
    return n;
}

/* ------------------------------------------------------------------ */
/* O1: direct circular convolution                                      */
/* y_j = sum_k x_k h_{(j-k) mod n}, per axis in d-D.                    */
/* ------------------------------------------------------------------ */

static void conv_one(int ndim, const int64_t *dims, const double *x,
                     const double *h, int64_t j, double *out)
{
    int64_t N = prod_dims(ndim, dims);
    int64_t jd[3] = {0, 0, 0}, kd[3] = {0, 0, 0};
    int64_t t = j;
    for (int a = ndim - 1; a >= 0; --a) { jd[a] = t % dims[a]; t /= dims[a]; }
    long double sr = 0.0L, si = 0.0L;
    for (int64_t k = 0; k < N; ++k) {
        /* index of h at (j - k) mod n, per axis */
        int64_t hi = 0;
        for (int a = 0; a < ndim; ++a) {
            int64_t d = jd[a] - kd[a];
            if (d < 0) d += dims[a];
            hi = hi * dims[a] + d;
        }
        long double xr = x[2 * k], xi = x[2 * k + 1];
        long double hr = h[2 * hi], hm = h[2 * hi + 1];
        sr += xr * hr - xi * hm;
        si += xr * hm + xi * hr;
        /* advance the multi-index of k (last axis fastest) */
        for (int a = ndim - 1; a >= 0; --a) {
            if (++kd[a] < dims[a]) break;
            kd[a] = 0;
        }
    }
    out[0] = (double)sr;
    out[1] = (double)si;
}

int orc_conv_direct(int ndim, const int64_t *dims, const double *x,
                    const double *h, double *y)
{
    if (ndim < 1 || ndim > 3) return -1;
    int64_t N = prod_dims(ndim, dims);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < N; ++j) conv_one(ndim, dims, x, h, j, y + 2 * j);
    return 0;
}

int orc_conv_direct_at(int ndim, const int64_t *dims, const double *x,
                       const double *h, int64_t nidx, const int64_t *idx,
                       double *out)
{
    if (ndim < 1 || ndim > 3) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nidx; ++i)
        conv_one(ndim, dims, x, h, idx[i], out + 2 * i);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Index-reversal permutation P_rho (Sec. "Mixed-radix framework").    */
/*                                                                      */
/* P_rho = Pi_{r_t,n} (I (x) Pi_{r_{t-1},k_{t-1}}) ... (I (x) Pi_{r_1,r_1})*/
/* with k_q = r_1...r_q and Pi_{r,m} the modulo-r perfect shuffle, the  */
/* inverse of the modulo-r sort R_{r,m} of eq. r-ary-sorting:           */
/*   (R_{r,m} x)[a*(m/r) + b] = x[b*r + a],  a < r, b < m/r.            */
/* The routine returns perm[] with (P_rho z)[i] = z[perm[i]].           */
/* ------------------------------------------------------------------ */

/* Apply z <- (I_{n/m} (x) Pi_{r,m}) z to an index vector. */
static void apply_shuffle(int64_t n, int64_t m, int64_t r, int64_t *z, int64_t *tmp)
{
    int64_t mr = m / r;
    for (int64_t blk = 0; blk < n; blk += m)
        for (int64_t a = 0; a < r; ++a)
            for (int64_t b = 0; b < mr; ++b)
                tmp[blk + b * r + a] = z[blk + a * mr + b];  /* Pi = R^{-1} */
    memcpy(z, tmp, (size_t)n * sizeof(int64_t));
}

int orc_perm_index(int64_t n, int t, const int *rho, int64_t *perm)
{
    int64_t prod = 1;
    for (int q = 0; q < t; ++q) {
        if (rho[q] < 2 || rho[q] > 16) return -1;
        prod *= rho[q];
    }
    if (prod != n) return -1;
    int64_t *tmp = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!tmp) return -2;
    /* Track where each entry of z lands: start with z = identity, so that
       after applying the product, perm[i] = source index of entry i. */
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    /* rightmost factor first: I_{n/r_1} (x) Pi_{r_1,r_1}, ..., Pi_{r_t,n} */
    int64_t k = 1;
    for (int q = 0; q < t; ++q) {
        k *= rho[q];
        apply_shuffle(n, k, rho[q], perm, tmp);
    }
    free(tmp);
    return 0;
}

/* ------------------------------------------------------------------ */
/* O2: the standard ordered FFT (explicit permutation + butterflies).  */
/* ------------------------------------------------------------------ */

/* u <- A_rho u (or conj(A_rho) u): stages q = 1..t, block k_q = r_1..r_q,
   (B_{r,k} x)[m*(k/r) + j] = sum_p w_r^{m p} w_k^{p j} x[p*(k/r) + j]
   (eq. 25 with Omega_{r,k/r} = diag(w_k^j)); conj flips every twiddle.
   The twiddles of a stage are evaluated once per stage into tw[] (hoisted
   out of the block loop; nothing is kept across calls). */
static void butterflies(int64_t n, int t, const int *rho, int conj, double *u,
                        double *tmp, long double *tw)
{
    int64_t k = 1;
    for (int q = 0; q < t; ++q) {
        int64_t r = rho[q];
        k *= r;
        int64_t m = k / r;
        long double fr[2 * 16 * 16];        /* w_r^{mo p}, r <= 16 */
        for (int64_t mo = 0; mo < r; ++mo)
            for (int64_t p = 0; p < r; ++p)
                orc_omega(r, mo * p, &fr[2 * (mo * r + p)], &fr[2 * (mo * r + p) + 1]);
        for (int64_t p = 0; p < r; ++p)     /* w_k^{p j} */
            for (int64_t j = 0; j < m; ++j)
                orc_omega(k, p * j, &tw[2 * (p * m + j)], &tw[2 * (p * m + j) + 1]);
        for (int64_t b = 0; b < n; b += k) {
            for (int64_t j = 0; j < m; ++j) {
                for (int64_t mo = 0; mo < r; ++mo) {
                    long double sr = 0.0L, si = 0.0L;
                    for (int64_t p = 0; p < r; ++p) {
                        long double c1 = tw[2 * (p * m + j)], s1 = tw[2 * (p * m + j) + 1];
                        long double c2 = fr[2 * (mo * r + p)], s2 = fr[2 * (mo * r + p) + 1];
                        long double wr = c1 * c2 - s1 * s2;
                        long double wi = c1 * s2 + s1 * c2;
                        if (conj) wi = -wi;
                        long double xr = u[2 * (b + p * m + j)];
                        long double xi = u[2 * (b + p * m + j) + 1];
                        sr += wr * xr - wi * xi;
                        si += wr * xi + wi * xr;
                    }
                    tmp[2 * (b + mo * m + j)] = (double)sr;
                    tmp[2 * (b + mo * m + j) + 1] = (double)si;
                }
            }
        }
        memcpy(u, tmp, (size_t)n * 2 * sizeof(double));
    }
}

/* One pencil: v <- F v (dir = -1) or F^{-1} v (dir = +1), with
   F = A_rho P_rho^T and F^{-1} = conj(A_rho) P_rho^T / n. */
static void fft_pencil(int64_t n, int t, const int *rho, const int64_t *perm,
                       int dir, double *v, double *u, double *tmp,
                       long double *tw)
{
    /* u = P_rho^T v:  (P z)[i] = z[perm[i]]  =>  (P^T v)[perm[i]] = v[i] */
    for (int64_t i = 0; i < n; ++i) {
        u[2 * perm[i]] = v[2 * i];
        u[2 * perm[i] + 1] = v[2 * i + 1];
    }
    butterflies(n, t, rho, dir > 0, u, tmp, tw);
    double s = dir > 0 ? 1.0 / (double)n : 1.0;
    for (int64_t i = 0; i < 2 * n; ++i) v[i] = u[i] * s;
}

/* rho_flat holds the radix sequences of the axes back to back, rho_len[a]
   entries for axis a, each listed r_1 first (innermost stage first). */
int orc_fft(int ndim, const int64_t *dims, const int *rho_flat,
            const int *rho_len, int dir, double *data)
{
    if (ndim < 1 || ndim > 3) return -1;
    int64_t N = prod_dims(ndim, dims);
    int off = 0;
    /* last axis first, as in Alg. alg:uFFT3D; the axes commute */
    int offs[3];
    for (int a = 0; a < ndim; ++a) { offs[a] = off; off += rho_len[a]; }
    for (int a = ndim - 1; a >= 0; --a) {
        int64_t n = dims[a];
        const int *rho = rho_flat + offs[a];
        int t = rho_len[a];
        int64_t *perm = (int64_t *)malloc((size_t)n * sizeof(int64_t));
        if (!perm) return -2;
        if (orc_perm_index(n, t, rho, perm) != 0) { free(perm); return -3; }
        int64_t stride = 1;
        for (int b = a + 1; b < ndim; ++b) stride *= dims[b];
        int64_t npencil = N / n;
        int err = 0;
#pragma omp parallel
        {
            double *v = (double *)malloc((size_t)n * 2 * sizeof(double));
            double *u = (double *)malloc((size_t)n * 2 * sizeof(double));
            double *tmp = (double *)malloc((size_t)n * 2 * sizeof(double));
            long double *tw = (long double *)malloc((size_t)n * 2 * sizeof(long double));
            if (!v || !u || !tmp || !tw) {
#pragma omp atomic write
                err = 1;
            } else {
#pragma omp for schedule(static)
                for (int64_t pcl = 0; pcl < npencil; ++pcl) {
                    int64_t outer = pcl / stride, inner = pcl % stride;
                    int64_t base = outer * n * stride + inner;
                    for (int64_t i = 0; i < n; ++i) {
                        v[2 * i] = data[2 * (base + i * stride)];
                        v[2 * i + 1] = data[2 * (base + i * stride) + 1];
                    }
                    fft_pencil(n, t, rho, perm, dir, v, u, tmp, tw);
                    for (int64_t i = 0; i < n; ++i) {
                        data[2 * (base + i * stride)] = v[2 * i];
                        data[2 * (base + i * stride) + 1] = v[2 * i + 1];
                    }
                }
            }
            free(v); free(u); free(tmp); free(tw);
        }
        free(perm);
        if (err) return -2;
    }
    return 0;
}

/* Standard FFT-based convolution (Alg. alg:fft-based-convolution):
   h := FFT(h), x := FFT(x), x := h o x, return iFFT(x).  x and h are not
   modified; y receives the result. */
int orc_conv_fft(int ndim, const int64_t *dims, const int *rho_flat,
                 const int *rho_len, const double *x, const double *h,
                 double *y)
{
    int64_t N = prod_dims(ndim, dims);
    double *hh = (double *)malloc((size_t)N * 2 * sizeof(double));
    if (!hh) return -2;
    memcpy(hh, h, (size_t)N * 2 * sizeof(double));
    memcpy(y, x, (size_t)N * 2 * sizeof(double));
    int rc = orc_fft(ndim, dims, rho_flat, rho_len, -1, hh);
    if (rc == 0) rc = orc_fft(ndim, dims, rho_flat, rho_len, -1, y);
    if (rc == 0) {
        for (int64_t i = 0; i < N; ++i) {
            double ar = y[2 * i], ai = y[2 * i + 1];
            double br = hh[2 * i], bi = hh[2 * i + 1];
            y[2 * i] = ar * br - ai * bi;
            y[2 * i + 1] = ar * bi + ai * br;
        }
        rc = orc_fft(ndim, dims, rho_flat, rho_len, +1, y);
    }
    free(hh);
    return rc;
}

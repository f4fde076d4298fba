/*
 * Plain FP64 stencil loops: the oracle for the FFT stencil solver.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg use it.  It shares no code, header or table with the HIP library.
 *
 * What it computes is the plain definition of the result, not the FFT algorithm:
 *
 *  - periodic:  T sweeps of the nested-loop periodic update (the periodic looping
 *    algorithm of the paper's looping-code figure, extended to d dimensions as in
 *    the appendix on d-D grids): every cell i gets
 *        b[i] = sum over offsets o in [-r, r]^d, row-major order, of c[o] * a[(i + o) mod n]
 *    accumulated in double from +0.0, multiply then add (build with
 *    -ffp-contract=off so no fused multiply-add changes the rounding);
 *
 *  - aperiodic: the same on an array whose extents are n_i + 2r; the outer r-wide
 *    frame holds fixed (Dirichlet) boundary values and is copied unchanged each step;
 *    interior cells use the same sum without the modulo (the aperiodic looping
 *    algorithm of the same figure, with r boundary cells on each side).
 *    With the reflecting (zero-flux, Neumann) boundary instead, the frame is
 *    refilled before every step as the mirror image of the interior: along each
 *    axis, frame cell r-1-k takes the value of interior cell r+k and frame cell
 *    n+r+k that of n+r-1-k (the even extension of the grid about the cell faces),
 *    corners mirrored along every axis they lie outside of; Sec. 4 lists such
 *    boundaries among those the base case may apply.
 *
 *  - periodic fields: m scalar fields a^(0..m-1) on the same periodic grid, each
 *    step computing b^(i)[x] = sum over j (field order), then over offsets o (row-major),
 *    of c^(i,j)[o] * a^(j)[(x + o) mod n] (the vector-valued extension: every field
 *    at t+1 is a sum of stencils applied to every field at t).
 *
 * Coefficients are a (2r+1)^d row-major array; c[o] multiplies the neighbour at
 * offset +o (the periodic loop's S[i, (i + j) % N] convention).  Sweeps are double
 * buffered; OpenMP splits the outermost spatial index, which does not change any
 * result because each cell is computed by one thread in a fixed order.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int64_t wrap(int64_t i, int64_t n) {
    int64_t m = i % n;
    return m < 0 ? m + n : m;
}

/* Expand (ndim, dims, r) to three axes; missing leading axes have extent 1 and radius 0. */
static void expand3(int ndim, const int64_t* dims, int r, int64_t n[3], int rr[3]) {
    for (int k = 0; k < 3; ++k) { n[k] = 1; rr[k] = 0; }
    for (int k = 0; k < ndim; ++k) { n[3 - ndim + k] = dims[k]; rr[3 - ndim + k] = r; }
}

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* a: prod(dims) doubles, overwritten with the state after T periodic sweeps. */
int oracle_periodic(double* a, int ndim, const int64_t* dims, const double* coeffs,
                    int r, int64_t T, int nthreads) {
    if (ndim < 1 || ndim > 3 || r < 0 || T < 0 || !a || !dims || !coeffs) return -1;
    int64_t n[3]; int rr[3];
    expand3(ndim, dims, r, n, rr);
    for (int k = 0; k < 3; ++k) if (n[k] < 1) return -1;
    const int64_t N = n[0] * n[1] * n[2];
    const int w0 = 2 * rr[0] + 1, w1 = 2 * rr[1] + 1, w2 = 2 * rr[2] + 1;
    double* b = (double*)malloc(sizeof(double) * (size_t)N);
    if (!b) return -3;
    double* src = a;
    double* dst = b;
    if (nthreads <= 0) nthreads = oracle_threads();
    for (int64_t t = 0; t < T; ++t) {
#pragma omp parallel for collapse(3) schedule(static) num_threads(nthreads)
        for (int64_t i0 = 0; i0 < n[0]; ++i0) {
            for (int64_t i1 = 0; i1 < n[1]; ++i1) {
                for (int64_t i2 = 0; i2 < n[2]; ++i2) {
                    double acc = 0.0;
                    for (int o0 = -rr[0]; o0 <= rr[0]; ++o0) {
                        const int64_t j0 = wrap(i0 + o0, n[0]);
                        for (int o1 = -rr[1]; o1 <= rr[1]; ++o1) {
                            const int64_t j1 = wrap(i1 + o1, n[1]);
                            for (int o2 = -rr[2]; o2 <= rr[2]; ++o2) {
                                const int64_t j2 = wrap(i2 + o2, n[2]);
                                const double c = coeffs[((o0 + rr[0]) * w1 + (o1 + rr[1])) * w2 + (o2 + rr[2])];
                                const double prod = c * src[(j0 * n[1] + j1) * n[2] + j2];
                                acc = acc + prod;
                            }
                        }
                    }
                    dst[(i0 * n[1] + i1) * n[2] + i2] = acc;
                }
            }
        }
        double* tmp = src; src = dst; dst = tmp;
    }
    (void)w0;
    if (src != a) memcpy(a, src, sizeof(double) * (size_t)N);
    free(b);
    return 0;
}

/* Mirror image of storage coordinate g along an axis with interior extent n and
 * frame width r: frame cells reflect about the nearer cell face, interior cells
 * map to themselves. */
static int64_t mirror(int64_t g, int64_t n, int r) {
    if (g < r) return 2 * (int64_t)r - 1 - g;
    if (g >= n + r) return 2 * (n + r) - 1 - g;
    return g;
}

/* a: prod(dims[k] + 2r) doubles (interior plus an r-wide frame on every side);
 * the interior evolves T steps.  bc 0: the frame holds fixed values and is left
 * unchanged.  bc 1: reflecting boundary; the frame's input values are ignored and
 * on return it holds the mirror image of the final interior (every interior
 * extent must be at least r, so that each mirror image lies inside). */
int oracle_aperiodic_bc(double* a, int ndim, const int64_t* dims, const double* coeffs,
                        int r, int64_t T, int bc, int nthreads) {
    if (ndim < 1 || ndim > 3 || r < 0 || T < 0 || !a || !dims || !coeffs) return -1;
    if (bc != 0 && bc != 1) return -1;
    int64_t n[3]; int rr[3];
    expand3(ndim, dims, r, n, rr);
    for (int k = 0; k < 3; ++k) if (n[k] < 1) return -1;
    if (bc == 1)
        for (int k = 0; k < ndim; ++k) if (dims[k] < r) return -1;
    int64_t s[3]; /* storage extents */
    for (int k = 0; k < 3; ++k) s[k] = n[k] + 2 * rr[k];
    const int64_t S = s[0] * s[1] * s[2];
    const int w1 = 2 * rr[1] + 1, w2 = 2 * rr[2] + 1;
    double* b = (double*)malloc(sizeof(double) * (size_t)S);
    if (!b) return -3;
    memcpy(b, a, sizeof(double) * (size_t)S); /* frame values in both buffers */
    double* src = a;
    double* dst = b;
    if (nthreads <= 0) nthreads = oracle_threads();
    for (int64_t t = 0; t <= T; ++t) {
        if (bc == 1) {
            /* frame of the current state := mirror image of its interior */
            for (int64_t i0 = 0; i0 < s[0]; ++i0)
                for (int64_t i1 = 0; i1 < s[1]; ++i1)
                    for (int64_t i2 = 0; i2 < s[2]; ++i2) {
                        const int64_t m0 = mirror(i0, n[0], rr[0]), m1 = mirror(i1, n[1], rr[1]),
                                      m2 = mirror(i2, n[2], rr[2]);
                        if (m0 != i0 || m1 != i1 || m2 != i2)
                            src[(i0 * s[1] + i1) * s[2] + i2] = src[(m0 * s[1] + m1) * s[2] + m2];
                    }
        }
        if (t == T) break;
#pragma omp parallel for collapse(3) schedule(static) num_threads(nthreads)
        for (int64_t i0 = rr[0]; i0 < rr[0] + n[0]; ++i0) {
            for (int64_t i1 = rr[1]; i1 < rr[1] + n[1]; ++i1) {
                for (int64_t i2 = rr[2]; i2 < rr[2] + n[2]; ++i2) {
                    double acc = 0.0;
                    for (int o0 = -rr[0]; o0 <= rr[0]; ++o0) {
                        for (int o1 = -rr[1]; o1 <= rr[1]; ++o1) {
                            for (int o2 = -rr[2]; o2 <= rr[2]; ++o2) {
                                const double c = coeffs[((o0 + rr[0]) * w1 + (o1 + rr[1])) * w2 + (o2 + rr[2])];
                                const double prod = c * src[((i0 + o0) * s[1] + (i1 + o1)) * s[2] + (i2 + o2)];
                                acc = acc + prod;
                            }
                        }
                    }
                    dst[(i0 * s[1] + i1) * s[2] + i2] = acc;
                }
            }
        }
        double* tmp = src; src = dst; dst = tmp;
    }
    if (src != a) memcpy(a, src, sizeof(double) * (size_t)S);
    free(b);
    return 0;
}

int oracle_aperiodic(double* a, int ndim, const int64_t* dims, const double* coeffs,
                     int r, int64_t T, int nthreads) {
    return oracle_aperiodic_bc(a, ndim, dims, coeffs, r, T, 0, nthreads);
}

/* a: m * prod(dims) doubles, field-major ([m][dims...]), overwritten with the state
 * after T sweeps; coeffs: m * m * (2r+1)^d doubles ([i][j][offsets...]), block
 * (i, j) applied to field j contributes to field i. */
int oracle_periodic_fields(double* a, int m, int ndim, const int64_t* dims, const double* coeffs,
                           int r, int64_t T, int nthreads) {
    if (m < 1 || ndim < 1 || ndim > 3 || r < 0 || T < 0 || !a || !dims || !coeffs) return -1;
    int64_t n[3]; int rr[3];
    expand3(ndim, dims, r, n, rr);
    for (int k = 0; k < 3; ++k) if (n[k] < 1) return -1;
    const int64_t N = n[0] * n[1] * n[2];
    const int w0 = 2 * rr[0] + 1, w1 = 2 * rr[1] + 1, w2 = 2 * rr[2] + 1;
    const int64_t nc = (int64_t)w0 * w1 * w2;
    double* b = (double*)malloc(sizeof(double) * (size_t)(N * m));
    if (!b) return -3;
    double* src = a;
    double* dst = b;
    if (nthreads <= 0) nthreads = oracle_threads();
    for (int64_t t = 0; t < T; ++t) {
        for (int i = 0; i < m; ++i) {
#pragma omp parallel for collapse(3) schedule(static) num_threads(nthreads)
            for (int64_t i0 = 0; i0 < n[0]; ++i0) {
                for (int64_t i1 = 0; i1 < n[1]; ++i1) {
                    for (int64_t i2 = 0; i2 < n[2]; ++i2) {
                        double acc = 0.0;
                        for (int j = 0; j < m; ++j) {
                            const double* cij = coeffs + ((int64_t)i * m + j) * nc;
                            const double* aj = src + (int64_t)j * N;
                            for (int o0 = -rr[0]; o0 <= rr[0]; ++o0) {
                                const int64_t j0 = wrap(i0 + o0, n[0]);
                                for (int o1 = -rr[1]; o1 <= rr[1]; ++o1) {
                                    const int64_t j1 = wrap(i1 + o1, n[1]);
                                    for (int o2 = -rr[2]; o2 <= rr[2]; ++o2) {
                                        const int64_t j2 = wrap(i2 + o2, n[2]);
                                        const double c = cij[((o0 + rr[0]) * w1 + (o1 + rr[1])) * w2 + (o2 + rr[2])];
                                        const double prod = c * aj[(j0 * n[1] + j1) * n[2] + j2];
                                        acc = acc + prod;
                                    }
                                }
                            }
                        }
                        dst[(int64_t)i * N + (i0 * n[1] + i1) * n[2] + i2] = acc;
                    }
                }
            }
        }
        double* tmp = src; src = dst; dst = tmp;
    }
    if (src != a) memcpy(a, src, sizeof(double) * (size_t)(N * m));
    free(b);
    return 0;
}

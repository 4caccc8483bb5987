/*
 * Seeded synthetic inputs for the Wilson-Dirac solver: SU(3) gauge links,
 * Gaussian and point sources, random SU(3) gauge transformations.
 *
 * This file is input generation only.  It contains none of the solver's
 * arithmetic (no Dirac operator, no Krylov step, no rescaling); both the
 * CPU oracle and the GPU path receive the arrays it fills.
 *
 * Random numbers: the counter-based form of SplitMix64 (G. Steele, D. Lea,
 * C. Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014;
 * the 64-bit finaliser constants are those published with S. Vigna's
 * splitmix64.c).  Draw n of stream `seed` is mix(key(seed) + (n+1)*G), so
 * every value depends only on (seed, n) and never on thread count or order.
 * Normals come from the Box-Muller transform (Box & Muller 1958).
 *
 * Canonical layouts (complex128, interleaved re/im):
 *   site index  s = x + Lx*(y + Ly*(z + Lz*t)),   mu = 0..3 is x,y,z,t
 *   links       U[s][mu][a][b]     (link from s to s+mu)
 *   spinor      psi[s][spin][colour]
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define GOLDEN 0x9e3779b97f4a7c15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static inline uint64_t stream_key(uint64_t seed) { return mix64(seed + GOLDEN); }

/* draw n of the stream with key k */
static inline uint64_t draw(uint64_t k, uint64_t n) { return mix64(k + (n + 1) * GOLDEN); }

/* uniform in (0, 1]: 53 random bits, never zero so log() is finite */
static inline double unif(uint64_t k, uint64_t n) {
    return (double)((draw(k, n) >> 11) + 1) * (1.0 / 9007199254740992.0);
}

/* Box-Muller: draws n, n+1 give two independent N(0,1) values */
static inline void box_muller(uint64_t k, uint64_t n, double *g0, double *g1) {
    double u1 = unif(k, n), u2 = unif(k, n + 1);
    double r = sqrt(-2.0 * log(u1));
    double th = 6.283185307179586476925286766559 * u2;
    *g0 = r * cos(th);
    *g1 = r * sin(th);
}

typedef struct { double re, im; } cplx;

static inline cplx cmul(cplx a, cplx b) { cplx c = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; return c; }

/* 3x3 complex product C = A B */
static void mat_mul(const cplx A[9], const cplx B[9], cplx C[9]) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cplx s = {0, 0};
            for (int k = 0; k < 3; k++) {
                cplx p = cmul(A[3 * i + k], B[3 * k + j]);
                s.re += p.re; s.im += p.im;
            }
            C[3 * i + j] = s;
        }
}

/* Hermitian traceless H = sum_a c_a lambda_a with the Gell-Mann matrices
 * (normalised tr lambda_a lambda_b = 2 delta_ab). */
static void gell_mann_combination(const double c[8], cplx H[9]) {
    const double r3 = 0.57735026918962576451; /* 1/sqrt(3) */
    memset(H, 0, 9 * sizeof(cplx));
    /* diagonal: lambda_3 = diag(1,-1,0), lambda_8 = diag(1,1,-2)/sqrt3 */
    H[0].re = c[2] + c[7] * r3;
    H[4].re = -c[2] + c[7] * r3;
    H[8].re = -2.0 * c[7] * r3;
    /* (0,1): lambda_1 real, lambda_2 imaginary (-i above the diagonal) */
    H[1].re = c[0]; H[1].im = -c[1];
    H[3].re = c[0]; H[3].im = c[1];
    /* (0,2): lambda_4, lambda_5 */
    H[2].re = c[3]; H[2].im = -c[4];
    H[6].re = c[3]; H[6].im = c[4];
    /* (1,2): lambda_6, lambda_7 */
    H[5].re = c[5]; H[5].im = -c[6];
    H[7].re = c[5]; H[7].im = c[6];
}

/* exp(A) for a 3x3 complex A by scaling and squaring with a degree-20 Taylor
 * polynomial; the scaled norm is below 1/2, so the truncation error is far
 * under double rounding. */
static void mat_exp(const cplx A[9], cplx E[9]) {
    double nrm = 0;
    for (int i = 0; i < 9; i++) nrm += A[i].re * A[i].re + A[i].im * A[i].im;
    nrm = sqrt(nrm);
    int k = 0;
    while (nrm > 0.5) { nrm *= 0.5; k++; }
    double sc = ldexp(1.0, -k);
    cplx As[9], term[9], tmp[9];
    for (int i = 0; i < 9; i++) { As[i].re = A[i].re * sc; As[i].im = A[i].im * sc; }
    memset(E, 0, 9 * sizeof(cplx));
    memset(term, 0, 9 * sizeof(cplx));
    for (int i = 0; i < 3; i++) { E[4 * i].re = 1; term[4 * i].re = 1; }
    for (int n = 1; n <= 20; n++) {
        mat_mul(term, As, tmp);
        for (int i = 0; i < 9; i++) {
            term[i].re = tmp[i].re / n; term[i].im = tmp[i].im / n;
            E[i].re += term[i].re; E[i].im += term[i].im;
        }
    }
    for (int s = 0; s < k; s++) {
        mat_mul(E, E, tmp);
        memcpy(E, tmp, 9 * sizeof(cplx));
    }
}

/* Re-unitarise: Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1);
 * the result is in SU(3) (unitary, det = 1) up to rounding. */
static void reunitarise(cplx U[9]) {
    double n0 = 0;
    for (int j = 0; j < 3; j++) n0 += U[j].re * U[j].re + U[j].im * U[j].im;
    n0 = 1.0 / sqrt(n0);
    for (int j = 0; j < 3; j++) { U[j].re *= n0; U[j].im *= n0; }
    cplx d = {0, 0}; /* <row0, row1> = sum conj(row0) row1 */
    for (int j = 0; j < 3; j++) {
        d.re += U[j].re * U[3 + j].re + U[j].im * U[3 + j].im;
        d.im += U[j].re * U[3 + j].im - U[j].im * U[3 + j].re;
    }
    for (int j = 0; j < 3; j++) {
        cplx p = cmul(d, U[j]);
        U[3 + j].re -= p.re; U[3 + j].im -= p.im;
    }
    double n1 = 0;
    for (int j = 0; j < 3; j++) n1 += U[3 + j].re * U[3 + j].re + U[3 + j].im * U[3 + j].im;
    n1 = 1.0 / sqrt(n1);
    for (int j = 0; j < 3; j++) { U[3 + j].re *= n1; U[3 + j].im *= n1; }
    for (int j = 0; j < 3; j++) {
        int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
        cplx a = cmul(U[j1], U[3 + j2]), b = cmul(U[j2], U[3 + j1]);
        U[6 + j].re = a.re - b.re;
        U[6 + j].im = -(a.im - b.im);
    }
}

/* One SU(3) matrix exp(i eps sum_a c_a lambda_a), c_a ~ N(0,1) from draws
 * [8*idx, 8*idx+8) of the stream with key k. */
static void su3_element(uint64_t k, uint64_t idx, double eps, cplx U[9]) {
    double c[8];
    for (int j = 0; j < 4; j++) box_muller(k, 8 * idx + 2 * j, &c[2 * j], &c[2 * j + 1]);
    cplx H[9], A[9];
    gell_mann_combination(c, H);
    for (int i = 0; i < 9; i++) { A[i].re = -eps * H[i].im; A[i].im = eps * H[i].re; } /* A = i eps H */
    mat_exp(A, U);
    reunitarise(U);
}

/* Gauge field: U[s][mu] = exp(i eps sum_a c_a lambda_a), stream index s*4+mu. */
void qi_gauge(double *U, int64_t volume, double eps, uint64_t seed) {
    uint64_t k = stream_key(seed);
    int64_t n = volume * 4;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) su3_element(k, (uint64_t)i, eps, (cplx *)(U + 18 * i));
}

/* Random SU(3) gauge transformation g[s] (one matrix per site). */
void qi_gauge_transform(double *g, int64_t volume, double eps, uint64_t seed) {
    uint64_t k = stream_key(seed ^ 0x5bd1e995ULL);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < volume; i++) su3_element(k, (uint64_t)i, eps, (cplx *)(g + 18 * i));
}

/* Gaussian complex source: re, im ~ N(0, 1/2) so E|z|^2 = 1, draws 2j, 2j+1
 * for complex component j = (s*4 + spin)*3 + colour. */
void qi_gaussian(double *psi, int64_t ncomplex, uint64_t seed) {
    uint64_t k = stream_key(seed);
    const double h = 0.70710678118654752440;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < ncomplex; j++) {
        double a, b;
        box_muller(k, 2 * (uint64_t)j, &a, &b);
        psi[2 * j] = a * h;
        psi[2 * j + 1] = b * h;
    }
}

/* Uniform (0,1] values, for tests of the generator itself. */
void qi_uniform(double *out, int64_t n, uint64_t seed) {
    uint64_t k = stream_key(seed);
    for (int64_t j = 0; j < n; j++) out[j] = unif(k, (uint64_t)j);
}

/* Raw 64-bit draws, for the published-value check of SplitMix64. */
void qi_splitmix_raw(uint64_t state, uint64_t *out, int64_t n) {
    /* the sequential generator: state += G; out = mix(state) */
    for (int64_t j = 0; j < n; j++) { state += GOLDEN; out[j] = mix64(state); }
}

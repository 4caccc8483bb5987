/*
 * CPU oracle: the Wilson-Dirac operator in FP64, written straight from its
 * definition.  TEST INFRASTRUCTURE ONLY: the product path never calls,
 * links or loads this file; only the tests, the smoke check and the
 * benchmark's CPU-baseline leg do.
 *
 * Definition (the Wilson matrix, eq. (1) of Kanamori et al., Sec. 2):
 *   (D phi)(x) = phi(x) - kappa * sum_mu [ (1 - gamma_mu) U_mu(x)            phi(x+mu)
 *                                        + (1 + gamma_mu) U_mu(x-mu)^dagger phi(x-mu) ]
 * with periodic boundaries in all four directions.  The hopping term H is
 * the bracketed sum, so D = 1 - kappa H.
 *
 * The spin matrices are applied as full 4x4 complex matrices; the
 * half-spinor projection of Sec. 2 (Alg. 1 and the (1 - gamma_1) example)
 * is deliberately not used, so that a GPU kernel built on projection is
 * checked against an independent route.
 *
 * Gamma basis: the paper fixes gamma_1 through the printed matrix
 * (1 - gamma_1) in Sec. 2 and calls the rest "our convention".  We take the
 * Dirac representation consistent with that gamma_1:
 *   gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]  (k = 1,2,3),
 *   gamma_4 = diag(1, 1, -1, -1),
 * where sigma_k are the Pauli matrices.  Directions mu = 0..3 of the code are
 * the paper's 1..4 (x, y, z, t).
 *
 * Layouts (complex128, interleaved re/im), site s = x + Lx*(y + Ly*(z + Lz*t)):
 *   U[s][mu][a][b],  phi[s][spin][colour]
 */
#include <stdint.h>
#include <string.h>

typedef struct { double re, im; } cplx;

/* Pauli matrices sigma_1..3, row-major 2x2 */
static const cplx PAULI[3][4] = {
    {{0, 0}, {1, 0}, {1, 0}, {0, 0}},
    {{0, 0}, {0, -1}, {0, 1}, {0, 0}},
    {{1, 0}, {0, 0}, {0, 0}, {-1, 0}},
};

static cplx GAMMA[4][4][4]; /* GAMMA[mu][i][j] */
static int gamma_ready = 0;

/* Build the Dirac-representation gamma matrices from the Pauli matrices. */
static void build_gamma(void) {
    if (gamma_ready) return;
    memset(GAMMA, 0, sizeof(GAMMA));
    for (int k = 0; k < 3; k++) {
        for (int i = 0; i < 2; i++)
            for (int j = 0; j < 2; j++) {
                cplx s = PAULI[k][2 * i + j];
                /* upper-right block: -i sigma_k;  (-i)(a + ib) = b - ia */
                GAMMA[k][i][2 + j].re = s.im;
                GAMMA[k][i][2 + j].im = -s.re;
                /* lower-left block: +i sigma_k;  i(a + ib) = -b + ia */
                GAMMA[k][2 + i][j].re = -s.im;
                GAMMA[k][2 + i][j].im = s.re;
            }
    }
    GAMMA[3][0][0].re = 1; GAMMA[3][1][1].re = 1;
    GAMMA[3][2][2].re = -1; GAMMA[3][3][3].re = -1;
    gamma_ready = 1;
}

/* Copy the gamma matrices out (complex128 [4][4][4]) for inspection by tests. */
void or_gamma(double *out) {
    build_gamma();
    memcpy(out, GAMMA, sizeof(GAMMA));
}

static inline cplx cmul(cplx a, cplx b) { cplx c = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; return c; }
static inline cplx cmulc(cplx a, cplx b) { /* conj(a) * b */ cplx c = {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re}; return c; }

/* neighbour of site s one step along +mu (dir = +1) or -mu (dir = -1), periodic */
static int64_t neighbour(const int dims[4], int64_t s, int mu, int dir) {
    int64_t c[4];
    int64_t r = s;
    for (int m = 0; m < 4; m++) { c[m] = r % dims[m]; r /= dims[m]; }
    c[mu] = (c[mu] + dir + dims[mu]) % dims[mu];
    return c[0] + (int64_t)dims[0] * (c[1] + (int64_t)dims[1] * (c[2] + (int64_t)dims[2] * c[3]));
}

/*
 * Hopping term at one site: out[12] = sum_mu [ (1 - sg*gamma_mu) U_mu(s) phi(s+mu)
 *                                            + (1 + sg*gamma_mu) U_mu(s-mu)^dag phi(s-mu) ]
 * sg = +1 gives H (eq. (1)); sg = -1 gives H^dagger, the matrix adjoint of H
 * (gamma_mu is Hermitian, and the adjoint of the forward term at x is the
 * backward term at x with the spin factor unchanged).
 */
static void hop_site(const int dims[4], const cplx *U, const cplx *phi, int64_t s, double sg, cplx out[12]) {
    for (int k = 0; k < 12; k++) out[k].re = out[k].im = 0;
    for (int mu = 0; mu < 4; mu++) {
        for (int dir = +1; dir >= -1; dir -= 2) {
            int64_t n = neighbour(dims, s, mu, dir);
            /* colour part: w[j][a] = (U or U^dag)[a][b] phi(n)[j][b] */
            cplx w[4][3];
            for (int j = 0; j < 4; j++)
                for (int a = 0; a < 3; a++) {
                    cplx acc = {0, 0};
                    for (int b = 0; b < 3; b++) {
                        cplx p;
                        if (dir > 0) /* U_mu(s)[a][b] */
                            p = cmul(U[(s * 4 + mu) * 9 + 3 * a + b], phi[n * 12 + 3 * j + b]);
                        else /* U_mu(s-mu)^dag[a][b] = conj(U_mu(s-mu)[b][a]) */
                            p = cmulc(U[(n * 4 + mu) * 9 + 3 * b + a], phi[n * 12 + 3 * j + b]);
                        acc.re += p.re; acc.im += p.im;
                    }
                    w[j][a] = acc;
                }
            /* spin part: (1 -/+ sg*gamma_mu)[i][j] */
            double pm = (dir > 0) ? -sg : +sg;
            for (int i = 0; i < 4; i++)
                for (int j = 0; j < 4; j++) {
                    cplx P = GAMMA[mu][i][j];
                    P.re *= pm; P.im *= pm;
                    if (i == j) P.re += 1.0;
                    if (P.re == 0 && P.im == 0) continue;
                    for (int a = 0; a < 3; a++) {
                        cplx q = cmul(P, w[j][a]);
                        out[3 * i + a].re += q.re;
                        out[3 * i + a].im += q.im;
                    }
                }
        }
    }
}

/*
 * op = 0: out = D phi;  op = 1: out = H phi;  op = 2: out = D^dagger phi;  op = 3: out = H^dagger phi
 * U: complex128 [V][4][3][3]; phi, out: complex128 [V][4][3]; out must not alias phi.
 */
void or_dslash(const int dims[4], const double *U, const double *phi, double *out, double kappa, int op) {
    build_gamma();
    int64_t V = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
    const cplx *Uc = (const cplx *)U;
    const cplx *pc = (const cplx *)phi;
    cplx *oc = (cplx *)out;
    double sg = (op == 0 || op == 1) ? 1.0 : -1.0;
    int hop_only = (op == 1 || op == 3);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; s++) {
        cplx h[12];
        hop_site(dims, Uc, pc, s, sg, h);
        for (int k = 0; k < 12; k++) {
            if (hop_only) {
                oc[s * 12 + k] = h[k];
            } else {
                oc[s * 12 + k].re = pc[s * 12 + k].re - kappa * h[k].re;
                oc[s * 12 + k].im = pc[s * 12 + k].im - kappa * h[k].im;
            }
        }
    }
}

/* D phi at a list of sites only (for sampled checks on large lattices):
 * out[i] = (D phi)(sites[i]), complex128 [n][4][3]. */
void or_dslash_sites(const int dims[4], const double *U, const double *phi, double *out, double kappa,
                     const int64_t *sites, int64_t n) {
    build_gamma();
    const cplx *Uc = (const cplx *)U;
    const cplx *pc = (const cplx *)phi;
    cplx *oc = (cplx *)out;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        int64_t s = sites[i];
        cplx h[12];
        hop_site(dims, Uc, pc, s, 1.0, h);
        for (int k = 0; k < 12; k++) {
            oc[i * 12 + k].re = pc[s * 12 + k].re - kappa * h[k].re;
            oc[i * 12 + k].im = pc[s * 12 + k].im - kappa * h[k].im;
        }
    }
}

/*
 * CPU FP64 oracle: the Wilson kernel operator.  TEST INFRASTRUCTURE ONLY --
 * this file is compiled into the oracle's private library, which only the
 * test suite, the smoke check and the CPU-baseline timing load.
 *
 * Plain definitions, written out directly (paper Sec. 1, eq. 2 and the text
 * after it):
 *
 *   H psi(x) = sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                     + (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu) ]
 *   D_W(-rho) psi = (4 - rho) psi - 1/2 H psi
 *   K psi = gamma_5 D_W(-rho) psi
 *
 * K here is the paper's kernel times 1/(2 kappa) with kappa = 1/(8 - 2 rho);
 * the sign function does not see a positive rescaling.  Spin is applied as a
 * full 4x4 matrix product and colour as a full 3x3 product, with no
 * spin-projection shortcut, so each line can be checked against the formula.
 *
 * Layouts (canonical): psi[site][spin][colour], U[site][mu][a][b],
 * complex128; site = x + Lx*(y + Ly*(z + Lz*t)); mu = 0..3 is x, y, z, t;
 * periodic boundaries in all four directions.
 *
 * Gamma basis (chiral, Hermitian): gamma_k = [[0, -i s_k], [i s_k, 0]]
 * (k = 1, 2, 3, s_k the Pauli matrices), gamma_4 = [[0, 1], [1, 0]],
 * gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 = diag(1, 1, -1, -1).
 */
#include <complex.h>
#include <stdint.h>
#include <string.h>

typedef double complex cplx;

static cplx G[5][4][4];
static int g_ready = 0;

static void build_gamma(void)
{
    if (g_ready) return;
    const cplx s[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(G, 0, sizeof(G));
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                G[k][a][2 + b] = -I * s[k][a][b];
                G[k][2 + a][b] = I * s[k][a][b];
            }
    for (int a = 0; a < 2; ++a) {
        G[3][a][2 + a] = 1;
        G[3][2 + a][a] = 1;
    }
    /* gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4, by explicit products */
    cplx t1[4][4], t2[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx acc = 0;
            for (int k = 0; k < 4; ++k) acc += G[0][i][k] * G[1][k][j];
            t1[i][j] = acc;
        }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx acc = 0;
            for (int k = 0; k < 4; ++k) acc += t1[i][k] * G[2][k][j];
            t2[i][j] = acc;
        }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            cplx acc = 0;
            for (int k = 0; k < 4; ++k) acc += t2[i][k] * G[3][k][j];
            G[4][i][j] = acc;
        }
    g_ready = 1;
}

/* Copy the 5 gamma matrices (gamma_1..gamma_4, gamma_5) out, [5][4][4]. */
void ora_gamma(cplx *out)
{
    build_gamma();
    memcpy(out, G, sizeof(G));
}

static inline int64_t site_index(const int *L, int x, int y, int z, int t)
{
    return (int64_t)x + (int64_t)L[0] * ((int64_t)y + (int64_t)L[1] * ((int64_t)z + (int64_t)L[2] * t));
}

static void neighbour(const int *L, int64_t s, int mu, int64_t *fwd, int64_t *bwd)
{
    int c[4];
    int64_t r = s;
    c[0] = (int)(r % L[0]); r /= L[0];
    c[1] = (int)(r % L[1]); r /= L[1];
    c[2] = (int)(r % L[2]); r /= L[2];
    c[3] = (int)r;
    int cf[4] = {c[0], c[1], c[2], c[3]};
    int cb[4] = {c[0], c[1], c[2], c[3]};
    cf[mu] = (c[mu] + 1) % L[mu];
    cb[mu] = (c[mu] + L[mu] - 1) % L[mu];
    *fwd = site_index(L, cf[0], cf[1], cf[2], cf[3]);
    *bwd = site_index(L, cb[0], cb[1], cb[2], cb[3]);
}

/* out = H in  (hopping term; see header) */
void ora_hopping(const int *L, const cplx *U, const cplx *in, cplx *out)
{
    build_gamma();
    const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        cplx acc[4][3];
        memset(acc, 0, sizeof(acc));
        for (int mu = 0; mu < 4; ++mu) {
            int64_t f, b;
            neighbour(L, s, mu, &f, &b);
            const cplx *Uf = U + (s * 4 + mu) * 9;  /* U_mu(x)      */
            const cplx *Ub = U + (b * 4 + mu) * 9;  /* U_mu(x - mu) */
            const cplx *pf = in + f * 12;
            const cplx *pb = in + b * 12;
            cplx uf[4][3], ub[4][3];
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) {
                    cplx af = 0, ab = 0;
                    for (int c = 0; c < 3; ++c) {
                        af += Uf[a * 3 + c] * pf[sp * 3 + c];
                        ab += conj(Ub[c * 3 + a]) * pb[sp * 3 + c];
                    }
                    uf[sp][a] = af;
                    ub[sp][a] = ab;
                }
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) {
                    cplx gf = 0, gb = 0;
                    for (int t = 0; t < 4; ++t) {
                        gf += G[mu][sp][t] * uf[t][a];
                        gb += G[mu][sp][t] * ub[t][a];
                    }
                    acc[sp][a] += (uf[sp][a] - gf) + (ub[sp][a] + gb);
                }
        }
        cplx *o = out + s * 12;
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) o[sp * 3 + a] = acc[sp][a];
    }
}

/* out = D_W(-rho) in = (4 - rho) in - 1/2 H in */
void ora_dw(const int *L, const cplx *U, double rho, const cplx *in, cplx *out)
{
    const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
    ora_hopping(L, U, in, out);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < V * 12; ++i) out[i] = (4.0 - rho) * in[i] - 0.5 * out[i];
}

/* out = K in = gamma_5 D_W(-rho) in */
void ora_kernel(const int *L, const cplx *U, double rho, const cplx *in, cplx *out)
{
    build_gamma();
    const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
    ora_dw(L, U, rho, in, out);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < V; ++s) {
        cplx t[4][3];
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) {
                cplx acc = 0;
                for (int k = 0; k < 4; ++k) acc += G[4][sp][k] * out[s * 12 + k * 3 + a];
                t[sp][a] = acc;
            }
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) out[s * 12 + sp * 3 + a] = t[sp][a];
    }
}

/* out = (K^2 + sigma) in, through a caller-provided temporary tmp */
void ora_kernel_sq_shift(const int *L, const cplx *U, double rho, double sigma,
                         const cplx *in, cplx *tmp, cplx *out)
{
    const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
    ora_kernel(L, U, rho, in, tmp);
    ora_kernel(L, U, rho, tmp, out);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < V * 12; ++i) out[i] += sigma * in[i];
}

/* out[i] = (H in)(sites[i]) for a list of sites: the same sum as ora_hopping,
 * evaluated one site at a time (used to check large fields on samples). */
void ora_hopping_sites(const int *L, const cplx *U, const cplx *in,
                       const int64_t *sites, int64_t nsites, cplx *out)
{
    build_gamma();
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nsites; ++i) {
        const int64_t s = sites[i];
        cplx acc[4][3];
        memset(acc, 0, sizeof(acc));
        for (int mu = 0; mu < 4; ++mu) {
            int64_t f, b;
            neighbour(L, s, mu, &f, &b);
            const cplx *Uf = U + (s * 4 + mu) * 9;
            const cplx *Ub = U + (b * 4 + mu) * 9;
            const cplx *pf = in + f * 12;
            const cplx *pb = in + b * 12;
            cplx uf[4][3], ub[4][3];
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) {
                    cplx af = 0, ab = 0;
                    for (int c = 0; c < 3; ++c) {
                        af += Uf[a * 3 + c] * pf[sp * 3 + c];
                        ab += conj(Ub[c * 3 + a]) * pb[sp * 3 + c];
                    }
                    uf[sp][a] = af;
                    ub[sp][a] = ab;
                }
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) {
                    cplx gf = 0, gb = 0;
                    for (int t = 0; t < 4; ++t) {
                        gf += G[mu][sp][t] * uf[t][a];
                        gb += G[mu][sp][t] * ub[t][a];
                    }
                    acc[sp][a] += (uf[sp][a] - gf) + (ub[sp][a] + gb);
                }
        }
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) out[i * 12 + sp * 3 + a] = acc[sp][a];
    }
}

/* Vector updates of the multi-shift CG on n complex entries, one IEEE
 * multiply and one add per real component, in the order written:
 *   ora_axpy_real:  y = y + a x
 *   ora_axpby_real: y = a x + b y
 * (a, b real; the same values numpy's y + a * x and a * x + b * y give). */
void ora_axpy_real(int64_t n, double a, const cplx *x, cplx *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) y[i] = y[i] + a * x[i];
}

void ora_axpby_real(int64_t n, double a, const cplx *x, double b, cplx *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) y[i] = a * x[i] + b * y[i];
}

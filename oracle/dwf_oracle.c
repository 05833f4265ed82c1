/*
 * Plain C / OpenMP FP64 oracle of the Shamir domain-wall fermion operator.
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the bench.  The HIP library shares no code with this file.
 *
 * The paper names the domain-wall Dirac operator and its node-local Wilson
 * hopping matrix as the kernels that dominate its run time (Introduction;
 * Performance results; Conclusion) without writing them down.  This file
 * writes out the same standard definitions as the numpy reference, as
 * straight loops over sites, directions, spins and colours:
 *
 *   (D_h psi)(x,s) = sum_mu (1 -/+ gamma_mu) eta_mu(x) U_mu(x) psi(x+mu,s)
 *                         + (1 +/- gamma_mu) eta_mu(x-mu) U_mu(x-mu)^dag psi(x-mu,s)
 *   (upper signs: D_h, lower signs: D_h^dag), eta_3 = -1 on links leaving t = Lt-1
 *   (M5op psi)(s) = (5-M5) psi(s) - P_- psi~(s+1) - P_+ psi~(s-1), wraps -mf
 *   M_pc = M5op - 1/4 D_h^{o<-e} M5op^-1 D_h^{e<-o}
 *
 * Layouts are the canonical ones: gauge [t][z][y][x][mu][3][3], checkerboard
 * field [V/2][Ls][4][3] with row c(x) = lex(x) >> 1, complex = (re, im).
 */
#include <complex.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* gamma_mu, chiral basis: [[0, e_mu], [e_mu^dag, 0]] with
 * e_0 = -i sigma_1, e_1 = -i sigma_2, e_2 = -i sigma_3, e_3 = 1. */
static void gamma_matrix(int mu, cplx g[4][4]) {
    cplx e[2][2];
    memset(g, 0, sizeof(cplx) * 16);
    switch (mu) {
        case 0: e[0][0] = 0; e[0][1] = -I; e[1][0] = -I; e[1][1] = 0; break;
        case 1: e[0][0] = 0; e[0][1] = -1; e[1][0] = 1; e[1][1] = 0; break;
        case 2: e[0][0] = -I; e[0][1] = 0; e[1][0] = 0; e[1][1] = I; break;
        default: e[0][0] = 1; e[0][1] = 0; e[1][0] = 0; e[1][1] = 1; break;
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            g[a][2 + b] = e[a][b];
            g[2 + a][b] = conj(e[b][a]);
        }
}

static long lex_of(const int L[4], const int x[4]) {
    return x[0] + (long)L[0] * (x[1] + (long)L[1] * (x[2] + (long)L[2] * x[3]));
}

static void site_of_row(const int L[4], int par, long c, int x[4]) {
    long xh = c % (L[0] / 2);
    long rest = c / (L[0] / 2);
    x[1] = (int)(rest % L[1]);
    x[2] = (int)((rest / L[1]) % L[2]);
    x[3] = (int)(rest / ((long)L[1] * L[2]));
    x[0] = (int)(2 * xh + ((par + x[1] + x[2] + x[3]) & 1));
}

/* out[row] for rows in [row_begin, row_end) of parity out_parity. */
void oracle_dhop_cb(const cplx *U, const cplx *in, cplx *out, const int *dims, int Ls, int out_parity,
                    int dagger, int antiperiodic_t, long row_begin, long row_end) {
    cplx proj[8][4][4];
    for (int mu = 0; mu < 4; ++mu) {
        cplx g[4][4];
        gamma_matrix(mu, g);
        double sf = dagger ? 1.0 : -1.0; /* forward hop: 1 + sf*gamma */
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                proj[mu][i][j] = (i == j ? 1.0 : 0.0) + sf * g[i][j];
                proj[4 + mu][i][j] = (i == j ? 1.0 : 0.0) - sf * g[i][j];
            }
    }
    const int L[4] = {dims[0], dims[1], dims[2], dims[3]};
#pragma omp parallel for schedule(static)
    for (long c = row_begin; c < row_end; ++c) {
        int x[4];
        site_of_row(L, out_parity, c, x);
        cplx *o = out + c * (long)Ls * 12;
        for (int s = 0; s < Ls; ++s)
            for (int sp = 0; sp < 4; ++sp)
                for (int a = 0; a < 3; ++a) o[(s * 4 + sp) * 3 + a] = 0;
        for (int dir = 0; dir < 8; ++dir) {
            int mu = dir & 3, fwd = dir < 4;
            int y[4] = {x[0], x[1], x[2], x[3]};
            y[mu] = fwd ? (x[mu] + 1) % L[mu] : (x[mu] - 1 + L[mu]) % L[mu];
            /* link: forward U_mu(x), backward U_mu(x-mu)^dag; eta of the link's base site */
            const int *base = fwd ? x : y;
            double eta = (antiperiodic_t && mu == 3 && base[3] == L[3] - 1) ? -1.0 : 1.0;
            const cplx *u = U + (lex_of(L, base) * 4 + mu) * 9;
            cplx w[3][3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) w[a][b] = eta * (fwd ? u[a * 3 + b] : conj(u[b * 3 + a]));
            const cplx *nb = in + (lex_of(L, y) >> 1) * (long)Ls * 12;
            for (int s = 0; s < Ls; ++s) {
                cplx t[4][3];
                for (int sp = 0; sp < 4; ++sp)
                    for (int a = 0; a < 3; ++a) {
                        cplx v = 0;
                        for (int b = 0; b < 3; ++b) v += w[a][b] * nb[(s * 4 + sp) * 3 + b];
                        t[sp][a] = v;
                    }
                for (int i = 0; i < 4; ++i)
                    for (int a = 0; a < 3; ++a) {
                        cplx v = 0;
                        for (int j = 0; j < 4; ++j) v += proj[dir][i][j] * t[j][a];
                        o[(s * 4 + i) * 3 + a] += v;
                    }
            }
        }
    }
}

/* M5op (dagger = 0) or M5op^dag (dagger = 1) on nsites rows of [Ls][4][3]. */
void oracle_m5op(const cplx *in, cplx *out, long nsites, int Ls, double M5, double mf, int dagger) {
#pragma omp parallel for schedule(static)
    for (long n = 0; n < nsites; ++n) {
        const cplx *p = in + n * Ls * 12;
        cplx *o = out + n * Ls * 12;
        for (int s = 0; s < Ls; ++s) {
            int su = (s + 1) % Ls, sd = (s - 1 + Ls) % Ls;
            double fu = (s + 1 < Ls) ? 1.0 : -mf, fd = (s >= 1) ? 1.0 : -mf;
            for (int sp = 0; sp < 4; ++sp) {
                int plus = sp < 2; /* P_+ keeps spins 0,1; P_- keeps spins 2,3 */
                /* M5op: P_- takes psi~(s+1), P_+ takes psi~(s-1); the adjoint swaps them */
                int take_up = dagger ? plus : !plus;
                for (int a = 0; a < 3; ++a) {
                    cplx nbv = take_up ? fu * p[(su * 4 + sp) * 3 + a] : fd * p[(sd * 4 + sp) * 3 + a];
                    o[(s * 4 + sp) * 3 + a] = (5.0 - M5) * p[(s * 4 + sp) * 3 + a] - nbv;
                }
            }
        }
    }
}

/* Inverse of the real (4 Ls) x (4 Ls) matrix of M5op over (s, spin) by Gauss-Jordan
 * elimination with partial pivoting, then applied to every site and colour. */
void oracle_m5inv(const cplx *in, cplx *out, long nsites, int Ls, double M5, double mf, int dagger) {
    int n = 4 * Ls;
    double *m = calloc((size_t)n * n, sizeof(double));
    double *inv = calloc((size_t)n * n, sizeof(double));
    for (int s = 0; s < Ls; ++s)
        for (int sp = 0; sp < 4; ++sp) {
            int row = s * 4 + sp;
            m[row * n + row] += 5.0 - M5;
            int su = (s + 1) % Ls, sd = (s - 1 + Ls) % Ls;
            double fu = (s + 1 < Ls) ? 1.0 : -mf, fd = (s >= 1) ? 1.0 : -mf;
            int plus = sp < 2;
            if (!plus) m[row * n + su * 4 + sp] -= fu;
            else m[row * n + sd * 4 + sp] -= fd;
        }
    if (dagger) { /* real matrix: adjoint = transpose */
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) {
                double t = m[i * n + j];
                m[i * n + j] = m[j * n + i];
                m[j * n + i] = t;
            }
    }
    for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (m[r * n + col] * m[r * n + col] > m[piv * n + col] * m[piv * n + col]) piv = r;
        if (piv != col)
            for (int j = 0; j < n; ++j) {
                double t = m[col * n + j]; m[col * n + j] = m[piv * n + j]; m[piv * n + j] = t;
                t = inv[col * n + j]; inv[col * n + j] = inv[piv * n + j]; inv[piv * n + j] = t;
            }
        double d = m[col * n + col];
        for (int j = 0; j < n; ++j) { m[col * n + j] /= d; inv[col * n + j] /= d; }
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            double f = m[r * n + col];
            if (f == 0.0) continue;
            for (int j = 0; j < n; ++j) { m[r * n + j] -= f * m[col * n + j]; inv[r * n + j] -= f * inv[col * n + j]; }
        }
    }
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nsites; ++k) {
        const cplx *p = in + k * n * 3;
        cplx *o = out + k * n * 3;
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) {
                cplx v = 0;
                for (int j = 0; j < n; ++j) v += inv[i * n + j] * p[j * 3 + a];
                o[i * 3 + a] = v;
            }
    }
    free(m);
    free(inv);
}

/* M_pc (dagger = 0) or M_pc^dag (dagger = 1) on the odd checkerboard. */
void oracle_mpc(const cplx *U, const cplx *in, cplx *out, const int *dims, int Ls, double M5, double mf,
                int dagger, int antiperiodic_t) {
    long half = (long)dims[0] * dims[1] * dims[2] * dims[3] / 2;
    long n = half * Ls * 12;
    cplx *t1 = malloc(sizeof(cplx) * n), *t2 = malloc(sizeof(cplx) * n);
    oracle_dhop_cb(U, in, t1, dims, Ls, 0, dagger, antiperiodic_t, 0, half);
    oracle_m5inv(t1, t2, half, Ls, M5, mf, dagger);
    oracle_dhop_cb(U, t2, t1, dims, Ls, 1, dagger, antiperiodic_t, 0, half);
    oracle_m5op(in, out, half, Ls, M5, mf, dagger);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) out[i] -= 0.25 * t1[i];
    free(t1);
    free(t2);
}

/* M_pc^dag M_pc on the odd checkerboard. */
void oracle_mdagm(const cplx *U, const cplx *in, cplx *out, const int *dims, int Ls, double M5, double mf,
                  int antiperiodic_t) {
    long n = (long)dims[0] * dims[1] * dims[2] * dims[3] / 2 * Ls * 12;
    cplx *t = malloc(sizeof(cplx) * n);
    oracle_mpc(U, in, t, dims, Ls, M5, mf, 0, antiperiodic_t);
    oracle_mpc(U, t, out, dims, Ls, M5, mf, 1, antiperiodic_t);
    free(t);
}

int oracle_num_threads(void) {
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}

/* Thread count of the later parallel regions (timing on one core or all of them). */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

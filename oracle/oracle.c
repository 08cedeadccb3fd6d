/*
 * oracle.c -- reference Coulomb/exchange (J/K) build on the CPU.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the tests, the smoke check and
 * the benchmark's CPU-baseline leg call this file.  It shares no source,
 * header, table or constant generator with the GPU library.
 *
 * What it computes is the plain definition of the paper's result:
 *
 *   J^s_ab = sum_cd (ab|cd) D^s_cd,   K^s_ac = sum_bd (ab|cd) D^s_bd
 *
 * (Section 2, eq. jk) over every AO quartet whose shell quartet passes the
 * Schwarz test Q_IJ * Q_KL >= cutoff (Section 2, eq. schwartz; threshold of
 * Section 4.2), with Q_IJ = sqrt(max_{a in I, b in J} |(ab|ab)|).
 *
 * The contracted integrals follow eq. rys0 (sum over primitive quartets of
 * coefficient products times primitive integrals).  The primitive integrals
 * are NOT evaluated by the paper's Rys quadrature: this file uses the
 * McMurchie-Davidson Hermite expansion (the alternative the paper names in
 * Section 2), so that the GPU path is checked against a different
 * formulation:
 *
 *   (ab|cd) = 2 pi^(5/2) / (p q sqrt(p+q)) * sum_tuv E^ab_tuv
 *             sum_tau,nu,phi (-1)^(tau+nu+phi) E^cd_tau,nu,phi R_(t+tau)(u+nu)(v+phi)
 *
 * with Hermite coefficients E from the standard two-term recurrence and
 * R^n_000 = (-2 alpha)^n F_n(alpha |PQ|^2).
 *
 * Two digestion modes:
 *   mode 0 (brute): every ordered shell quartet, J_ab += v D_cd, K_ac += v D_bd.
 *   mode 1 (8-fold): unique quartets I>=J, K>=L, IJ>=KL (Section 2's
 *      permutational symmetry) with degeneracy weight
 *      w = 1/2^[I=J] * 1/2^[K=L] * 1/2^[IJ=KL]; every element feeds two J
 *      and four K updates, then J = J' + J'^T, K = K' + K'^T.
 *
 * Spherical shells: D_cart = T^T D T and J = T J_cart T^T with T the real
 * solid harmonic coefficients (Section 2: spherical functions are fixed
 * linear combinations of Cartesian ones), built here from the closed formula
 * for real solid harmonics and normalised numerically.
 *
 * Range separation (the paper's omega, Tables 1 and 2): the same contraction
 * over the long-range operator erf(omega r)/r (omega > 0) or the short-range
 * operator erfc(|omega| r)/r (omega < 0), through the attenuated Boys values
 * of op_boys; screening keeps the full-range Schwarz factors.
 *
 * Parity pins live in tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_LMAX 4
#define OR_NC(l) (((l) + 1) * ((l) + 2) / 2)
#define OR_MAXNC 15
#define OR_LTOT (4 * OR_LMAX)
#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* basis bookkeeping                                                   */
/* ------------------------------------------------------------------ */
typedef struct {
    int ns, natom, spherical;
    const int *l, *nprim, *atom;
    const double *exps, *coefs, *coords;
    int *poff;      /* first primitive of each shell */
    int *coff;      /* Cartesian AO offset */
    int *eoff;      /* external (spherical or Cartesian) AO offset */
    int nao_cart, nao_ext;
    double omega;   /* operator: 0 full range, > 0 long range, < 0 short range */
} obasis;

static int ob_init(obasis *b, int ns, int natom, int spherical, const int *l, const int *nprim,
                   const int *atom, const double *exps, const double *coefs, const double *coords) {
    b->ns = ns; b->natom = natom; b->spherical = spherical;
    b->l = l; b->nprim = nprim; b->atom = atom;
    b->exps = exps; b->coefs = coefs; b->coords = coords;
    b->omega = 0.0;
    b->poff = (int *)malloc(sizeof(int) * (ns + 1));
    b->coff = (int *)malloc(sizeof(int) * (ns + 1));
    b->eoff = (int *)malloc(sizeof(int) * (ns + 1));
    if (!b->poff || !b->coff || !b->eoff) return -1;
    b->poff[0] = b->coff[0] = b->eoff[0] = 0;
    for (int i = 0; i < ns; ++i) {
        if (l[i] < 0 || l[i] > OR_LMAX) return -1;
        b->poff[i + 1] = b->poff[i] + nprim[i];
        b->coff[i + 1] = b->coff[i] + OR_NC(l[i]);
        b->eoff[i + 1] = b->eoff[i] + (spherical ? 2 * l[i] + 1 : OR_NC(l[i]));
    }
    b->nao_cart = b->coff[ns];
    b->nao_ext = b->eoff[ns];
    return 0;
}

static void ob_free(obasis *b) { free(b->poff); free(b->coff); free(b->eoff); }

/* Cartesian exponents of component c of a shell with angular momentum l,
 * reversed lexicographic order (xx, xy, xz, yy, yz, zz for d). */
static void cart_xyz(int l, int xyz[][3]) {
    int n = 0;
    for (int x = l; x >= 0; --x)
        for (int y = l - x; y >= 0; --y) {
            xyz[n][0] = x; xyz[n][1] = y; xyz[n][2] = l - x - y; ++n;
        }
}

/* ------------------------------------------------------------------ */
/* Boys function F_m(T) = int_0^1 t^(2m) exp(-T t^2) dt, m = 0..mmax    */
/* ------------------------------------------------------------------ */
void oracle_boys(int mmax, double T, double *F) {
    if (T < 30.0) {
        /* F_m(T) = exp(-T) sum_k (2T)^k / ((2m+1)(2m+3)...(2m+2k+1)), then
         * downward recursion F_m = (2T F_(m+1) + exp(-T)) / (2m+1). */
        double e = exp(-T);
        double term = 1.0 / (2 * mmax + 1), sum = term;
        for (int k = 1; k < 2000; ++k) {
            term *= 2.0 * T / (2 * mmax + 2 * k + 1);
            sum += term;
            if (term < 1e-18 * sum) break;
        }
        F[mmax] = e * sum;
        for (int m = mmax - 1; m >= 0; --m) F[m] = (2.0 * T * F[m + 1] + e) / (2 * m + 1);
    } else {
        /* F_0 = (1/2) sqrt(pi/T) erf(sqrt T), upward recursion
         * F_(m+1) = ((2m+1) F_m - exp(-T)) / (2T), stable for m < T. */
        double e = exp(-T);
        F[0] = 0.5 * sqrt(OR_PI / T) * erf(sqrt(T));
        for (int m = 0; m < mmax; ++m) F[m + 1] = ((2 * m + 1) * F[m] - e) / (2.0 * T);
    }
}

/* ------------------------------------------------------------------ */
/* Range-separated operators (the paper's range-separation parameter    */
/* omega, Table 1 rys_type and Table 2).  With the Gaussian transform   */
/* 1/r = (2/sqrt(pi)) int_0^inf exp(-s^2 r^2) ds, the error-function    */
/* operator erf(w r)/r keeps s in [0, w]; in the Boys variable t^2 =    */
/* s^2 / (alpha + s^2) that is t in [0, theta], theta^2 = w^2/(w^2 +    */
/* alpha), and int_0^theta t^(2n) exp(-T t^2) dt = theta^(2n+1)          */
/* F_n(theta^2 T).  These satisfy the same derivative relation as F_n,  */
/* so R^n_000 = (-2 alpha)^n Ftilde_n(T) carries over unchanged.        */
/*   omega > 0: long range  erf(omega r)/r:  Ftilde_n = theta^(2n+1) F_n(theta^2 T)       */
/*   omega < 0: short range erfc(|omega| r)/r: Ftilde_n = F_n(T) - (the long-range one)  */
/* ------------------------------------------------------------------ */
static void op_boys(int mmax, double T, double alpha, double omega, double *F) {
    oracle_boys(mmax, T, F);
    if (omega == 0.0) return;
    const double w2 = omega * omega, th2 = w2 / (w2 + alpha);
    double G[4 * OR_LMAX + 1];
    oracle_boys(mmax, th2 * T, G);
    double f = sqrt(th2);
    for (int n = 0; n <= mmax; ++n) {
        const double lr = f * G[n];
        F[n] = omega > 0.0 ? lr : F[n] - lr;
        f *= th2;
    }
}

/* ------------------------------------------------------------------ */
/* McMurchie-Davidson pieces                                            */
/* ------------------------------------------------------------------ */
#define E_DIM (OR_LMAX + 1)
#define T_DIM (2 * OR_LMAX + 1)

/* One Cartesian direction: E[i][j][t], i <= la, j <= lb, t <= i + j, for the
 * product of x_A^i exp(-a x_A^2) and x_B^j exp(-b x_B^2) expanded in Hermite
 * Gaussians at P.  The exp(-ab/p X_AB^2) factor is left out (applied once per
 * primitive pair). */
static void md_E(int la, int lb, double p, double PA, double PB, double E[E_DIM][E_DIM][T_DIM]) {
    memset(E, 0, sizeof(double) * E_DIM * E_DIM * T_DIM);
    const double h = 0.5 / p;
    E[0][0][0] = 1.0;
    for (int i = 0; i <= la; ++i)
        for (int j = 0; j <= lb; ++j) {
            if (i == 0 && j == 0) continue;
            if (i > 0) {
                for (int t = 0; t <= i + j; ++t) {
                    double v = PA * E[i - 1][j][t];
                    if (t > 0) v += h * E[i - 1][j][t - 1];
                    if (t + 1 <= i - 1 + j) v += (t + 1) * E[i - 1][j][t + 1];
                    E[i][j][t] = v;
                }
            } else {
                for (int t = 0; t <= i + j; ++t) {
                    double v = PB * E[i][j - 1][t];
                    if (t > 0) v += h * E[i][j - 1][t - 1];
                    if (t + 1 <= i + j - 1) v += (t + 1) * E[i][j - 1][t + 1];
                    E[i][j][t] = v;
                }
            }
        }
}

#define R_DIM (OR_LTOT + 1)
#define RIDX(n, t, u, v) ((((n) * R_DIM + (t)) * R_DIM + (u)) * R_DIM + (v))

/* Hermite Coulomb integrals R_tuv = R^0_tuv for t+u+v <= L.
 * work: R_DIM^4 doubles. out: R_DIM^3 doubles indexed (t*R_DIM+u)*R_DIM+v. */
static void md_R(int L, double alpha, double omega, double X, double Y, double Z, double *work, double *out) {
    double F[OR_LTOT + 1];
    op_boys(L, alpha * (X * X + Y * Y + Z * Z), alpha, omega, F);
    double f = 1.0;
    for (int n = 0; n <= L; ++n) { work[RIDX(n, 0, 0, 0)] = f * F[n]; f *= -2.0 * alpha; }
    for (int s = 1; s <= L; ++s)
        for (int t = 0; t <= s; ++t)
            for (int u = 0; u <= s - t; ++u) {
                int v = s - t - u;
                for (int n = 0; n <= L - s; ++n) {
                    double r;
                    if (t > 0) {
                        r = X * work[RIDX(n + 1, t - 1, u, v)];
                        if (t > 1) r += (t - 1) * work[RIDX(n + 1, t - 2, u, v)];
                    } else if (u > 0) {
                        r = Y * work[RIDX(n + 1, t, u - 1, v)];
                        if (u > 1) r += (u - 1) * work[RIDX(n + 1, t, u - 2, v)];
                    } else {
                        r = Z * work[RIDX(n + 1, t, u, v - 1)];
                        if (v > 1) r += (v - 1) * work[RIDX(n + 1, t, u, v - 2)];
                    }
                    work[RIDX(n, t, u, v)] = r;
                }
            }
    for (int t = 0; t <= L; ++t)
        for (int u = 0; u <= L - t; ++u)
            for (int v = 0; v <= L - t - u; ++v)
                out[(t * R_DIM + u) * R_DIM + v] = work[RIDX(0, t, u, v)];
}

typedef struct {
    double *rwork, *R, *W;
} md_ws;

static int ws_init(md_ws *w) {
    w->rwork = (double *)malloc(sizeof(double) * R_DIM * R_DIM * R_DIM * R_DIM);
    w->R = (double *)malloc(sizeof(double) * R_DIM * R_DIM * R_DIM);
    /* W[tuv][cd]: bra Hermite index (dims (2*LMAX+1)^3) x ket Cartesian pairs */
    w->W = (double *)malloc(sizeof(double) * T_DIM * T_DIM * T_DIM * OR_MAXNC * OR_MAXNC);
    return (w->rwork && w->R && w->W) ? 0 : -1;
}
static void ws_free(md_ws *w) { free(w->rwork); free(w->R); free(w->W); }

/* Contracted Cartesian block (IJ|KL), row-major [a][b][c][d]. */
static void eri_block(const obasis *B, int I, int J, int K, int L, double *out, md_ws *ws) {
    const int li = B->l[I], lj = B->l[J], lk = B->l[K], ll = B->l[L];
    const int ni = OR_NC(li), nj = OR_NC(lj), nk = OR_NC(lk), nl = OR_NC(ll);
    const int nab = ni * nj, ncd = nk * nl;
    const double *A = B->coords + 3 * B->atom[I], *Bc = B->coords + 3 * B->atom[J];
    const double *C = B->coords + 3 * B->atom[K], *Dc = B->coords + 3 * B->atom[L];
    int xi[OR_MAXNC][3], xj[OR_MAXNC][3], xk[OR_MAXNC][3], xl[OR_MAXNC][3];
    cart_xyz(li, xi); cart_xyz(lj, xj); cart_xyz(lk, xk); cart_xyz(ll, xl);
    const int Lab = li + lj, Lcd = lk + ll, Ltot = Lab + Lcd;
    const double AB2 = (A[0] - Bc[0]) * (A[0] - Bc[0]) + (A[1] - Bc[1]) * (A[1] - Bc[1]) + (A[2] - Bc[2]) * (A[2] - Bc[2]);
    const double CD2 = (C[0] - Dc[0]) * (C[0] - Dc[0]) + (C[1] - Dc[1]) * (C[1] - Dc[1]) + (C[2] - Dc[2]) * (C[2] - Dc[2]);
    static const int TD = T_DIM;
    double Eab[3][E_DIM][E_DIM][T_DIM], Ecd[3][E_DIM][E_DIM][T_DIM];
    memset(out, 0, sizeof(double) * nab * ncd);
    for (int ip = 0; ip < B->nprim[I]; ++ip)
        for (int jp = 0; jp < B->nprim[J]; ++jp) {
            const double a = B->exps[B->poff[I] + ip], b = B->exps[B->poff[J] + jp];
            const double p = a + b;
            const double kab = exp(-a * b / p * AB2) * B->coefs[B->poff[I] + ip] * B->coefs[B->poff[J] + jp];
            double P[3];
            for (int x = 0; x < 3; ++x) {
                P[x] = (a * A[x] + b * Bc[x]) / p;
                md_E(li, lj, p, P[x] - A[x], P[x] - Bc[x], Eab[x]);
            }
            for (int kp = 0; kp < B->nprim[K]; ++kp)
                for (int lp = 0; lp < B->nprim[L]; ++lp) {
                    const double c = B->exps[B->poff[K] + kp], d = B->exps[B->poff[L] + lp];
                    const double q = c + d;
                    const double kcd = exp(-c * d / q * CD2) * B->coefs[B->poff[K] + kp] * B->coefs[B->poff[L] + lp];
                    double Q[3];
                    for (int x = 0; x < 3; ++x) {
                        Q[x] = (c * C[x] + d * Dc[x]) / q;
                        md_E(lk, ll, q, Q[x] - C[x], Q[x] - Dc[x], Ecd[x]);
                    }
                    const double alpha = p * q / (p + q);
                    md_R(Ltot, alpha, B->omega, P[0] - Q[0], P[1] - Q[1], P[2] - Q[2], ws->rwork, ws->R);
                    const double pref = 2.0 * pow(OR_PI, 2.5) / (p * q * sqrt(p + q)) * kab * kcd;
                    /* ket first: W[tuv][cd] */
                    for (int cd = 0; cd < ncd; ++cd) {
                        const int *ck = xk[cd / nl], *dl = xl[cd % nl];
                        for (int t = 0; t <= Lab; ++t)
                            for (int u = 0; u <= Lab - t; ++u)
                                for (int v = 0; v <= Lab - t - u; ++v) {
                                    double s = 0.0;
                                    for (int tt = 0; tt <= ck[0] + dl[0]; ++tt)
                                        for (int uu = 0; uu <= ck[1] + dl[1]; ++uu)
                                            for (int vv = 0; vv <= ck[2] + dl[2]; ++vv) {
                                                double e = Ecd[0][ck[0]][dl[0]][tt] * Ecd[1][ck[1]][dl[1]][uu] *
                                                           Ecd[2][ck[2]][dl[2]][vv];
                                                if ((tt + uu + vv) & 1) e = -e;
                                                s += e * ws->R[((t + tt) * R_DIM + (u + uu)) * R_DIM + (v + vv)];
                                            }
                                    ws->W[((t * TD + u) * TD + v) * (OR_MAXNC * OR_MAXNC) + cd] = s;
                                }
                    }
                    for (int ab = 0; ab < nab; ++ab) {
                        const int *ai = xi[ab / nj], *bj = xj[ab % nj];
                        for (int cd = 0; cd < ncd; ++cd) {
                            double s = 0.0;
                            for (int t = 0; t <= ai[0] + bj[0]; ++t)
                                for (int u = 0; u <= ai[1] + bj[1]; ++u)
                                    for (int v = 0; v <= ai[2] + bj[2]; ++v)
                                        s += Eab[0][ai[0]][bj[0]][t] * Eab[1][ai[1]][bj[1]][u] * Eab[2][ai[2]][bj[2]][v] *
                                             ws->W[((t * TD + u) * TD + v) * (OR_MAXNC * OR_MAXNC) + cd];
                            out[ab * ncd + cd] += pref * s;
                        }
                    }
                }
        }
}

/* ------------------------------------------------------------------ */
/* real solid harmonics                                                 */
/* ------------------------------------------------------------------ */
static double fact(int n) { double r = 1; for (int i = 2; i <= n; ++i) r *= i; return r; }
static double binom(int n, int k) { return (k < 0 || k > n) ? 0.0 : fact(n) / (fact(k) * fact(n - k)); }
static double dfact(int n) { double r = 1; for (int i = n; i > 1; i -= 2) r *= i; return r; }

/* Angular overlap of x^a1.. and x^a2.. for a common radial part, in units
 * where x^l has unit norm: prod (a1+a2-1)!! / (2l-1)!!. */
static double cart_ovl(int l, const int *e1, const int *e2) {
    double r = 1.0;
    for (int x = 0; x < 3; ++x) {
        int s = e1[x] + e2[x];
        if (s & 1) return 0.0;
        r *= dfact(s - 1);
    }
    return r / dfact(2 * l - 1);
}

/* T[(2l+1) x ncart]: row m (m = -l..l; for l = 1 the rows are x, y, z) of
 * real solid harmonics in Cartesian monomials.  Unnormalised coefficients
 * follow the closed formula
 *   S_lm ~ sum_{t,u,v} (-1)^(t+v-vm) (1/4)^t C(l,t) C(l-t,|m|+t) C(t,u) C(|m|,2v)
 *          x^(2t+|m|-2(u+v)) y^(2(u+v)) z^(l-2t-|m|)
 * (vm = 0 for m >= 0, 1/2 for m < 0, with 2v then odd), then each row is
 * scaled to unit norm with the Cartesian overlap above. */
int oracle_c2s(int l, double *T) {
    if (l < 0 || l > OR_LMAX) return -1;
    int xyz[OR_MAXNC][3];
    cart_xyz(l, xyz);
    const int nc = OR_NC(l), ns = 2 * l + 1;
    memset(T, 0, sizeof(double) * nc * ns);
    if (l == 1) { for (int i = 0; i < 3; ++i) T[i * 3 + i] = 1.0; return 0; }
    for (int m = -l; m <= l; ++m) {
        double *row = T + (m + l) * nc;
        const int am = abs(m);
        for (int t = 0; t <= (l - am) / 2; ++t)
            for (int u = 0; u <= t; ++u) {
                /* 2v runs over even values (m >= 0) or odd values (m < 0) up to |m| */
                for (int v2 = (m < 0 ? 1 : 0); v2 <= am; v2 += 2) {
                    double c = pow(0.25, t) * binom(l, t) * binom(l - t, am + t) * binom(t, u) * binom(am, v2);
                    /* sign (-1)^(t + v - vm) with v - vm = (v2 - (m<0)) / 2 */
                    int sg = t + (v2 - (m < 0 ? 1 : 0)) / 2;
                    if (sg & 1) c = -c;
                    int ex = 2 * t + am - 2 * u - v2, ey = 2 * u + v2, ez = l - 2 * t - am;
                    if (ex < 0) continue;
                    for (int k = 0; k < nc; ++k)
                        if (xyz[k][0] == ex && xyz[k][1] == ey && xyz[k][2] == ez) row[k] += c;
                }
            }
        double n2 = 0.0;
        for (int a = 0; a < nc; ++a)
            for (int b = 0; b < nc; ++b) n2 += row[a] * row[b] * cart_ovl(l, xyz[a], xyz[b]);
        const double s = 1.0 / sqrt(n2);
        for (int a = 0; a < nc; ++a) row[a] *= s;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* public helpers                                                       */
/* ------------------------------------------------------------------ */
#define BASIS_ARGS int ns, int natom, int spherical, const int *l, const int *nprim, const int *atom, \
                   const double *exps, const double *coefs, const double *coords
#define BASIS_PASS ns, natom, spherical, l, nprim, atom, exps, coefs, coords

int oracle_nao(BASIS_ARGS, int *nao_ext, int *nao_cart) {
    obasis b;
    if (ob_init(&b, BASIS_PASS)) { ob_free(&b); return -1; }
    *nao_ext = b.nao_ext; *nao_cart = b.nao_cart;
    ob_free(&b);
    return 0;
}

/* Cartesian contracted block (IJ|KL) into out[ni*nj*nk*nl]; omega selects
 * the operator (0 full range, > 0 erf(omega r)/r, < 0 erfc(|omega| r)/r). */
int oracle_eri_block_op(BASIS_ARGS, double omega, int I, int J, int K, int L, double *out) {
    obasis b; md_ws w;
    if (ob_init(&b, BASIS_PASS) || ws_init(&w)) return -1;
    b.omega = omega;
    eri_block(&b, I, J, K, L, out, &w);
    ws_free(&w); ob_free(&b);
    return 0;
}

int oracle_eri_block(BASIS_ARGS, int I, int J, int K, int L, double *out) {
    return oracle_eri_block_op(BASIS_PASS, 0.0, I, J, K, L, out);
}

/* Schwarz table Q[I*ns+J] = sqrt(max_{a in I, b in J} |(ab|ab)|). */
static void schwarz(const obasis *b, double *Q) {
    const int ns = b->ns;
#pragma omp parallel
    {
        md_ws w; ws_init(&w);
        double *blk = (double *)malloc(sizeof(double) * OR_MAXNC * OR_MAXNC * OR_MAXNC * OR_MAXNC);
#pragma omp for schedule(dynamic, 4)
        for (int I = 0; I < ns; ++I)
            for (int J = 0; J <= I; ++J) {
                eri_block(b, I, J, I, J, blk, &w);
                const int nab = OR_NC(b->l[I]) * OR_NC(b->l[J]);
                double m = 0.0;
                for (int ab = 0; ab < nab; ++ab) m = fmax(m, fabs(blk[ab * nab + ab]));
                Q[I * ns + J] = Q[J * ns + I] = sqrt(m);
            }
        free(blk); ws_free(&w);
    }
}

int oracle_schwarz(BASIS_ARGS, double *Q) {
    obasis b;
    if (ob_init(&b, BASIS_PASS)) return -1;
    schwarz(&b, Q);
    ob_free(&b);
    return 0;
}

/* external -> Cartesian density: Dc = T^T D T, per density */
static void d_to_cart(const obasis *b, const double *Dext, double *Dc, const double *Tl[OR_LMAX + 1]) {
    const int ne = b->nao_ext, nc = b->nao_cart;
    if (!b->spherical) { memcpy(Dc, Dext, sizeof(double) * nc * nc); return; }
    for (int I = 0; I < b->ns; ++I)
        for (int J = 0; J < b->ns; ++J) {
            const int li = b->l[I], lj = b->l[J];
            const double *Ti = Tl[li], *Tj = Tl[lj];
            for (int a = 0; a < OR_NC(li); ++a)
                for (int bb = 0; bb < OR_NC(lj); ++bb) {
                    double s = 0.0;
                    for (int m = 0; m < 2 * li + 1; ++m)
                        for (int n = 0; n < 2 * lj + 1; ++n)
                            s += Ti[m * OR_NC(li) + a] * Dext[(b->eoff[I] + m) * ne + b->eoff[J] + n] * Tj[n * OR_NC(lj) + bb];
                    Dc[(b->coff[I] + a) * nc + b->coff[J] + bb] = s;
                }
        }
}

/* Cartesian -> external result block: Xe[I,J] = T_I Xc[I,J] T_J^T */
static void block_to_ext(int li, int lj, int spherical, const double *Xc /* [nci][ncj] */, double *Xe, const double *Tl[OR_LMAX + 1]) {
    const int nci = OR_NC(li), ncj = OR_NC(lj);
    if (!spherical) { memcpy(Xe, Xc, sizeof(double) * nci * ncj); return; }
    const int nsi = 2 * li + 1, nsj = 2 * lj + 1;
    for (int m = 0; m < nsi; ++m)
        for (int n = 0; n < nsj; ++n) {
            double s = 0.0;
            for (int a = 0; a < nci; ++a)
                for (int bb = 0; bb < ncj; ++bb) s += Tl[li][m * nci + a] * Xc[a * ncj + bb] * Tl[lj][n * ncj + bb];
            Xe[m * nsj + n] = s;
        }
}

static void mat_to_ext(const obasis *b, const double *Xc, double *Xe, const double *Tl[OR_LMAX + 1]) {
    const int ne = b->nao_ext, nc = b->nao_cart;
    double blk[OR_MAXNC * OR_MAXNC], eb[OR_MAXNC * OR_MAXNC];
    for (int I = 0; I < b->ns; ++I)
        for (int J = 0; J < b->ns; ++J) {
            const int li = b->l[I], lj = b->l[J];
            for (int a = 0; a < OR_NC(li); ++a)
                for (int bb = 0; bb < OR_NC(lj); ++bb) blk[a * OR_NC(lj) + bb] = Xc[(b->coff[I] + a) * nc + b->coff[J] + bb];
            block_to_ext(li, lj, b->spherical, blk, eb, Tl);
            const int nei = b->eoff[I + 1] - b->eoff[I], nej = b->eoff[J + 1] - b->eoff[J];
            for (int m = 0; m < nei; ++m)
                for (int n = 0; n < nej; ++n) Xe[(b->eoff[I] + m) * ne + b->eoff[J] + n] = eb[m * nej + n];
        }
}

static void load_c2s(double store[OR_LMAX + 1][OR_MAXNC * (2 * OR_LMAX + 1)], const double *Tl[OR_LMAX + 1]) {
    for (int l = 0; l <= OR_LMAX; ++l) { oracle_c2s(l, store[l]); Tl[l] = store[l]; }
}

/*
 * Full J/K.  D, J, K: [nset][nao_ext][nao_ext] row-major.  Q: optional
 * precomputed Schwarz table [ns*ns] (NULL -> computed here).  mode 0 brute,
 * 1 eight-fold.  *nsig receives the number of significant unique shell
 * quartets (I>=J, K>=L, IJ>=KL) in either mode.
 */
/*
 * Density screening (the direct-SCF screening by the density matrix, at
 * shell-pair level like the Schwarz test): with dscreen > 0 a quartet is
 * kept only if Q_IJ Q_KL max(Dm_IJ, Dm_KL, Dm_IK, Dm_IL, Dm_JK, Dm_JL) >=
 * dscreen, Dm_XY = max over densities and the Cartesian components of the
 * block (X, Y) of |D| (the Cartesian density, double precision).  Applied
 * to a density
 * change Delta D this is the incremental-SCF screening; it bounds every
 * dropped contribution to J and K by dscreen.
 */
static double *dmax_table(const obasis *b, const double *Dc, int nset) {
    const int ns = b->ns, nc = b->nao_cart;
    double *dm = (double *)malloc(sizeof(double) * ns * ns);
    for (int I = 0; I < ns; ++I)
        for (int J = 0; J < ns; ++J) {
            double m = 0.0;
            for (int s = 0; s < nset; ++s)
                for (int a = b->coff[I]; a < b->coff[I + 1]; ++a)
                    for (int c = b->coff[J]; c < b->coff[J + 1]; ++c) m = fmax(m, fabs(Dc[(size_t)s * nc * nc + (size_t)a * nc + c]));
            dm[I * ns + J] = m;
        }
    return dm;
}

static int density_kept(const double *Q, const double *dm, int ns, double dscreen, int I, int J, int K, int L) {
    if (dscreen <= 0.0) return 1;
    double m = dm[I * ns + J];
    m = fmax(m, dm[K * ns + L]);
    m = fmax(m, dm[I * ns + K]);
    m = fmax(m, dm[I * ns + L]);
    m = fmax(m, dm[J * ns + K]);
    m = fmax(m, dm[J * ns + L]);
    return Q[I * ns + J] * Q[K * ns + L] * m >= dscreen;
}

int oracle_jk_screen(BASIS_ARGS, double omega, double dscreen, const double *D, int nset, double cutoff,
                     const double *Qin, int mode, double *Jout, double *Kout, long long *nsig);

int oracle_jk_op(BASIS_ARGS, double omega, const double *D, int nset, double cutoff, const double *Qin, int mode,
                 double *Jout, double *Kout, long long *nsig) {
    return oracle_jk_screen(BASIS_PASS, omega, 0.0, D, nset, cutoff, Qin, mode, Jout, Kout, nsig);
}

int oracle_jk_screen(BASIS_ARGS, double omega, double dscreen, const double *D, int nset, double cutoff,
                     const double *Qin, int mode, double *Jout, double *Kout, long long *nsig) {
    obasis b;
    if (ob_init(&b, BASIS_PASS)) return -1;
    const int ns_ = b.ns, nc = b.nao_cart, ne = b.nao_ext;
    double c2s_store[OR_LMAX + 1][OR_MAXNC * (2 * OR_LMAX + 1)];
    const double *Tl[OR_LMAX + 1];
    load_c2s(c2s_store, Tl);
    double *Q = (double *)malloc(sizeof(double) * ns_ * ns_);
    /* screening always by the full-range Schwarz factors: they bound the
     * long- and short-range integrals too (both operators are 1/r minus a
     * positive semidefinite kernel) */
    if (Qin) memcpy(Q, Qin, sizeof(double) * ns_ * ns_); else schwarz(&b, Q);
    b.omega = omega;
    double *Dc = (double *)malloc(sizeof(double) * nset * nc * nc);
    double *Jc = (double *)calloc((size_t)nset * nc * nc, sizeof(double));
    double *Kc = (double *)calloc((size_t)nset * nc * nc, sizeof(double));
    for (int s = 0; s < nset; ++s) d_to_cart(&b, D + (size_t)s * ne * ne, Dc + (size_t)s * nc * nc, Tl);
    double *dm = dmax_table(&b, Dc, nset);
    long long count = 0;
    const int npair = ns_ * (ns_ + 1) / 2;
#pragma omp parallel reduction(+ : count)
    {
        md_ws w; ws_init(&w);
        double *blk = (double *)malloc(sizeof(double) * OR_MAXNC * OR_MAXNC * OR_MAXNC * OR_MAXNC);
        double *Jp = (double *)calloc((size_t)nset * nc * nc, sizeof(double));
        double *Kp = (double *)calloc((size_t)nset * nc * nc, sizeof(double));
        if (mode == 0) {
#pragma omp for schedule(dynamic, 1)
            for (int IJ = 0; IJ < ns_ * ns_; ++IJ) {
                const int I = IJ / ns_, J = IJ % ns_;
                for (int K = 0; K < ns_; ++K)
                    for (int L = 0; L < ns_; ++L) {
                        if (Q[I * ns_ + J] * Q[K * ns_ + L] < cutoff) continue;
                        if (!density_kept(Q, dm, ns_, dscreen, I, J, K, L)) continue;
                        if (I >= J && K >= L && I * (I + 1) / 2 + J >= K * (K + 1) / 2 + L) ++count;
                        eri_block(&b, I, J, K, L, blk, &w);
                        const int ni = OR_NC(b.l[I]), nj = OR_NC(b.l[J]), nk = OR_NC(b.l[K]), nl = OR_NC(b.l[L]);
                        for (int s = 0; s < nset; ++s) {
                            const double *d = Dc + (size_t)s * nc * nc;
                            double *jj = Jp + (size_t)s * nc * nc, *kk = Kp + (size_t)s * nc * nc;
                            for (int a = 0; a < ni; ++a)
                                for (int bb = 0; bb < nj; ++bb)
                                    for (int c = 0; c < nk; ++c)
                                        for (int dd = 0; dd < nl; ++dd) {
                                            const double v = blk[((a * nj + bb) * nk + c) * nl + dd];
                                            const int ia = b.coff[I] + a, ib = b.coff[J] + bb, ic = b.coff[K] + c, id = b.coff[L] + dd;
                                            jj[ia * nc + ib] += v * d[ic * nc + id];
                                            kk[ia * nc + ic] += v * d[ib * nc + id];
                                        }
                        }
                    }
            }
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int ij = 0; ij < npair; ++ij) {
                int I = (int)((sqrt(8.0 * ij + 1.0) - 1.0) / 2.0);
                while (I * (I + 1) / 2 > ij) --I;
                while ((I + 1) * (I + 2) / 2 <= ij) ++I;
                const int J = ij - I * (I + 1) / 2;
                for (int kl = 0; kl <= ij; ++kl) {
                    int K = (int)((sqrt(8.0 * kl + 1.0) - 1.0) / 2.0);
                    while (K * (K + 1) / 2 > kl) --K;
                    while ((K + 1) * (K + 2) / 2 <= kl) ++K;
                    const int L = kl - K * (K + 1) / 2;
                    if (Q[I * ns_ + J] * Q[K * ns_ + L] < cutoff) continue;
                    if (!density_kept(Q, dm, ns_, dscreen, I, J, K, L)) continue;
                    ++count;
                    double wgt = 1.0;
                    if (I == J) wgt *= 0.5;
                    if (K == L) wgt *= 0.5;
                    if (ij == kl) wgt *= 0.5;
                    eri_block(&b, I, J, K, L, blk, &w);
                    const int ni = OR_NC(b.l[I]), nj = OR_NC(b.l[J]), nk = OR_NC(b.l[K]), nl = OR_NC(b.l[L]);
                    for (int s = 0; s < nset; ++s) {
                        const double *d = Dc + (size_t)s * nc * nc;
                        double *jj = Jp + (size_t)s * nc * nc, *kk = Kp + (size_t)s * nc * nc;
                        for (int a = 0; a < ni; ++a)
                            for (int bb = 0; bb < nj; ++bb)
                                for (int c = 0; c < nk; ++c)
                                    for (int dd = 0; dd < nl; ++dd) {
                                        const double v = wgt * blk[((a * nj + bb) * nk + c) * nl + dd];
                                        const int ia = b.coff[I] + a, ib = b.coff[J] + bb, ic = b.coff[K] + c, id = b.coff[L] + dd;
                                        jj[ia * nc + ib] += 2.0 * v * d[ic * nc + id];
                                        jj[ic * nc + id] += 2.0 * v * d[ia * nc + ib];
                                        kk[ia * nc + ic] += v * d[ib * nc + id];
                                        kk[ia * nc + id] += v * d[ib * nc + ic];
                                        kk[ib * nc + ic] += v * d[ia * nc + id];
                                        kk[ib * nc + id] += v * d[ia * nc + ic];
                                    }
                    }
                }
            }
        }
#pragma omp critical
        {
            for (size_t x = 0; x < (size_t)nset * nc * nc; ++x) { Jc[x] += Jp[x]; Kc[x] += Kp[x]; }
        }
        free(Jp); free(Kp); free(blk); ws_free(&w);
    }
    if (mode == 1) {
        for (int s = 0; s < nset; ++s) {
            double *jj = Jc + (size_t)s * nc * nc, *kk = Kc + (size_t)s * nc * nc;
            for (int a = 0; a < nc; ++a)
                for (int bb = 0; bb <= a; ++bb) {
                    const double js = jj[a * nc + bb] + jj[bb * nc + a];
                    const double ks = kk[a * nc + bb] + kk[bb * nc + a];
                    jj[a * nc + bb] = jj[bb * nc + a] = js;
                    kk[a * nc + bb] = kk[bb * nc + a] = ks;
                }
        }
    }
    for (int s = 0; s < nset; ++s) {
        mat_to_ext(&b, Jc + (size_t)s * nc * nc, Jout + (size_t)s * ne * ne, Tl);
        mat_to_ext(&b, Kc + (size_t)s * nc * nc, Kout + (size_t)s * ne * ne, Tl);
    }
    if (nsig) *nsig = count;
    free(dm); free(Q); free(Dc); free(Jc); free(Kc); ob_free(&b);
    return 0;
}

/*
 * Mixed-precision classification (the split of the benchmark's config 3, a
 * reading of the paper's mixed-precision outlook in Section 6): over the
 * unique quartets I>=J, K>=L, IJ>=KL that pass the Schwarz test, count
 * those whose bound Q_IJ Q_KL max(Dm_IJ, Dm_KL, Dm_IK, Dm_IL, Dm_JK, Dm_JL)
 * is below thr (they may run in single precision).  Dm as in the density
 * screening above (FP64 block maxima of the Cartesian density).
 */
int oracle_mixed_count(BASIS_ARGS, const double *D, int nset, double cutoff, double thr, const double *Qin,
                       long long *nsig, long long *nlow) {
    obasis b;
    if (ob_init(&b, BASIS_PASS)) return -1;
    const int ns_ = b.ns, nc = b.nao_cart, ne = b.nao_ext;
    double c2s_store[OR_LMAX + 1][OR_MAXNC * (2 * OR_LMAX + 1)];
    const double *Tl[OR_LMAX + 1];
    load_c2s(c2s_store, Tl);
    double *Q = (double *)malloc(sizeof(double) * ns_ * ns_);
    if (Qin) memcpy(Q, Qin, sizeof(double) * ns_ * ns_); else schwarz(&b, Q);
    double *Dc = (double *)malloc(sizeof(double) * nset * nc * nc);
    for (int s = 0; s < nset; ++s) d_to_cart(&b, D + (size_t)s * ne * ne, Dc + (size_t)s * nc * nc, Tl);
    double *dm = dmax_table(&b, Dc, nset);
    const int npair = ns_ * (ns_ + 1) / 2;
    long long cs = 0, cl = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : cs, cl)
    for (int ij = 0; ij < npair; ++ij) {
        int I = (int)((sqrt(8.0 * ij + 1.0) - 1.0) / 2.0);
        while (I * (I + 1) / 2 > ij) --I;
        while ((I + 1) * (I + 2) / 2 <= ij) ++I;
        const int J = ij - I * (I + 1) / 2;
        for (int kl = 0; kl <= ij; ++kl) {
            int K = (int)((sqrt(8.0 * kl + 1.0) - 1.0) / 2.0);
            while (K * (K + 1) / 2 > kl) --K;
            while ((K + 1) * (K + 2) / 2 <= kl) ++K;
            const int L = kl - K * (K + 1) / 2;
            const double qq = Q[I * ns_ + J] * Q[K * ns_ + L];
            if (qq < cutoff) continue;
            ++cs;
            double m = dm[I * ns_ + J];
            m = fmax(m, dm[K * ns_ + L]);
            m = fmax(m, dm[I * ns_ + K]);
            m = fmax(m, dm[I * ns_ + L]);
            m = fmax(m, dm[J * ns_ + K]);
            m = fmax(m, dm[J * ns_ + L]);
            if (qq * m < thr) ++cl;
        }
    }
    *nsig = cs;
    *nlow = cl;
    free(dm); free(Dc); free(Q);
    ob_free(&b);
    return 0;
}

int oracle_jk(BASIS_ARGS, const double *D, int nset, double cutoff, const double *Qin, int mode,
              double *Jout, double *Kout, long long *nsig) {
    return oracle_jk_op(BASIS_PASS, 0.0, D, nset, cutoff, Qin, mode, Jout, Kout, nsig);
}

/*
 * Sampled blocks of J and K, straight from the definition (every ordered
 * shell quartet that passes the Schwarz test):
 *   J[I,J] block = sum_{K,L} sum_cd (ab|cd) D_cd      for each (I,J) in jpairs
 *   K[I,K] block = sum_{J,L} sum_bd (ab|cd) D_bd      for each (I,K) in kpairs
 * Output: blocks in the external basis, concatenated in request order, each
 * [nset][nI_ext][nJ_ext].  Q must be the full [ns*ns] Schwarz table.
 */
int oracle_jk_blocks(BASIS_ARGS, const double *D, int nset, double cutoff, const double *Q,
                     int nj_req, const int *jpairs, int nk_req, const int *kpairs,
                     double *Jout, double *Kout) {
    obasis b;
    if (ob_init(&b, BASIS_PASS)) return -1;
    const int ns_ = b.ns, nc = b.nao_cart, ne = b.nao_ext;
    double c2s_store[OR_LMAX + 1][OR_MAXNC * (2 * OR_LMAX + 1)];
    const double *Tl[OR_LMAX + 1];
    load_c2s(c2s_store, Tl);
    double *Dc = (double *)malloc(sizeof(double) * nset * nc * nc);
    for (int s = 0; s < nset; ++s) d_to_cart(&b, D + (size_t)s * ne * ne, Dc + (size_t)s * nc * nc, Tl);
    const int nreq = nj_req + nk_req;
    size_t *ooff = (size_t *)malloc(sizeof(size_t) * (nreq + 1));
    ooff[0] = 0;
    for (int r = 0; r < nreq; ++r) {
        const int *pr = r < nj_req ? jpairs + 2 * r : kpairs + 2 * (r - nj_req);
        ooff[r + 1] = ooff[r] + (size_t)nset * (b.eoff[pr[0] + 1] - b.eoff[pr[0]]) * (b.eoff[pr[1] + 1] - b.eoff[pr[1]]);
    }
    for (int r = 0; r < nreq; ++r) {
        const int isJ = r < nj_req;
        const int *pr = isJ ? jpairs + 2 * r : kpairs + 2 * (r - nj_req);
        const int X = pr[0], Y = pr[1];
        const int nx = OR_NC(b.l[X]), ny = OR_NC(b.l[Y]);
        double *acc = (double *)calloc((size_t)nset * nx * ny, sizeof(double));
#pragma omp parallel
        {
            md_ws w; ws_init(&w);
            double *blk = (double *)malloc(sizeof(double) * OR_MAXNC * OR_MAXNC * OR_MAXNC * OR_MAXNC);
            double *loc = (double *)calloc((size_t)nset * nx * ny, sizeof(double));
#pragma omp for schedule(dynamic, 4)
            for (int P = 0; P < ns_; ++P)
                for (int R = 0; R < ns_; ++R) {
                    /* J: quartet (X Y | P R); K: quartet (X P | Y R) */
                    const int I = X, J = isJ ? Y : P, K = isJ ? P : Y, L = R;
                    if (Q[I * ns_ + J] * Q[K * ns_ + L] < cutoff) continue;
                    eri_block(&b, I, J, K, L, blk, &w);
                    const int ni = OR_NC(b.l[I]), nj = OR_NC(b.l[J]), nk = OR_NC(b.l[K]), nl = OR_NC(b.l[L]);
                    for (int s = 0; s < nset; ++s) {
                        const double *d = Dc + (size_t)s * nc * nc;
                        double *o = loc + (size_t)s * nx * ny;
                        for (int a = 0; a < ni; ++a)
                            for (int bb = 0; bb < nj; ++bb)
                                for (int c = 0; c < nk; ++c)
                                    for (int dd = 0; dd < nl; ++dd) {
                                        const double v = blk[((a * nj + bb) * nk + c) * nl + dd];
                                        if (isJ) o[a * ny + bb] += v * d[(b.coff[K] + c) * nc + b.coff[L] + dd];
                                        else o[a * ny + c] += v * d[(b.coff[J] + bb) * nc + b.coff[L] + dd];
                                    }
                    }
                }
#pragma omp critical
            for (size_t x = 0; x < (size_t)nset * nx * ny; ++x) acc[x] += loc[x];
            free(loc); free(blk); ws_free(&w);
        }
        const int nex = b.eoff[X + 1] - b.eoff[X], ney = b.eoff[Y + 1] - b.eoff[Y];
        double *dst = isJ ? Jout : Kout;
        const size_t base = isJ ? ooff[r] : ooff[r] - ooff[nj_req];
        for (int s = 0; s < nset; ++s)
            block_to_ext(b.l[X], b.l[Y], b.spherical, acc + (size_t)s * nx * ny, dst + base + (size_t)s * nex * ney, Tl);
        free(acc);
    }
    free(ooff); free(Dc); ob_free(&b);
    return 0;
}

/*
 * Eight-fold digestion restricted to the bra pair indices ij in sel[0..nsel)
 * (ij = I(I+1)/2 + J, every canonical ket kl <= ij): a bounded sample of the
 * full build, used only to time the reference on the host.  J', K' are the
 * unsymmetrised partial accumulators [nset][nao_cart][nao_cart] (Cartesian);
 * *nsig receives the number of significant quartets processed.
 */
int oracle_jk_subset(BASIS_ARGS, const double *D, int nset, double cutoff, const double *Q, int nsel,
                     const int *sel, double *Jp_out, double *Kp_out, long long *nsig) {
    obasis b;
    if (ob_init(&b, BASIS_PASS)) return -1;
    const int ns_ = b.ns, nc = b.nao_cart, ne = b.nao_ext;
    double c2s_store[OR_LMAX + 1][OR_MAXNC * (2 * OR_LMAX + 1)];
    const double *Tl[OR_LMAX + 1];
    load_c2s(c2s_store, Tl);
    double *Dc = (double *)malloc(sizeof(double) * nset * nc * nc);
    for (int s = 0; s < nset; ++s) d_to_cart(&b, D + (size_t)s * ne * ne, Dc + (size_t)s * nc * nc, Tl);
    memset(Jp_out, 0, sizeof(double) * nset * nc * nc);
    memset(Kp_out, 0, sizeof(double) * nset * nc * nc);
    long long count = 0;
#pragma omp parallel reduction(+ : count)
    {
        md_ws w; ws_init(&w);
        double *blk = (double *)malloc(sizeof(double) * OR_MAXNC * OR_MAXNC * OR_MAXNC * OR_MAXNC);
        double *Jp = (double *)calloc((size_t)nset * nc * nc, sizeof(double));
        double *Kp = (double *)calloc((size_t)nset * nc * nc, sizeof(double));
#pragma omp for schedule(dynamic, 1)
        for (int si = 0; si < nsel; ++si) {
            const int ij = sel[si];
            int I = (int)((sqrt(8.0 * ij + 1.0) - 1.0) / 2.0);
            while (I * (I + 1) / 2 > ij) --I;
            while ((I + 1) * (I + 2) / 2 <= ij) ++I;
            const int J = ij - I * (I + 1) / 2;
            for (int kl = 0; kl <= ij; ++kl) {
                int K = (int)((sqrt(8.0 * kl + 1.0) - 1.0) / 2.0);
                while (K * (K + 1) / 2 > kl) --K;
                while ((K + 1) * (K + 2) / 2 <= kl) ++K;
                const int L = kl - K * (K + 1) / 2;
                if (Q[I * ns_ + J] * Q[K * ns_ + L] < cutoff) continue;
                ++count;
                double wgt = 1.0;
                if (I == J) wgt *= 0.5;
                if (K == L) wgt *= 0.5;
                if (ij == kl) wgt *= 0.5;
                eri_block(&b, I, J, K, L, blk, &w);
                const int ni = OR_NC(b.l[I]), nj = OR_NC(b.l[J]), nk = OR_NC(b.l[K]), nl = OR_NC(b.l[L]);
                for (int s = 0; s < nset; ++s) {
                    const double *d = Dc + (size_t)s * nc * nc;
                    double *jj = Jp + (size_t)s * nc * nc, *kk = Kp + (size_t)s * nc * nc;
                    for (int a = 0; a < ni; ++a)
                        for (int bb = 0; bb < nj; ++bb)
                            for (int c = 0; c < nk; ++c)
                                for (int dd = 0; dd < nl; ++dd) {
                                    const double v = wgt * blk[((a * nj + bb) * nk + c) * nl + dd];
                                    const int ia = b.coff[I] + a, ib = b.coff[J] + bb, ic = b.coff[K] + c, id = b.coff[L] + dd;
                                    jj[ia * nc + ib] += 2.0 * v * d[ic * nc + id];
                                    jj[ic * nc + id] += 2.0 * v * d[ia * nc + ib];
                                    kk[ia * nc + ic] += v * d[ib * nc + id];
                                    kk[ia * nc + id] += v * d[ib * nc + ic];
                                    kk[ib * nc + ic] += v * d[ia * nc + id];
                                    kk[ib * nc + id] += v * d[ia * nc + ic];
                                }
                }
            }
        }
#pragma omp critical
        {
            for (size_t x = 0; x < (size_t)nset * nc * nc; ++x) { Jp_out[x] += Jp[x]; Kp_out[x] += Kp[x]; }
        }
        free(Jp); free(Kp); free(blk); ws_free(&w);
    }
    if (nsig) *nsig = count;
    free(Dc); ob_free(&b);
    return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

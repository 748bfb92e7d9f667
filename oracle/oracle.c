/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, CPU reference for the quantities the GPU library computes:
 *
 *   (P|ab)  3-center 2-electron Coulomb integrals over contracted Gaussian
 *           shells: Cartesian orbital shells a, b and an auxiliary shell P that
 *           is solid-harmonic (pure = 1) or Cartesian (pure = 0);
 *   J_ab  = sum_P (ab|P) d_P                     (density-fitted Coulomb matrix);
 *   dL/dR for L = sum_ab G_ab J_ab                (nuclear gradient).
 *
 * Definitions follow the paper's Appendix "Notation": a primitive Cartesian
 * Gaussian is (x-A_x)^ax (y-A_y)^ay (z-A_z)^az exp(-zeta |r-A|^2), the
 * integral [ab|c] is the double integral of phi_a phi_b (r1) |r1-r2|^-1
 * phi_c (r2), and contracted integrals (ab|c) sum primitive ones weighted by
 * the contraction coefficients.  The ket is projected on real solid harmonics
 * (Section 2.2 / 2.5.1: the ket is always a solid-harmonic Gaussian).
 *
 * The integrals are evaluated by the McMurchie-Davidson Hermite expansion,
 * the method the paper rejects for the GPU on FLOP count (Section 2.3, Design
 * Pivot 2).  It shares no recurrence with the Obara-Saika scheme of the GPU
 * path: Hermite expansion coefficients E per Cartesian axis, Hermite Coulomb
 * integrals R from the Boys function, and their contraction.  The formulas are
 * the textbook ones (Helgaker, Jorgensen, Olsen, "Molecular Electronic-Structure
 * Theory", chapter 9):
 *
 *   E^{00}_0 = exp(-mu X_AB^2),  mu = za zb / p,  p = za + zb
 *   E^{i+1,j}_t = E^{ij}_{t-1} / (2p) + X_PA E^{ij}_t + (t+1) E^{ij}_{t+1}
 *   E^{i,j+1}_t = E^{ij}_{t-1} / (2p) + X_PB E^{ij}_t + (t+1) E^{ij}_{t+1}
 *   single ket Gaussian (centre C, exponent q): E^0_0 = 1,
 *   E^{k+1}_t = E^k_{t-1} / (2q) + (t+1) E^k_{t+1}
 *   R^n_{000} = (-2 alpha)^n F_n(alpha |PC|^2),  alpha = p q / (p + q)
 *   R^n_{t+1,u,v} = t R^{n+1}_{t-1,u,v} + X_PC R^{n+1}_{t,u,v}  (same in u, v)
 *   [ab|c] = 2 pi^{5/2} / (p q sqrt(p+q))
 *            sum_{tuv} E^{ab}_{tuv} sum_{tau nu phi} (-1)^{tau+nu+phi}
 *                                   E^c_{tau nu phi} R_{t+tau,u+nu,v+phi}
 *
 * The Boys function F_m(T) (Appendix "Notation") is evaluated by its power
 * series for T < 35 followed by downward recursion, and from erf plus upward
 * recursion above.  The gradient differentiates each of the three centres
 * explicitly (d/dA_i phi_a = 2 za phi_{a+1_i} - a_i phi_{a-1_i}), without
 * translational invariance, so that the sum over atoms vanishing is a real
 * check.
 *
 * Built twice: in double (liboracle.so) and, with -DORACLE_LONG, in x87 long
 * double (liboracle_ld.so) for adjudicating disagreements at the 1e-11 level.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef ORACLE_LONG
typedef long double real;
#define R_EXP expl
#define R_SQRT sqrtl
#define R_ERF erfl
#define R_PI 3.141592653589793238462643383279502884L
#else
typedef double real;
#define R_EXP exp
#define R_SQRT sqrt
#define R_ERF erf
#define R_PI 3.141592653589793238462643383279502884
#endif

#define LMAX_ORB 9  /* orbital shells, including the +1 of the gradient */
#define LMAX_AUX 8  /* auxiliary shells, including the +1 of the gradient */
#define GRAD_LMAX_ORB 4  /* orbital shells of the gradient (its work arrays are sized for it) */
#define MMAX_BOYS 40

static int ncart(int l) { return (l + 1) * (l + 2) / 2; }

/* Cartesian component index of (x, y, z) within its shell; see oracle.h. */
static int cart_index(int x, int y, int z) {
  (void)x;
  int i = y + z;
  return i * (i + 1) / 2 + z;
}

static void cart_list(int l, int (*q)[3]) {
  int n = 0;
  for (int i = 0; i <= l; ++i)
    for (int j = 0; j <= i; ++j) {
      q[n][0] = l - i;
      q[n][1] = i - j;
      q[n][2] = j;
      ++n;
    }
}

/* ------------------------------------------------------------------------ */
/* Boys function F_m(T) = int_0^1 y^{2m} exp(-T y^2) dy                      */
/* ------------------------------------------------------------------------ */
static void boys_real(int mmax, real T, real *F) {
  if (T < 35) {
    /* F_M(T) = exp(-T) sum_k (2T)^k / ((2M+1)(2M+3)...(2M+2k+1)), then
     * F_m = (2T F_{m+1} + exp(-T)) / (2m+1) downwards. */
    real term = (real)1 / (2 * mmax + 1), sum = term;
    for (int k = 1; k < 2000; ++k) {
      term *= 2 * T / (2 * mmax + 2 * k + 1);
      sum += term;
      if (term < sum * (real)1e-21) break;
    }
    real et = R_EXP(-T);
    F[mmax] = et * sum;
    for (int m = mmax - 1; m >= 0; --m) F[m] = (2 * T * F[m + 1] + et) / (2 * m + 1);
  } else {
    /* F_0 = (1/2) sqrt(pi/T) erf(sqrt T), F_{m+1} = ((2m+1) F_m - exp(-T)) / (2T) */
    real st = R_SQRT(T), et = R_EXP(-T);
    F[0] = (real)0.5 * R_SQRT(R_PI / T) * R_ERF(st);
    for (int m = 0; m < mmax; ++m) F[m + 1] = ((2 * m + 1) * F[m] - et) / (2 * T);
  }
}

int oracle_boys(int mmax, double T, double *F) {
  if (mmax < 0 || mmax > MMAX_BOYS || !(T >= 0) || !F) return -1;
  real Fr[MMAX_BOYS + 1];
  boys_real(mmax, (real)T, Fr);
  for (int m = 0; m <= mmax; ++m) F[m] = (double)Fr[m];
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Real solid harmonics                                                      */
/* ------------------------------------------------------------------------ */
static real binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  real r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

static real dfact(int n) { /* n!!, with (-1)!! = 1 */
  real r = 1;
  for (int i = n; i > 1; i -= 2) r *= i;
  return r;
}

/* Unnormalised real solid harmonic S_lm as coefficients over the Cartesian
 * monomials of degree l (closed form of Helgaker et al., eq. 6.4.47-6.4.50):
 *   S_lm ~ sum_{t,u,v} C_tuv x^{2t+|m|-2(u+v)} y^{2(u+v)} z^{l-2t-|m|},
 *   C_tuv = (-1)^{t+v-vm} 4^{-t} C(l,t) C(l-t,|m|+t) C(t,u) C(|m|,2v),
 * with vm = 0 (m >= 0) or 1/2 (m < 0) and 2v running over integers of the
 * parity of 2vm up to |m|. */
static void solid_unnormalised(int l, int m, real *row) {
  int am = m < 0 ? -m : m;
  int twovm = m < 0 ? 1 : 0;
  for (int c = 0; c < ncart(l); ++c) row[c] = 0;
  for (int t = 0; t <= (l - am) / 2; ++t)
    for (int u = 0; u <= t; ++u)
      for (int twov = twovm; twov <= am; twov += 2) {
        int sgnexp = t + (twov - twovm) / 2;
        real c = ((sgnexp & 1) ? -1 : 1) * binom(l, t) * binom(l - t, am + t) *
                 binom(t, u) * binom(am, twov);
        for (int k = 0; k < t; ++k) c /= 4;
        int py = 2 * u + twov;
        int px = 2 * t + am - py;
        int pz = l - 2 * t - am;
        row[cart_index(px, py, pz)] += c;
      }
}

/* Overlap of Cartesian components a, b of one contracted shell whose x^l
 * member has unit norm: prod_i (a_i+b_i-1)!! / (2l-1)!!  (0 if any sum odd). */
static real cart_overlap(const int *a, const int *b, int l) {
  real r = 1;
  for (int i = 0; i < 3; ++i) {
    int s = a[i] + b[i];
    if (s & 1) return 0;
    r *= dfact(s - 1);
  }
  return r / dfact(2 * l - 1);
}

static void solid_transform_real(int l, real *T) {
  int nc = ncart(l);
  int q[64][3];
  cart_list(l, q);
  for (int m = -l; m <= l; ++m) {
    real *row = T + (m + l) * nc;
    solid_unnormalised(l, m, row);
    real nrm = 0;
    for (int i = 0; i < nc; ++i)
      for (int j = 0; j < nc; ++j) nrm += row[i] * row[j] * cart_overlap(q[i], q[j], l);
    real s = 1 / R_SQRT(nrm);
    for (int i = 0; i < nc; ++i) row[i] *= s;
  }
}

int oracle_solid_transform(int l, double *T) {
  if (l < 0 || l > LMAX_AUX || !T) return -1;
  real Tr[(2 * LMAX_AUX + 1) * 45];
  solid_transform_real(l, Tr);
  for (int i = 0; i < (2 * l + 1) * ncart(l); ++i) T[i] = (double)Tr[i];
  return 0;
}

/* ------------------------------------------------------------------------ */
/* McMurchie-Davidson primitive integrals                                    */
/* ------------------------------------------------------------------------ */
#define NT (2 * LMAX_ORB + 1)                    /* t range of a bra pair      */
#define NR (2 * LMAX_ORB + LMAX_AUX + 1)         /* t+tau range                */

typedef struct {
  real Ex[LMAX_ORB + 1][LMAX_ORB + 1][NT], Ey[LMAX_ORB + 1][LMAX_ORB + 1][NT],
      Ez[LMAX_ORB + 1][LMAX_ORB + 1][NT];
  real Ec[LMAX_AUX + 1][LMAX_AUX + 1];
  real Rn[NR][NR][NR][NR]; /* Rn[n][t][u][v] */
  real X[NT][NT][NT];      /* ket-contracted Hermite integrals for one c */
} md_work;

/* Hermite coefficients of a bra pair along one axis, E[i][j][t]. */
static void hermite_pair(int imax, int jmax, real za, real zb, real Xab,
                         real E[LMAX_ORB + 1][LMAX_ORB + 1][NT]) {
  real p = za + zb, mu = za * zb / p;
  real Xpa = -zb / p * Xab, Xpb = za / p * Xab, h = 1 / (2 * p);
  memset(E, 0, sizeof(real) * (LMAX_ORB + 1) * (LMAX_ORB + 1) * NT);
  E[0][0][0] = R_EXP(-mu * Xab * Xab);
  for (int i = 0; i <= imax; ++i) {
    if (i > 0)
      for (int t = 0; t <= i; ++t) {
        real v = Xpa * E[i - 1][0][t];
        if (t > 0) v += h * E[i - 1][0][t - 1];
        if (t + 1 <= i - 1) v += (t + 1) * E[i - 1][0][t + 1];
        E[i][0][t] = v;
      }
    for (int j = 1; j <= jmax; ++j)
      for (int t = 0; t <= i + j; ++t) {
        real v = (t <= i + j - 1) ? Xpb * E[i][j - 1][t] : 0;
        if (t > 0) v += h * E[i][j - 1][t - 1];
        if (t + 1 <= i + j - 1) v += (t + 1) * E[i][j - 1][t + 1];
        E[i][j][t] = v;
      }
  }
}

/* Hermite coefficients of a single Gaussian x_C^k exp(-q x_C^2), E[k][t]. */
static void hermite_single(int kmax, real q, real E[LMAX_AUX + 1][LMAX_AUX + 1]) {
  memset(E, 0, sizeof(real) * (LMAX_AUX + 1) * (LMAX_AUX + 1));
  E[0][0] = 1;
  real h = 1 / (2 * q);
  for (int k = 1; k <= kmax; ++k)
    for (int t = 0; t <= k; ++t) {
      real v = 0;
      if (t > 0) v += h * E[k - 1][t - 1];
      if (t + 1 <= k - 1) v += (t + 1) * E[k - 1][t + 1];
      E[k][t] = v;
    }
}

/* Hermite Coulomb integrals R^n_{tuv} for t+u+v+n <= N. */
static void hermite_R(int N, real alpha, real X, real Y, real Z, md_work *w) {
  real F[MMAX_BOYS + 1];
  boys_real(N, alpha * (X * X + Y * Y + Z * Z), F);
  real f = 1;
  for (int n = 0; n <= N; ++n) {
    w->Rn[n][0][0][0] = f * F[n];
    f *= -2 * alpha;
  }
  for (int s = 1; s <= N; ++s)
    for (int n = 0; n <= N - s; ++n)
      for (int t = 0; t <= s; ++t)
        for (int u = 0; u <= s - t; ++u) {
          int v = s - t - u;
          real r;
          if (t > 0) {
            r = X * w->Rn[n + 1][t - 1][u][v];
            if (t > 1) r += (t - 1) * w->Rn[n + 1][t - 2][u][v];
          } else if (u > 0) {
            r = Y * w->Rn[n + 1][t][u - 1][v];
            if (u > 1) r += (u - 1) * w->Rn[n + 1][t][u - 2][v];
          } else {
            r = Z * w->Rn[n + 1][t][u][v - 1];
            if (v > 1) r += (v - 1) * w->Rn[n + 1][t][u][v - 2];
          }
          w->Rn[n][t][u][v] = r;
        }
}

/* Primitive Cartesian block [c][a][b] (no contraction coefficients) for
 * exponents za, zb, zc at centres A, B, C, accumulated as out += scale * [..]. */
static void md_primitive(const real *A, const real *B, const real *C, int la, int lb,
                         int lc, real za, real zb, real zc, real scale, real *out,
                         md_work *w) {
  real p = za + zb, q = zc, alpha = p * q / (p + q);
  real P[3];
  for (int i = 0; i < 3; ++i) P[i] = (za * A[i] + zb * B[i]) / p;
  hermite_pair(la, lb, za, zb, A[0] - B[0], w->Ex);
  hermite_pair(la, lb, za, zb, A[1] - B[1], w->Ey);
  hermite_pair(la, lb, za, zb, A[2] - B[2], w->Ez);
  hermite_single(lc, q, w->Ec);
  int N = la + lb + lc;
  hermite_R(N, alpha, P[0] - C[0], P[1] - C[1], P[2] - C[2], w);
  real pref = scale * 2 * R_PI * R_PI * R_SQRT(R_PI) / (p * q * R_SQRT(p + q));

  int qa[64][3], qb[64][3], qc[64][3];
  cart_list(la, qa);
  cart_list(lb, qb);
  cart_list(lc, qc);
  int nab = la + lb;
  for (int ic = 0; ic < ncart(lc); ++ic) {
    const int *c = qc[ic];
    /* X[tuv] = sum (-1)^{tau+nu+phi} E^c_tau E^c_nu E^c_phi R_{t+tau,u+nu,v+phi} */
    for (int t = 0; t <= nab; ++t)
      for (int u = 0; u <= nab - t; ++u)
        for (int v = 0; v <= nab - t - u; ++v) {
          real s = 0;
          for (int ta = 0; ta <= c[0]; ++ta)
            for (int nu = 0; nu <= c[1]; ++nu)
              for (int ph = 0; ph <= c[2]; ++ph) {
                real e = w->Ec[c[0]][ta] * w->Ec[c[1]][nu] * w->Ec[c[2]][ph];
                if (e == 0) continue;
                if ((ta + nu + ph) & 1) e = -e;
                s += e * w->Rn[0][t + ta][u + nu][v + ph];
              }
          w->X[t][u][v] = s;
        }
    for (int ia = 0; ia < ncart(la); ++ia)
      for (int ib = 0; ib < ncart(lb); ++ib) {
        const int *a = qa[ia], *b = qb[ib];
        real s = 0;
        for (int t = 0; t <= a[0] + b[0]; ++t)
          for (int u = 0; u <= a[1] + b[1]; ++u)
            for (int v = 0; v <= a[2] + b[2]; ++v)
              s += w->Ex[a[0]][b[0]][t] * w->Ey[a[1]][b[1]][u] * w->Ez[a[2]][b[2]][v] *
                   w->X[t][u][v];
        out[(ic * ncart(la) + ia) * ncart(lb) + ib] += pref * s;
      }
  }
}

/* ------------------------------------------------------------------------ */
/* Contracted shell triplets                                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
  int l, K;
  const double *e, *c;
  real R[3];
  int atom;
} shell_view;

static shell_view view(const double *xyz, const oracle_basis *b, int s) {
  shell_view v;
  v.l = b->l[s];
  v.K = b->nprim[s];
  v.e = b->exps + b->prim_off[s];
  v.c = b->coefs + b->prim_off[s];
  v.atom = b->atom[s];
  for (int i = 0; i < 3; ++i) v.R[i] = xyz[3 * v.atom + i];
  return v;
}

static int nfunc(const oracle_basis *b, int l) { return b->pure ? 2 * l + 1 : ncart(l); }

/* Contracted Cartesian block [c][a][b] for shells P (ket), a, b. */
static void contracted_cart(const shell_view *P, const shell_view *a, const shell_view *b,
                            real *out, md_work *w) {
  int n = ncart(P->l) * ncart(a->l) * ncart(b->l);
  for (int i = 0; i < n; ++i) out[i] = 0;
  for (int i = 0; i < a->K; ++i)
    for (int j = 0; j < b->K; ++j)
      for (int k = 0; k < P->K; ++k)
        md_primitive(a->R, b->R, P->R, a->l, b->l, P->l, a->e[i], b->e[j], P->e[k],
                     (real)a->c[i] * b->c[j] * P->c[k], out, w);
}

/* out[p][a][b] = sum_c T[p][c] cart[c][a][b] (copy if Cartesian). */
static void ket_to_pure(int lc, int pure, int nab, const real *cart, real *out) {
  int nc = ncart(lc);
  if (!pure) {
    for (int i = 0; i < nc * nab; ++i) out[i] = cart[i];
    return;
  }
  real T[(2 * LMAX_AUX + 1) * 45];
  solid_transform_real(lc, T);
  for (int p = 0; p < 2 * lc + 1; ++p)
    for (int x = 0; x < nab; ++x) {
      real s = 0;
      for (int c = 0; c < nc; ++c) s += T[p * nc + c] * cart[c * nab + x];
      out[p * nab + x] = s;
    }
}

static int check_basis(const oracle_basis *b, int lmax) {
  if (!b || b->nshell < 0) return -1;
  for (int s = 0; s < b->nshell; ++s)
    if (b->l[s] < 0 || b->l[s] > lmax || b->nprim[s] < 1) return -1;
  return 0;
}

static void set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

/* largest Cartesian block [c][a][b]: aux l <= LMAX_AUX - 1, orbital l <= LMAX_ORB - 1 */
#define NC_AUX ((LMAX_AUX) * (LMAX_AUX + 1) / 2)
#define NC_ORB ((LMAX_ORB) * (LMAX_ORB + 1) / 2)
#define BLK_MAX (NC_AUX * NC_ORB * NC_ORB)

int oracle_eval_batch(const double *xyz, const oracle_basis *aux, const oracle_basis *orb,
                      int64_t ntrip, const int32_t *trip, const int64_t *out_off, double *out,
                      int nthreads) {
  if (check_basis(aux, LMAX_AUX - 1) || check_basis(orb, LMAX_ORB - 1) || ntrip < 0) return -1;
  set_threads(nthreads);
  int err = 0;
#pragma omp parallel
  {
    md_work *w = (md_work *)malloc(sizeof(md_work));
    real *cart = (real *)malloc(sizeof(real) * BLK_MAX);
    real *pure = (real *)malloc(sizeof(real) * BLK_MAX);
#pragma omp for schedule(dynamic, 1)
    for (int64_t t = 0; t < ntrip; ++t) {
      int sP = trip[3 * t], sa = trip[3 * t + 1], sb = trip[3 * t + 2];
      if (sP < 0 || sP >= aux->nshell || sa < 0 || sa >= orb->nshell || sb < 0 ||
          sb >= orb->nshell) {
        err = -1;
        continue;
      }
      shell_view P = view(xyz, aux, sP), a = view(xyz, orb, sa), b = view(xyz, orb, sb);
      int nab = ncart(a.l) * ncart(b.l);
      contracted_cart(&P, &a, &b, cart, w);
      ket_to_pure(P.l, aux->pure, nab, cart, pure);
      int n = nfunc(aux, P.l) * nab;
      for (int i = 0; i < n; ++i) out[out_off[t] + i] = (double)pure[i];
    }
    free(w);
    free(cart);
    free(pure);
  }
  return err;
}

static void offsets(const oracle_basis *b, int64_t *off) {
  int64_t o = 0;
  for (int s = 0; s < b->nshell; ++s) {
    off[s] = o;
    o += nfunc(b, b->l[s]);
  }
  off[b->nshell] = o;
}

/* J block for orbital shells (sa, sb): Jblk[i][j] = sum_P sum_p (ab|P)_{pij} d_{P p}. */
static void J_block(const double *xyz, const oracle_basis *aux, const oracle_basis *orb,
                    const double *d, const int64_t *aoff, int sa, int sb, real *Jblk,
                    real *cart, real *pure, md_work *w) {
  shell_view a = view(xyz, orb, sa), b = view(xyz, orb, sb);
  int nab = ncart(a.l) * ncart(b.l);
  for (int x = 0; x < nab; ++x) Jblk[x] = 0;
  for (int sP = 0; sP < aux->nshell; ++sP) {
    shell_view P = view(xyz, aux, sP);
    contracted_cart(&P, &a, &b, cart, w);
    ket_to_pure(P.l, aux->pure, nab, cart, pure);
    for (int p = 0; p < nfunc(aux, P.l); ++p)
      for (int x = 0; x < nab; ++x) Jblk[x] += pure[p * nab + x] * d[aoff[sP] + p];
  }
}

/* Bra transform of one Cartesian block (of J, or of (P|ab) for one P) onto real solid harmonics on both
 * orbital shells: out[i'][j'] = sum_ij T_la[i'][i] T_lb[j'][j] cart[i][j]
 * (Section 2.5.1: the solid-harmonic transform is linear and acts on each
 * shell's Cartesian index; the same T as for the ket). */
static void bra_to_pure(int la, int lb, const real *cart, real *out) {
  int na = ncart(la), nb = ncart(lb);
  real Ta[(2 * LMAX_AUX + 1) * 45], Tb[(2 * LMAX_AUX + 1) * 45];
  solid_transform_real(la, Ta);
  solid_transform_real(lb, Tb);
  for (int ip = 0; ip < 2 * la + 1; ++ip)
    for (int jp = 0; jp < 2 * lb + 1; ++jp) {
      real v = 0;
      for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j) v += Ta[ip * na + i] * Tb[jp * nb + j] * cart[i * nb + j];
      out[ip * (2 * lb + 1) + jp] = v;
    }
}

/* gamma_P = sum_{a,b} (P|ab) D_ab over all ordered orbital shell pairs: the
 * definition written out (the contraction of the right-hand side of the fitting
 * equations, and dL/dd for L = sum_ab G_ab J_ab with D = G).  One loop
 * iteration owns one aux shell. */
int oracle_coulomb_gamma(const double *xyz, const oracle_basis *aux, const oracle_basis *orb,
                         const double *D, double *gamma, int nthreads) {
  if (check_basis(aux, LMAX_AUX - 1) || check_basis(orb, LMAX_ORB - 1) ||
      (orb->pure != 0 && orb->pure != 1))
    return -1;
  set_threads(nthreads);
  int64_t *aoff = (int64_t *)malloc(sizeof(int64_t) * (aux->nshell + 1));
  int64_t *ooff = (int64_t *)malloc(sizeof(int64_t) * (orb->nshell + 1));
  offsets(aux, aoff);
  offsets(orb, ooff);
  int64_t nao = ooff[orb->nshell];
#pragma omp parallel
  {
    md_work *w = (md_work *)malloc(sizeof(md_work));
    real *cart = (real *)malloc(sizeof(real) * BLK_MAX);
    real *pure = (real *)malloc(sizeof(real) * BLK_MAX);
    real blk[NC_ORB * NC_ORB], bp[NC_ORB * NC_ORB];
#pragma omp for schedule(dynamic, 1)
    for (int sP = 0; sP < aux->nshell; ++sP) {
      shell_view P = view(xyz, aux, sP);
      int np = nfunc(aux, P.l);
      real acc[2 * LMAX_AUX + 1 > 64 ? 2 * LMAX_AUX + 1 : 64];
      for (int p = 0; p < np; ++p) acc[p] = 0;
      for (int sa = 0; sa < orb->nshell; ++sa)
        for (int sb = 0; sb < orb->nshell; ++sb) {
          shell_view a = view(xyz, orb, sa), b = view(xyz, orb, sb);
          int na = ncart(a.l), nb = ncart(b.l), nab = na * nb;
          contracted_cart(&P, &a, &b, cart, w);
          ket_to_pure(P.l, aux->pure, nab, cart, pure);
          if (!orb->pure) {
            for (int p = 0; p < np; ++p)
              for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j)
                  acc[p] += pure[p * nab + i * nb + j] * D[(ooff[sa] + i) * nao + ooff[sb] + j];
            continue;
          }
          /* solid-harmonic orbital shells: (P|a'b') = sum_ij T_a[a'][i]
           * T_b[b'][j] (P|ij), contracted with D over the pure functions */
          int npa = 2 * a.l + 1, npb = 2 * b.l + 1;
          for (int p = 0; p < np; ++p) {
            for (int x = 0; x < nab; ++x) blk[x] = pure[p * nab + x];
            bra_to_pure(a.l, b.l, blk, bp);
            for (int i = 0; i < npa; ++i)
              for (int j = 0; j < npb; ++j)
                acc[p] += bp[i * npb + j] * D[(ooff[sa] + i) * nao + ooff[sb] + j];
          }
        }
      for (int p = 0; p < np; ++p) gamma[aoff[sP] + p] = (double)acc[p];
    }
    free(w);
    free(cart);
    free(pure);
  }
  free(aoff);
  free(ooff);
  return 0;
}

/* V[P][Q] = (P|Q), the two-centre Coulomb integrals of the aux basis: the
 * three-centre integral with Q as the bra shell and a unit s function
 * (exponent 0, coefficient 1) as its partner, the bra then taken to the same
 * (pure or Cartesian) functions as the ket. */
int oracle_coulomb_metric(const double *xyz, const oracle_basis *aux, double *V, int nthreads) {
  /* Q is the bra: aux l <= LMAX_AUX - 1 is within the orbital range */
  if (check_basis(aux, LMAX_AUX - 1)) return -1;
  set_threads(nthreads);
  int64_t *aoff = (int64_t *)malloc(sizeof(int64_t) * (aux->nshell + 1));
  offsets(aux, aoff);
  int64_t naux = aoff[aux->nshell];
  static const double zero_exp = 0.0, unit_coef = 1.0;
#pragma omp parallel
  {
    md_work *w = (md_work *)malloc(sizeof(md_work));
    real *cart = (real *)malloc(sizeof(real) * BLK_MAX);
    real *pure = (real *)malloc(sizeof(real) * BLK_MAX);
    real Tq[(2 * LMAX_AUX + 1) * 45];
#pragma omp for schedule(dynamic, 1)
    for (int sP = 0; sP < aux->nshell; ++sP) {
      shell_view P = view(xyz, aux, sP);
      int npP = nfunc(aux, P.l);
      for (int sQ = 0; sQ < aux->nshell; ++sQ) {
        shell_view Q = view(xyz, aux, sQ);
        shell_view one = Q;
        one.l = 0;
        one.K = 1;
        one.e = &zero_exp;
        one.c = &unit_coef;
        int nq = ncart(Q.l), npQ = nfunc(aux, Q.l);
        contracted_cart(&P, &Q, &one, cart, w);       /* [c][q] */
        ket_to_pure(P.l, aux->pure, nq, cart, pure);  /* [p][q] */
        if (aux->pure) solid_transform_real(Q.l, Tq);
        for (int p = 0; p < npP; ++p)
          for (int q = 0; q < npQ; ++q) {
            real v = 0;
            if (aux->pure)
              for (int c = 0; c < nq; ++c) v += Tq[q * nq + c] * pure[p * nq + c];
            else
              v = pure[p * nq + q];
            V[(aoff[sP] + p) * naux + aoff[sQ] + q] = (double)v;
          }
      }
    }
    free(w);
    free(cart);
    free(pure);
  }
  free(aoff);
  return 0;
}

int oracle_coulomb_J(const double *xyz, const oracle_basis *aux, const oracle_basis *orb,
                     const double *d, double *J, int nthreads) {
  if (check_basis(aux, LMAX_AUX - 1) || check_basis(orb, LMAX_ORB - 1) ||
      (orb->pure != 0 && orb->pure != 1))
    return -1;
  set_threads(nthreads);
  int64_t *aoff = (int64_t *)malloc(sizeof(int64_t) * (aux->nshell + 1));
  int64_t *ooff = (int64_t *)malloc(sizeof(int64_t) * (orb->nshell + 1));
  offsets(aux, aoff);
  offsets(orb, ooff);
  int64_t nao = ooff[orb->nshell];
  int64_t npair = (int64_t)orb->nshell * (orb->nshell + 1) / 2;
#pragma omp parallel
  {
    md_work *w = (md_work *)malloc(sizeof(md_work));
    real *cart = (real *)malloc(sizeof(real) * BLK_MAX);
    real *pure = (real *)malloc(sizeof(real) * BLK_MAX);
    real Jblk[NC_ORB * NC_ORB], Jp[NC_ORB * NC_ORB];
#pragma omp for schedule(dynamic, 1)
    for (int64_t k = 0; k < npair; ++k) {
      /* k -> (sa >= sb) */
      int sa = (int)((sqrt(8.0 * (double)k + 1) - 1) / 2);
      while ((int64_t)sa * (sa + 1) / 2 > k) --sa;
      while ((int64_t)(sa + 1) * (sa + 2) / 2 <= k) ++sa;
      int sb = (int)(k - (int64_t)sa * (sa + 1) / 2);
      J_block(xyz, aux, orb, d, aoff, sa, sb, Jblk, cart, pure, w);
      const real *out = Jblk;
      if (orb->pure) {
        bra_to_pure(orb->l[sa], orb->l[sb], Jblk, Jp);
        out = Jp;
      }
      int na = nfunc(orb, orb->l[sa]), nb = nfunc(orb, orb->l[sb]);
      for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j) {
          J[(ooff[sa] + i) * nao + ooff[sb] + j] = (double)out[i * nb + j];
          J[(ooff[sb] + j) * nao + ooff[sa] + i] = (double)out[i * nb + j];
        }
    }
    free(w);
    free(cart);
    free(pure);
  }
  free(aoff);
  free(ooff);
  return 0;
}

int oracle_coulomb_J_masked(const double *xyz, const oracle_basis *aux, const oracle_basis *orb,
                            const double *d, const uint8_t *mask, double *J, int nthreads) {
  if (check_basis(aux, LMAX_AUX - 1) || check_basis(orb, LMAX_ORB - 1) || orb->pure || !mask)
    return -1;
  set_threads(nthreads);
  int64_t *aoff = (int64_t *)malloc(sizeof(int64_t) * (aux->nshell + 1));
  int64_t *ooff = (int64_t *)malloc(sizeof(int64_t) * (orb->nshell + 1));
  offsets(aux, aoff);
  offsets(orb, ooff);
  int64_t nao = ooff[orb->nshell];
  int64_t npair = (int64_t)orb->nshell * (orb->nshell + 1) / 2;
  for (int64_t x = 0; x < nao * nao; ++x) J[x] = 0.0;
#pragma omp parallel
  {
    md_work *w = (md_work *)malloc(sizeof(md_work));
    real *cart = (real *)malloc(sizeof(real) * BLK_MAX);
    real *pure = (real *)malloc(sizeof(real) * BLK_MAX);
    real Jblk[NC_ORB * NC_ORB];
#pragma omp for schedule(dynamic, 1)
    for (int64_t k = 0; k < npair; ++k) {
      int sa = (int)((sqrt(8.0 * (double)k + 1) - 1) / 2);
      while ((int64_t)sa * (sa + 1) / 2 > k) --sa;
      while ((int64_t)(sa + 1) * (sa + 2) / 2 <= k) ++sa;
      int sb = (int)(k - (int64_t)sa * (sa + 1) / 2);
      if (!mask[(int64_t)sa * orb->nshell + sb]) continue;
      J_block(xyz, aux, orb, d, aoff, sa, sb, Jblk, cart, pure, w);
      int na = ncart(orb->l[sa]), nb = ncart(orb->l[sb]);
      for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j) {
          J[(ooff[sa] + i) * nao + ooff[sb] + j] = (double)Jblk[i * nb + j];
          J[(ooff[sb] + j) * nao + ooff[sa] + i] = (double)Jblk[i * nb + j];
        }
    }
    free(w);
    free(cart);
    free(pure);
  }
  free(aoff);
  free(ooff);
  return 0;
}

int oracle_screen_pairs(const double *xyz, const oracle_basis *orb, double tau, uint8_t *mask,
                        double *S) {
  if (check_basis(orb, LMAX_ORB - 1) || !mask) return -1;
  const double pi = 3.14159265358979323846;
  for (int a = 0; a < orb->nshell; ++a)
    for (int b = 0; b <= a; ++b) {
      const double *A = xyz + 3 * orb->atom[a], *B = xyz + 3 * orb->atom[b];
      const double ab2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) +
                         (A[2] - B[2]) * (A[2] - B[2]);
      double smax = 0.0;
      for (int i = 0; i < orb->nprim[a]; ++i)
        for (int j = 0; j < orb->nprim[b]; ++j) {
          const double za = orb->exps[orb->prim_off[a] + i], zb = orb->exps[orb->prim_off[b] + j];
          const double ca = orb->coefs[orb->prim_off[a] + i], cb = orb->coefs[orb->prim_off[b] + j];
          const double g = za + zb;
          const double v = fabs(ca * cb) * pow(pi / g, 1.5) * exp(-za * zb / g * ab2);
          if (v > smax) smax = v;
        }
      const uint8_t keep = smax >= tau;
      mask[(int64_t)a * orb->nshell + b] = mask[(int64_t)b * orb->nshell + a] = keep;
      if (S) S[(int64_t)a * orb->nshell + b] = S[(int64_t)b * orb->nshell + a] = smax;
    }
  return 0;
}

/* Schwarz-type bounds of the 3-center integrals (not in the paper; the
 * screening reading of this build).  A primitive Cartesian component of l
 * quanta satisfies |x^i y^j z^k| e^{-a r^2} <= r^l e^{-a r^2}
 * <= M_l(a) e^{-theta a r^2}, with theta = 1, M_0 = 1 for l = 0 and
 * theta = 1/2, M_l(a) = (l / (a e))^{l/2} (the maximum of r^l e^{-a r^2 / 2})
 * for l > 0.  So |phi_a phi_b| is bounded pointwise by a positive sum of
 * s-type Gaussians, |phi_P| likewise (times t_l = max_m sum_c |T_mc| for a
 * solid-harmonic shell), and, the Coulomb kernel being positive and positive
 * definite, |(ab|P_m)| <= (env_ab|env_P) <= Q_ab Q_P with
 *   Q_ab = sum_ij |c_i c_j| M(a_i) M(b_j) e^{-mu_ij AB^2} sqrt((g|g)_ij),
 * (g|g) = 2 pi^{5/2} / (gamma^2 sqrt(2 gamma)) the self-repulsion of
 * e^{-gamma r^2}, gamma and mu from the envelope exponents theta a_i,
 * theta b_j; Q_P = t_l sum_k |c_k| M(z_k) sqrt((g|g)) with gamma = theta z_k. */
static double env_m(int l, double a) {
  return l == 0 ? 1.0 : pow(l / (a * 2.718281828459045235360287), 0.5 * l);
}
static double env_theta(int l) { return l == 0 ? 1.0 : 0.5; }
static double self_rep(double g) {
  return sqrt(2.0 * 17.493418327624862 / (g * g * sqrt(2.0 * g)));  /* 2 pi^{5/2}: 34.98.. */
}

int oracle_schwarz_bounds(const double *xyz, const oracle_basis *aux, const oracle_basis *orb,
                          double *Qab, double *QP) {
  if (check_basis(aux, LMAX_AUX - 1) || check_basis(orb, LMAX_ORB - 1) || !Qab || !QP) return -1;
  for (int a = 0; a < orb->nshell; ++a)
    for (int b = 0; b <= a; ++b) {
      const double *A = xyz + 3 * orb->atom[a], *B = xyz + 3 * orb->atom[b];
      const double ab2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) +
                         (A[2] - B[2]) * (A[2] - B[2]);
      const int la = orb->l[a], lb = orb->l[b];
      double q = 0.0;
      for (int i = 0; i < orb->nprim[a]; ++i)
        for (int j = 0; j < orb->nprim[b]; ++j) {
          const double za = orb->exps[orb->prim_off[a] + i], zb = orb->exps[orb->prim_off[b] + j];
          const double ca = orb->coefs[orb->prim_off[a] + i], cb = orb->coefs[orb->prim_off[b] + j];
          const double ea = env_theta(la) * za, eb = env_theta(lb) * zb, g = ea + eb;
          q += fabs(ca * cb) * env_m(la, za) * env_m(lb, zb) * exp(-ea * eb / g * ab2) *
               self_rep(g);
        }
      Qab[(int64_t)a * orb->nshell + b] = Qab[(int64_t)b * orb->nshell + a] = q;
    }
  for (int p = 0; p < aux->nshell; ++p) {
    const int l = aux->l[p];
    double t = 1.0;
    if (aux->pure) {
      double T[(2 * LMAX_AUX + 1) * 45];
      oracle_solid_transform(l, T);
      const int nc = (l + 1) * (l + 2) / 2;
      t = 0.0;
      for (int m = 0; m < 2 * l + 1; ++m) {
        double r = 0.0;
        for (int c = 0; c < nc; ++c) r += fabs(T[m * nc + c]);
        if (r > t) t = r;
      }
    }
    double q = 0.0;
    for (int k = 0; k < aux->nprim[p]; ++k) {
      const double z = aux->exps[aux->prim_off[p] + k], c = aux->coefs[aux->prim_off[p] + k];
      q += fabs(c) * env_m(l, z) * self_rep(env_theta(l) * z);
    }
    QP[p] = t * q;
  }
  return 0;
}

/* mask[a][b] = (Q_ab S_d >= tau), S_d = sum_P Q_P sum_m |d_Pm|: the J blocks
 * of the dropped pairs are bounded by tau element by element. */
int oracle_screen_pairs_schwarz(const double *xyz, const oracle_basis *aux,
                                const oracle_basis *orb, const double *d, double tau,
                                uint8_t *mask, double *Sd) {
  if (!mask || !d || !(tau >= 0.0)) return -1;
  const int64_t n = orb->nshell;
  double *Qab = (double *)malloc(sizeof(double) * (n * n > 0 ? n * n : 1));
  double *QP = (double *)malloc(sizeof(double) * (aux->nshell > 0 ? aux->nshell : 1));
  int rc = oracle_schwarz_bounds(xyz, aux, orb, Qab, QP);
  if (!rc) {
    double s = 0.0;
    int64_t off = 0;
    for (int p = 0; p < aux->nshell; ++p) {
      const int l = aux->l[p], nf = aux->pure ? 2 * l + 1 : (l + 1) * (l + 2) / 2;
      double a1 = 0.0;
      for (int m = 0; m < nf; ++m) a1 += fabs(d[off + m]);
      off += nf;
      s += QP[p] * a1;
    }
    for (int64_t x = 0; x < n * n; ++x) mask[x] = Qab[x] * s >= tau;
    if (Sd) *Sd = s;
  }
  free(Qab);
  free(QP);
  return rc;
}

int oracle_coulomb_J_pairs(const double *xyz, const oracle_basis *aux, const oracle_basis *orb,
                           const double *d, int64_t npair, const int32_t *pairs,
                           const int64_t *out_off, double *out, int nthreads) {
  if (check_basis(aux, LMAX_AUX - 1) || check_basis(orb, LMAX_ORB - 1) || orb->pure) return -1;
  set_threads(nthreads);
  int64_t *aoff = (int64_t *)malloc(sizeof(int64_t) * (aux->nshell + 1));
  offsets(aux, aoff);
  int err = 0;
#pragma omp parallel
  {
    md_work *w = (md_work *)malloc(sizeof(md_work));
    real *cart = (real *)malloc(sizeof(real) * BLK_MAX);
    real *pure = (real *)malloc(sizeof(real) * BLK_MAX);
    real Jblk[NC_ORB * NC_ORB];
#pragma omp for schedule(dynamic, 1)
    for (int64_t k = 0; k < npair; ++k) {
      int sa = pairs[2 * k], sb = pairs[2 * k + 1];
      if (sa < 0 || sa >= orb->nshell || sb < 0 || sb >= orb->nshell) {
        err = -1;
        continue;
      }
      J_block(xyz, aux, orb, d, aoff, sa, sb, Jblk, cart, pure, w);
      int n = ncart(orb->l[sa]) * ncart(orb->l[sb]);
      for (int x = 0; x < n; ++x) out[out_off[k] + x] = (double)Jblk[x];
    }
    free(w);
    free(cart);
    free(pure);
  }
  free(aoff);
  return err;
}

/* ------------------------------------------------------------------------ */
/* Gradient                                                                  */
/* ------------------------------------------------------------------------ */
/* Contracted derivative blocks of one triplet.  D[3 centres][3 axes] each a
 * Cartesian block [c][a][b]; centre 0 = a, 1 = b, 2 = P. */
static void contracted_deriv(const shell_view *P, const shell_view *a, const shell_view *b,
                             real *D /* [9][nblk] */, real *tmp, md_work *w) {
  int la = a->l, lb = b->l, lc = P->l;
  int na = ncart(la), nb = ncart(lb), nc = ncart(lc);
  int nblk = nc * na * nb;
  int qa[64][3], qb[64][3], qc[64][3];
  cart_list(la, qa);
  cart_list(lb, qb);
  cart_list(lc, qc);
  for (int i = 0; i < 9 * nblk; ++i) D[i] = 0;
  /* tmp holds six primitive blocks: a+1, a-1, b+1, b-1, c+1, c-1 */
  int nA1 = ncart(lc) * ncart(la + 1) * nb, nAm = la > 0 ? nc * ncart(la - 1) * nb : 0;
  int nB1 = nc * na * ncart(lb + 1), nBm = lb > 0 ? nc * na * ncart(lb - 1) : 0;
  int nC1 = ncart(lc + 1) * na * nb, nCm = lc > 0 ? ncart(lc - 1) * na * nb : 0;
  real *A1 = tmp, *Am = A1 + nA1, *B1 = Am + nAm, *Bm = B1 + nB1, *C1 = Bm + nBm,
       *Cm = C1 + nC1;
  for (int i = 0; i < a->K; ++i)
    for (int j = 0; j < b->K; ++j)
      for (int k = 0; k < P->K; ++k) {
        real za = a->e[i], zb = b->e[j], zc = P->e[k];
        real cf = (real)a->c[i] * b->c[j] * P->c[k];
        int tot = nA1 + nAm + nB1 + nBm + nC1 + nCm;
        for (int x = 0; x < tot; ++x) tmp[x] = 0;
        md_primitive(a->R, b->R, P->R, la + 1, lb, lc, za, zb, zc, 1, A1, w);
        if (la > 0) md_primitive(a->R, b->R, P->R, la - 1, lb, lc, za, zb, zc, 1, Am, w);
        md_primitive(a->R, b->R, P->R, la, lb + 1, lc, za, zb, zc, 1, B1, w);
        if (lb > 0) md_primitive(a->R, b->R, P->R, la, lb - 1, lc, za, zb, zc, 1, Bm, w);
        md_primitive(a->R, b->R, P->R, la, lb, lc + 1, za, zb, zc, 1, C1, w);
        if (lc > 0) md_primitive(a->R, b->R, P->R, la, lb, lc - 1, za, zb, zc, 1, Cm, w);
        for (int ic = 0; ic < nc; ++ic)
          for (int ia = 0; ia < na; ++ia)
            for (int ib = 0; ib < nb; ++ib) {
              const int *qa_ = qa[ia], *qb_ = qb[ib], *qc_ = qc[ic];
              int o = (ic * na + ia) * nb + ib;
              for (int ax = 0; ax < 3; ++ax) {
                int up[3], dn[3];
                /* centre a */
                for (int r = 0; r < 3; ++r) up[r] = dn[r] = qa_[r];
                up[ax]++;
                dn[ax]--;
                real v = 2 * za *
                         A1[(ic * ncart(la + 1) + cart_index(up[0], up[1], up[2])) * nb + ib];
                if (qa_[ax] > 0)
                  v -= qa_[ax] *
                       Am[(ic * ncart(la - 1) + cart_index(dn[0], dn[1], dn[2])) * nb + ib];
                D[(0 * 3 + ax) * nblk + o] += cf * v;
                /* centre b */
                for (int r = 0; r < 3; ++r) up[r] = dn[r] = qb_[r];
                up[ax]++;
                dn[ax]--;
                v = 2 * zb *
                    B1[(ic * na + ia) * ncart(lb + 1) + cart_index(up[0], up[1], up[2])];
                if (qb_[ax] > 0)
                  v -= qb_[ax] *
                       Bm[(ic * na + ia) * ncart(lb - 1) + cart_index(dn[0], dn[1], dn[2])];
                D[(1 * 3 + ax) * nblk + o] += cf * v;
                /* centre P */
                for (int r = 0; r < 3; ++r) up[r] = dn[r] = qc_[r];
                up[ax]++;
                dn[ax]--;
                v = 2 * zc * C1[(cart_index(up[0], up[1], up[2]) * na + ia) * nb + ib];
                if (qc_[ax] > 0)
                  v -= qc_[ax] * Cm[(cart_index(dn[0], dn[1], dn[2]) * na + ia) * nb + ib];
                D[(2 * 3 + ax) * nblk + o] += cf * v;
              }
            }
      }
}

int oracle_coulomb_J_grad(const double *xyz, int32_t natom, const oracle_basis *aux,
                          const oracle_basis *orb, const double *d, const double *G,
                          const uint8_t *atom_mask, const uint8_t *pair_mask, double *grad,
                          int nthreads) {
  if (check_basis(aux, LMAX_AUX - 2) || check_basis(orb, GRAD_LMAX_ORB) ||
      (orb->pure != 0 && orb->pure != 1) || natom < 0)
    return -1;
  set_threads(nthreads);
  int64_t *aoff = (int64_t *)malloc(sizeof(int64_t) * (aux->nshell + 1));
  int64_t *ooff = (int64_t *)malloc(sizeof(int64_t) * (orb->nshell + 1));
  offsets(aux, aoff);
  offsets(orb, ooff);
  int64_t nao = ooff[orb->nshell];
  int64_t npair = (int64_t)orb->nshell * orb->nshell; /* all ordered pairs */
  real *gacc = (real *)calloc((size_t)natom * 3, sizeof(real));
  int err = 0;
#pragma omp parallel
  {
    md_work *w = (md_work *)malloc(sizeof(md_work));
    int nblk_max = 45 * 28 * 28;
    real *D = (real *)malloc(sizeof(real) * 9 * nblk_max);
    real *tmp = (real *)malloc(sizeof(real) * 6 * 55 * 36 * 36);
    real *pure = (real *)malloc(sizeof(real) * nblk_max);
    real T[(2 * LMAX_AUX + 1) * 45], Ta[(2 * LMAX_AUX + 1) * 45], Tb[(2 * LMAX_AUX + 1) * 45];
    real Gblk[NC_ORB * NC_ORB];
    real *g = (real *)calloc((size_t)natom * 3, sizeof(real));
#pragma omp for schedule(dynamic, 1)
    for (int64_t k = 0; k < npair; ++k) {
      int sa = (int)(k / orb->nshell), sb = (int)(k % orb->nshell);
      if (pair_mask && !pair_mask[k]) continue;
      shell_view a = view(xyz, orb, sa), b = view(xyz, orb, sb);
      if (a.atom < 0 || a.atom >= natom || b.atom < 0 || b.atom >= natom) {
        err = -1;
        continue;
      }
      int na = ncart(a.l), nb = ncart(b.l), nab = na * nb;
      /* weights of the Cartesian J block: G itself, or for solid-harmonic
       * orbital shells (J_pure = T_a J_cart T_b^T) the pulled-back
       * G_cart = T_a^T G_pure T_b */
      if (orb->pure) {
        solid_transform_real(a.l, Ta);
        solid_transform_real(b.l, Tb);
      }
      for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j) {
          if (!orb->pure) {
            Gblk[i * nb + j] = G[(ooff[sa] + i) * nao + ooff[sb] + j];
            continue;
          }
          real v = 0;
          for (int ip = 0; ip < 2 * a.l + 1; ++ip)
            for (int jp = 0; jp < 2 * b.l + 1; ++jp)
              v += Ta[ip * na + i] * Tb[jp * nb + j] * G[(ooff[sa] + ip) * nao + ooff[sb] + jp];
          Gblk[i * nb + j] = v;
        }
      for (int sP = 0; sP < aux->nshell; ++sP) {
        shell_view P = view(xyz, aux, sP);
        if (P.atom < 0 || P.atom >= natom) {
          err = -1;
          continue;
        }
        if (atom_mask && !atom_mask[a.atom] && !atom_mask[b.atom] && !atom_mask[P.atom])
          continue;
        contracted_deriv(&P, &a, &b, D, tmp, w);
        int nc = ncart(P.l), np = nfunc(aux, P.l);
        if (aux->pure) solid_transform_real(P.l, T);
        int atoms[3] = {a.atom, b.atom, P.atom};
        for (int cen = 0; cen < 3; ++cen)
          for (int ax = 0; ax < 3; ++ax) {
            const real *blk = D + (cen * 3 + ax) * nc * nab;
            real s = 0;
            for (int p = 0; p < np; ++p) {
              real dp = d[aoff[sP] + p];
              for (int x = 0; x < nab; ++x) {
                real v;
                if (aux->pure) {
                  v = 0;
                  for (int c = 0; c < nc; ++c) v += T[p * nc + c] * blk[c * nab + x];
                } else {
                  v = blk[p * nab + x];
                }
                s += v * dp * Gblk[x];
              }
            }
            g[atoms[cen] * 3 + ax] += s;
          }
      }
    }
#pragma omp critical
    for (int i = 0; i < natom * 3; ++i) gacc[i] += g[i];
    free(w);
    free(D);
    free(tmp);
    free(pure);
    free(g);
  }
  for (int i = 0; i < natom * 3; ++i) grad[i] = (double)gacc[i];
  free(gacc);
  free(aoff);
  free(ooff);
  return err;
}

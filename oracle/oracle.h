/*
 * oracle.h -- test infrastructure only (see oracle.c).
 *
 * Plain CPU reference for 3-center Coulomb integrals (P|ab), the density-fitted
 * Coulomb matrix J_ab = sum_P (ab|P) d_P and the nuclear gradient of
 * L = sum_ab G_ab J_ab.  All arrays are HOST arrays.  Only tests/, the smoke
 * check and the CPU-baseline leg of the benchmark may call it.
 *
 * Conventions (the paper leaves them open; Appendix "Notation" defines the
 * integrals, Section 2.5.1 fixes the ket as a solid-harmonic Gaussian):
 *   - Cartesian component order inside a shell of l quanta:
 *       for i = 0..l, for j = 0..i: (l-i, i-j, j)       (xx,xy,xz,yy,yz,zz)
 *   - real solid harmonics ordered m = -l..+l, leading monomial positive,
 *     scaled so that T S_cart T^T = I where S_cart is the overlap of the
 *     Cartesian components of one contracted shell whose x^l member has unit
 *     norm.
 *   - contraction coefficients passed in already include all normalisation.
 *   - a block (P|ab) is stored [p][i][j] row-major (P slowest, b fastest).
 */
#ifndef DF3C_ORACLE_H
#define DF3C_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t nshell;
  const int32_t *l;        /* [nshell] angular momentum */
  const int32_t *nprim;    /* [nshell] contraction degree K >= 1 */
  const int64_t *prim_off; /* [nshell] offset into exps/coefs */
  const int32_t *atom;     /* [nshell] index into xyz */
  const double *exps;      /* primitive exponents */
  const double *coefs;     /* contraction coefficients (normalised) */
  int32_t pure;            /* 1: solid-harmonic functions, 0: Cartesian */
} oracle_basis;

/* F_m(T) for m = 0..mmax (mmax <= 40). Returns 0, or -1 on bad arguments. */
int oracle_boys(int mmax, double T, double *F);

/* Real solid-harmonic transform for l <= 8: T[(2l+1) x ncart(l)], row-major. */
int oracle_solid_transform(int l, double *T);

/* Contracted blocks for ntrip triplets trip[t] = (P, a, b) (aux shell P,
 * orbital shells a and b); block t written at out + out_off[t]. */
int oracle_eval_batch(const double *xyz, const oracle_basis *aux,
                      const oracle_basis *orb, int64_t ntrip,
                      const int32_t *trip, const int64_t *out_off, double *out,
                      int nthreads);

/* J[nao][nao] = sum_P (ab|P) d_P over all shell pairs (both triangles).
 * orb->pure = 1 takes the orbital shells as real solid harmonics: each
 * Cartesian block is transformed on both sides (nao = sum 2l+1). */
int oracle_coulomb_J(const double *xyz, const oracle_basis *aux,
                     const oracle_basis *orb, const double *d, double *J,
                     int nthreads);

/* J restricted to the orbital shell pairs with mask[a * nshell + b] != 0
 * (mask symmetric, nshell x nshell, host); the blocks of the other pairs are
 * zero.  Same arithmetic as oracle_coulomb_J per kept pair. */
int oracle_coulomb_J_masked(const double *xyz, const oracle_basis *aux,
                            const oracle_basis *orb, const double *d,
                            const uint8_t *mask, double *J, int nthreads);

/* Screening of orbital shell pairs by the largest primitive overlap bound
 *   S_ab = max_ij |c_ai c_bj| (pi / (z_ai + z_bj))^{3/2}
 *          exp(-z_ai z_bj / (z_ai + z_bj) |A - B|^2):
 * mask[a * nshell + b] = mask[b * nshell + a] = (S_ab >= tau); S is also
 * returned (nshell x nshell, may be NULL). */
int oracle_screen_pairs(const double *xyz, const oracle_basis *orb, double tau,
                        uint8_t *mask, double *S);

/* Schwarz-type bounds |(ab|P_m)| <= Qab[a*nshell+b] QP[P] from positive
 * s-type envelopes of the shells (see oracle.c). */
int oracle_schwarz_bounds(const double *xyz, const oracle_basis *aux, const oracle_basis *orb,
                          double *Qab, double *QP);

/* mask[a*nshell+b] = (Qab S_d >= tau) with S_d = sum_P QP sum_m |d_Pm|
 * (returned in *Sd if non-null): dropped J blocks are bounded by tau. */
int oracle_screen_pairs_schwarz(const double *xyz, const oracle_basis *aux,
                                const oracle_basis *orb, const double *d, double tau,
                                uint8_t *mask, double *Sd);

/* gamma[naux] = sum_{a,b} (P|ab) D_ab over all ordered orbital shell pairs;
 * D is nao x nao row-major (not assumed symmetric).  With orb->pure = 1 the
 * pairs run over real solid-harmonic orbital functions. */
int oracle_coulomb_gamma(const double *xyz, const oracle_basis *aux,
                         const oracle_basis *orb, const double *D, double *gamma,
                         int nthreads);

/* V[naux][naux] = (P|Q), the two-centre Coulomb integrals of the aux basis
 * (pure or Cartesian as the basis says). */
int oracle_coulomb_metric(const double *xyz, const oracle_basis *aux, double *V, int nthreads);

/* J blocks for selected orbital shell pairs pairs[t] = (a, b):
 * out + out_off[t] receives the ncart(a) x ncart(b) block of J. */
int oracle_coulomb_J_pairs(const double *xyz, const oracle_basis *aux,
                           const oracle_basis *orb, const double *d,
                           int64_t npair, const int32_t *pairs,
                           const int64_t *out_off, double *out, int nthreads);

/* grad[natom][3] = dL/dR for L = sum_ab G_ab J_ab (d, G fixed).  Derivatives
 * with respect to all three centres are taken explicitly.  If atom_mask is not
 * NULL only triplets with a centre on a masked atom are visited, and only the
 * masked atoms' rows are meaningful.  If pair_mask (nshell x nshell,
 * symmetric) is not NULL, J and so L run over the kept orbital shell pairs
 * only (the screened DF-J).  With orb->pure = 1, G and J are over real
 * solid-harmonic orbital functions (J as in oracle_coulomb_J). */
int oracle_coulomb_J_grad(const double *xyz, int32_t natom,
                          const oracle_basis *aux, const oracle_basis *orb,
                          const double *d, const double *G,
                          const uint8_t *atom_mask, const uint8_t *pair_mask, double *grad,
                          int nthreads);

#ifdef __cplusplus
}
#endif
#endif

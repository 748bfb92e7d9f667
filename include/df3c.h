/*
 * df3c.h -- C ABI of libdf3c: 3-center 2-electron Coulomb integrals (P|ab) and
 * the density-fitted Coulomb matrix on AMD MI355X (gfx950), FP64 throughout.
 *
 * The operations are those of Asadchev & Valeev, "Memory-Efficient Recursive
 * Evaluation of 3-Center Gaussian Integrals":
 *   - integrals over contracted Gaussian shells (Appendix "Notation"): orbital
 *     shells a, b are Cartesian, the auxiliary (ket) shell P is a real
 *     solid-harmonic shell (Section 2.2, first design assumption);
 *   - evaluated by the HGPA scheme of Section 2.5.1: Boys function (2.5.2),
 *     2-quantal VRR1 (2.5.3), early-contracted n-quantal CVRR2 (2.5.4), ket
 *     transform, n-quantal HRR (2.5.5);
 *   - digested into J_ab = sum_P (ab|P) d_P, the DF-J build of Sections 3 and 4
 *     (Table "dfj"), and its nuclear gradient.
 *
 * Conventions
 *   - Units: bohr, atomic units.  All arithmetic is IEEE FP64.
 *   - Cartesian order inside a shell of l quanta: for i = 0..l, for j = 0..i:
 *     (l-i, i-j, j), i.e. xx, xy, xz, yy, yz, zz.
 *   - Solid harmonics ordered m = -l..+l, leading monomial positive, scaled so
 *     that a solid-harmonic member of a contracted shell has unit norm when the
 *     shell's x^l Cartesian member has unit norm.
 *   - Contraction coefficients passed in already include all normalisation.
 *   - A block (P|ab) is stored row-major [p][i][j] (P slowest, b fastest).
 *   - AO order: shell order, then component order; aux functions likewise.
 *
 * Memory: every pointer marked DEVICE must point to device memory of the
 * current HIP device; HOST pointers to host memory.  The caller owns every
 * buffer, including the workspace; the library never allocates device memory
 * (its read-only tables, the Boys table included, are part of its code
 * object).  Calls that read counts or status words back take a small pinned
 * host slot of their own from a pool (allocated on first use, a few hundred
 * bytes each).  All device work is ordered on `stream`: the calls whose class
 * groups write disjoint outputs (J, masked J, the gradient, gamma, a
 * mixed-class eval_batch, the batched DF-J) fork them onto three internal side
 * streams of the device (default priority, created on first use), and
 * df3c_fit_solve runs its trailing updates on a side stream of its own; all
 * of them join back to `stream` before returning, so a call's work still starts after
 * `stream`'s earlier work and ends before its later work, also under graph
 * capture (the branches become parallel graph branches).  The fork and join
 * are enqueued under a per-device lock; calls from several host threads on one
 * device share the side streams and serialise there.
 *
 * Errors: every function returns DF3C_OK (0) or a negative status; no C++
 * exception crosses the ABI.  After an error the outputs are unspecified.
 * Host-side arguments (pointers, sizes, l_host, flags) are checked before any
 * device work is enqueued.  Device-side data (atom indices, contraction
 * degrees, shell indices of triplets, l against l_host) is checked by the
 * first kernels of a call, which set a status word at the start of the
 * workspace; every later kernel of the call reads it and does nothing when
 * it is set.  Without DF3C_ASYNC a call reads the word back at its end (one
 * synchronisation of `stream`) and returns the status; with DF3C_ASYNC it
 * returns after enqueueing and df3c_workspace_status reads the word later.
 */
#ifndef DF3C_H
#define DF3C_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DF3C_OK 0
#define DF3C_E_ARG (-1)          /* null pointer, bad size, index out of range */
#define DF3C_E_UNSUPPORTED (-2)  /* angular momentum or option beyond the build */
#define DF3C_E_WORKSPACE (-3)    /* workspace missing or too small */
#define DF3C_E_HIP (-4)          /* a HIP runtime call failed */
#define DF3C_E_NUMERIC (-5)      /* matrix not positive definite in working precision */

/* Limits of this build. */
#define DF3C_LMAX_ORB 4  /* orbital shells: s..g */
#define DF3C_LMAX_AUX 6  /* auxiliary shells: s..i */
#define DF3C_LMAX_GRAD_ORB 4  /* orbital shells in df3c_coulomb_J_grad: s..g */
#define DF3C_KMAX 64          /* primitives per shell */

/* flags */
#define DF3C_FLAG_NONE 0u
#define DF3C_SCHED_PER_CLASS 0u  /* batched J: one launch per (molecule, class) */
#define DF3C_SCHED_PERSISTENT 1u /* batched J: one persistent work-queue launch per class */
#define DF3C_GRAPH 2u            /* batched J: capture the launches in a HIP graph on the
                                    first call and replay it on calls with the same
                                    arguments */
#define DF3C_ASYNC 4u            /* return right after enqueueing: no synchronisation of
                                    `stream` and no host memory read after the call
                                    returns, so the call may be captured into a HIP
                                    graph; the status is left in the workspace
                                    (df3c_workspace_status).  Accepted by
                                    df3c_eval_batch, df3c_coulomb_J(_masked),
                                    df3c_coulomb_J_grad(_masked), df3c_coulomb_gamma
                                    and df3c_coulomb_J_batched */

/* A basis: nshell shells.  l_host is a HOST array; the other arrays are DEVICE
 * arrays.  exps/coefs are indexed by prim_off[s] .. prim_off[s] + nprim[s]-1.
 * l_host is required whenever nshell > 0 (the launches are sized from it);
 * the device plans compare its per-l counts with those of l (DF3C_E_ARG on a
 * mismatch). */
typedef struct {
  int32_t nshell;
  const int32_t *l_host;   /* HOST   [nshell] angular momentum */
  const int32_t *l;        /* DEVICE [nshell] angular momentum (same values) */
  const int32_t *nprim;    /* DEVICE [nshell] contraction degree K >= 1 */
  const int64_t *prim_off; /* DEVICE [nshell] offset into exps / coefs */
  const int32_t *atom;     /* DEVICE [nshell] index of the shell's centre in xyz */
  const double *exps;      /* DEVICE primitive exponents (> 0) */
  const double *coefs;     /* DEVICE contraction coefficients (normalised) */
  int32_t pure;            /* aux: 1 solid-harmonic; 0 Cartesian (every l in
                              df3c_eval_batch, l <= 1 in the other calls);
                              orbital: 0 Cartesian; 1 solid-harmonic, accepted by
                              df3c_coulomb_J, df3c_coulomb_J_grad (and their
                              masked and batched forms) and df3c_coulomb_gamma */
  const int32_t *nprim_host; /* HOST [nshell] copy of nprim, or NULL.  Optional, read
                              by df3c_coulomb_J_batched only: when given, its host plan
                              orders the orbital shells of each l by decreasing
                              contraction degree, as the device plans of the
                              single-molecule calls always do (from nprim), so that
                              the shell pairs that share a wavefront have equal
                              primitive loops; results do not depend on the order
                              beyond rounding */
} df3c_shells;

/* Set-up for the current device (kernel registry, the device address of the
 * code object's Boys table, CU count).  Called implicitly by the entry
 * points; call it explicitly before capturing a HIP graph.  Returns
 * DF3C_E_HIP on failure. */
int df3c_init(void);

/* Status of the last call that used workspace ws on `stream` (reads the
 * status word back: synchronises `stream`).  For calls made with DF3C_ASYNC. */
int df3c_workspace_status(const void *ws, void *stream);

/* Bytes of workspace df3c_eval_batch needs for ntrip triplets. */
size_t df3c_eval_batch_workspace(int64_t ntrip);

/* (P|ab) blocks for a batch of shell triplets (Section 2.5.1; the batch may mix
 * classes and is unordered, Section 3).
 *   xyz      DEVICE [natom][3] centres
 *   aux, orb bases of P and of a, b (orb->pure must be 0); every shell's atom
 *            index must lie in [0, natom) and 1 <= nprim <= DF3C_KMAX
 *            (checked on the device; DF3C_E_ARG otherwise)
 *   trip     DEVICE [ntrip][3] = (P, a, b) shell indices
 *   out_off  DEVICE [ntrip] offset (in doubles) of each block in out
 *   out      DEVICE output; block t is npure(l_P) x ncart(l_a) x ncart(l_b)
 *            (ncart(l_P) for a Cartesian aux basis) at out + out_off[t]
 *   ws       DEVICE workspace of at least df3c_eval_batch_workspace(ntrip) bytes
 * A Cartesian aux shell of l >= 2 keeps the ket term that the paper's VRR2
 * drops (Eq. vrr2 is exact for solid-harmonic kets only, Section 2.2): its
 * block is the class-l block plus the lower-degree terms l - 2, l - 4, ...
 * of the Cartesian-to-Hermite expansion, each from one more launch of class
 * l - 2k with a modified Boys sequence, added in stream order.
 * Shell indices in trip are checked on the device.  Without DF3C_ASYNC the
 * call synchronises `stream` once to read the class counts, which size one
 * launch per class present.  With DF3C_ASYNC nothing is read back: every
 * class the bases allow is launched over the device counts (empty classes
 * exit at once, about 0.3 ms of launches in all). */
int df3c_eval_batch(const double *xyz, int32_t natom, const df3c_shells *aux,
                    const df3c_shells *orb,
                    int64_t ntrip, const int32_t *trip, const int64_t *out_off, double *out,
                    void *ws, size_t ws_bytes, uint32_t flags, void *stream);

/* Bytes of workspace df3c_coulomb_J needs. */
size_t df3c_coulomb_J_workspace(const df3c_shells *aux, const df3c_shells *orb);

/* J_ab = sum_P (ab|P) d_P over all orbital shell pairs (DF-J, Section 3).
 *   xyz, natom, aux, orb as for df3c_eval_batch, except that orb->pure = 1
 *       is accepted: the orbital shells are then real solid harmonics (the
 *       same transform as the ket's, Section 2.5.1, applied to both sides of
 *       each Cartesian J block) and nao = sum over shells of 2l+1
 *   d   DEVICE [naux] fitting coefficients, aux function order
 *   J   DEVICE [nao][nao] output, overwritten, both triangles written
 *   ws  DEVICE workspace of at least df3c_coulomb_J_workspace bytes (with
 *       pure orbital shells it also holds the Cartesian J)
 *   flags  0 or DF3C_ASYNC
 * The shell lists (grouped by l, orbital shells by decreasing contraction
 * degree within l) and function offsets are built on the device, so with
 * DF3C_ASYNC the call only enqueues kernels and can be captured. */
int df3c_coulomb_J(const double *xyz, int32_t natom, const df3c_shells *aux,
                   const df3c_shells *orb, const double *d, double *J, void *ws, size_t ws_bytes,
                   uint32_t flags, void *stream);

/* Bytes of workspace df3c_fit_solve needs (a status word and a scalar). */
size_t df3c_fit_solve_workspace(int64_t n);

/* The density-fitting solve d = V^{-1} gamma (Introduction: the fitting
 * equations of the DF-J method; Section 3's DF-J builder takes d as given):
 * a blocked right-looking Cholesky factorisation V = L L^T in FP64 (64-wide
 * block columns: diagonal block in LDS, panel by forward substitution per row,
 * trailing update of the lower triangle in 64 x 64 tiles) and the two
 * triangular solves.
 *   V     DEVICE [n][n] row-major, symmetric positive definite (e.g. from
 *         df3c_coulomb_metric); overwritten: L in its lower triangle and L^T
 *         in its upper triangle (the diagonal is L's)
 *   rhs   DEVICE [n] right-hand side (e.g. gamma from df3c_coulomb_gamma)
 *   x     DEVICE [n] solution (may be rhs)
 *   ws    DEVICE workspace of df3c_fit_solve_workspace(n) bytes
 *   flags 0 or DF3C_ASYNC
 * Conditioning policy: no regularisation; a pivot below DBL_EPSILON times
 * the largest diagonal element of V (or a non-positive or NaN diagonal) stops
 * the factorisation and the call returns DF3C_E_NUMERIC (with DF3C_ASYNC,
 * df3c_workspace_status does).  A basis whose metric passes can still be
 * ill-conditioned: the solution then carries a relative error of about
 * cond(V) DBL_EPSILON. */
int df3c_fit_solve(double *V, int64_t n, const double *rhs, double *x, void *ws, size_t ws_bytes,
                   uint32_t flags, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): DF-J as df3c_coulomb_J
 * with DF3C_ASYNC, the workspace being the library's own device array of
 * DF3C_NOALLOC_SCRATCH_BYTES (one per device, held until the process ends)
 * instead of a caller's buffer.  The call makes no allocation of any kind
 * (no hipMalloc/hipFree, no host allocation, no event: launch timing is
 * off for it) and no synchronisation.
 *   xyz, natom, aux, orb, d, J  as for df3c_coulomb_J
 *   status  DEVICE int or NULL: receives the call's device-side status word
 *           (0 = ok; nonzero: a device-side argument check failed and J is
 *           unspecified) when the call's kernels have run
 *   flags   must be 0
 * Returns DF3C_E_WORKSPACE when df3c_coulomb_J_workspace(aux, orb) exceeds
 * DF3C_NOALLOC_SCRATCH_BYTES (solid-harmonic orbital shells need the
 * Cartesian J there too: about 1000 Cartesian AOs at most).  All calls on one
 * device share its array: calls that overlap on a device (other streams or
 * threads) race and give wrong results; each call rewrites every part of the
 * array it reads. */
#define DF3C_NOALLOC_SCRATCH_BYTES (8u << 20)
int df3c_coulomb_J_noalloc(const double *xyz, int32_t natom, const df3c_shells *aux,
                           const df3c_shells *orb, const double *d, double *J, int32_t *status,
                           uint32_t flags, void *stream);

/* Screening of orbital shell pairs.  The paper's DF-J timings use screening
 * without stating its criterion (Section 4); here the largest primitive
 * overlap bound of a pair,
 *   S_ab = max_ij |c_ai c_bj| (pi / (z_ai + z_bj))^{3/2}
 *          exp(-z_ai z_bj / (z_ai + z_bj) |A - B|^2),
 * keeps the pair when S_ab >= tau.
 *   orb   orbital basis (as for df3c_coulomb_J)
 *   tau   threshold (>= 0)
 *   mask  DEVICE [nshell][nshell] uint8 output, symmetric: 1 = pair kept
 * Asynchronous on `stream`; DF3C_E_ARG for a bad basis or tau < 0. */
int df3c_screen_pairs(const double *xyz, int32_t natom, const df3c_shells *orb, double tau,
                      uint8_t *mask, void *stream);

/* Schwarz-type screening with an error guarantee (Section 4 screens the
 * DF-J runs without stating how; this is the reading of this build).  Every
 * shell and pair is bounded by positive s-type envelopes (a primitive
 * component of l quanta by M_l(a) e^{-th a r^2}: th = 1, M_0 = 1 for l = 0;
 * th = 1/2, M_l = (l / (a e))^{l/2} otherwise), so by the positivity and the
 * Schwarz inequality of the Coulomb kernel |(ab|P_m)| <= Q_ab Q_P with
 *   Q_ab = sum_ij |c_i c_j| M(a_i) M(b_j) e^{-mu_ij AB^2} (g|g)_ij^{1/2},
 *   Q_P  = t_l sum_k |c_k| M(z_k) (g|g)_k^{1/2},
 * (g|g) = 2 pi^{5/2} / (g^2 (2g)^{1/2}) at the envelope exponents, t_l the
 * largest row 1-norm of the solid-harmonic table.  A pair is kept when
 * Q_ab S_d >= tau, S_d = sum_P Q_P sum_m |d_Pm|: every element of a dropped
 * pair's J block is below tau.
 *   aux, orb, d  as for df3c_coulomb_J (d DEVICE [naux])
 *   mask         DEVICE [nshell][nshell] uint8 output (exactly symmetric)
 *   ws           DEVICE workspace of df3c_screen_pairs_schwarz_workspace() bytes
 *   flags        0 or DF3C_ASYNC */
size_t df3c_screen_pairs_schwarz_workspace(void);
int df3c_screen_pairs_schwarz(const double *xyz, int32_t natom, const df3c_shells *aux,
                              const df3c_shells *orb, const double *d, double tau, uint8_t *mask,
                              void *ws, size_t ws_bytes, uint32_t flags, void *stream);

/* Bytes of workspace df3c_coulomb_J_masked needs. */
size_t df3c_coulomb_J_masked_workspace(const df3c_shells *aux, const df3c_shells *orb);

/* J_ab = sum_P (ab|P) d_P over the orbital shell pairs (a, b) with
 * mask[a * nshell + b] != 0 (mask DEVICE, symmetric, e.g. from
 * df3c_screen_pairs); the J blocks of the other pairs are zero.  The kept
 * pairs of each (l_a, l_b) class are compacted on the device and run by the
 * same kernels as df3c_coulomb_J, so an all-ones mask gives the same J
 * bitwise.  Without DF3C_ASYNC the kept counts are read back once (one
 * synchronisation) and size the launches; with it the launches are sized for
 * every candidate pair and the kernels read the kept counts.  Other arguments
 * as for df3c_coulomb_J; ws of at least df3c_coulomb_J_masked_workspace bytes. */
int df3c_coulomb_J_masked(const double *xyz, int32_t natom, const df3c_shells *aux,
                          const df3c_shells *orb, const double *d, const uint8_t *mask,
                          double *J, void *ws, size_t ws_bytes, uint32_t flags, void *stream);

/* Bytes of workspace df3c_coulomb_J_grad needs (depends on the current device's
 * CU count). */
size_t df3c_coulomb_J_grad_workspace(const df3c_shells *aux, const df3c_shells *orb,
                                     int32_t natom);

/* Nuclear gradient of L = sum_ab G_ab J_ab with J from df3c_coulomb_J, d and G
 * held fixed (the backward of the DF-J build; not in the paper).  Derivative
 * integrals come from raising and lowering the bra angular momentum,
 * d/dA (ab|P) = (a+1 b|P)^{2 zeta_a} - a (a-1 b|P) and likewise for B; the aux
 * centre follows from translational invariance.  Integrals are recomputed.
 *   xyz, natom, aux, orb, d as for df3c_coulomb_J (with orb->pure = 1, G and J
 *          are over the solid-harmonic functions; G is pulled back to the
 *          Cartesian blocks, T_a^T G T_b, in the workspace first)
 *   G      DEVICE [nao][nao] = dL/dJ (need not be symmetric)
 *   grad   DEVICE [natom][3] output, overwritten
 * Orbital shells up to DF3C_LMAX_GRAD_ORB.  The result is bitwise reproducible
 * (fixed-order reductions).  Returns DF3C_E_UNSUPPORTED when natom is too large
 * for the per-team LDS accumulators (about 1500 atoms). */
int df3c_coulomb_J_grad(const double *xyz, int32_t natom, const df3c_shells *aux,
                        const df3c_shells *orb, const double *d, const double *G, double *grad,
                        void *ws, size_t ws_bytes, uint32_t flags, void *stream);

/* Bytes of workspace df3c_coulomb_J_grad_masked needs. */
size_t df3c_coulomb_J_grad_masked_workspace(const df3c_shells *aux, const df3c_shells *orb,
                                            int32_t natom);

/* The gradient of L = sum_ab G_ab J_ab for the screened J of
 * df3c_coulomb_J_masked: only the orbital shell pairs with
 * mask[a * nshell + b] != 0 (DEVICE, symmetric) contribute.  The kept pairs of
 * every class are compacted on the device (launches sized as for
 * df3c_coulomb_J_masked); the result is bitwise reproducible.  Other arguments as for
 * df3c_coulomb_J_grad; ws of at least df3c_coulomb_J_grad_masked_workspace
 * bytes. */
int df3c_coulomb_J_grad_masked(const double *xyz, int32_t natom, const df3c_shells *aux,
                               const df3c_shells *orb, const double *d, const double *G,
                               const uint8_t *mask, double *grad, void *ws, size_t ws_bytes,
                               uint32_t flags, void *stream);

/* The J gradient for nmol independent molecules in one call (the batched form
 * of df3c_coulomb_J_grad, matching df3c_coulomb_J_batched's layout).
 *   mol_orb, mol_aux  HOST [nmol+1] shell ranges per molecule (as for
 *                     df3c_coulomb_J_batched)
 *   mol_atom          HOST [nmol+1]: molecule m owns atoms [mol_atom[m],
 *                     mol_atom[m+1]) and its shells' atom indices must lie there
 *                     (checked on the device); mol_atom[nmol] = natom
 *   d                 DEVICE, the molecules' fitting coefficients in aux order
 *   G                 DEVICE, molecule m's nao_m x nao_m dL/dJ at offset
 *                     sum_{m' < m} nao_m'^2
 *   grad              DEVICE [natom][3] output, overwritten
 *   ws                DEVICE workspace of df3c_coulomb_J_grad_batched_workspace
 *   flags             0 or DF3C_ASYNC
 * The molecules run in turn on `stream` through the single-molecule gradient
 * engines on their own atom ranges (each molecule's rows equal
 * df3c_coulomb_J_grad of that molecule bitwise). */
size_t df3c_coulomb_J_grad_batched_workspace(const df3c_shells *aux, const df3c_shells *orb,
                                             int32_t nmol, const int32_t *mol_orb,
                                             const int32_t *mol_aux, const int32_t *mol_atom);
int df3c_coulomb_J_grad_batched(const double *xyz, int32_t natom, const df3c_shells *aux,
                                const df3c_shells *orb, int32_t nmol, const int32_t *mol_orb,
                                const int32_t *mol_aux, const int32_t *mol_atom, const double *d,
                                const double *G, double *grad, void *ws, size_t ws_bytes,
                                uint32_t flags, void *stream);

/* Per-class schedule parameters of the persistent batched J (written by the
 * project's autotuner).  A table has DF3C_NCLASS entries indexed by
 * (l_P * 5 + l_a) * 5 + l_b with l_a >= l_b. */
typedef struct {
  int32_t chunk;        /* consecutive shell pairs per team and queue grab, >= 1 */
  int32_t grid_per_cu;  /* persistent workgroups per CU, >= 1 */
  int32_t enabled;      /* 0 skips the class (lets the autotuner time one class) */
  int32_t order;        /* launch order key, smaller first */
} df3c_class_tune;
#define DF3C_NCLASS 175

/* Bytes of workspace df3c_coulomb_J_batched needs.  mol_orb (HOST [nmol+1], as
 * for df3c_coulomb_J_batched) is read only for solid-harmonic orbital shells
 * (orb->pure = 1: the Cartesian J of every molecule is kept in the workspace)
 * and may be NULL otherwise; 0 on bad arguments. */
size_t df3c_coulomb_J_batched_workspace(const df3c_shells *aux, const df3c_shells *orb,
                                        int32_t nmol, const int32_t *mol_orb);

/* DF-J for nmol independent molecules in one call: the batched form of
 * df3c_coulomb_J for uneven molecule sizes, L classes and contraction degrees.
 *   mol_orb, mol_aux  HOST [nmol+1]: molecule m owns orbital shells
 *                     [mol_orb[m], mol_orb[m+1]) and aux shells
 *                     [mol_aux[m], mol_aux[m+1]); mol_*[0] = 0, mol_*[nmol] = nshell
 *   d                 DEVICE, the molecules' fitting coefficients in aux order
 *   J                 DEVICE output, molecule m's nao_m x nao_m matrix at offset
 *                     sum_{m' < m} nao_m'^2 (both triangles; nao_m counts 2l+1
 *                     functions per shell for solid-harmonic orbital shells, whose
 *                     Cartesian J is transformed on both sides per molecule, the
 *                     transform captured with the other launches under DF3C_GRAPH)
 *   tune              HOST [DF3C_NCLASS] schedule parameters, or NULL for defaults
 *   flags             DF3C_SCHED_PER_CLASS or DF3C_SCHED_PERSISTENT, optionally
 *                     | DF3C_GRAPH and | DF3C_ASYNC.  The plan is built on the host
 *                     and uploaded into ws on every call.  With DF3C_GRAPH the
 *                     launches are captured on the first call and replayed on later
 *                     calls with the same arguments (including ws); the cached graph
 *                     owns its plan, and at most 8 graphs are kept (the oldest is
 *                     destroyed, after a device synchronisation).  `stream` must not
 *                     be the legacy default stream (it cannot be captured).  Without
 *                     DF3C_GRAPH the call synchronises `stream` once (the plan's host
 *                     memory ends with the call).
 * The persistent schedule runs one launch per class in which workgroups take
 * shell pairs of all molecules from an atomic counter until the queue is empty. */
int df3c_coulomb_J_batched(const double *xyz, int32_t natom, const df3c_shells *aux,
                           const df3c_shells *orb, int32_t nmol, const int32_t *mol_orb,
                           const int32_t *mol_aux, const double *d, double *J,
                           const df3c_class_tune *tune, void *ws, size_t ws_bytes,
                           uint32_t flags, void *stream);

/* ---------------------------------------------------------------- timing
 * Launch timing for measurement.  While enabled, every class-kernel launch of
 * the entry points above that is not being captured into a graph is bracketed
 * by two HIP events recorded on the launch's stream (one record per launch:
 * kind, class id (L_P * 5 + l_a) * 5 + l_b, duration).  Recording adds two
 * event records per launch and nothing else.  Not thread-safe against calls
 * that launch on other threads while df3c_timing_read runs. */
#define DF3C_KERNEL_STORE 0  /* df3c_eval_batch block kernel */
#define DF3C_KERNEL_J 1      /* DF-J pair kernel (single molecule, per-class batched) */
#define DF3C_KERNEL_GRAD 2   /* J-gradient kernel */
#define DF3C_KERNEL_JQ 3     /* persistent work-queue DF-J kernel */
#define DF3C_KERNEL_GAMMA 4  /* adjoint digestion (gamma) kernel */
int df3c_timing_enable(int32_t on);

/* Waits for the recorded launches, writes the first min(n, cap) of them to
 * kind/cls/ms (HOST arrays of cap entries) and forgets all n of them.  Returns
 * n (>= 0) or a negative status (DF3C_E_ARG for cap < 0 or a null array with
 * cap > 0, DF3C_E_HIP). */
int64_t df3c_timing_read(int32_t *kind, int32_t *cls, float *ms, int64_t cap);

/* Bytes of workspace df3c_coulomb_metric needs. */
size_t df3c_coulomb_metric_workspace(const df3c_shells *aux);

/* Two-centre Coulomb metric V[P][Q] = (P|Q) of the auxiliary basis, the matrix
 * of the density-fitting equations V d = gamma (Section 3's DF-J builder takes
 * d as given).  Evaluated as the three-centre class (L_P, l_Q, 0) with a unit
 * s function of exponent 0 as Q's partner.
 *   V  DEVICE output [naux][naux] row-major, both triangles (symmetric)
 * aux->l_host is read.  DF3C_E_UNSUPPORTED for l > DF3C_LMAX_AUX or a
 * Cartesian aux shell with l > 1. */
int df3c_coulomb_metric(const double *xyz, int32_t natom, const df3c_shells *aux, double *V,
                        void *ws, size_t ws_bytes, uint32_t flags, void *stream);

/* Bytes of workspace df3c_coulomb_gamma needs (the first call on a device
 * initialises it, as df3c_init does; 0 on error). */
size_t df3c_coulomb_gamma_workspace(const df3c_shells *aux, const df3c_shells *orb);

/* Adjoint digestion: gamma_P = sum_{a,b} (P|ab) D_ab over all ordered orbital
 * function pairs -- the right-hand side of the density-fitting equations
 * (Section 3, the digestion of a 3-index batch) and dL/dd of L = sum G_ab J_ab
 * with D = G.
 *   D      DEVICE [nao][nao] row-major, any symmetry (over the solid-harmonic
 *          functions when orb->pure = 1; pulled back to the Cartesian
 *          blocks, T_a^T D T_b, in the workspace first)
 *   gamma  DEVICE output [naux] in aux-shell order, then component order
 *          (overwritten)
 * Work items are (aux shell, chunk of shell pairs); every item writes its own
 * partial sum and one fixed-order reduction per class adds them: bitwise
 * reproducible.  DF3C_E_UNSUPPORTED for a Cartesian aux shell with l > 1. */
int df3c_coulomb_gamma(const double *xyz, int32_t natom, const df3c_shells *aux,
                       const df3c_shells *orb, const double *D, double *gamma, void *ws,
                       size_t ws_bytes, uint32_t flags, void *stream);

/* Readable name of a status code (static string). */
const char *df3c_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif

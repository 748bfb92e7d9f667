// Compile-time metadata for the Obara-Saika / HGPA evaluation of (ab|P).
//
// Section 3 of the paper generates kernels from constexpr metadata (Cartesian
// orbital lists, recurrence index maps).  Here the class geometry (sizes and
// offsets of every intermediate) is constexpr; the larger index maps are
// literal arrays written by gen_tables.py at build time (the C++ constant
// evaluator is too slow for them) and compiled into the code object.
//
// Notation (Section 2.5.1, Appendix "Notation"):
//   levels j of VRR1 hold [e 0|0]^(m) with |e| = j;  m runs over
//   [L_P, L_P + L - j] where L = l_a + l_b (+1 when gradients need the raised
//   bra).  The contracted VRR2 prerequisites are
//   pi_k(e', n) = sum_prim (rho/(2 gamma zeta_c))^k (rho/zeta_c)^|n| PC^n
//                 [e' 0|0]^(L_P),      k + |n| = L_P           (Eq. a0cv2)
//   and the n-quantal CVRR2 gives the targets (e 0|c), |c| = L_P, as
//   (e 0|c) = sum_{u <= min(e, c)} prod_i C(c_i, u_i) e_i!/(e_i - u_i)!
//             pi_{|u|}(e - u, c - u)                      (Eq. cVRR2, n-q form)
//   (the coefficient of the printed n-q formula is garbled; this is the form
//   obtained by applying Eq. cVRR2 repeatedly, and it reproduces the worked
//   example of Section 2.5.4 with the last coefficient of (d_xx s|d_xx) equal
//   to 2).
#pragma once
#include <array>
#include <cstdint>

namespace df3c {

constexpr int ncart(int l) { return l < 0 ? 0 : (l + 1) * (l + 2) / 2; }
constexpr int npure(int l) { return 2 * l + 1; }
// number of Cartesian components of all levels below j
constexpr int offT(int j) { return j <= 0 ? 0 : j * (j + 1) * (j + 2) / 6; }
// index of (x, y, z) inside its shell: for i = 0..l, for j = 0..i: (l-i, i-j, j)
constexpr int cidx(int x, int y, int z) {
  int i = y + z;
  return i * (i + 1) / 2 + z;
}
constexpr int imax(int a, int b) { return a > b ? a : b; }
constexpr int imin(int a, int b) { return a < b ? a : b; }

struct C3 {
  int v[3];
  constexpr int operator[](int i) const { return v[i]; }
  constexpr int sum() const { return v[0] + v[1] + v[2]; }
};

// c-th Cartesian component of a shell with l quanta
constexpr C3 cart(int l, int c) {
  int i = 0;
  while ((i + 1) * (i + 2) / 2 <= c) ++i;
  int z = c - i * (i + 1) / 2;
  return C3{{l - i, i - z, z}};
}
constexpr int cidx3(C3 q) { return cidx(q[0], q[1], q[2]); }

// recurrence direction of a Cartesian with l >= 1 quanta: first axis with e_i > 0
constexpr int rdir(C3 e) { return e[0] > 0 ? 0 : (e[1] > 0 ? 1 : 2); }

constexpr long binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}
constexpr long falling(int n, int k) {  // n! / (n-k)!
  long r = 1;
  for (int i = 0; i < k; ++i) r *= (n - i);
  return r;
}

// ---------------------------------------------------------------------------
// Class geometry
// ---------------------------------------------------------------------------
// A class computes (e 0|P) for target levels e in [EA, EB] (EA = l_a,
// EB = l_a + l_b, or raised/lowered ranges for derivative integrals) with ket
// angular momentum LP.
template <int LP_, int EA_, int EB_>
struct Geo {
  static constexpr int LP = LP_, EA = EA_, EB = EB_;
  static constexpr int L = EB;                       // top VRR1 level
  static constexpr int NPURE = npure(LP), NCP = ncart(LP);
  static constexpr int NE = offT(EB + 1) - offT(EA);  // target e components
  // prerequisite blocks pi_k: e' in [max(0, EA-k), EB-k]
  static constexpr int emin(int k) { return imax(0, EA - k); }
  static constexpr int emax(int k) { return EB - k; }
  static constexpr int nek(int k) {
    return emax(k) >= emin(k) ? offT(emax(k) + 1) - offT(emin(k)) : 0;
  }
  static constexpr int pi_off(int k) {
    int o = 0;
    for (int q = 0; q < k; ++q) o += ncart(LP - q) * nek(q);
    return o;
  }
  static constexpr int NPI = pi_off(LP + 1);
  static constexpr int sw_off(int k) {
    int o = 0;
    for (int q = 0; q < k; ++q) o += ncart(LP - q);
    return o;
  }
  static constexpr int NSW = sw_off(LP + 1);
  // VRR1 storage per primitive: targets [e]^(LP) for all levels 0..L, then the
  // higher-m work area of the two most recent levels (2-quantal stages)
  static constexpr int NT = offT(L + 1);
  static constexpr int wsize(int lo, int hi) {  // higher-m storage of levels lo, hi
    return (lo >= 0 ? ncart(lo) * (L - lo) : 0) + (hi >= 0 ? ncart(hi) * (L - hi) : 0);
  }
  static constexpr int NW = [] {
    int w = L;  // level 0 alone
    for (int j = 1; j <= L; ++j) w = imax(w, wsize(j - 1, j));
    return w;
  }();
  static constexpr int NV1 = NT + NW;
};

// ---------------------------------------------------------------------------
// VRR1 (Eq. vrr1) 2-quantal stages.  A stage builds levels (j-1, j) from the
// stored levels (j-2, j-3); level j items compute their level j-1 inputs
// internally (Section 2.5.3).  For odd L a single 1-quantal stage building
// level 1 runs first.  Items are (component, m) pairs.
// ---------------------------------------------------------------------------
template <int L>
struct VStages {
  // stage s builds levels hi(s) (and hi(s)-1 when two_q(s))
  static constexpr int first_hi = (L % 2) ? 1 : 2;
  static constexpr int nstage = L == 0 ? 0 : ((L % 2) ? 1 + (L - 1) / 2 : L / 2);
  static constexpr int hi(int s) { return (L % 2) ? (s == 0 ? 1 : 1 + 2 * s) : 2 + 2 * s; }
  static constexpr bool two_q(int s) { return !((L % 2) && s == 0); }
  static constexpr int nitems(int s) {
    int j = hi(s);
    int n = ncart(j) * (L - j + 1);
    if (two_q(s)) n += ncart(j - 1) * (L - j + 2);
    return n;
  }
  static constexpr int maxitems() {
    int n = 0;
    for (int s = 0; s < nstage; ++s) n = imax(n, nitems(s));
    return n;
  }
  static constexpr int items_off(int s) {
    int o = 0;
    for (int q = 0; q < s; ++q) o += nitems(q);
    return o;
  }
  static constexpr int NITEMS = items_off(nstage);
};


// VRR1 stage item: operand and destination offsets (doubles) relative to the
// T region of a primitive record, and the coefficients of Eq. vrr1.
//   1-quantal (q = 0), step along i:
//     [e]^(m) = PA_i [e-1_i]^(m) - (rho/gamma) PC_i [e-1_i]^(m+1)
//               + f1/(2 gamma) ([e-2_i]^(m) - (rho/gamma) [e-2_i]^(m+1))
//   2-quantal (q = 1): the same step along ip gives [x]^(m), [x]^(m+1) of
//     x = e - 1_i in registers, then one step along i (lower term via y = e-2_i).
// A missing operand points at offset 0 and carries a zero coefficient.
struct alignas(16) VO {
  int16_t u0, u1, u2;  // upper input at m, m+1, m+2
  int16_t l0, l1, l2;  // lower input at m, m+1, m+2
  int16_t y0, y1;      // 2-q: e-2_i (upper input level) at m, m+1
  int16_t dst;         // output
  int16_t ax;          // i | ip << 2 | q << 4
  int16_t f1, f2;      // integer coefficients (e_ip - 1 or e_i - 1; e_i - 1)
  int16_t pad[4];      // 32 bytes: two 16-byte loads per item
};

// Generated tables (gen_tables.py):
//   GenTab<LP, EA, EB>: CVRR2 contraction map (pi_sw, pi_v) and n-q CVRR2
//                        combine (cb_start, cb_pw)
//   GenSolid<l>:        solid-harmonic transform, CSR rows m = -l..l
//   GenHrr<LA, LB>:     n-q HRR terms
//   GenV<L>:            VRR1 stage items (operand offsets)
//   GenY<LP, EA, EB>:   per-primitive digested ket of the derivative engine
template <int LP, int EA, int EB> struct GenTab;
template <int LP, int EA, int EB> struct GenY;
template <int LA, int LB> struct GenOmega;  // transposed shifted HRRs of the gradient engine
template <int LA, int LB> struct GenHrrT;   // HRR transposed onto D~ (gamma engine)
template <int l> struct GenSolid;
template <int LA, int LB> struct GenHrr;
template <int L> struct GenV;

}  // namespace df3c

#include "gen/tables_common.hpp"
#include "gen/tables_lp0.hpp"
#include "gen/tables_lp1.hpp"
#include "gen/tables_lp2.hpp"
#include "gen/tables_lp3.hpp"
#include "gen/tables_lp4.hpp"
#include "gen/tables_lp5.hpp"
#include "gen/tables_lp6.hpp"

// Class kernels of the (ab|P) pipeline for gfx950.
//
// Per contracted triplet (Section 2.5.1):
//   setup + Boys -> [00|0]^(m)      per primitive triplet (Section 2.5.2)
//   VRR1 2-quantal -> [e0|0]^(LP)   per primitive triplet (Section 2.5.3)
//   pi_k(e', n)    += sW x [e'0|0]  early contraction of the CVRR2 prerequisites,
//                                   accumulated in registers across primitives
//   (e0|c)          = n-q CVRR2      once per triplet, in place on pi_0 (Section 2.5.4)
//   (e0|P)          = solid-harmonic transform, constant coefficients
//   (ab|P)          = n-q HRR, factorised per Cartesian axis, in registers (Section 2.5.5)
//   digestion: store the block (staged through LDS for coalesced writes), or
//   accumulate J_ab += sum_P (ab|P) d_P.
//
// A team of TS lanes owns one triplet; TS <= 64 packs 64/TS teams in a
// single-wave workgroup, TS = 128 / 256 spreads one triplet over 2 / 4 waves
// of a workgroup.  Team synchronisation is a workgroup barrier.
#pragma once
#include "device.hpp"

namespace df3c {

struct StoreArgs {
  const double *boys;       // Boys table
  const double *xyz;
  ShellsDev aux, orb;
  const int32_t *trip;      // [ntrip][3] = (P, a, b)
  const int64_t *out_off;   // [ntrip]
  double *out;
  const uint32_t *bucket;   // triplet ids of this class; bit 31: a and b swapped
  int64_t count;
  int32_t pure;             // ket solid-harmonic (1) or Cartesian (0)
  const int *err;           // device status word: nothing is done when it is non-zero
  const int *dcount;        // optional device count and bucket offset of the class
  const int *dstart;        //   (replace count and shift bucket; asynchronous calls)
  int32_t cexp;             // Cartesian ket of l = LP + 2 cexp: this launch adds its
                            //   degree-LP term (0: the plain block of the class)
};

struct JArgs {
  const double *boys;       // Boys table
  const double *xyz;
  ShellsDev aux, orb;
  const int32_t *ash;       // orbital shells of l = LA (sorted)
  const int32_t *bsh;       // orbital shells of l = LB
  int32_t na, nb;           // lengths of ash / bsh
  int32_t same;             // LA == LB: pairs are a >= b within one list
  const int32_t *psh;       // aux shells of l = LP
  int32_t np;
  const int64_t *ao_off;    // AO offset of each orbital shell
  const int64_t *aux_off;   // function offset of each aux shell
  const double *d;          // fitting coefficients
  double *J;                // [nao][nao]
  int64_t nao;
  int64_t npair;
  int64_t ao_base;          // subtracted from ao_off (first AO of the molecule)
  int32_t pure;
  int32_t nsub;             // register engine: lanes per shell pair (power of two,
                            // 1..16), which split the aux shells between them
  const double *arec;       // aux-shell records, aligned with psh (see AREC)
  const int64_t *plist;     // optional: indices q of the class's pairs to run
  const int64_t *pcount;    //   (device count of plist), null for all npair
  const int *err;           // device status word: nothing is done when it is non-zero
};

// Aux-shell record, one per position of the sorted aux list, built once per
// call: centre, primitive offset, contraction degree, atom (as doubles, exact),
// exponent and coefficient of the first primitive, and d' = T^T d_P, the
// Cartesian image of the shell's fitting coefficients (d_P itself for a
// Cartesian aux basis), so that an engine's aux loop reads one contiguous,
// aligned record instead of a chain of dependent loads (and an uncontracted
// shell needs no further load at all).
enum { AR_CX = 0, AR_CY, AR_CZ, AR_PRIM, AR_K, AR_ATOM, AR_Z0, AR_C0, AR_DQ };
constexpr int AREC = AR_DQ + 28;  // doubles per record (d' of l <= 6)

// LDS layout of one team (in doubles).  Regions are reused once dead:
//   PRIM [0, PCH*REC)             primitive records of the current chunk (loop only)
//   PI   [0, NPI)                 pi, written after the loop; its block k = 0 is
//                                 the target (e0|c) ([c][e''])
//   EM   (e0|P) [m][e'']          in the dead tail of pi, else after everything
//   STG  output staging          at 0 (dead pi_0) when EM starts beyond it, else extra
template <int LP, int LA, int LB, int PCH, bool CART = false>
struct Layout {
  using G = Geo<LP, LA, LA + LB>;
  // ket rows of the transformed block: solid harmonics, or every Cartesian
  // component for a Cartesian aux shell (CART)
  static constexpr int NKET = CART ? G::NCP : G::NPURE;
  static constexpr int REC = PS_N + G::NV1 + G::NSW;
  static constexpr int NEC = G::NCP * G::NE;
  static constexpr int NEM = NKET * G::NE;
  static constexpr int NOUT = NKET * ncart(LA) * ncart(LB);
  static constexpr int PI = 0;
  // the primitive records live only during the primitive loop, pi is written
  // to LDS only after it: the two share the start of the slice
  static constexpr int PRIM = 0;
  static constexpr int PRIM_END = PCH * REC;
  static constexpr int END_LOOP = imax(G::NPI, PRIM_END);
  // EM: after pi_0 if the tail of pi is large enough, else after everything
  static constexpr bool EM_IN_PI = NEM <= G::NPI - NEC;
  static constexpr int EM = EM_IN_PI ? NEC : END_LOOP;
  static constexpr int EM_END = EM + NEM;
  static constexpr int END0 = imax(END_LOOP, EM_END);
  // STG (written by the HRR) must not overlap EM (read by the HRR)
  static constexpr int STG = (EM >= NOUT) ? 0 : END0;
  // odd number of doubles: the slices of the teams of one workgroup start on
  // different LDS banks
  static constexpr int TOTAL = imax(END0, STG + NOUT) | 1;
};

// Team size and primitive chunk per class: small classes run one triplet per
// lane (or per few lanes), large ones one triplet per one to four wavefronts.
// Minimum waves per SIMD asked of the register allocator for teams of 2-4
// waves and of one wave.  Two waves per SIMD let one team's barriers and LDS
// latency overlap another's work; measured faster than one wave with more
// registers even where it costs a few spills.
#ifndef DF3C_MIN_WAVES_BIG
#define DF3C_MIN_WAVES_BIG 2
#endif
#ifndef DF3C_MIN_WAVES_WAVE
#define DF3C_MIN_WAVES_WAVE 2
#endif
// J kernels of the register engine (one lane per shell pair)
#ifndef DF3C_MIN_WAVES_JREG
#define DF3C_MIN_WAVES_JREG 1
#endif

// Small classes whose J runs on the register engine (jr_pair): VRR1 over all
// m, the d-contracted ket and X fit the registers of one lane.
// limits of the register J engine: l_a + l_b and the live doubles per lane
#ifndef DF3C_JREG_LMAX
#define DF3C_JREG_LMAX 6
#endif
#ifndef DF3C_JREG_COST
#define DF3C_JREG_COST 300
#endif
template <int LP, int LA, int LB>
struct JReg {
  static constexpr int L = LA + LB, EA = LA, EB = LA + LB;
  static constexpr int NE = offT(EB + 1) - offT(EA);
  static constexpr int KU = imin(LP, EB);  // |u| of the H_u that can meet a target
  static constexpr int NU = offT(KU + 1);
  // VRR1 in registers: level l holds m = 0..L-l (relative to LP)
  static constexpr int voff(int l) {
    int o = 0;
    for (int q = 0; q < l; ++q) o += ncart(q) * (L - q + 1);
    return o;
  }
  static constexpr int NVR = voff(L + 1);
  static constexpr int COST = ncart(LP) + NU + NE + NVR;
  static constexpr bool OK = L <= DF3C_JREG_LMAX && COST <= DF3C_JREG_COST;
};

template <class G>
struct MTiles {
  static constexpr int nr(int k) { return (ncart(k) + 15) / 16; }
  static constexpr int nc(int k) { return (G::nek(k) + 15) / 16; }
  static constexpr int count() {
    int n = 0;
    for (int k = 0; k <= G::LP; ++k)
      if (G::nek(k) > 0) n += nr(k) * nc(k);
    return n;
  }
  static constexpr int N = count();
  static constexpr int field(int t, int which) {
    for (int k = 0; k <= G::LP; ++k) {
      if (G::nek(k) == 0) continue;
      const int n = nr(k) * nc(k);
      if (t < n) return which == 0 ? k : which == 1 ? 16 * (t / nc(k)) : 16 * (t % nc(k));
      t -= n;
    }
    return -1;
  }
  static constexpr int moff(int k) {
    int o = 0;
    for (int q = 0; q < k; ++q) o += ncart(q) * G::nek(q);
    return o;
  }
  static constexpr int NM = moff(G::LP + 1);
};

// LDS layout of one J-engine team (doubles):
//   PRIM [0, PCH*REC)    records [PS_N][T][W][sW][H] of the current chunk
//   DP   [.., +PCH*NCP)  d' of the aux shell of each primitive of the chunk
//   MJ   [0, NM)         M after the aux loop (over the dead PRIM / DP)
//   XD   [.., +NE)       X_e for the HRR
template <int LP, int LA, int LB, int PCH>
struct JELayout {
  using G = Geo<LP, LA, LA + LB>;
  static constexpr int HU = PS_N + G::NV1 + G::NSW;
  static constexpr int REC = HU + G::NSW;
  static constexpr int DP = PCH * REC;
  static constexpr int MJ = 0;
  static constexpr int XD = imax(DP + PCH * G::NCP, MTiles<G>::NM);
  static constexpr int TOTAL = XD + G::NE;
};

template <int LP, int LA, int LB>
struct Cfg {
  using G = Geo<LP, LA, LA + LB>;
  static constexpr int work = G::NPI + G::NE * G::NCP + G::NPURE * G::NE +
                              G::NPURE * ncart(LA) * ncart(LB);
  static constexpr int TS = work >= 6000 ? 256 : work >= 2500 ? 128 : work >= 1024 ? 64
                            : work >= 256 ? 16 : work >= 48 ? 4 : 1;
  // primitives per chunk: whole-wave teams take as many groups of 4 (the K
  // extent of one MFMA) as fit in the pi region, up to 16
  static constexpr int REC = PS_N + G::NV1 + G::NSW;
  static constexpr int PCH = TS >= 64 ? 4 * imax(1, imin(4, G::NPI / (4 * REC)))
                             : TS >= 16 ? 4 : TS == 4 ? 2 : 1;
  static constexpr int BLK = TS > 64 ? TS : 64;
  static constexpr int LDS = (BLK / TS) * Layout<LP, LA, LB, PCH>::TOTAL * 8;
  // store kernels also run the pipeline with the shells swapped (the second
  // HRR direction of a split contracted pair); a team's slice holds either
  static constexpr int STORE_TEAM =
      imax(Layout<LP, LA, LB, PCH>::TOTAL, LA > LB ? Layout<LP, LB, LA, PCH>::TOTAL : 0) | 1;
  static constexpr int STORE_LDS = (BLK / TS) * STORE_TEAM * 8;
  // the same for the Cartesian-ket instantiation (aux shells with pure = 0)
  static constexpr int STORE_TEAM_C =
      imax(Layout<LP, LA, LB, PCH, true>::TOTAL,
           LA > LB ? Layout<LP, LB, LA, PCH, true>::TOTAL : 0) | 1;
  static constexpr int STORE_LDS_C = (BLK / TS) * STORE_TEAM_C * 8;
  // the store kernels stage the VRR1 item records in LDS after the team
  // slices (words 0-3 and 4-5 of each record, 16-byte aligned)
  static constexpr int VT_BYTES = VStages<LA + LB>::NITEMS * 24;
  static constexpr int STORE_LDS_V = ((BLK / TS) * STORE_TEAM * 8 + 15) / 16 * 16 + VT_BYTES;
  static constexpr int STORE_LDS_CV = ((BLK / TS) * STORE_TEAM_C * 8 + 15) / 16 * 16 + VT_BYTES;
  // minimum waves per SIMD requested from the register allocator
  static constexpr int WPE = TS >= 128 ? DF3C_MIN_WAVES_BIG : TS == 64 ? DF3C_MIN_WAVES_WAVE : 1;
  // J kernels: one lane per shell pair on the register engine, else the J
  // engine with whole-wave teams (at least one wave per shell pair)
  static constexpr bool JREG = JReg<LP, LA, LB>::OK;
  static constexpr int TSJ = JREG ? 1 : TS >= 64 ? TS : 64;
  // J engine: 16 primitive triplets per chunk where the team's LDS stays
  // within 48 kB, else 8, else 4
  static constexpr int PCHJ = JREG ? 1
                              : JELayout<LP, LA, LB, 16>::TOTAL * 8 <= 48 * 1024 ? 16
                              : JELayout<LP, LA, LB, 8>::TOTAL * 8 <= 48 * 1024  ? 8
                                                                                  : 4;
  static constexpr int BLKJ = TSJ > 64 ? TSJ : 64;
  static constexpr int WPEJ = JREG ? DF3C_MIN_WAVES_JREG : TSJ >= 128 ? DF3C_MIN_WAVES_BIG
                                                                    : DF3C_MIN_WAVES_WAVE;
  static_assert(LDS <= 160 * 1024, "class does not fit the LDS of a CU");
  static_assert(STORE_LDS <= 160 * 1024, "class does not fit the LDS of a CU");
  static_assert(STORE_LDS_C <= 160 * 1024, "class does not fit the LDS of a CU");
  static_assert(STORE_LDS_V <= 160 * 1024 && STORE_LDS_CV <= 160 * 1024,
                "class does not fit the LDS of a CU");
};

// ---------------------------------------------------------------------------
// Per-lane slots of the prerequisite array pi: slot q of lane tid holds entry
// r = tid + q TS, packed as (sW index << 16) | (VRR1 target index).
// ---------------------------------------------------------------------------
template <class G>
__device__ __forceinline__ int pi_slot(int r) {
  int code = -1;
  static_for<G::LP + 1>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if constexpr (G::nek(k) > 0) {
      constexpr int o0 = G::pi_off(k), o1 = G::pi_off(k + 1), ne = G::nek(k);
      if (r >= o0 && r < o1) {
        const int n = (r - o0) / ne, e = r - o0 - n * ne;
        code = ((G::sw_off(k) + n) << 16) | (offT(G::emin(k)) + e);
      }
    }
  });
  return code;
}

// ---------------------------------------------------------------------------
// Prerequisite contraction on the FP64 matrix cores.  For each k the block
//   pi_k[n][e'] = sum_prim sW_k[n](prim) V[e'](prim),  V = [e'0|0]^(LP),
// is an ncart(LP-k) x K times K x nek(k) product over the K primitives of the
// triplet.  The output is cut into 16 x 16 tiles; each chunk of 4 primitives
// adds one v_mfma_f64_16x16x4 per tile (lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; it holds D[4v + l/16][l%16], v < 4).  Tiles are dealt
// round-robin to the waves of the team.
// ---------------------------------------------------------------------------
typedef double dbl4 __attribute__((ext_vector_type(4)));

template <class G>
struct PiTiles {
  static constexpr int nr(int k) { return (ncart(G::LP - k) + 15) / 16; }
  static constexpr int nc(int k) { return (G::nek(k) + 15) / 16; }
  static constexpr int count() {
    int n = 0;
    for (int k = 0; k <= G::LP; ++k)
      if (G::nek(k) > 0) n += nr(k) * nc(k);
    return n;
  }
  static constexpr int N = count();
  // tile t -> (k, first row, first column), tiles ordered by k, row, column
  static constexpr int field(int t, int which) {
    for (int k = 0; k <= G::LP; ++k) {
      if (G::nek(k) == 0) continue;
      const int n = nr(k) * nc(k);
      if (t < n) return which == 0 ? k : which == 1 ? 16 * (t / nc(k)) : 16 * (t % nc(k));
      t -= n;
    }
    return -1;
  }
};

// ---------------------------------------------------------------------------
// Setup of primitive triplet p of a shell triplet (p = (ia Kb + ib) Kc + ic)
// into its record R: the scalars, Boys, level 0 of VRR1 at every m and the
// CVRR2 monomials sW.  setup_chunk runs it for p0 .. p0+npc-1 (lanes over
// primitives), record of primitive pp at prims + pp * REC:
//   [PS_N scalars][T: NT][W: NW][sW: NSW]...
// WM selects the contraction weights: 0 -> c_a c_b c_c, 1 -> 2 zeta_a c_a c_b c_c,
// 2 -> 2 zeta_b c_a c_b c_c (the raised bra of the derivative integrals).
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Split of a contracted shell pair by HRR direction.  Eq. hrr transfers quanta
// from the centre that carries the VRR1 quanta to the other one with powers of
// AB, applied to the contracted (e0| of all primitive pairs at once.  A pair
// (ia, ib) whose Gaussian product centre P lies near the other centre
// (zeta_a < zeta_b) gives (e0| terms of order |PA|^e that the transfer
// cancels, so with contracted shells mixing tight and diffuse primitives at a
// few bohr the single-direction result loses up to ~1e-9 relative (and a
// single pair with the tight exponent on the lower-l shell, whose quanta
// would go to the higher-l shell, loses accuracy the same way).  The store
// kernels therefore contract the pairs with zeta_a >= zeta_b with the quanta
// on A (group 1) and the others with the quanta on B (group 2, the pipeline
// with the shells swapped: zeta_b > zeta_a strictly), and add the two blocks.
// Group 0 keeps every pair (no split).  Pairs of a group are taken in
// row-major (ia, ib) order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool split_keep(int grp, double za, double zb) {
  return grp == 1 ? za >= zb : za > zb;
}

__device__ __forceinline__ int split_count(int grp, int Ka, int Kb, const double *ea,
                                           const double *eb) {
  if (grp == 0) return Ka * Kb;
  int n = 0;
  for (int i = 0; i < Ka; ++i) {
    const double za = ea[i];
    for (int j = 0; j < Kb; ++j) n += split_keep(grp, za, eb[j]) ? 1 : 0;
  }
  return n;
}

// index of the k-th (0-based) set bit of m (k < popcount(m)), by halving
__device__ __forceinline__ int nth_set_bit(uint64_t m, int k) {
  int pos = 0;
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) {
    const uint64_t low = m & ((uint64_t(1) << s) - 1);
    const int c = __popcll(low);
    if (k >= c) {
      k -= c;
      m >>= s;
      pos += s;
    } else {
      m = low;
    }
  }
  return pos;
}

// split_pair for the lanes of one whole wavefront (every lane calls it): the
// candidate pairs are flagged 64 at a time, a ballot and a prefix count rank
// them, and a lane takes the pair ranked q; O(Ka Kb / 64) steps instead of a
// serial scan per lane
__device__ __forceinline__ void split_pair_wave(int lane, int q, int grp, int Ka, int Kb,
                                                const double *ea, const double *eb, int &ia,
                                                int &ib) {
  const int n = Ka * Kb;
  int base = 0;
  for (int w0 = 0; w0 < n; w0 += 64) {
    const int c = w0 + lane;
    bool keep = false;
    if (c < n) {
      const int i = c / Kb;
      keep = split_keep(grp, ea[i], eb[c - i * Kb]);
    }
    const uint64_t m = __ballot(keep);
    const int cnt = __popcll(m);
    if (q >= base && q < base + cnt) {
      const int pos = w0 + nth_set_bit(m, q - base);
      ia = pos / Kb;
      ib = pos - ia * Kb;
    }
    base += cnt;
  }
}

// (ia, ib) of the q-th pair of group grp (q < split_count)
__device__ __forceinline__ void split_pair(int q, int grp, int Ka, int Kb, const double *ea,
                                           const double *eb, int &ia, int &ib) {
  ia = q / Kb;
  ib = q - ia * Kb;
  if (grp == 0) return;
  for (int i = 0; i < Ka; ++i) {
    const double za = ea[i];
    for (int j = 0; j < Kb; ++j)
      if (split_keep(grp, za, eb[j])) {
        if (q == 0) {
          ia = i;
          ib = j;
          return;
        }
        --q;
      }
  }
}

// Largest row 1-norm of the solid-harmonic table of l (a constant): a pure
// function is bounded by it times r^l.
template <int L>
constexpr double solid_row_norm() {
  double t = 0.0;
  for (int m = 0; m < 2 * L + 1; ++m) {
    double r = 0.0;
    for (int q = GenSolid<L>::start[m]; q < GenSolid<L>::start[m + 1]; ++q)
      r += GenSolid<L>::val[q] < 0 ? -GenSolid<L>::val[q] : GenSolid<L>::val[q];
    t = r > t ? r : t;
  }
  return t;
}

// Positive s-type envelope of a primitive Cartesian component of l quanta:
// r^l e^{-z r^2} <= env_m(l, z) e^{-env_theta(l) z r^2} (theta = 1 for l = 0,
// else 1/2 with env_m = (l / (z e))^{l/2}); self-repulsion root of e^{-g r^2}.
__device__ __forceinline__ double env_m(int l, double z) {
  return l == 0 ? 1.0 : pow(double(l) / (z * 2.718281828459045235360287), 0.5 * l);
}
__device__ __forceinline__ double env_theta(int l) { return l == 0 ? 1.0 : 0.5; }
__device__ __forceinline__ double env_self(double g) {
  return sqrt(34.98683665524972497 / (g * g * sqrt(2.0 * g)));
}

// Bound on the rounding error a shell pair's group-2 primitive pairs
// (zeta_a < zeta_b) would carry if their VRR1 quanta stayed on A: the HRR
// adds sum_k C(LB,k) |AB|^{LB-k} [(LA+k) 0|P], whose terms are bounded by the
// Schwarz-type envelope bounds (bra: l = LA+k on A, s on B; ket: the aux
// shell), times the unit roundoff.  One wavefront's lanes take the primitive
// pairs and sum by a butterfly, so every lane of every wave of a team gets the
// same value (the decision is uniform over the team).
template <int LP, int LA, int LB>
__device__ double split_error_bound(int lane, int Ka, const double *ea, const double *ca, int Kb,
                                    const double *eb, const double *cb, double AB2, int Kc,
                                    const double *ec, const double *cc, int pure) {
  const double R = sqrt(AB2);
  double s = 0.0;
  for (int q = lane; q < Ka * Kb; q += 64) {
    const int i = q / Kb, j = q - i * Kb;
    const double za = ea[i], zb = eb[j];
    if (!(za < zb)) continue;
    double b = 1.0, rp = 1.0;  // C(LB, k), R^{LB-k} built from the top
    double t = 0.0;
    for (int k = LB; k >= 0; --k) {
      const double a1 = env_theta(LA + k) * za, g = a1 + zb;
      t += b * rp * env_m(LA + k, za) * exp(-a1 * zb / g * AB2) * env_self(g);
      b = b * double(k) / double(LB - k + 1);
      rp *= R;
    }
    s += fabs(ca[i] * cb[j]) * t;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  double qp = 0.0;
  for (int k = 0; k < Kc; ++k)
    qp += fabs(cc[k]) * env_m(LP, ec[k]) * env_self(env_theta(LP) * ec[k]);
  return 1.1102230246251565e-16 * s * qp * (pure ? solid_row_norm<LP>() : 1.0);
}

template <class G, int WM>
__device__ __forceinline__ void setup_prim(const double *btab, double *R, int p, int Kb, int Kc,
                                           const double *A, const double *B, const double *C,
                                           double AB2, const double *ea, const double *ca,
                                           const double *eb, const double *cb,
                                           const double *ec, const double *cc, int grp = 0,
                                           int Ka = 0, int cs = 0, int ia_in = -1,
                                           int ib_in = 0) {
  constexpr int LP = G::LP, L = G::L;
  {
    const int ic = p % Kc, rest = p / Kc;
    int ia = ia_in, ib = ib_in;
    if (ia_in < 0) split_pair(rest, grp, Ka, Kb, ea, eb, ia, ib);
    const double za = ea[ia], zb = eb[ib], zc = ec[ic];
    const double g = za + zb, ig = 1.0 / g;
    const double Px = (za * A[0] + zb * B[0]) * ig, Py = (za * A[1] + zb * B[1]) * ig,
                 Pz = (za * A[2] + zb * B[2]) * ig;
    const double PCx = Px - C[0], PCy = Py - C[1], PCz = Pz - C[2];
    const double gz = g + zc;
    const double rho = g * zc / gz;
    const double T = rho * (PCx * PCx + PCy * PCy + PCz * PCz);
    // 2 pi^{5/2} / ((g+zc)^{1/2} g zc) exp(-za zb/g AB^2) x contraction coefficients
    double pre = 34.98683665524972497 / (sqrt(gz) * g * zc) * exp(-za * zb * ig * AB2) *
                 (ca[ia] * cb[ib] * cc[ic]);
    if constexpr (WM == 1) pre *= 2.0 * za;
    if constexpr (WM == 2) pre *= 2.0 * zb;
    double Fm[L + 1];
    if (LP + L + 3 > BOYS_MTOP_MAX || cs == 0) {
      boys<LP, L + 1>(btab, T, Fm);
    } else if constexpr (LP + L + 3 <= BOYS_MTOP_MAX) {
      // degree-LP term of a Cartesian ket of l = LP + 2 cs (cs <= 3): the
      // Boys values become F'_m = (4 zc)^{-cs} sum_j C(cs, j) (-rho/zc)^j F_{m+j}
      double Fx[L + 4];
      boys<LP, L + 4>(btab, T, Fx);
      const double q = -rho / zc;
      double sc = 1.0;
      for (int k = 0; k < cs; ++k) sc *= 0.25 / zc;
#pragma unroll
      for (int mm = 0; mm <= L; ++mm) {
        double acc = Fx[mm], bq = 1.0;
        for (int j = 1; j <= cs; ++j) {
          bq *= q * double(cs - j + 1) / double(j);
          acc += bq * Fx[mm + j];
        }
        Fm[mm] = sc * acc;
      }
    }
    R[PS_PAX] = Px - A[0];
    R[PS_PAY] = Py - A[1];
    R[PS_PAZ] = Pz - A[2];
    const double rg = rho * ig;
    R[PS_RPX] = rg * PCx;
    R[PS_RPY] = rg * PCy;
    R[PS_RPZ] = rg * PCz;
    R[PS_I2G] = 0.5 * ig;
    R[PS_RG] = rg;
    double *Tr = R + PS_N;
    double *W = Tr + G::NT;
    Tr[0] = pre * Fm[0];
#pragma unroll
    for (int mm = 1; mm <= L; ++mm) W[mm - 1] = pre * Fm[mm];
    // sW[k][n] = (rho/(2 g zc))^k (rho/zc PC)^n, k + |n| = LP   (Eq. a0cv2)
    double *SW = Tr + G::NV1;
    const double s = rho * ig * (0.5 / zc), rz = rho / zc;
    double wx[LP + 1], wy[LP + 1], wz[LP + 1], sk[LP + 1];
    wx[0] = wy[0] = wz[0] = sk[0] = 1.0;
#pragma unroll
    for (int q = 1; q <= LP; ++q) {
      wx[q] = wx[q - 1] * (rz * PCx);
      wy[q] = wy[q - 1] * (rz * PCy);
      wz[q] = wz[q - 1] * (rz * PCz);
      sk[q] = sk[q - 1] * s;
    }
    static_for<LP + 1>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      static_for<ncart(LP - k)>([&](auto nc) {
        constexpr int n = decltype(nc)::value;
        constexpr C3 q = cart(LP - k, n);
        SW[G::sw_off(k) + n] = sk[k] * wx[q[0]] * wy[q[1]] * wz[q[2]];
      });
    });
  }
}

template <class G, int TS, int REC, int WM>
__device__ __forceinline__ void setup_chunk(const double *btab, double *prims, int lt, int p0,
                                            int npc, int Kb, int Kc, const double *A,
                                            const double *B, const double *C, double AB2,
                                            const double *ea, const double *ca,
                                            const double *eb, const double *cb,
                                            const double *ec, const double *cc, int grp = 0,
                                            int Ka = 0, int cs = 0) {
  if constexpr (TS % 64 == 0 && REC > 0) {
    // whole-wave teams: npc <= 64, the first wave sets the chunk up; with a
    // split the pairs of the group are ranked by the whole wave
    if (lt < 64) {
      int ia = -1, ib = 0;
      if (grp != 0)
        split_pair_wave(lt, (p0 + lt) / imax(Kc, 1), grp, Ka, Kb, ea, eb, ia, ib);
      if (lt < npc)
        setup_prim<G, WM>(btab, prims + lt * REC, p0 + lt, Kb, Kc, A, B, C, AB2, ea, ca, eb, cb,
                          ec, cc, grp, Ka, cs, grp != 0 ? ia : (p0 + lt) / Kc / Kb,
                          grp != 0 ? ib : (p0 + lt) / Kc % Kb);
    }
  } else {
    for (int pp = lt; pp < npc; pp += TS)
      setup_prim<G, WM>(btab, prims + pp * REC, p0 + pp, Kb, Kc, A, B, C, AB2, ea, ca, eb, cb, ec,
                        cc, grp, Ka, cs);
  }
}

// ---------------------------------------------------------------------------
// The per-triplet pipeline up to (e0|P) in LDS (region EM of the layout).
// ---------------------------------------------------------------------------
// WM selects the contraction weights (see setup_chunk).  slot is the per-lane
// prerequisite map of make_slots, or nullptr to decode it inline.
template <int LP, int LA, int LB, int TS, int PCH, int WM = 0, bool CART = false>
__device__ __forceinline__ void triplet_to_e0P(const double *btab, double *S, int tid,
                                               const int *slot, int npmax, const double *A,
                                               const double *B, const double *C, int Ka,
                                               const double *ea, const double *ca, int Kb,
                                               const double *eb, const double *cb, int Kc,
                                               const double *ec, const double *cc, int pure,
                                               int grp = 0, int cs = 0, int nkept = -1,
                                               const uint4 *vt0 = nullptr,
                                               const uint2 *vt1 = nullptr) {
  using G = Geo<LP, LA, LA + LB>;
  using LY = Layout<LP, LA, LB, PCH, CART>;
  using TB = GenTab<LP, G::EA, G::EB>;
  static_assert(TB::NPI == G::NPI && TB::NTGT == G::NE * G::NCP, "generated tables out of date");
  constexpr int L = G::L;
  constexpr int REC = LY::REC;
  constexpr int NQ = (G::NPI + TS - 1) / TS;
  double *PI = S + LY::PI;
  double *prims = S + LY::PRIM;

  const double ABx = A[0] - B[0], ABy = A[1] - B[1], ABz = A[2] - B[2];
  const double AB2 = ABx * ABx + ABy * ABy + ABz * ABz;
  // primitive triplets of the group (nkept: its pair count, when the caller has it)
  const int K = (nkept >= 0 ? nkept : split_count(grp, Ka, Kb, ea, eb)) * Kc;

  // matrix-core contraction for whole-wave teams (chunks of 4 primitives = the
  // K extent of one MFMA); per-lane register slots otherwise
  constexpr bool MF = (TS % 64 == 0) && PCH % 4 == 0;
  using PT = PiTiles<G>;
  constexpr int NWV = TS >= 64 ? TS / 64 : 1;
  constexpr int NTW = MF ? (PT::N + NWV - 1) / NWV : 1;
  constexpr int NQA = MF ? 1 : NQ;
  const int wv = tid >> 6, pl = (tid & 63) >> 4, il = tid & 15;
  dbl4 macc[NTW];
#pragma unroll
  for (int j = 0; j < NTW; ++j) macc[j] = dbl4{0.0, 0.0, 0.0, 0.0};
  double acc[NQA];
#pragma unroll
  for (int q = 0; q < NQA; ++q) acc[q] = 0.0;

  for (int p0 = 0; p0 < npmax; p0 += PCH) {
    const int npc = imax(0, imin(PCH, K - p0));
    // the lane index is re-read every chunk: lane-dependent addresses are then
    // recomputed per chunk instead of being hoisted and kept live (spilled)
    int lt = tid;
    __asm__ volatile("" : "+v"(lt));
    setup_chunk<G, TS, REC, WM>(btab, prims, lt, p0, npc, Kb, Kc, A, B, C, AB2, ea, ca, eb, cb, ec,
                                cc, grp, Ka, cs);
    team_sync();
    // ---- VRR1, 2-quantal stages in place
    vrr1<G, TS, PCH, REC>(prims, npc, lt, vt0, vt1);
    // ---- early contraction of the CVRR2 prerequisites
    if constexpr (MF) {
      // lane (pl, il): primitive pl of the chunk, row / column il of a tile
      const int wl = lt >> 6, pc = (lt & 63) >> 4, cl = lt & 15;
      // groups of 4 primitives: the K extent of one MFMA (empty groups skipped,
      // uniformly over the team)
      static_for<PCH / 4>([&](auto gc) {
        constexpr int gq = decltype(gc)::value;
        if (4 * gq < npc) {
          const double *Rl = prims + (4 * gq + pc) * REC + PS_N + cl;
          const bool pv = 4 * gq + pc < npc;
          static_for<NWV>([&](auto wc) {
            constexpr int W = decltype(wc)::value;
            if (wl == W) {
              static_for<NTW>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                constexpr int t = j * NWV + W;
                if constexpr (t < PT::N) {
                  constexpr int k = PT::field(t, 0), r0 = PT::field(t, 1), c0 = PT::field(t, 2);
                  constexpr int nr = ncart(LP - k) - r0, nc = G::nek(k) - c0;
                  const double av = (pv && cl < nr) ? Rl[G::NV1 + G::sw_off(k) + r0] : 0.0;
                  const double bv = (pv && cl < nc) ? Rl[offT(G::emin(k)) + c0] : 0.0;
                  macc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, macc[j], 0, 0, 0);
                }
              });
            }
          });
        }
      });
    } else {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int r = lt + q * TS;
        const int code = slot ? slot[q] : (r < G::NPI ? pi_slot<G>(r) : -1);
        if (code >= 0) {
          const int isw = G::NV1 + (code >> 16), iv = code & 0xffff;
          double a = acc[q];
          for (int pp = 0; pp < npc; ++pp) {
            const double *R = prims + pp * REC + PS_N;
            a += R[isw] * R[iv];
          }
          acc[q] = a;
        }
      }
    }
    team_sync();
  }
  if constexpr (MF) {
    static_for<NWV>([&](auto wc) {
      constexpr int W = decltype(wc)::value;
      if (wv == W) {
        static_for<NTW>([&](auto jc) {
          constexpr int j = decltype(jc)::value;
          constexpr int t = j * NWV + W;
          if constexpr (t < PT::N) {
            constexpr int k = PT::field(t, 0), r0 = PT::field(t, 1), c0 = PT::field(t, 2);
            constexpr int nr = ncart(LP - k) - r0, nc = G::nek(k) - c0;
            constexpr int base = G::pi_off(k) + r0 * G::nek(k) + c0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int r = 4 * v + pl;
              if (r < nr && il < nc) PI[base + r * G::nek(k) + il] = macc[j][v];
            }
          }
        });
      }
    });
  } else {
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      if (tid + q * TS < G::NPI) PI[tid + q * TS] = acc[q];
  }
  team_sync();
  // ---- n-quantal CVRR2 in place on pi_0: (e0|c) += sum_{u != 0} w pi_{|u|}(e-u, c-u)
  // (reads only the blocks k >= 1, so the targets may be updated in any order)
  if constexpr (MF) {
    // whole waves take blocks of 64 targets of equal term count, terms
    // interleaved across the lanes: uniform loops, coalesced table loads; all
    // table words of a block are loaded first, then all pi operands, so each
    // block waits for one table and one LDS latency
    constexpr int MM = TB::CBM > 0 ? TB::CBM : 1;
    const int wv2 = tid >> 6, ln = tid & 63;
    for (int b = wv2; b < TB::NCB; b += NWV) {
      const int t = TB::cb_tg[b * 64 + ln];
      const int m = TB::cb_bm[b];
      const uint32_t *w = TB::cb_il + TB::cb_boff[b] + ln;
      uint32_t cw[MM];
#pragma unroll
      for (int j = 0; j < MM; ++j) cw[j] = j < m ? w[j * 64] : 0u;
      double pv[MM];
#pragma unroll
      for (int j = 0; j < MM; ++j) pv[j] = j < m ? PI[cw[j] & 0xffffu] : 0.0;
      double a = 0.0;
#pragma unroll
      for (int j = 0; j < MM; ++j) a += double(cw[j] >> 16) * pv[j];
      if (t != 0xffff) PI[t] += a;
    }
  } else {
    for (int t = tid; t < TB::NTGT; t += TS) {
      const int q0 = TB::cb_start[t], q1 = TB::cb_start[t + 1];
      if (q1 > q0) {
        double a = PI[t];
        // independent table loads, batched so their latencies overlap
#pragma unroll 8
        for (int q = q0; q < q1; ++q) {
          const uint32_t c = TB::cb_pw[q];
          a += double(c >> 16) * PI[c & 0xffffu];
        }
        PI[t] = a;
      }
    }
  }
  team_sync();
  // ---- ket to solid harmonics: lanes over e'', constant coefficients
  if (pure) {
    double *EM = S + LY::EM;
    using SH = GenSolid<LP>;
    for (int e = tid; e < G::NE; e += TS) {
      double ecv[G::NCP];
#pragma unroll
      for (int c = 0; c < G::NCP; ++c) ecv[c] = PI[c * G::NE + e];
      static_for<G::NPURE>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        double v = 0.0;
        static_for<G::NCP>([&](auto cc_) {
          constexpr int c = decltype(cc_)::value;
          constexpr double t = SH::dense[m * G::NCP + c];
          if constexpr (t != 0.0) v += t * ecv[c];
        });
        EM[m * G::NE + e] = v;
      });
    }
  } else if constexpr (LY::EM != 0) {
    // Cartesian ket (LP <= 1): (e0|c) is already the result; move it to EM
    double *EM = S + LY::EM;
    for (int t = tid; t < G::NCP * G::NE; t += TS) EM[t] = PI[t];
  }
  team_sync();
}

// ---------------------------------------------------------------------------
// n-quantal HRR for one (ket component m, bra component a):
//   (a b|m) = sum_{i <= b} prod_x C(b_x, i_x) AB_x^{b_x - i_x} (a+i 0|m),
// evaluated axis by axis (z, then y, then x) in registers.  out[b] for all
// Cartesian b of l = LB.
// ---------------------------------------------------------------------------
template <int LA, int LB>
__device__ __forceinline__ void hrr_nq(const double *EMm, int a, const double *pwx,
                                       const double *pwy, const double *pwz, double *out) {
  constexpr int NI = offT(LB + 1);  // all Cartesians i with |i| <= LB
  // components of a (y, z suffice for the index)
  int ay = 0, az = 0;
  static_for<ncart(LA)>([&](auto ac) {
    constexpr int c = decltype(ac)::value;
    constexpr C3 q = cart(LA, c);
    if (a == c) {
      ay = q[1];
      az = q[2];
    }
  });
  double X[NI];
  // X[i] = (a+i 0|m); e'' index of a + i relative to level LA
  static_for<LB + 1>([&](auto lc) {
    constexpr int li = decltype(lc)::value;
    static_for<ncart(li)>([&](auto ic) {
      constexpr int c = decltype(ic)::value;
      constexpr C3 i = cart(li, c);
      const int s = ay + az + i[1] + i[2];
      const int idx = offT(LA + li) - offT(LA) + (s * (s + 1)) / 2 + az + i[2];
      X[offT(li) + c] = EMm[idx];
    });
  });
  // z: Z(ix, iy, bz) = sum_{iz <= bz} C(bz, iz) ABz^{bz-iz} X(ix, iy, iz)
  double Z[NI];
  static_for<LB + 1>([&](auto xc) {
    constexpr int ix = decltype(xc)::value;
    static_for<LB + 1 - ix>([&](auto yc) {
      constexpr int iy = decltype(yc)::value;
      static_for<LB + 1 - ix - iy>([&](auto zc) {
        constexpr int bz = decltype(zc)::value;
        double v = 0.0;
        static_for<bz + 1>([&](auto kc) {
          constexpr int iz = decltype(kc)::value;
          constexpr double bn = double(binom(bz, iz));
          v += (bn * pwz[bz - iz]) * X[offT(ix + iy + iz) + cidx(ix, iy, iz)];
        });
        Z[offT(ix + iy + bz) + cidx(ix, iy, bz)] = v;
      });
    });
  });
  // y: Y(ix, by, bz) = sum_{iy <= by} C(by, iy) ABy^{by-iy} Z(ix, iy, bz)
  double Y[NI];
  static_for<LB + 1>([&](auto xc) {
    constexpr int ix = decltype(xc)::value;
    static_for<LB + 1 - ix>([&](auto yc) {
      constexpr int by = decltype(yc)::value;
      static_for<LB + 1 - ix - by>([&](auto zc) {
        constexpr int bz = decltype(zc)::value;
        double v = 0.0;
        static_for<by + 1>([&](auto kc) {
          constexpr int iy = decltype(kc)::value;
          constexpr double bn = double(binom(by, iy));
          v += (bn * pwy[by - iy]) * Z[offT(ix + iy + bz) + cidx(ix, iy, bz)];
        });
        Y[offT(ix + by + bz) + cidx(ix, by, bz)] = v;
      });
    });
  });
  // x: out(b) = sum_{ix <= bx} C(bx, ix) ABx^{bx-ix} Y(ix, by, bz), |b| = LB
  static_for<ncart(LB)>([&](auto bc) {
    constexpr int b = decltype(bc)::value;
    constexpr C3 q = cart(LB, b);
    double v = 0.0;
    static_for<q[0] + 1>([&](auto kc) {
      constexpr int ix = decltype(kc)::value;
      constexpr double bn = double(binom(q[0], ix));
      v += (bn * pwx[q[0] - ix]) * Y[offT(ix + q[1] + q[2]) + cidx(ix, q[1], q[2])];
    });
    out[b] = v;
  });
}

// HRR of the whole block into the staging area STG: [m][a][b] (or [m][b][a]
// when the triplet's a and b were swapped to orient the transfer).
template <int LP, int LA, int LB, int TS, int PCH, bool CART = false>
__device__ __forceinline__ void hrr_block(double *S, int tid, const double *A, const double *B,
                                          int np_out, bool swp) {
  using G = Geo<LP, LA, LA + LB>;
  using LY = Layout<LP, LA, LB, PCH, CART>;
  constexpr int NA = ncart(LA), NB = ncart(LB);
  const double *EM = S + LY::EM;
  double *STG = S + LY::STG;
  double pwx[LB + 1], pwy[LB + 1], pwz[LB + 1];
  pwx[0] = pwy[0] = pwz[0] = 1.0;
#pragma unroll
  for (int k = 1; k <= LB; ++k) {
    pwx[k] = pwx[k - 1] * (A[0] - B[0]);
    pwy[k] = pwy[k - 1] * (A[1] - B[1]);
    pwz[k] = pwz[k - 1] * (A[2] - B[2]);
  }
  for (int it = tid; it < np_out * NA; it += TS) {
    const int m = it / NA, a = it - m * NA;
    double o[NB];
    hrr_nq<LA, LB>(EM + m * G::NE, a, pwx, pwy, pwz, o);
    if (!swp) {
#pragma unroll
      for (int b = 0; b < NB; ++b) STG[(m * NA + a) * NB + b] = o[b];
    } else {
#pragma unroll
      for (int b = 0; b < NB; ++b) STG[(m * NB + b) * NA + a] = o[b];
    }
  }
}

// per-lane contraction slots, decoded once per launch
template <int LP, int LA, int LB, int TS>
__device__ __forceinline__ void make_slots(int *slot, int tid) {
  using G = Geo<LP, LA, LA + LB>;
  constexpr int NQ = (G::NPI + TS - 1) / TS;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int r = tid + q * TS;
    slot[q] = r < G::NPI ? pi_slot<G>(r) : -1;
  }
}

// ---------------------------------------------------------------------------
// Cartesian ket of l = LQ + 2 cs from the degree-LQ term of its expansion: a
// Cartesian Gaussian x^c e^{-zc r^2} (per axis) is the sum over k of
// c!/(k!(c-2k)!) (4 zc)^{-k} (2 zc)^{-(c-2k)} times the Hermite Gaussian of
// order c - 2k, and a Hermite ket of order t is the sum over j of
// t!/(j!(t-2j)!) (-rho/(4 zc^2))^j times the two-term VRR2 ket of order t - 2j
// with the Boys orders raised by j.  Collected by the total lowering d = k + j
// (Vandermonde over the axes), the part of degree LQ = l - 2 cs is
//   (c|  +=  sum_{|d| = cs, 2d <= c} c! / ((c - 2d)! d!)  (c - 2d|',
// where (t|' is the two-term ket of class LQ with the Boys sequence of
// setup_prim (cs > 0).  The launch of class LQ adds this into the block of the
// class LQ + 2 cs, rows [c][a b] from the staging rows [t][a b].
// ---------------------------------------------------------------------------
template <int LQ, int TS>
__device__ __forceinline__ void store_cart_expand(double *out, const double *STG, int tid, int cs,
                                                  int nab) {
  constexpr double fact[11] = {1, 1, 2, 6, 24, 120, 720, 5040, 40320, 362880, 3628800};
  const int l = LQ + 2 * cs;
  const int nc = (l + 1) * (l + 2) / 2;
  for (int o = tid; o < nc * nab; o += TS) {
    const int c = o / nab, r = o - c * nab;
    // Cartesian order: for i = 0..l, j = 0..i: (l - i, i - j, j)
    int i = 0;
    while ((i + 1) * (i + 2) / 2 <= c) ++i;
    const int cz = c - i * (i + 1) / 2, cy = i - cz, cx = l - i;
    double v = 0.0;
    for (int dx = 0; dx <= cs && 2 * dx <= cx; ++dx)
      for (int dy = 0; dx + dy <= cs && 2 * dy <= cy; ++dy) {
        const int dz = cs - dx - dy;
        if (2 * dz > cz) continue;
        const int tx = cx - 2 * dx, ty = cy - 2 * dy, tz = cz - 2 * dz;
        const int ti = (ty + tz) * (ty + tz + 1) / 2 + tz;
        const double w = fact[cx] / (fact[tx] * fact[dx]) * fact[cy] / (fact[ty] * fact[dy]) *
                         fact[cz] / (fact[tz] * fact[dz]);
        v += w * STG[ti * nab + r];
      }
    out[o] += v;
  }
}

// ---------------------------------------------------------------------------
// store digestion: one triplet per team, blocks written to out + out_off[t]
// ---------------------------------------------------------------------------
template <int LP, int LA, int LB, int TS, int PCH, bool CART = false>
__global__ void __launch_bounds__(TS > 64 ? TS : 64)
    __attribute__((amdgpu_waves_per_eu(Cfg<LP, LA, LB>::WPE))) k_store(StoreArgs a) {
  using G = Geo<LP, LA, LA + LB>;
  using LY = Layout<LP, LA, LB, PCH, CART>;
  constexpr int BLK = TS > 64 ? TS : 64;
  constexpr int TPB = BLK / TS;
  constexpr int NA = ncart(LA), NB = ncart(LB);
  constexpr int NQ = (G::NPI + TS - 1) / TS;
  extern __shared__ double smem[];
  const int team = threadIdx.x / TS, tid = threadIdx.x % TS;
  double *S = smem + team * (CART ? Cfg<LP, LA, LB>::STORE_TEAM_C : Cfg<LP, LA, LB>::STORE_TEAM);
  const int np_out = a.pure ? npure(LP) : ncart(LP);
  // the lower-degree Cartesian terms run only in the Cartesian-ket kernels
  // (a compile-time 0 elsewhere keeps their Boys branch out of the pure kernels)
  const int cexp = CART ? a.cexp : 0;
  if (a.err && *a.err) return;
  // the VRR1 item records, staged once per workgroup after the team slices
  constexpr int STEAM = CART ? Cfg<LP, LA, LB>::STORE_TEAM_C : Cfg<LP, LA, LB>::STORE_TEAM;
  constexpr int VTO = (TPB * STEAM * 8 + 15) / 16 * 16;
  constexpr int NVT = VStages<LA + LB>::NITEMS;
  uint4 *vt0 = reinterpret_cast<uint4 *>(reinterpret_cast<char *>(smem) + VTO);
  uint2 *vt1 = reinterpret_cast<uint2 *>(reinterpret_cast<char *>(smem) + VTO + NVT * 16);
  stage_vrr1_table<LA + LB>(vt0, vt1);
  __syncthreads();
  const int64_t count = a.dcount ? int64_t(*a.dcount) : a.count;
  const uint32_t *bucket = a.bucket + (a.dstart ? *a.dstart : 0);
  int slot[NQ];
  make_slots<LP, LA, LB, TS>(slot, tid);

  for (int64_t base = int64_t(blockIdx.x) * TPB; base < count; base += int64_t(gridDim.x) * TPB) {
    const int64_t item = base + team;
    const bool valid = item < count;
    uint32_t code = valid ? bucket[item] : 0u;
    const bool swp = (code >> 31) != 0;
    const int64_t t = int64_t(code & 0x7fffffffu);
    int sP = 0, s1 = 0, s2 = 0;
    if (valid) {
      sP = a.trip[3 * t];
      s1 = a.trip[3 * t + 1];
      s2 = a.trip[3 * t + 2];
    }
    const int sa = swp ? s2 : s1, sb = swp ? s1 : s2;
    const int Ka = valid ? a.orb.nprim[sa] : 0, Kb = valid ? a.orb.nprim[sb] : 0;
    const int Kc = valid ? a.aux.nprim[sP] : 0;
    const int64_t oa = valid ? a.orb.prim_off[sa] : 0, ob = valid ? a.orb.prim_off[sb] : 0,
                  oc = valid ? a.aux.prim_off[sP] : 0;
    double Ar[3] = {0, 0, 0}, Br[3] = {0, 0, 0}, Cr[3] = {0, 0, 0};
    if (valid) {
      const int ia = a.orb.atom[sa], ib = a.orb.atom[sb], ic = a.aux.atom[sP];
      for (int x = 0; x < 3; ++x) {
        Ar[x] = a.xyz[3 * ia + x];
        Br[x] = a.xyz[3 * ib + x];
        Cr[x] = a.xyz[3 * ic + x];
      }
    }
    const double *ea = a.orb.exps + oa, *eb = a.orb.exps + ob;
    // HRR direction per primitive pair: pass 1 puts the VRR1 quanta on A
    // (pairs with zeta_a >= zeta_b), pass 2 on B (the rest), and the blocks
    // add.  A shell pair whose pairs all prefer A runs pass 1 alone over all
    // of them; one whose pairs all prefer B (possible for l_a > l_b, where the
    // quanta would otherwise always go to the higher-l shell) pass 2 alone;
    // A == B needs no transfer and runs pass 1.
    int n1 = 0;
    bool far = false;
    if (valid) {
      const double ABx = Ar[0] - Br[0], ABy = Ar[1] - Br[1], ABz = Ar[2] - Br[2];
      far = ABx * ABx + ABy * ABy + ABz * ABz > 0.0;
      n1 = split_count(1, Ka, Kb, ea, eb);
    }
    const int nab = Ka * Kb;
    bool run1 = valid && (!far || n1 > 0), run2 = valid && far && n1 < nab;
    // a mixed pair whose group 2 is too weak to matter stays in one pass with
    // the quanta on A: the bound on its HRR rounding lies below 1e-16 (a
    // thousandth of the absolute floor of the element bar).  Whole-wave teams
    // only (smaller teams share a wave, whose passes must agree).
    if constexpr (TS >= 64) {
      if (run1 && run2 && cexp == 0) {
        int lane = tid & 63;
        __asm__ volatile("" : "+v"(lane));
        const double ABx = Ar[0] - Br[0], ABy = Ar[1] - Br[1], ABz = Ar[2] - Br[2];
        const double bound = split_error_bound<LP, LA, LB>(
            lane, Ka, ea, a.orb.coefs + oa, Kb, eb, a.orb.coefs + ob,
            ABx * ABx + ABy * ABy + ABz * ABz, Kc, a.aux.exps + oc, a.aux.coefs + oc, a.pure);
        if (bound < 1e-16) {
          run2 = false;
          n1 = nab;
        }
      }
    }
    // the passes are uniform over the workgroup (teams of one wave share
    // barriers); a team without work in a pass runs it over no primitives
    const bool do1 = TS >= 64 ? run1 : wave_any(run1);
    const bool do2 = TS >= 64 ? run2 : wave_any(run2);
    const int nout = np_out * NA * NB;
    if (do1) {
      const int K1 = (run1 ? (run2 ? n1 : nab) : 0) * Kc;
      triplet_to_e0P<LP, LA, LB, TS, PCH, 0, CART>(a.boys, S, tid, slot,
                                                   TS >= 64 ? K1 : wave_max(K1),
                                          Ar, Br, Cr, Ka, ea, a.orb.coefs + oa, Kb, eb,
                                          a.orb.coefs + ob, run1 ? Kc : 0, a.aux.exps + oc,
                                          a.aux.coefs + oc, a.pure, run2 ? 1 : 0, cexp,
                                          run2 ? n1 : nab, vt0, vt1);
      hrr_block<LP, LA, LB, TS, PCH, CART>(S, tid, Ar, Br, np_out, swp);
      team_sync();
      if (run1) {
        double *out = a.out + a.out_off[t];
        const double *STG = S + LY::STG;
        if (cexp)
          store_cart_expand<LP, TS>(out, STG, tid, cexp, NA * NB);
        else
          for (int o = tid; o < nout; o += TS) out[o] = STG[o];
      }
      team_sync();
    }
    if (do2) {
      // quanta on B: for l_a > l_b the pipeline of the swapped class
      // (LP, LB, LA), whose VRR1 builds e = LB..LA+LB on B and whose HRR
      // moves LA quanta to A
      const int K2 = run2 ? (nab - n1) * Kc : 0;
      triplet_to_e0P<LP, LB, LA, TS, PCH, 0, CART>(a.boys, S, tid, LA == LB ? slot : nullptr,
                                          TS >= 64 ? K2 : wave_max(K2), Br, Ar, Cr, Kb, eb,
                                          a.orb.coefs + ob, Ka, ea, a.orb.coefs + oa,
                                          run2 ? Kc : 0, a.aux.exps + oc, a.aux.coefs + oc,
                                          a.pure, 2, cexp, nab - n1, vt0, vt1);
      hrr_block<LP, LB, LA, TS, PCH, CART>(S, tid, Br, Ar, np_out, !swp);
      team_sync();
      if (run2) {
        double *out = a.out + a.out_off[t];
        const double *STG = S + Layout<LP, LB, LA, PCH, CART>::STG;
        if (cexp)
          store_cart_expand<LP, TS>(out, STG, tid, cexp, NA * NB);
        else if (run1)
          for (int o = tid; o < nout; o += TS) out[o] += STG[o];
        else
          for (int o = tid; o < nout; o += TS) out[o] = STG[o];
      }
      team_sync();
    }
  }
}

// lanes per work item of the gradient and gamma engines: four waves share one
// item's LDS (the LDS per item, not the lanes, bounds the items per CU)
constexpr int ENG_TS = 256;

// ---------------------------------------------------------------------------
// HRR orientation of a pair of equal l: the VRR1 quanta go to the shell with
// the larger (max exponent x min exponent), for which the Gaussian product
// centre P lies closest to its own centre and the HRR transfers are best
// conditioned.  The J kernels write both J blocks of a pair, so the choice is
// free; the batched (P|ab) path makes the same choice.
// ---------------------------------------------------------------------------
template <int LA, int LB>
__device__ __forceinline__ void orient_pair(const ShellsDev &orb, int &sa, int &sb) {
  if (LA != LB || sa == sb) return;
  auto tight = [&](int sh) {
    const double *e = orb.exps + orb.prim_off[sh];
    double lo = e[0], hi = e[0];
    for (int i = 1; i < orb.nprim[sh]; ++i) {
      lo = fmin(lo, e[i]);
      hi = fmax(hi, e[i]);
    }
    return lo * hi;
  };
  if (tight(sb) > tight(sa)) {
    const int t = sa;
    sa = sb;
    sb = t;
  }
}

// ---------------------------------------------------------------------------
// J digestion: one orbital shell pair per team (per lane group on the register
// engine); the team loops over all aux shells of l = LP.  The HRR and the ket transform are linear in the ket, and
// the HRR coefficients depend only on A - B, so d_P is contracted into (e0|P)
// right after the transform and accumulated over all aux shells,
//   X_e = sum_P sum_m d_Pm (e0|Pm),
// and one single-component HRR per pair gives J_ab = (ab|X) -- the same sum as
// sum_P (ab|P) d_P in another order (the contraction of the density with
// intermediates that Section 4 names as the better J strategy).  The block and
// its transpose are added into J; each pair is owned by exactly one team, so
// no atomics are needed, and launches of different LP run in stream order.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Register J engine for small classes: one lane owns one shell pair and runs
// every aux shell and primitive triplet of it with all intermediates in
// registers (compile-time indices, no LDS, no index tables).  Per primitive:
// setup, Boys, VRR1 (Eq. vrr1, 1-quantal steps over all m), then the digested
// ket of the J engine below with the sW monomials formed on the fly:
//   H_u = s^{|u|} sum_{c >= u} C(c,u) d'_c W^{c-u},  W = rho/zeta_c PC,
//   X_e += sum_u e!/(e-u)! H_u [e-u 0|0]^(LP);
// one HRR of X per pair adds the J block (both triangles).
// ---------------------------------------------------------------------------
template <int LP, int LA, int LB>
__device__ __forceinline__ void jr_pair(const JArgs &a, bool valid, int sa, int sb, int sub) {
  using R = JReg<LP, LA, LB>;
  constexpr int L = R::L, NE = R::NE, NCP = ncart(LP), NA = ncart(LA), NB = ncart(LB);
  if (!valid) return;
  orient_pair<LA, LB>(a.orb, sa, sb);
  const int Ka = a.orb.nprim[sa], Kb = a.orb.nprim[sb];
  const double *ea = a.orb.exps + a.orb.prim_off[sa], *ca = a.orb.coefs + a.orb.prim_off[sa];
  const double *eb = a.orb.exps + a.orb.prim_off[sb], *cb = a.orb.coefs + a.orb.prim_off[sb];
  double A[3], B[3];
  {
    const int ia = a.orb.atom[sa], ib = a.orb.atom[sb];
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      A[x] = a.xyz[3 * ia + x];
      B[x] = a.xyz[3 * ib + x];
    }
  }
  const double AB2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) +
                     (A[2] - B[2]) * (A[2] - B[2]);
  double X[NE];
#pragma unroll
  for (int e = 0; e < NE; ++e) X[e] = 0.0;

  // primitive pairs outermost: 1/gamma, P and the pair's exponential are
  // formed once per primitive pair, not once per (primitive pair, aux shell);
  // the nsub lanes of the pair take every nsub-th aux shell
  const int nsub = a.nsub;
  for (int ia = 0; ia < Ka; ++ia)
    for (int ib = 0; ib < Kb; ++ib) {
      const double za = ea[ia], zb = eb[ib];
      const double g = za + zb, ig = 1.0 / g;
      const double P[3] = {(za * A[0] + zb * B[0]) * ig, (za * A[1] + zb * B[1]) * ig,
                           (za * A[2] + zb * B[2]) * ig};
      const double PA[3] = {P[0] - A[0], P[1] - A[1], P[2] - A[2]};
      const double eab = exp(-za * zb * ig * AB2) * ca[ia] * cb[ib];
      for (int ip = sub; ip < a.np; ip += nsub) {
        const double *rc = a.arec + int64_t(ip) * AREC;
        const double C[3] = {rc[AR_CX], rc[AR_CY], rc[AR_CZ]};
        const int64_t po = int64_t(rc[AR_PRIM]);
        const int Kc = int(rc[AR_K]);
        const double *ec = a.aux.exps + po, *cc = a.aux.coefs + po;
        double zc = rc[AR_Z0], ccv = rc[AR_C0];
        double dq[NCP];
#pragma unroll
        for (int c = 0; c < NCP; ++c) dq[c] = rc[AR_DQ + c];
        for (int ic = 0; ic < Kc; ++ic) {
          if (ic > 0) {
            zc = ec[ic];
            ccv = cc[ic];
          }
          const double PC[3] = {P[0] - C[0], P[1] - C[1], P[2] - C[2]};
          const double gz = g + zc, rho = g * zc / gz, rg = rho * ig, i2g = 0.5 * ig;
          const double T = rho * (PC[0] * PC[0] + PC[1] * PC[1] + PC[2] * PC[2]);
          // 2 pi^{5/2} / ((g+zc)^{1/2} g zc) exp(-za zb/g AB^2) x contraction coefficients
          const double pre = 34.98683665524972497 / (sqrt(gz) * g * zc) * eab * ccv;
          const double RP[3] = {rg * PC[0], rg * PC[1], rg * PC[2]};
          double Fm[L + 1];
          boys<LP, L + 1>(a.boys, T, Fm);
          // VRR1: vr[voff(l) + c (L-l+1) + m] = [e 0|0]^(LP+m), e = cart(l, c)
          double vr[R::NVR];
#pragma unroll
          for (int m = 0; m <= L; ++m) vr[m] = pre * Fm[m];
          static_for<L>([&](auto lc) {
            constexpr int l = decltype(lc)::value + 1;
            static_for<ncart(l)>([&](auto cc_) {
              constexpr int c = decltype(cc_)::value;
              constexpr C3 e = cart(l, c);
              constexpr int i = rdir(e);
              constexpr int c1 = cidx(e[0] - (i == 0), e[1] - (i == 1), e[2] - (i == 2));
              constexpr int o1 = R::voff(l - 1) + c1 * (L - l + 2);
              constexpr int o = R::voff(l) + c * (L - l + 1);
              static_for<L - l + 1>([&](auto mc) {
                constexpr int m = decltype(mc)::value;
                double v = PA[i] * vr[o1 + m] - RP[i] * vr[o1 + m + 1];
                if constexpr (e[i] >= 2) {
                  constexpr int c2 = cidx(e[0] - 2 * (i == 0), e[1] - 2 * (i == 1),
                                          e[2] - 2 * (i == 2));
                  constexpr int o2 = R::voff(l - 2) + c2 * (L - l + 3);
                  v += double(e[i] - 1) * i2g * (vr[o2 + m] - rg * vr[o2 + m + 1]);
                }
                vr[o + m] = v;
              });
            });
          });
          // H_u, |u| <= KU
          const double s = rho * ig * (0.5 / zc), rz = rho / zc;
          double wx[LP + 1], wy[LP + 1], wz[LP + 1], sk[R::KU + 1];
          wx[0] = wy[0] = wz[0] = sk[0] = 1.0;
#pragma unroll
          for (int q = 1; q <= LP; ++q) {
            wx[q] = wx[q - 1] * (rz * PC[0]);
            wy[q] = wy[q - 1] * (rz * PC[1]);
            wz[q] = wz[q - 1] * (rz * PC[2]);
          }
#pragma unroll
          for (int q = 1; q <= R::KU; ++q) sk[q] = sk[q - 1] * s;
          double H[R::NU];
          static_for<R::KU + 1>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            static_for<ncart(k)>([&](auto uc) {
              constexpr int ui = decltype(uc)::value;
              constexpr C3 u = cart(k, ui);
              double h = 0.0;
              static_for<NCP>([&](auto cc_) {
                constexpr int c = decltype(cc_)::value;
                constexpr C3 q = cart(LP, c);
                if constexpr (q[0] >= u[0] && q[1] >= u[1] && q[2] >= u[2]) {
                  constexpr double bn =
                      double(binom(q[0], u[0]) * binom(q[1], u[1]) * binom(q[2], u[2]));
                  h += (bn * dq[c]) * (wx[q[0] - u[0]] * wy[q[1] - u[1]] * wz[q[2] - u[2]]);
                }
              });
              H[offT(k) + ui] = sk[k] * h;
            });
          });
          // X_e += sum_u e!/(e-u)! H_u V_{e-u}
          static_for<L - LA + 1>([&](auto lc) {
            constexpr int le = LA + decltype(lc)::value;
            static_for<ncart(le)>([&](auto ec_) {
              constexpr int ce = decltype(ec_)::value;
              constexpr C3 e = cart(le, ce);
              double v = X[offT(le) - offT(LA) + ce];
              static_for<e[0] + 1>([&](auto xc) {
                constexpr int ux = decltype(xc)::value;
                static_for<e[1] + 1>([&](auto yc) {
                  constexpr int uy = decltype(yc)::value;
                  static_for<e[2] + 1>([&](auto zc_) {
                    constexpr int uz = decltype(zc_)::value;
                    constexpr int k = ux + uy + uz;
                    if constexpr (k <= LP) {
                      constexpr int lr = le - k;
                      constexpr int cr = cidx(e[0] - ux, e[1] - uy, e[2] - uz);
                      constexpr double f = double(falling(e[0], ux) * falling(e[1], uy) *
                                                  falling(e[2], uz));
                      v += (f * H[offT(k) + cidx(ux, uy, uz)]) *
                           vr[R::voff(lr) + cr * (L - lr + 1)];
                    }
                  });
                });
              });
              X[offT(le) - offT(LA) + ce] = v;
            });
          });
        }
      }
  }
  // sum the partial X of the pair's lanes p + k 64/nsub by a butterfly: every
  // lane ends with the same bits, (x0 + x1) + (x2 + x3) for nsub = 4
  for (int m = 64 / nsub; m < 64; m <<= 1) {
#pragma unroll
    for (int e = 0; e < NE; ++e) X[e] += __shfl_xor(X[e], m);
  }
  if (sub != 0) return;
  // one HRR of X, both J triangles
  double pwx[LB + 1], pwy[LB + 1], pwz[LB + 1];
  pwx[0] = pwy[0] = pwz[0] = 1.0;
#pragma unroll
  for (int k = 1; k <= LB; ++k) {
    pwx[k] = pwx[k - 1] * (A[0] - B[0]);
    pwy[k] = pwy[k - 1] * (A[1] - B[1]);
    pwz[k] = pwz[k - 1] * (A[2] - B[2]);
  }
  const int64_t ra = a.ao_off[sa] - a.ao_base, rb = a.ao_off[sb] - a.ao_base;
  static_for<NA>([&](auto ac) {
    constexpr int ia = decltype(ac)::value;
    double o[NB];
    hrr_nq<LA, LB>(X, ia, pwx, pwy, pwz, o);
#pragma unroll
    for (int ib = 0; ib < NB; ++ib) {
      a.J[(ra + ia) * a.nao + rb + ib] += o[ib];
      if (sa != sb) a.J[(rb + ib) * a.nao + ra + ia] += o[ib];
    }
  });
}

// ---------------------------------------------------------------------------
// J engine: the fitting coefficients are digested into the ket before the
// CVRR2 combination.  For one aux shell with Cartesian image
// d'_c = sum_m d_m T_mc of its coefficients,
//   sum_c d'_c (e0|c) = sum_prim sum_u e!/(e-u)! H_u V_{e-u},
//   H_u = sum_{c >= u, |c| = LP} C(c,u) d'_c sW_{|u|}[c-u],  V = [e'0|0]^(LP),
// which is Eq. cVRR2 in n-quantal form applied to the prerequisites of
// Eq. a0cv2 (the powers of rho/(2 gamma zeta_c) cancel between the two).  Per
// shell pair the team accumulates M_{u,e'} = sum_{aux shells} sum_prim H_u V_{e'}
// on the matrix cores (block k = |u|: ncart(k) rows, nek(k) columns, 16 x 16 x 4
// tiles) and forms X_e = sum_u e!/(e-u)! M_{u,e-u} once; one HRR of X gives the
// J block.  No per-triplet CVRR2 combination, ket transform or digestion remains.
// ---------------------------------------------------------------------------
// classes whose J runs on the engine: whole-wave teams, chunks of 4, 8 or 16
// primitive triplets (groups of 4 = the K extent of one MFMA)
template <int LP, int LA, int LB, int TS, int PCH>
constexpr bool use_jengine() {
  return TS % 64 == 0 && PCH % 4 == 0 && PCH <= 16;
}

template <int LP, int LA, int LB, int TS, int PCH>
__device__ __forceinline__ void jeng_pair(const JArgs &a, double *S, int tid, bool valid, int sa,
                                          int sb, int np_loop) {
  using G = Geo<LP, LA, LA + LB>;
  using JE = JELayout<LP, LA, LB, PCH>;
  using MT = MTiles<G>;
  using SH = GenSolid<LP>;
  using TB = GenTab<LP, G::EA, G::EB>;
  static_assert(TB::NM == MT::NM, "generated J-engine tables out of date");
  static_assert(use_jengine<LP, LA, LB, TS, PCH>(), "the J engine runs whole-wave teams");
  constexpr int REC = JE::REC;
  constexpr int NA = ncart(LA), NB = ncart(LB);
  constexpr int NWV = TS / 64;
  constexpr int NTW = (MT::N + NWV - 1) / NWV;
  constexpr int NU = offT(imin(LP, G::EB) + 1);  // H_u with |u| <= min(LP, EB)
  if (valid) orient_pair<LA, LB>(a.orb, sa, sb);
  const int Ka = valid ? a.orb.nprim[sa] : 0, Kb = valid ? a.orb.nprim[sb] : 0;
  const int64_t oa = valid ? a.orb.prim_off[sa] : 0, ob = valid ? a.orb.prim_off[sb] : 0;
  double Ar[3] = {0, 0, 0}, Br[3] = {0, 0, 0};
  if (valid) {
    const int ia = a.orb.atom[sa], ib = a.orb.atom[sb];
    for (int x = 0; x < 3; ++x) {
      Ar[x] = a.xyz[3 * ia + x];
      Br[x] = a.xyz[3 * ib + x];
    }
  }
  const double ABx = Ar[0] - Br[0], ABy = Ar[1] - Br[1], ABz = Ar[2] - Br[2];
  const double AB2 = ABx * ABx + ABy * ABy + ABz * ABz;
  double *prims = S;
  double *DP = S + JE::DP;
  dbl4 macc[NTW];
#pragma unroll
  for (int j = 0; j < NTW; ++j) macc[j] = dbl4{0.0, 0.0, 0.0, 0.0};
  const int Kab = Ka * Kb;
  // The pair's primitive triplets over all its aux shells, (aux shell, p) in
  // order, are cut into chunks of PCH: M sums over aux shells as well, so a
  // chunk may mix shells and every chunk but the last is full.  The cursor
  // (cip, cp) is uniform over the team.
  auto shell_prims = [&](int ip) {
    return (valid && ip < a.np) ? Kab * int(a.arec[int64_t(ip) * AREC + AR_K]) : 0;
  };
  int cip = 0, cp = 0, cK = shell_prims(0);
  while (cip < np_loop && cK == 0) cK = shell_prims(++cip);
  while (cip < np_loop) {
    // slots of this chunk: aux shell position and primitive in the shell
    int sl_ip[PCH], sl_p[PCH];
    int npc = 0;
#pragma unroll
    for (int pp = 0; pp < PCH; ++pp) {
      sl_ip[pp] = cip;
      sl_p[pp] = cp;
      if (cip < np_loop) {
        npc = pp + 1;
        if (++cp == cK) {
          cp = 0;
          cK = shell_prims(++cip);
          while (cip < np_loop && cK == 0) cK = shell_prims(++cip);
        }
      }
    }
    int lt = tid;
    __asm__ volatile("" : "+v"(lt));
    // d' of the aux shell of every slot, from the shell's record
    for (int it = lt; it < npc * G::NCP; it += TS) {
      const int pp = it / G::NCP, c = it - pp * G::NCP;
      int ip = sl_ip[0];
#pragma unroll
      for (int q = 1; q < PCH; ++q)
        if (pp == q) ip = sl_ip[q];
      DP[pp * G::NCP + c] = a.arec[int64_t(ip) * AREC + AR_DQ + c];
    }
    // one lane per slot: record setup (primitive of its own aux shell)
    if (lt < npc) {
      int ip = sl_ip[0], p = sl_p[0];
#pragma unroll
      for (int q = 1; q < PCH; ++q)
        if (lt == q) {
          ip = sl_ip[q];
          p = sl_p[q];
        }
      const double *rc = a.arec + int64_t(ip) * AREC;
      const int Kc = int(rc[AR_K]);
      const int64_t oc = int64_t(rc[AR_PRIM]);
      const double Cr[3] = {rc[AR_CX], rc[AR_CY], rc[AR_CZ]};
      setup_prim<G, 0>(a.boys, prims + lt * REC, p, Kb, Kc, Ar, Br, Cr, AB2, a.orb.exps + oa,
                       a.orb.coefs + oa, a.orb.exps + ob, a.orb.coefs + ob, a.aux.exps + oc,
                       a.aux.coefs + oc);
    }
    team_sync();
    vrr1<G, TS, PCH, REC>(prims, npc, lt);
    // H_u of the chunk, u-major so the long sums (small |u|) spread over lanes
    for (int it = lt; it < npc * NU; it += TS) {
      const int u = it / npc, pp = it - u * npc;
      const double *SWp = prims + pp * REC + PS_N + G::NV1;
      const double *DPp = DP + pp * G::NCP;
      double h = 0.0;
#pragma unroll 4
      for (int q = SH::jh_start[u]; q < SH::jh_start[u + 1]; ++q) {
        const uint32_t t = SH::jh_t[q];
        h += double(t >> 16) * DPp[t & 0xffu] * SWp[(t >> 8) & 0xffu];
      }
      prims[pp * REC + JE::HU + u] = h;
    }
    team_sync();
    // M += H V on the matrix cores, one MFMA per tile and group of 4
    // primitives; lane (pc, cl): primitive 4 g + pc of group g, row / column cl
    const int wl = lt >> 6, pc = (lt & 63) >> 4, cl = lt & 15;
    static_for<PCH / 4>([&](auto gc) {
      constexpr int g4 = decltype(gc)::value;
      if (4 * g4 < npc) {
        const double *Rl = prims + (4 * g4 + pc) * REC + cl;
        const bool pv = 4 * g4 + pc < npc;
        static_for<NWV>([&](auto wc) {
          constexpr int W = decltype(wc)::value;
          if (wl == W) {
            static_for<NTW>([&](auto jc) {
              constexpr int j = decltype(jc)::value;
              constexpr int t = j * NWV + W;
              if constexpr (t < MT::N) {
                constexpr int k = MT::field(t, 0), r0 = MT::field(t, 1), c0 = MT::field(t, 2);
                constexpr int nr = ncart(k) - r0, nc = G::nek(k) - c0;
                const double av = (pv && cl < nr) ? Rl[JE::HU + offT(k) + r0] : 0.0;
                const double bv = (pv && cl < nc) ? Rl[PS_N + offT(G::emin(k)) + c0] : 0.0;
                macc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, macc[j], 0, 0, 0);
              }
            });
          }
        });
      }
    });
    team_sync();
  }
  // M to LDS, then X_e = sum_u e!/(e-u)! M_{u,e-u}
  double *MJ = S + JE::MJ;
  {
    const int wl = tid >> 6, pc = (tid & 63) >> 4, cl = tid & 15;
    static_for<NWV>([&](auto wc) {
      constexpr int W = decltype(wc)::value;
      if (wl == W) {
        static_for<NTW>([&](auto jc) {
          constexpr int j = decltype(jc)::value;
          constexpr int t = j * NWV + W;
          if constexpr (t < MT::N) {
            constexpr int k = MT::field(t, 0), r0 = MT::field(t, 1), c0 = MT::field(t, 2);
            constexpr int nr = ncart(k) - r0, nc = G::nek(k) - c0;
            constexpr int base = MT::moff(k) + r0 * G::nek(k) + c0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int r = 4 * v + pc;
              if (r < nr && cl < nc) MJ[base + r * G::nek(k) + cl] = macc[j][v];
            }
          }
        });
      }
    });
  }
  team_sync();
  double *XD = S + JE::XD;
  for (int e = tid; e < G::NE; e += TS) {
    double v = 0.0;
#pragma unroll 8
    for (int q = TB::jx_start[e]; q < TB::jx_start[e + 1]; ++q) {
      const uint32_t t = TB::jx_mc[q];
      v += double(t >> 16) * MJ[t & 0xffffu];
    }
    XD[e] = v;
  }
  team_sync();
  double pwx[LB + 1], pwy[LB + 1], pwz[LB + 1];
  pwx[0] = pwy[0] = pwz[0] = 1.0;
#pragma unroll
  for (int k = 1; k <= LB; ++k) {
    pwx[k] = pwx[k - 1] * ABx;
    pwy[k] = pwy[k - 1] * ABy;
    pwz[k] = pwz[k - 1] * ABz;
  }
  if (valid) {
    const int64_t ra = a.ao_off[sa] - a.ao_base, rb = a.ao_off[sb] - a.ao_base;
    for (int ia = tid; ia < NA; ia += TS) {
      double o[NB];
      hrr_nq<LA, LB>(XD, ia, pwx, pwy, pwz, o);
#pragma unroll
      for (int ib = 0; ib < NB; ++ib) {
        a.J[(ra + ia) * a.nao + rb + ib] += o[ib];
        if (sa != sb) a.J[(rb + ib) * a.nao + ra + ia] += o[ib];
      }
    }
  }
  team_sync();
}

template <int LP, int LA, int LB, int TS, int PCH>
struct JLayout {
  // the register engine keeps everything in registers; the J engine runs
  // whole-wave teams with chunks of 4 primitive triplets
  static constexpr bool REG = TS == 1 && JReg<LP, LA, LB>::OK;
  static_assert(REG || use_jengine<LP, LA, LB, TS, PCH>(), "J runs on one of the two engines");
  static constexpr int TOTAL = REG ? 0 : JELayout<LP, LA, LB, PCH>::TOTAL;
  static constexpr int BYTES_WG = ((TS > 64 ? TS : 64) / TS) * TOTAL * 8;
  static_assert(BYTES_WG <= 160 * 1024, "J layout does not fit the LDS of a CU");
};

template <int LP, int LA, int LB, int TS, int PCH>
__device__ __forceinline__ void j_pair(const JArgs &a, double *S, int tid, bool valid, int sa,
                                       int sb, int np_loop, int sub) {
  if constexpr (JLayout<LP, LA, LB, TS, PCH>::REG)
    jr_pair<LP, LA, LB>(a, valid, sa, sb, sub);
  else
    jeng_pair<LP, LA, LB, TS, PCH>(a, S, tid, valid, sa, sb, np_loop);
}

template <int LP, int LA, int LB, int TS, int PCH>
__global__ void __launch_bounds__(TS > 64 ? TS : 64)
    __attribute__((amdgpu_waves_per_eu(Cfg<LP, LA, LB>::WPEJ))) k_J(JArgs a) {
  using JL = JLayout<LP, LA, LB, TS, PCH>;
  constexpr int BLK = TS > 64 ? TS : 64;
  constexpr int TPB = BLK / TS;
  constexpr bool REG = JL::REG;
  extern __shared__ double smem[];
  // register engine: lane = sub (64 / nsub) + team, nsub lanes per pair
  const int tpb = REG ? TPB / a.nsub : TPB;
  const int team = REG ? int(threadIdx.x) % tpb : int(threadIdx.x) / TS;
  const int sub = REG ? int(threadIdx.x) / tpb : 0;
  const int tid = threadIdx.x % TS;
  double *S = smem + (REG ? 0 : team * JL::TOTAL);
  if (a.err && *a.err) return;

  // all pairs of the class, or the compacted list of kept pairs
  const int64_t nitem = a.plist ? *a.pcount : a.npair;
  for (int64_t base = int64_t(blockIdx.x) * tpb; base < nitem; base += int64_t(gridDim.x) * tpb) {
    const bool valid = base + team < nitem;
    const int64_t q = valid && a.plist ? a.plist[base + team] : base + team;
    int sa = 0, sb = 0;
    if (valid) {
      if (a.same) {  // q -> (i >= j)
        int i = int((sqrt(8.0 * double(q) + 1.0) - 1.0) * 0.5);
        while (int64_t(i) * (i + 1) / 2 > q) --i;
        while (int64_t(i + 1) * (i + 2) / 2 <= q) ++i;
        const int j = int(q - int64_t(i) * (i + 1) / 2);
        sa = a.ash[i];
        sb = a.ash[j];
      } else {
        const int i = int(q / a.nb), j = int(q - int64_t(i) * a.nb);
        sa = a.ash[i];
        sb = a.bsh[j];
      }
    }
    j_pair<LP, LA, LB, TS, PCH>(a, S, tid, valid, sa, sb, a.np, sub);
  }
}

}  // namespace df3c

// Class kernels of the (ab|P) pipeline for gfx950.
//
// Per contracted triplet (Section 2.5.1):
//   setup + Boys -> [00|0]^(m)      per primitive triplet (Section 2.5.2)
//   VRR1 2-quantal -> [e0|0]^(LP)   per primitive triplet (Section 2.5.3)
//   pi_k(e', n)    += sW x [e'0|0]  early contraction of the CVRR2 prerequisites
//   (e0|c)          = n-q CVRR2      once per triplet (Section 2.5.4)
//   (e0|P)          = solid-harmonic transform of the ket
//   (ab|P)          = n-q HRR        once per triplet (Section 2.5.5)
//   digestion: store the block, or accumulate J_ab += sum_P (ab|P) d_P.
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
  int32_t pure;             // ket solid-harmonic (1) or Cartesian (0, LP <= 1)
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
  int32_t pure;
};


// LDS footprint (doubles) of one team
template <int LP, int LA, int LB, int PCH>
struct Foot {
  using G = Geo<LP, LA, LA + LB>;
  static constexpr int REC = PS_N + G::NV1 + G::NSW;      // per primitive record
  static constexpr int PRIM = PCH * REC;
  static constexpr int EC = G::NE * G::NCP;
  static constexpr int EM = G::NPURE * G::NE;
  static constexpr int NHC = GenHrr<LA, LB>::NHC;
  static constexpr int R0 = imax(PRIM, EC);               // prim records, then (e0|c)
  static constexpr int R1 = imax(G::NPI, EM);             // pi, then (e0|P)
  static constexpr int TOTAL = R0 + R1 + NHC;
};

// ---------------------------------------------------------------------------
// The per-triplet pipeline up to (e0|P) in LDS.  The team's LDS slice S holds
// [R0: primitive records / (e0|c)] [R1: pi / (e0|P)] [HC].
// A, B, C: centres; shell data of a (l = LA), b (l = LB), P (l = LP).
// ---------------------------------------------------------------------------
template <int LP, int LA, int LB, int TS, int PCH>
__device__ __forceinline__ void triplet_to_e0P(const double *btab, double *S, int tid, int npmax,
                                               const double *A,
                                               const double *B, const double *C, int Ka,
                                               const double *ea, const double *ca, int Kb,
                                               const double *eb, const double *cb, int Kc,
                                               const double *ec, const double *cc, int pure) {
  using G = Geo<LP, LA, LA + LB>;
  using F = Foot<LP, LA, LB, PCH>;
  constexpr int L = G::L;
  constexpr int REC = F::REC;
  double *prims = S;
  double *PI = S + F::R0;
  double *EC = S;
  double *EM = S + F::R0;
  using TB = GenTab<LP, G::EA, G::EB>;
  static_assert(TB::NPI == G::NPI && TB::NTGT == G::NE * G::NCP, "generated tables out of date");

  const double ABx = A[0] - B[0], ABy = A[1] - B[1], ABz = A[2] - B[2];
  const double AB2 = ABx * ABx + ABy * ABy + ABz * ABz;
  const int K = Ka * Kb * Kc;

  for (int r = tid; r < G::NPI; r += TS) PI[r] = 0.0;

  for (int p0 = 0; p0 < npmax; p0 += PCH) {
    const int npc = imax(0, imin(PCH, K - p0));
    // ---- setup, Boys, level 0 of VRR1 and the CVRR2 monomials sW
    for (int pp = tid; pp < npc; pp += TS) {
      const int p = p0 + pp;
      const int ic = p % Kc, rest = p / Kc;
      const int ib = rest % Kb, ia = rest / Kb;
      const double za = ea[ia], zb = eb[ib], zc = ec[ic];
      const double g = za + zb, ig = 1.0 / g;
      const double Px = (za * A[0] + zb * B[0]) * ig, Py = (za * A[1] + zb * B[1]) * ig,
                   Pz = (za * A[2] + zb * B[2]) * ig;
      const double PCx = Px - C[0], PCy = Py - C[1], PCz = Pz - C[2];
      const double gz = g + zc;
      const double rho = g * zc / gz;
      const double T = rho * (PCx * PCx + PCy * PCy + PCz * PCz);
      // 2 pi^{5/2} / ((g+zc)^{1/2} g zc) exp(-za zb/g AB^2) x contraction coefficients
      const double pre = 34.98683665524972497 / (sqrt(gz) * g * zc) * exp(-za * zb * ig * AB2) *
                         (ca[ia] * cb[ib] * cc[ic]);
      double Fm[L + 1];
      boys<LP, L + 1>(btab, T, Fm);
      double *R = prims + pp * REC;
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
    team_sync();
    // ---- VRR1, 2-quantal stages in place
    vrr1<G, TS, PCH, REC>(prims, npc, tid);
    // ---- early contraction of the CVRR2 prerequisites
    for (int r = tid; r < G::NPI; r += TS) {
      const int isw = TB::pi_sw[r], iv = TB::pi_v[r];
      double acc = PI[r];
      for (int pp = 0; pp < npc; ++pp) {
        const double *R = prims + pp * REC + PS_N;
        acc += R[G::NV1 + isw] * R[iv];
      }
      PI[r] = acc;
    }
    team_sync();
  }
  // ---- n-quantal CVRR2: (e0|c) = sum_u w pi_{|u|}(e-u, c-u)
  for (int t = tid; t < TB::NTGT; t += TS) {
    double acc = 0.0;
    for (int q = TB::cb_start[t]; q < TB::cb_start[t + 1]; ++q)
      acc += double(TB::cb_w[q]) * PI[TB::cb_pi[q]];
    EC[t] = acc;
  }
  team_sync();
  // ---- ket to solid harmonics (or keep Cartesian for LP <= 1)
  if (pure) {
    using sh = GenSolid<LP>;
    for (int t = tid; t < G::NPURE * G::NE; t += TS) {
      const int m = t / G::NE, e = t - m * G::NE;
      double acc = 0.0;
      for (int q = sh::start[m]; q < sh::start[m + 1]; ++q) acc += sh::val[q] * EC[e * G::NCP + sh::col[q]];
      EM[t] = acc;
    }
  } else {
    for (int t = tid; t < G::NCP * G::NE; t += TS) {
      const int m = t / G::NE, e = t - m * G::NE;
      EM[t] = EC[e * G::NCP + m];
    }
  }
  team_sync();
}

// HRR coefficients prod_x C(b_x, i_x) AB_x^{b_x - i_x} for all (b, i)
template <int LA, int LB>
__device__ __forceinline__ void hrr_coefs(double *HC, int tid, int TS, const double *A,
                                          const double *B) {
  using h = GenHrr<LA, LB>;
  const double AB[3] = {A[0] - B[0], A[1] - B[1], A[2] - B[2]};
  for (int n = tid; n < h::NHC; n += TS) {
    double v = double(h::hc_binom[n]);
    for (int x = 0; x < 3; ++x)
      for (int k = 0; k < h::hc_pow[4 * n + x]; ++k) v *= AB[x];
    HC[n] = v;
  }
}

// ---------------------------------------------------------------------------
// store digestion: one triplet per team, blocks written to out + out_off[t]
// ---------------------------------------------------------------------------
template <int LP, int LA, int LB, int TS, int PCH>
__global__ void __launch_bounds__(64) k_store(StoreArgs a) {
  using G = Geo<LP, LA, LA + LB>;
  using F = Foot<LP, LA, LB, PCH>;
  constexpr int TPW = 64 / TS;
  constexpr int NA = ncart(LA), NB = ncart(LB);
  extern __shared__ double smem[];
  const int team = threadIdx.x / TS, tid = threadIdx.x % TS;
  double *S = smem + team * F::TOTAL;
  double *HC = S + F::R0 + F::R1;
  double *EM = S + F::R0;
  using h = GenHrr<LA, LB>;
  const int np_out = a.pure ? npure(LP) : ncart(LP);

  for (int64_t base = int64_t(blockIdx.x) * TPW; base < a.count; base += int64_t(gridDim.x) * TPW) {
    const int64_t item = base + team;
    const bool valid = item < a.count;
    uint32_t code = valid ? a.bucket[item] : 0u;
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
    const int npmax = wave_max(Ka * Kb * Kc);
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
    triplet_to_e0P<LP, LA, LB, TS, PCH>(a.boys, S, tid, npmax, Ar, Br, Cr, Ka, a.orb.exps + oa,
                                        a.orb.coefs + oa, Kb, a.orb.exps + ob, a.orb.coefs + ob,
                                        Kc, a.aux.exps + oc, a.aux.coefs + oc, a.pure);
    hrr_coefs<LA, LB>(HC, tid, TS, Ar, Br);
    team_sync();
    if (valid) {
      double *out = a.out + a.out_off[t];
      const int nout = np_out * NA * NB;
      for (int o = tid; o < nout; o += TS) {
        const int m = o / (NA * NB), ab = o - m * (NA * NB);
        const int ia = ab / NB, ib = ab - ia * NB;
        double acc = 0.0;
        const int16_t *ep = &h::e[ia * h::NHC];
        for (int n = h::hc_start[ib]; n < h::hc_start[ib + 1]; ++n) acc += HC[n] * EM[m * G::NE + ep[n]];
        const int dst = swp ? (m * NB + ib) * NA + ia : o;
        out[dst] = acc;
      }
    }
    team_sync();
  }
}

// ---------------------------------------------------------------------------
// J digestion: one orbital shell pair per team; the team loops over all aux
// shells of l = LP and accumulates J_ab += sum_P (ab|P) d_P for its pair, then
// adds the block (and its transpose) into J.  Each pair is owned by exactly one
// team, so no atomics are needed; launches of different LP run in stream order.
// ---------------------------------------------------------------------------
template <int LP, int LA, int LB, int TS, int PCH>
__global__ void __launch_bounds__(64) k_J(JArgs a) {
  using G = Geo<LP, LA, LA + LB>;
  using F = Foot<LP, LA, LB, PCH>;
  constexpr int TPW = 64 / TS;
  constexpr int NA = ncart(LA), NB = ncart(LB);
  constexpr int NAB = NA * NB;
  constexpr int NACC = (NAB + TS - 1) / TS;
  extern __shared__ double smem[];
  const int team = threadIdx.x / TS, tid = threadIdx.x % TS;
  double *S = smem + team * F::TOTAL;
  double *HC = S + F::R0 + F::R1;
  double *EM = S + F::R0;
  using h = GenHrr<LA, LB>;
  const int np_out = a.pure ? npure(LP) : ncart(LP);

  for (int64_t base = int64_t(blockIdx.x) * TPW; base < a.npair; base += int64_t(gridDim.x) * TPW) {
    const int64_t q = base + team;
    const bool valid = q < a.npair;
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
    if (valid && LA == LB && sa != sb) {
      // orient the pair for a well-conditioned HRR (see the runtime's k_scatter):
      // VRR1 quanta on the shell with the larger (max exponent x min exponent);
      // both J blocks are written below, so the orientation is free.
      auto tight = [&](int sh) {
        const double *e = a.orb.exps + a.orb.prim_off[sh];
        double lo = e[0], hi = e[0];
        for (int i = 1; i < a.orb.nprim[sh]; ++i) {
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
    double acc[NACC];
#pragma unroll
    for (int k = 0; k < NACC; ++k) acc[k] = 0.0;
    hrr_coefs<LA, LB>(HC, tid, TS, Ar, Br);
    for (int ip = 0; ip < a.np; ++ip) {
      const int sP = a.psh[ip];
      const int Kc = a.aux.nprim[sP];
      const int npmax = wave_max(Ka * Kb * Kc);
      const int64_t oc = a.aux.prim_off[sP];
      const int ic = a.aux.atom[sP];
      const double Cr[3] = {a.xyz[3 * ic], a.xyz[3 * ic + 1], a.xyz[3 * ic + 2]};
      triplet_to_e0P<LP, LA, LB, TS, PCH>(a.boys, S, tid, npmax, Ar, Br, Cr, Ka, a.orb.exps + oa,
                                          a.orb.coefs + oa, Kb, a.orb.exps + ob,
                                          a.orb.coefs + ob, Kc, a.aux.exps + oc,
                                          a.aux.coefs + oc, a.pure);
      const double *dP = a.d + a.aux_off[sP];
#pragma unroll
      for (int k = 0; k < NACC; ++k) {
        const int ab = tid + k * TS;
        if (ab < NAB) {
          const int ia = ab / NB, ib = ab - ia * NB;
          const int16_t *ep = &h::e[ia * h::NHC];
          double s = acc[k];
          for (int m = 0; m < np_out; ++m) {
            double v = 0.0;
            for (int n = h::hc_start[ib]; n < h::hc_start[ib + 1]; ++n) v += HC[n] * EM[m * G::NE + ep[n]];
            s += v * dP[m];
          }
          acc[k] = s;
        }
      }
      team_sync();
    }
    if (valid) {
      const int64_t ra = a.ao_off[sa], rb = a.ao_off[sb];
#pragma unroll
      for (int k = 0; k < NACC; ++k) {
        const int ab = tid + k * TS;
        if (ab < NAB) {
          const int ia = ab / NB, ib = ab - ia * NB;
          a.J[(ra + ia) * a.nao + rb + ib] += acc[k];
          if (sa != sb) a.J[(rb + ib) * a.nao + ra + ia] += acc[k];
        }
      }
    }
  }
}

}  // namespace df3c

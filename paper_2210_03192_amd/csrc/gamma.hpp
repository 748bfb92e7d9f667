// Adjoint digestion: gamma_P = sum_{a,b} (P|ab) D_ab, the right-hand side of
// the fitting equations and dL/dd of L = sum_ab G_ab J_ab (with D = G).
//
// Per shell pair (a >= b) with D~ = D_ab (+ D_ba^T for a != b), the HRR of
// Eq. hrr is transposed onto the targets: sum_ab D~_ab (ab|c) = sum_e w_e (e0|c)
// with w_{a+i} += D~_ab C(b,i) AB^{b-i}.  Written out with the n-quantal CVRR2
// (Eq. cVRR2 on the prerequisites of Eq. a0cv2), per primitive triplet
//   G_u = sum_{e >= u} w_e e!/(e-u)! [e-u 0|0]^(LP),
//   y_c += sum_{u <= c} C(c,u) sW_{|u|}[c-u] G_u,      gamma_m = sum_c T_mc y_c.
//
// Work items (range of shell pairs, subset of the aux shells) write partial
// gammas that one reduction per class adds in a fixed order (no atomics,
// bitwise reproducible); the register engine serves the classes whose
// intermediates fit a lane, the gamma engine the others.
#pragma once
#include "kernels.hpp"

namespace df3c {

struct GamArgs {
  const double *boys;
  const double *xyz;
  ShellsDev aux, orb;
  const int32_t *ash, *bsh;   // orbital shells of l = LA / LB (sorted)
  int32_t na, nb, same;
  const int32_t *psh;         // aux shells of l = LP
  const double *arec;         // their aux-shell records (AREC), aligned with psh
  int32_t np;
  const int64_t *ao_off;      // AO offset of each orbital shell
  const double *D;            // [nao][nao]
  int64_t nao, npair;
  int32_t pure;
  // items (pair range r, aux subset s); subset s holds the aux shells s,
  // s + nsplit, ... (at most nps of them), range r the pairs
  // [r prange, (r + 1) prange)
  int32_t nsplit, nps;
  int64_t prange;
  int64_t nrange;
  double *partial;            // [nrange][nsplit][nps][np_out]
  const int *err;             // device status word: nothing is done when it is non-zero
};

// Register engine with the primitive pairs outermost (l_P <= 2): the per-lane
// accumulators y of up to NPS aux shells live in LDS, YBYTES per wavefront.
template <int LP>
struct GamSwap {
  static constexpr bool ON = LP <= 2;
  static constexpr int YBYTES = 12 * 1024;
  static constexpr int NPS = ON ? YBYTES / (ncart(LP) * 64 * 8) : 0;
};
inline int gam_nps_cap(int lp) {
  switch (lp) {
    case 0: return GamSwap<0>::NPS;
    case 1: return GamSwap<1>::NPS;
    case 2: return GamSwap<2>::NPS;
    default: return 0;
  }
}

// pair q of the class -> (sa, sb)
__device__ __forceinline__ void gam_pair(const GamArgs &g, int64_t q, int &sa, int &sb) {
  if (g.same) {
    int i = int((sqrt(8.0 * double(q) + 1.0) - 1.0) * 0.5);
    while (int64_t(i) * (i + 1) / 2 > q) --i;
    while (int64_t(i + 1) * (i + 2) / 2 <= q) ++i;
    const int j = int(q - int64_t(i) * (i + 1) / 2);
    sa = g.ash[i];
    sb = g.ash[j];
  } else {
    const int i = int(q / g.nb), j = int(q - int64_t(i) * g.nb);
    sa = g.ash[i];
    sb = g.bsh[j];
  }
}

// ---------------------------------------------------------------------------
// Register engine (classes of the register J engine): one lane per shell pair.
// A workgroup is one wavefront and one item (pair range, aux subset).  Per
// round of 64 pairs each lane transposes the HRR onto its D~ once (w_e) and
// forms y of every aux shell of the subset over the pair's primitive triplets.
// l_P <= 2: primitive pairs outermost, y of each shell kept per lane in LDS
// over all rounds of the item, then one ket transform and one fixed butterfly
// over the wavefront per shell.  l_P >= 3: aux shells outermost, and each
// round's y is transformed and summed over the wavefront at once.  Lane 0
// accumulates the sums per aux shell in LDS, and the item writes them as its
// partial; a reduction adds the ranges in order.
// ---------------------------------------------------------------------------
template <int LP, int LA, int LB>
__global__ void __launch_bounds__(64) k_gam_r(GamArgs g) {
  using R = JReg<LP, LA, LB>;
  using SH = GenSolid<LP>;
  constexpr int L = R::L, NE = R::NE, NCP = ncart(LP), NA = ncart(LA), NB = ncart(LB);
  extern __shared__ double acc[];  // [nps][np_out]
  const int lane = threadIdx.x;
  const int nout = g.pure ? npure(LP) : NCP;
  if (g.err && *g.err) return;
  for (int64_t item = blockIdx.x; item < g.nrange * g.nsplit; item += gridDim.x) {
    const int64_t r = item / g.nsplit;
    const int sub = int(item - r * g.nsplit);
    for (int x = lane; x < g.nps * nout; x += 64) acc[x] = 0.0;
    // ket transform of the shell ks, sum over the wavefront's pairs, accumulate
    auto reduce_shell = [&](int ks, const double *y) {
      double o[NCP];
      if (g.pure) {
        static_for<npure(LP)>([&](auto mc) {
          constexpr int m = decltype(mc)::value;
          double v = 0.0;
          static_for<NCP>([&](auto cc_) {
            constexpr int c = decltype(cc_)::value;
            constexpr double t = SH::dense[m * NCP + c];
            if constexpr (t != 0.0) v += t * y[c];
          });
          o[m] = v;
        });
      } else {
#pragma unroll
        for (int c = 0; c < NCP; ++c) o[c] = y[c];
      }
#pragma unroll
      for (int m = 0; m < NCP; ++m) {
        if (m < nout) {
          double v = o[m];
#pragma unroll
          for (int sh = 32; sh > 0; sh >>= 1) v += __shfl_xor(v, sh, 64);
          if (lane == 0) acc[ks * nout + m] += v;
        }
      }
    };
    // primitive pairs outermost (l_P <= 2): per-lane y of the nks aux shells of
    // the subset in LDS, summed over all the item's pairs before one transform
    // and one wavefront sum per shell
    double *yb = acc + g.nps * nout;  // [nps][NCP][64]
    const int nks = sub < g.np ? (g.np - sub + g.nsplit - 1) / g.nsplit : 0;
    if constexpr (GamSwap<LP>::ON)
      for (int x = 0; x < nks * NCP; ++x) yb[x * 64 + lane] = 0.0;
    const int64_t qend = (r + 1) * g.prange < g.npair ? (r + 1) * g.prange : g.npair;
    for (int64_t q0 = r * g.prange; q0 < qend; q0 += 64) {
      const int64_t q = q0 + lane;
      const bool valid = q < qend;
      int sa = 0, sb = 0;
      if (valid) {
        gam_pair(g, q, sa, sb);
        orient_pair<LA, LB>(g.orb, sa, sb);
      }
      const int Ka = valid ? g.orb.nprim[sa] : 0, Kb = valid ? g.orb.nprim[sb] : 0;
      const double *ea = g.orb.exps + g.orb.prim_off[sa], *ca = g.orb.coefs + g.orb.prim_off[sa];
      const double *eb = g.orb.exps + g.orb.prim_off[sb], *cb = g.orb.coefs + g.orb.prim_off[sb];
      double A[3], B[3];
      {
        const int ia = g.orb.atom[sa], ib = g.orb.atom[sb];
#pragma unroll
        for (int x = 0; x < 3; ++x) {
          A[x] = g.xyz[3 * ia + x];
          B[x] = g.xyz[3 * ib + x];
        }
      }
      const double AB[3] = {A[0] - B[0], A[1] - B[1], A[2] - B[2]};
      const double AB2 = AB[0] * AB[0] + AB[1] * AB[1] + AB[2] * AB[2];
      // w_e: the HRR transposed onto D~
      double w[NE];
      {
        const int64_t ra = g.ao_off[sa], rb = g.ao_off[sb];
        double px[LB + 1], py[LB + 1], pz[LB + 1];
        px[0] = py[0] = pz[0] = 1.0;
#pragma unroll
        for (int k = 1; k <= LB; ++k) {
          px[k] = px[k - 1] * AB[0];
          py[k] = py[k - 1] * AB[1];
          pz[k] = pz[k - 1] * AB[2];
        }
#pragma unroll
        for (int e = 0; e < NE; ++e) w[e] = 0.0;
        static_for<NA>([&](auto ac) {
          constexpr int ai = decltype(ac)::value;
          constexpr C3 av = cart(LA, ai);
          static_for<NB>([&](auto bc) {
            constexpr int bi = decltype(bc)::value;
            constexpr C3 bv = cart(LB, bi);
            double dt = valid ? g.D[(ra + ai) * g.nao + rb + bi] : 0.0;
            if (valid && sa != sb) dt += g.D[(rb + bi) * g.nao + ra + ai];
            static_for<bv[0] + 1>([&](auto xc) {
              constexpr int ix = decltype(xc)::value;
              static_for<bv[1] + 1>([&](auto yc) {
                constexpr int iy = decltype(yc)::value;
                static_for<bv[2] + 1>([&](auto zc_) {
                  constexpr int iz = decltype(zc_)::value;
                  constexpr int le = LA + ix + iy + iz;
                  constexpr int idx = offT(le) - offT(LA) + cidx(av[0] + ix, av[1] + iy, av[2] + iz);
                  constexpr double bn = double(binom(bv[0], ix) * binom(bv[1], iy) * binom(bv[2], iz));
                  w[idx] += (bn * dt) * (px[bv[0] - ix] * py[bv[1] - iy] * pz[bv[2] - iz]);
                });
              });
            });
          });
        });
      }
      // one primitive triplet into y: primitive pair (gg, ig, P, PA, eab), aux
      // primitive (zc, cz) at C
      auto triplet = [&](const double zc, const double cz, const double *C, const double gg,
                         const double ig, const double *P, const double *PA,
                         const double eab, double *y) {
        const double PC[3] = {P[0] - C[0], P[1] - C[1], P[2] - C[2]};
        const double gz = gg + zc, rho = gg * zc / gz, rg = rho * ig, i2g = 0.5 * ig;
        const double T = rho * (PC[0] * PC[0] + PC[1] * PC[1] + PC[2] * PC[2]);
        const double pre = 34.98683665524972497 / (sqrt(gz) * gg * zc) * eab * cz;
        const double RP[3] = {rg * PC[0], rg * PC[1], rg * PC[2]};
        double Fm[L + 1];
        boys<LP, L + 1>(g.boys, T, Fm);
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
        // G_u = sum_{e >= u} w_e e!/(e-u)! V_{e-u}
        double Gu[R::NU];
#pragma unroll
        for (int u = 0; u < R::NU; ++u) Gu[u] = 0.0;
        static_for<L - LA + 1>([&](auto lc) {
          constexpr int le = LA + decltype(lc)::value;
          static_for<ncart(le)>([&](auto ec_) {
            constexpr int ce = decltype(ec_)::value;
            constexpr C3 e = cart(le, ce);
            const double we = w[offT(le) - offT(LA) + ce];
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
                    Gu[offT(k) + cidx(ux, uy, uz)] +=
                        (f * we) * vr[R::voff(lr) + cr * (L - lr + 1)];
                  }
                });
              });
            });
          });
        });
        // y_c += sum_{u <= c} C(c,u) s^{|u|} W^{c-u} G_u
        const double s = rho * ig * (0.5 / zc), rz = rho / zc;
        double wx[LP + 1], wy[LP + 1], wz[LP + 1], sk[R::KU + 1];
        wx[0] = wy[0] = wz[0] = sk[0] = 1.0;
#pragma unroll
        for (int k = 1; k <= LP; ++k) {
          wx[k] = wx[k - 1] * (rz * PC[0]);
          wy[k] = wy[k - 1] * (rz * PC[1]);
          wz[k] = wz[k - 1] * (rz * PC[2]);
        }
#pragma unroll
        for (int k = 1; k <= R::KU; ++k) sk[k] = sk[k - 1] * s;
        static_for<R::KU + 1>([&](auto kc) {
          constexpr int k = decltype(kc)::value;
          static_for<ncart(k)>([&](auto uc) {
            constexpr int ui = decltype(uc)::value;
            constexpr C3 u = cart(k, ui);
            const double gk = sk[k] * Gu[offT(k) + ui];
            static_for<NCP>([&](auto cc_) {
              constexpr int c = decltype(cc_)::value;
              constexpr C3 qq = cart(LP, c);
              if constexpr (qq[0] >= u[0] && qq[1] >= u[1] && qq[2] >= u[2]) {
                constexpr double bn =
                    double(binom(qq[0], u[0]) * binom(qq[1], u[1]) * binom(qq[2], u[2]));
                y[c] += (bn * gk) * (wx[qq[0] - u[0]] * wy[qq[1] - u[1]] * wz[qq[2] - u[2]]);
              }
            });
          });
        });
      };
      if constexpr (GamSwap<LP>::ON) {
        // as in the J engine: 1/gamma, P and the pair exponential once per
        // primitive pair for all the subset's aux shells
        for (int ia = 0; ia < Ka; ++ia)
          for (int ib = 0; ib < Kb; ++ib) {
            const double za = ea[ia], zb = eb[ib];
            const double gg = za + zb, ig = 1.0 / gg;
            const double P[3] = {(za * A[0] + zb * B[0]) * ig, (za * A[1] + zb * B[1]) * ig,
                                 (za * A[2] + zb * B[2]) * ig};
            const double PA[3] = {P[0] - A[0], P[1] - A[1], P[2] - A[2]};
            const double eab = exp(-za * zb * ig * AB2) * ca[ia] * cb[ib];
            for (int ks = 0, ip = sub; ip < g.np; ++ks, ip += g.nsplit) {  // uniform
              const double *rc = g.arec + int64_t(ip) * AREC;
              const double C[3] = {rc[AR_CX], rc[AR_CY], rc[AR_CZ]};
              const int Kc = int(rc[AR_K]);
              const int64_t po = int64_t(rc[AR_PRIM]);
              double y[NCP];
#pragma unroll
              for (int c = 0; c < NCP; ++c) y[c] = yb[(ks * NCP + c) * 64 + lane];
              double zc = rc[AR_Z0], cz = rc[AR_C0];
              for (int ic = 0; ic < Kc; ++ic) {
                if (ic > 0) {
                  zc = g.aux.exps[po + ic];
                  cz = g.aux.coefs[po + ic];
                }
                triplet(zc, cz, C, gg, ig, P, PA, eab, y);
              }
#pragma unroll
              for (int c = 0; c < NCP; ++c) yb[(ks * NCP + c) * 64 + lane] = y[c];
            }
          }
      } else {
        for (int ks = 0, ip = sub; ip < g.np; ++ks, ip += g.nsplit) {  // uniform over the wave
          const int sP = g.psh[ip];
          const int Kc = g.aux.nprim[sP];
          const double *ec = g.aux.exps + g.aux.prim_off[sP], *cc = g.aux.coefs + g.aux.prim_off[sP];
          const int icn = g.aux.atom[sP];
          const double C[3] = {g.xyz[3 * icn], g.xyz[3 * icn + 1], g.xyz[3 * icn + 2]};
          double y[NCP];
#pragma unroll
          for (int c = 0; c < NCP; ++c) y[c] = 0.0;
          for (int ia = 0; ia < Ka; ++ia)
            for (int ib = 0; ib < Kb; ++ib) {
              const double za = ea[ia], zb = eb[ib];
              const double gg = za + zb, ig = 1.0 / gg;
              const double P[3] = {(za * A[0] + zb * B[0]) * ig, (za * A[1] + zb * B[1]) * ig,
                                   (za * A[2] + zb * B[2]) * ig};
              const double PA[3] = {P[0] - A[0], P[1] - A[1], P[2] - A[2]};
              const double eab = exp(-za * zb * ig * AB2) * ca[ia] * cb[ib];
              for (int ic = 0; ic < Kc; ++ic) triplet(ec[ic], cc[ic], C, gg, ig, P, PA, eab, y);
            }
          reduce_shell(ks, y);
        }
      }
    }
    if constexpr (GamSwap<LP>::ON)
      for (int ks = 0; ks < nks; ++ks) {
        double y[NCP];
#pragma unroll
        for (int c = 0; c < NCP; ++c) y[c] = yb[(ks * NCP + c) * 64 + lane];
        reduce_shell(ks, y);
      }
    double *out = g.partial + item * g.nps * nout;
    for (int x = lane; x < g.nps * nout; x += 64) out[x] = acc[x];
  }
}

// ---------------------------------------------------------------------------
// Gamma engine (classes beyond the register engine): one workgroup per item
// (range of shell pairs, subset of the aux shells), the pairs of the range in
// turn.  Per pair the HRR is transposed onto D~ once (w_e, lanes over e); the
// pair's primitive triplets over the subset's aux shells are cut into chunks
// that span shells, and per primitive
//   G_u = sum_{e >= u} w_e e!/(e-u)! [e-u 0|0]^(LP),
//   y_c = sum_{u <= c} C(c,u) sW_{|u|}[c-u] G_u,
// which the lanes of the components c add to the accumulator of the
// primitive's aux shell in primitive order.  The ket transform runs once per
// item, on the accumulators.
// ---------------------------------------------------------------------------
template <int LP, int LA, int LB>
struct GamE {
  using G = Geo<LP, LA, LA + LB>;
  static constexpr int NA = ncart(LA), NB = ncart(LB), NCP = ncart(LP), NE = G::NE;
  static constexpr int NU = offT(imin(LP, G::EB) + 1);
  static constexpr int HU = PS_N + G::NV1 + G::NSW;   // record: scalars, VRR1, sW, G
  static constexpr int REC = HU + G::NSW;
  static constexpr int PCH = REC <= 200 ? 16 : 8;
  // lanes per item: four waves where a primitive carries much work (measured
  // on the water clusters), one wave for the (l_P <= 3, l_a l_b <= 3 2) classes
  static constexpr int TS = (LP >= 4 || LB >= 3) ? ENG_TS : 64;
  static constexpr int SL = PCH * REC;                // aux-shell slot of each primitive
  static constexpr int YC = SL + PCH;                 // y [PCH][NCP]
  static constexpr int W = YC + PCH * NCP;            // w_e of the pair
  static constexpr int DT = W + NE;                   // D~ of the pair [NA][NB]
  static constexpr int PW = DT + NA * NB;             // AB powers [3][LB + 1]
  static constexpr int TEAM = PW + 3 * (LB + 1);      // doubles before the accumulators
};

template <int LP, int LA, int LB>
__global__ void __launch_bounds__((GamE<LP, LA, LB>::TS))
    __attribute__((amdgpu_waves_per_eu(DF3C_MIN_WAVES_WAVE))) k_gam_e(GamArgs g) {
  using E = GamE<LP, LA, LB>;
  using G = typename E::G;
  using SH = GenSolid<LP>;
  using TB = GenTab<LP, LA, LA + LB>;
  constexpr int TS = E::TS, PCH = E::PCH, REC = E::REC, NU = E::NU, NE = E::NE;
  constexpr int NA = E::NA, NB = E::NB, NCP = E::NCP;
  extern __shared__ double smem[];
  double *prims = smem, *SLK = smem + E::SL, *Yc = smem + E::YC, *Wv = smem + E::W;
  double *DT = smem + E::DT, *PW = smem + E::PW, *acc = smem + E::TEAM;  // acc [nps][NCP]
  const int tid = threadIdx.x;
  if (g.err && *g.err) return;
  for (int64_t item = blockIdx.x; item < g.nrange * g.nsplit; item += gridDim.x) {
    const int64_t r = item / g.nsplit;
    const int sub = int(item - r * g.nsplit);
    for (int x = tid; x < g.nps * NCP; x += TS) acc[x] = 0.0;
    const int64_t qend = (r + 1) * g.prange < g.npair ? (r + 1) * g.prange : g.npair;
    for (int64_t q = r * g.prange; q < qend; ++q) {
      int sa, sb;
      gam_pair(g, q, sa, sb);
      orient_pair<LA, LB>(g.orb, sa, sb);
      const int Ka = g.orb.nprim[sa], Kb = g.orb.nprim[sb];
      const int64_t oa = g.orb.prim_off[sa], ob = g.orb.prim_off[sb];
      double Ar[3], Br[3];
      {
        const int ia = g.orb.atom[sa], ib = g.orb.atom[sb];
        for (int x = 0; x < 3; ++x) {
          Ar[x] = g.xyz[3 * ia + x];
          Br[x] = g.xyz[3 * ib + x];
        }
      }
      const double AB2 = (Ar[0] - Br[0]) * (Ar[0] - Br[0]) + (Ar[1] - Br[1]) * (Ar[1] - Br[1]) +
                         (Ar[2] - Br[2]) * (Ar[2] - Br[2]);
      {
        const int64_t ra = g.ao_off[sa], rb = g.ao_off[sb];
        for (int ab = tid; ab < NA * NB; ab += TS) {
          const int ia = ab / NB, ib = ab - ia * NB;
          double v = g.D[(ra + ia) * g.nao + rb + ib];
          if (sa != sb) v += g.D[(rb + ib) * g.nao + ra + ia];
          DT[ab] = v;
        }
        if (tid < 3) {
          const double d = Ar[tid] - Br[tid];
          double p = 1.0;
          for (int n = 0; n < LB + 1; ++n) {
            PW[tid * (LB + 1) + n] = p;
            p *= d;
          }
        }
      }
      team_sync();
      // w_e, the HRR transposed onto D~, from the generated terms
      for (int e = tid; e < NE; e += TS) {
        using TW = GenHrrT<LA, LB>;
        double v = 0.0;
        for (int q = TW::w_start[e]; q < TW::w_start[e + 1]; ++q) {
          const uint32_t t = TW::w_t[q];
          v += double(t >> 24) * DT[t & 0xfffu] * PW[(t >> 20) & 0xfu] *
               PW[(LB + 1) + ((t >> 16) & 0xfu)] * PW[2 * (LB + 1) + ((t >> 12) & 0xfu)];
        }
        Wv[e] = v;
      }
      team_sync();
      const int Kab = Ka * Kb;
      // the pair's primitive triplets over the subset's aux shells, in
      // (aux shell, p) order, in chunks of PCH; the cursor is uniform
      auto shell_prims = [&](int ip) { return ip < g.np ? Kab * g.aux.nprim[g.psh[ip]] : 0; };
      int cip = sub, cp = 0, cK = shell_prims(sub);
      while (cip < g.np && cK == 0) cK = shell_prims(cip += g.nsplit);
      while (cip < g.np) {
        int sl_ip[PCH], sl_p[PCH];
        int npc = 0;
#pragma unroll
        for (int pp = 0; pp < PCH; ++pp) {
          sl_ip[pp] = cip;
          sl_p[pp] = cp;
          if (cip < g.np) {
            npc = pp + 1;
            if (++cp == cK) {
              cp = 0;
              cK = shell_prims(cip += g.nsplit);
              while (cip < g.np && cK == 0) cK = shell_prims(cip += g.nsplit);
            }
          }
        }
        int lt = tid;
        __asm__ volatile("" : "+v"(lt));
        if (lt < npc) {
          int ip = sl_ip[0], p = sl_p[0];
#pragma unroll
          for (int qq = 1; qq < PCH; ++qq)
            if (lt == qq) {
              ip = sl_ip[qq];
              p = sl_p[qq];
            }
          const int sP = g.psh[ip];
          const int Kc = g.aux.nprim[sP];
          const int64_t oc = g.aux.prim_off[sP];
          const int atC = g.aux.atom[sP];
          const double Cr[3] = {g.xyz[3 * atC], g.xyz[3 * atC + 1], g.xyz[3 * atC + 2]};
          setup_prim<G, 0>(g.boys, prims + lt * REC, p, Kb, Kc, Ar, Br, Cr, AB2, g.orb.exps + oa,
                           g.orb.coefs + oa, g.orb.exps + ob, g.orb.coefs + ob,
                           g.aux.exps + oc, g.aux.coefs + oc);
          SLK[lt] = double((ip - sub) / g.nsplit);  // the shell's place in the subset
        }
        team_sync();
        vrr1<G, TS, PCH, REC>(prims, npc, lt);
        // G_u per primitive
        for (int it = lt; it < npc * NU; it += TS) {
          const int pp = it / NU, u = it - pp * NU;
          const double *R = prims + pp * REC;
          double v = 0.0;
#pragma unroll 4
          for (int qq = TB::g_start[u]; qq < TB::g_start[u + 1]; ++qq) {
            const uint32_t t = TB::g_t[qq];
            v += double(t >> 16) * Wv[(t >> 8) & 0xffu] * R[PS_N + (t & 0xffu)];
          }
          prims[pp * REC + E::HU + u] = v;
        }
        team_sync();
        // y_c per primitive
        for (int it = lt; it < npc * NCP; it += TS) {
          const int pp = it / NCP, c = it - pp * NCP;
          const double *R = prims + pp * REC;
          double v = 0.0;
#pragma unroll 4
          for (int qq = SH::jy_start[c]; qq < SH::jy_start[c + 1]; ++qq) {
            const uint32_t t = SH::jy_t[qq];
            const int u = int(t & 0xffu);
            if (u < NU) v += double(t >> 16) * R[PS_N + G::NV1 + ((t >> 8) & 0xffu)] * R[E::HU + u];
          }
          Yc[it] = v;
        }
        team_sync();
        // lanes of the components add the chunk to the shells' accumulators in order
        if (lt < NCP)
          for (int pp = 0; pp < npc; ++pp) acc[int(SLK[pp]) * NCP + lt] += Yc[pp * NCP + lt];
        team_sync();
      }
    }
    // ket transform of the accumulators: the item's partial
    const int nout = g.pure ? npure(LP) : NCP;
    double *out = g.partial + item * g.nps * nout;
    for (int x = tid; x < g.nps * nout; x += TS) {
      const int ks = x / nout, m = x - ks * nout;
      double v;
      if (g.pure) {
        v = 0.0;
        for (int c = 0; c < NCP; ++c) v += SH::dense[m * NCP + c] * acc[ks * NCP + c];
      } else {
        v = acc[ks * NCP + m];
      }
      out[x] = v;
    }
    team_sync();
  }
}

}  // namespace df3c

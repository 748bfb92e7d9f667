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
// Work items write partial gammas that one reduction per class adds in a fixed
// order (no atomics, bitwise reproducible): on the register engine an item is
// (range of shell pairs, subset of the aux shells), on the per-triplet
// pipeline (aux shell, chunk of consecutive shell pairs).
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
  int32_t np;
  const int64_t *ao_off;      // AO offset of each orbital shell
  const double *D;            // [nao][nao]
  int64_t nao, npair;
  int32_t pure;
  int32_t nchunk;             // chunks of pairs per aux shell
  int64_t chunk;              // pairs per chunk
  // register engine: items (pair range r, aux subset s); subset s holds the
  // aux shells s, s + nsplit, ... (at most nps of them), range r the pairs
  // [r prange, (r + 1) prange)
  int32_t nsplit, nps;
  int64_t prange;
  int64_t nrange;
  double *partial;            // per-triplet pipeline: [np * nchunk][np_out];
                              // register engine: [nrange][nsplit][nps][np_out]
};

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
// round of 64 pairs each lane transposes the HRR onto its D~ once (w_e); per
// aux shell of the subset it forms y over the pair's primitive triplets, the
// ket transform, and the wavefront sums the 64 pairs by a fixed butterfly.
// Lane 0 accumulates the sums per aux shell in LDS, and the item writes them
// as its partial; a reduction adds the ranges in order.
// ---------------------------------------------------------------------------
template <int LP, int LA, int LB>
__global__ void __launch_bounds__(64) k_gam_r(GamArgs g) {
  using R = JReg<LP, LA, LB>;
  using SH = GenSolid<LP>;
  constexpr int L = R::L, NE = R::NE, NCP = ncart(LP), NA = ncart(LA), NB = ncart(LB);
  extern __shared__ double acc[];  // [nps][np_out]
  const int lane = threadIdx.x;
  const int nout = g.pure ? npure(LP) : NCP;
  for (int64_t item = blockIdx.x; item < g.nrange * g.nsplit; item += gridDim.x) {
    const int64_t r = item / g.nsplit;
    const int sub = int(item - r * g.nsplit);
    for (int x = lane; x < g.nps * nout; x += 64) acc[x] = 0.0;
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
            for (int ic = 0; ic < Kc; ++ic) {
              const double zc = ec[ic];
              const double PC[3] = {P[0] - C[0], P[1] - C[1], P[2] - C[2]};
              const double gz = gg + zc, rho = gg * zc / gz, rg = rho * ig, i2g = 0.5 * ig;
              const double T = rho * (PC[0] * PC[0] + PC[1] * PC[1] + PC[2] * PC[2]);
              const double pre = 34.98683665524972497 / (sqrt(gz) * gg * zc) * eab * cc[ic];
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
            }
          }
        // ket transform, sum over the wavefront's pairs, accumulate for the shell
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
      }
    }
    double *out = g.partial + item * g.nps * nout;
    for (int x = lane; x < g.nps * nout; x += 64) out[x] = acc[x];
  }
}

// ---------------------------------------------------------------------------
// Per-triplet pipeline (all other classes): one team per item; per pair the
// block (P|ab) is formed in LDS (triplet_to_e0P + hrr_block) and contracted
// with D~ by the lanes owning the ket components.
// ---------------------------------------------------------------------------
template <int LP, int LA, int LB, int TS, int PCH>
struct GamLayout {
  static constexpr int DT = Layout<LP, LA, LB, PCH>::TOTAL;   // D~ of the current pair
  static constexpr int TOTAL = (DT + ncart(LA) * ncart(LB)) | 1;
  static constexpr int BYTES_WG = ((TS > 64 ? TS : 64) / TS) * TOTAL * 8;
  static_assert(BYTES_WG <= 160 * 1024, "gamma layout does not fit the LDS of a CU");
};

template <int LP, int LA, int LB, int TS, int PCH>
__global__ void __launch_bounds__(TS > 64 ? TS : 64)
    __attribute__((amdgpu_waves_per_eu(Cfg<LP, LA, LB>::WPE))) k_gam_p(GamArgs g) {
  using G = Geo<LP, LA, LA + LB>;
  using LY = Layout<LP, LA, LB, PCH>;
  using GL = GamLayout<LP, LA, LB, TS, PCH>;
  constexpr int BLK = TS > 64 ? TS : 64;
  constexpr int TPB = BLK / TS;
  constexpr int NA = ncart(LA), NB = ncart(LB);
  constexpr bool MF = (TS % 64 == 0) && PCH % 4 == 0;
  constexpr int NQ = MF ? 1 : (G::NPI + TS - 1) / TS;
  constexpr int NOUT = imax(npure(LP), ncart(LP));
  constexpr int NM = (NOUT + TS - 1) / TS;
  extern __shared__ double smem[];
  const int team = threadIdx.x / TS, tid = threadIdx.x % TS;
  double *S = smem + team * GL::TOTAL;
  double *DT = S + GL::DT;
  const double *STG = S + LY::STG;
  const int np_out = g.pure ? npure(LP) : ncart(LP);
  int slot[NQ];
  if constexpr (!MF) make_slots<LP, LA, LB, TS>(slot, tid);
  const int64_t items = int64_t(g.np) * g.nchunk;

  for (int64_t base = int64_t(blockIdx.x) * TPB; base < items; base += int64_t(gridDim.x) * TPB) {
    const int64_t item = base + team;
    const bool ivalid = item < items;
    const int ip = ivalid ? int(item / g.nchunk) : 0;
    const int64_t ch = ivalid ? item - int64_t(ip) * g.nchunk : 0;
    const int sP = g.psh[ip];
    const int64_t q0 = ch * g.chunk;
    const int64_t q1 = ivalid ? (q0 + g.chunk < g.npair ? q0 + g.chunk : g.npair) : q0;
    const int icn = g.aux.atom[sP];
    const double Cr[3] = {g.xyz[3 * icn], g.xyz[3 * icn + 1], g.xyz[3 * icn + 2]};
    const int64_t oc = g.aux.prim_off[sP];
    double acc[NM];
#pragma unroll
    for (int k = 0; k < NM; ++k) acc[k] = 0.0;
    // the same number of steps for every team of the workgroup (barriers)
    for (int64_t qi = 0; qi < g.chunk; ++qi) {
      const int64_t q = q0 + qi;
      const bool valid = q < q1;
      int sa = 0, sb = 0;
      if (valid) {
        gam_pair(g, q, sa, sb);
        orient_pair<LA, LB>(g.orb, sa, sb);
      }
      const int Ka = valid ? g.orb.nprim[sa] : 0, Kb = valid ? g.orb.nprim[sb] : 0;
      const int Kc = valid ? g.aux.nprim[sP] : 0;
      const int64_t oa = valid ? g.orb.prim_off[sa] : 0, ob = valid ? g.orb.prim_off[sb] : 0;
      double Ar[3] = {0, 0, 0}, Br[3] = {0, 0, 0};
      if (valid) {
        const int ia = g.orb.atom[sa], ib = g.orb.atom[sb];
        for (int x = 0; x < 3; ++x) {
          Ar[x] = g.xyz[3 * ia + x];
          Br[x] = g.xyz[3 * ib + x];
        }
        const int64_t ra = g.ao_off[sa], rb = g.ao_off[sb];
        for (int ab = tid; ab < NA * NB; ab += TS) {
          const int ia2 = ab / NB, ib2 = ab - ia2 * NB;
          double v = g.D[(ra + ia2) * g.nao + rb + ib2];
          if (sa != sb) v += g.D[(rb + ib2) * g.nao + ra + ia2];
          DT[ab] = v;
        }
      }
      const int npmax = TS >= 64 ? Ka * Kb * Kc : wave_max(Ka * Kb * Kc);
      triplet_to_e0P<LP, LA, LB, TS, PCH>(g.boys, S, tid, slot, npmax, Ar, Br, Cr, Ka,
                                          g.orb.exps + oa, g.orb.coefs + oa, Kb, g.orb.exps + ob,
                                          g.orb.coefs + ob, Kc, g.aux.exps + oc,
                                          g.aux.coefs + oc, g.pure);
      hrr_block<LP, LA, LB, TS, PCH>(S, tid, Ar, Br, np_out, false);
      team_sync();
      if (valid) {
#pragma unroll
        for (int k = 0; k < NM; ++k) {
          const int m = tid + k * TS;
          if (m < np_out) {
            double v = acc[k];
            for (int ab = 0; ab < NA * NB; ++ab) v += DT[ab] * STG[m * NA * NB + ab];
            acc[k] = v;
          }
        }
      }
      team_sync();
    }
    if (ivalid) {
#pragma unroll
      for (int k = 0; k < NM; ++k) {
        const int m = tid + k * TS;
        if (m < np_out) g.partial[item * np_out + m] = acc[k];
      }
    }
  }
}

}  // namespace df3c

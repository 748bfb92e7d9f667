// Backward kernel of the DF-J build: nuclear gradient of L = sum_ab G_ab J_ab
// with J_ab = sum_P (ab|P) d_P, for fixed d and G (G = dL/dJ).
//
// Derivative integrals come from raising and lowering the bra:
//   d/dA_x (ab|P) = (a+1_x b|P)^{2 zeta_a} - a_x (a-1_x b|P)
//   d/dB_x (ab|P) = (a b+1_x|P)^{2 zeta_b} - b_x (a b-1_x|P)
//   d/dC_x (ab|P) = -(d/dA_x + d/dB_x)            (translational invariance)
// where (..)^{2 zeta} is contracted with the extra primitive weight 2 zeta.
// Small classes run the register engine (one lane per shell pair, every
// intermediate in registers, per aux shell the shifted HRR blocks contracted
// with G~); the others run the gradient engine, which transposes the shifted
// HRRs onto G~ once per pair and takes dot products per primitive triplet.
// Integrals are recomputed, never stored.
//
// Owner computes: work items are (shell pairs, subset of the aux shells of
// l = LP).  Per-atom contributions are accumulated per workgroup in LDS in a
// fixed order and added to a per-workgroup partial array in global memory; a
// final kernel sums the partials in a fixed order, so the gradient is bitwise
// reproducible.
#pragma once
#include "kernels.hpp"

namespace df3c {

struct GradArgs {
  const double *boys;
  const double *xyz;
  ShellsDev aux, orb;
  const int32_t *ash, *bsh;
  int32_t na, nb, same;
  const int32_t *psh;
  int32_t np;
  const int64_t *ao_off, *aux_off;
  const double *d;          // fitting coefficients
  const double *G;          // [nao][nao] = dL/dJ
  int64_t nao, npair;
  int32_t pure;
  int32_t natom;
  int32_t nsplit;           // aux shells of a pair split into nsplit interleaved subsets
  double *partial;          // [gridDim.x][natom][3], accumulated
  const int64_t *plist;     // optional: indices q of the class's pairs to run
  const int64_t *pcount;    //   (device count of plist), null for all npair
  const int *err;           // device status word: nothing is done when it is non-zero
  int32_t atom_base;        // subtracted from the shells' atom indices (xyz, the
                            // atom arrays and partials start at that atom)
};

// Work items of the gradient kernels: blocks of tpb consecutive shell pairs
// (all pairs of the class, or the kept ones of a pair list) times nsplit
// subsets of the aux shells (subset k: aux shells k, k + nsplit, ...); every
// team of a workgroup takes the same subset, so the aux loop is uniform over
// the workgroup.  Block b -> subset b / nblk, pairs of block b % nblk.
__device__ __forceinline__ int64_t grad_items(const GradArgs &g) {
  return g.plist ? *g.pcount : g.npair;
}

// ---------------------------------------------------------------------------
// Register gradient engine for small classes: one lane per shell pair, every
// intermediate in registers (compile-time indices), one wavefront per
// workgroup.  Per primitive triplet: setup, Boys, 1-quantal VRR1 up to
// l_a + l_b + 1, the d-contracted ket digested as in the register J engine,
//   Y_e = sum_u e!/(e-u)! H_u [e-u 0|0]^(LP),
// accumulated with the weights of the shifted classes: Ya (2 zeta_a, targets of
// (l_a+1, l_b)), Yb (2 zeta_b, targets of (l_a, l_b+1)) and Y0 (1, targets of
// (l_a-1, l_b) and (l_a, l_b-1)).  Per aux shell the HRR of the shifted blocks
// is contracted with G~ in registers:
//   dA_x = sum_ab G~_ab [(a+1_x b|)^{2 zeta_a} - a_x (a-1_x b|)],
//   dB_x = sum_ab G~_ab [(a b+1_x|)^{2 zeta_b} - b_x (a b-1_x|)],
// dC = -(dA + dB) is summed over the wavefront (fixed butterfly order) and added
// to the aux shell's atom; dA, dB of the pairs are added lane by lane at the
// end, so the per-workgroup atom array is filled in a fixed order.
// ---------------------------------------------------------------------------
#ifndef DF3C_GREG_LMAX
#define DF3C_GREG_LMAX 5
#endif
#ifndef DF3C_GREG_COST
#define DF3C_GREG_COST 260
#endif

template <int LP, int LA, int LB>
struct GReg {
  static constexpr int L = LA + LB + 1;               // top VRR1 level
  static constexpr int EL = LA > 0 ? LA - 1 : 0;      // lowest target level
  static constexpr int NA = ncart(LA), NB = ncart(LB);
  static constexpr int KU = imin(LP, L);
  static constexpr int NU = offT(KU + 1);
  // target ranges of the accumulators (levels, inclusive)
  static constexpr int A0 = LA + 1, A1 = L;           // Ya
  static constexpr int B0 = LA, B1 = L;               // Yb
  static constexpr int Z0 = EL, Z1 = LA + LB - 1;     // Y0 (empty when LA = LB = 0)
  static constexpr int ny(int lo, int hi) { return hi >= lo ? offT(hi + 1) - offT(lo) : 0; }
  static constexpr int NYA = ny(A0, A1), NYB = ny(B0, B1), NY0 = ny(Z0, Z1);
  static constexpr int voff(int l) {
    int o = 0;
    for (int q = 0; q < l; ++q) o += ncart(q) * (L - q + 1);
    return o;
  }
  static constexpr int NVR = voff(L + 1);
  static constexpr int COST = NYA + NYB + NY0 + ncart(LP) + NU + NVR / 2 + NA * NB;
  static constexpr bool OK = L <= DF3C_GREG_LMAX && COST <= DF3C_GREG_COST;
};

template <int LP, int LA, int LB>
__global__ void __launch_bounds__(64) k_gradr(GradArgs g) {
  using R = GReg<LP, LA, LB>;
  using SH = GenSolid<LP>;
  constexpr int L = R::L, NCP = ncart(LP), NA = R::NA, NB = R::NB;
  extern __shared__ double smem[];
  double *ACC = smem;  // [natom][3] of this workgroup
  const int lane = threadIdx.x;
  if (g.err && *g.err) return;
  for (int x = lane; x < 3 * g.natom; x += 64) ACC[x] = 0.0;
  __syncthreads();

  const int64_t nitem = grad_items(g);
  const int64_t nblk = (nitem + 63) / 64;
  for (int64_t blk = blockIdx.x; blk < nblk * g.nsplit; blk += gridDim.x) {
    const int sub = int(blk / nblk);
    const int64_t qi = (blk - sub * nblk) * 64 + lane;
    const bool valid = qi < nitem;
    const int64_t q = valid && g.plist ? g.plist[qi] : qi;
    int sa = 0, sb = 0;
    if (valid) {
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
      orient_pair<LA, LB>(g.orb, sa, sb);
    }
    const int Ka = valid ? g.orb.nprim[sa] : 0, Kb = valid ? g.orb.nprim[sb] : 0;
    const double *ea = g.orb.exps + (valid ? g.orb.prim_off[sa] : 0);
    const double *ca = g.orb.coefs + (valid ? g.orb.prim_off[sa] : 0);
    const double *eb = g.orb.exps + (valid ? g.orb.prim_off[sb] : 0);
    const double *cb = g.orb.coefs + (valid ? g.orb.prim_off[sb] : 0);
    const int atA = valid ? g.orb.atom[sa] - g.atom_base : 0,
              atB = valid ? g.orb.atom[sb] - g.atom_base : 0;
    double A[3], B[3];
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      A[x] = g.xyz[3 * atA + x];
      B[x] = g.xyz[3 * atB + x];
    }
    const double AB2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) +
                       (A[2] - B[2]) * (A[2] - B[2]);
    // G~ of the pair (both J blocks of an off-diagonal pair)
    double gt[NA * NB];
    {
      const int64_t ra = valid ? g.ao_off[sa] : 0, rb = valid ? g.ao_off[sb] : 0;
#pragma unroll
      for (int ia = 0; ia < NA; ++ia)
#pragma unroll
        for (int ib = 0; ib < NB; ++ib) {
          double v = 0.0;
          if (valid) {
            v = g.G[(ra + ia) * g.nao + rb + ib];
            if (sa != sb) v += g.G[(rb + ib) * g.nao + ra + ia];
          }
          gt[ia * NB + ib] = v;
        }
    }
    double pwx[LB + 2], pwy[LB + 2], pwz[LB + 2];
    pwx[0] = pwy[0] = pwz[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= LB + 1; ++k) {
      pwx[k] = pwx[k - 1] * (A[0] - B[0]);
      pwy[k] = pwy[k - 1] * (A[1] - B[1]);
      pwz[k] = pwz[k - 1] * (A[2] - B[2]);
    }
    double GA[3] = {0, 0, 0}, GB[3] = {0, 0, 0};

    for (int ip = sub; ip < g.np; ip += g.nsplit) {  // uniform over the wavefront
      const int sP = g.psh[ip];
      const int Kc = g.aux.nprim[sP];
      const double *ec = g.aux.exps + g.aux.prim_off[sP];
      const double *cc = g.aux.coefs + g.aux.prim_off[sP];
      const int atC = g.aux.atom[sP] - g.atom_base;
      const double C[3] = {g.xyz[3 * atC], g.xyz[3 * atC + 1], g.xyz[3 * atC + 2]};
      const double *dP = g.d + g.aux_off[sP];
      double dq[NCP];
      if (g.pure) {
        static_for<NCP>([&](auto cc_) {
          constexpr int c = decltype(cc_)::value;
          double v = 0.0;
          static_for<npure(LP)>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            constexpr double t = SH::dense[m * NCP + c];
            if constexpr (t != 0.0) v += t * dP[m];
          });
          dq[c] = v;
        });
      } else {
#pragma unroll
        for (int c = 0; c < NCP; ++c) dq[c] = dP[c];
      }
      double Ya[R::NYA > 0 ? R::NYA : 1], Yb[R::NYB > 0 ? R::NYB : 1],
          Y0[R::NY0 > 0 ? R::NY0 : 1];
#pragma unroll
      for (int e = 0; e < R::NYA; ++e) Ya[e] = 0.0;
#pragma unroll
      for (int e = 0; e < R::NYB; ++e) Yb[e] = 0.0;
#pragma unroll
      for (int e = 0; e < R::NY0; ++e) Y0[e] = 0.0;
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
            double H[R::NU];
            static_for<R::KU + 1>([&](auto kc) {
              constexpr int k = decltype(kc)::value;
              static_for<ncart(k)>([&](auto uc) {
                constexpr int ui = decltype(uc)::value;
                constexpr C3 u = cart(k, ui);
                double h = 0.0;
                static_for<NCP>([&](auto cc_) {
                  constexpr int c = decltype(cc_)::value;
                  constexpr C3 qq = cart(LP, c);
                  if constexpr (qq[0] >= u[0] && qq[1] >= u[1] && qq[2] >= u[2]) {
                    constexpr double bn =
                        double(binom(qq[0], u[0]) * binom(qq[1], u[1]) * binom(qq[2], u[2]));
                    h += (bn * dq[c]) *
                         (wx[qq[0] - u[0]] * wy[qq[1] - u[1]] * wz[qq[2] - u[2]]);
                  }
                });
                H[offT(k) + ui] = sk[k] * h;
              });
            });
            const double wA = 2.0 * za, wB = 2.0 * zb;
            static_for<L - R::EL + 1>([&](auto lc) {
              constexpr int le = R::EL + decltype(lc)::value;
              static_for<ncart(le)>([&](auto ec_) {
                constexpr int ce = decltype(ec_)::value;
                constexpr C3 e = cart(le, ce);
                double y = 0.0;
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
                        y += (f * H[offT(k) + cidx(ux, uy, uz)]) *
                             vr[R::voff(lr) + cr * (L - lr + 1)];
                      }
                    });
                  });
                });
                if constexpr (le >= R::A0 && le <= R::A1) Ya[offT(le) - offT(R::A0) + ce] += wA * y;
                if constexpr (le >= R::B0 && le <= R::B1) Yb[offT(le) - offT(R::B0) + ce] += wB * y;
                if constexpr (le >= R::Z0 && le <= R::Z1) Y0[offT(le) - offT(R::Z0) + ce] += y;
              });
            });
          }
        }
      // HRR of the shifted blocks contracted with G~:
      //   (a' b'|) = sum_{i <= b'} C(b', i) AB^{b'-i} Y[a' + i]
      double pA[3] = {0, 0, 0}, pB[3] = {0, 0, 0};
      static_for<NA>([&](auto ac) {
        constexpr int ai = decltype(ac)::value;
        constexpr C3 av = cart(LA, ai);
        static_for<NB>([&](auto bc) {
          constexpr int bi = decltype(bc)::value;
          constexpr C3 bv = cart(LB, bi);
          const double gab = gt[ai * NB + bi];
          static_for<3>([&](auto xc) {
            constexpr int x = decltype(xc)::value;
            // hrr(Y, lo, a', b'): block element of Y's class with bra a', b'
            auto hrr = [&](auto &Y, auto loc, auto a3c, auto b3c) {
              constexpr int lo = decltype(loc)::value;
              constexpr int ax = decltype(a3c)::value / 100, ay = (decltype(a3c)::value / 10) % 10,
                            az = decltype(a3c)::value % 10;
              constexpr int bx = decltype(b3c)::value / 100, by = (decltype(b3c)::value / 10) % 10,
                            bz = decltype(b3c)::value % 10;
              double v = 0.0;
              static_for<bx + 1>([&](auto ixc) {
                constexpr int ix = decltype(ixc)::value;
                static_for<by + 1>([&](auto iyc) {
                  constexpr int iy = decltype(iyc)::value;
                  static_for<bz + 1>([&](auto izc) {
                    constexpr int iz = decltype(izc)::value;
                    constexpr int lev = ax + ay + az + ix + iy + iz;
                    constexpr int idx = offT(lev) - offT(lo) + cidx(ax + ix, ay + iy, az + iz);
                    constexpr double bn = double(binom(bx, ix) * binom(by, iy) * binom(bz, iz));
                    v += (bn * pwx[bx - ix] * pwy[by - iy] * pwz[bz - iz]) * Y[idx];
                  });
                });
              });
              return v;
            };
            constexpr int d100 = x == 0 ? 100 : x == 1 ? 10 : 1;
            constexpr int ac3 = av[0] * 100 + av[1] * 10 + av[2];
            constexpr int bc3 = bv[0] * 100 + bv[1] * 10 + bv[2];
            double vA = hrr(Ya, std::integral_constant<int, R::A0>{},
                            std::integral_constant<int, ac3 + d100>{},
                            std::integral_constant<int, bc3>{});
            if constexpr (av[x] > 0)
              vA -= double(av[x]) * hrr(Y0, std::integral_constant<int, R::Z0>{},
                                        std::integral_constant<int, ac3 - d100>{},
                                        std::integral_constant<int, bc3>{});
            double vB = hrr(Yb, std::integral_constant<int, R::B0>{},
                            std::integral_constant<int, ac3>{},
                            std::integral_constant<int, bc3 + d100>{});
            if constexpr (bv[x] > 0)
              vB -= double(bv[x]) * hrr(Y0, std::integral_constant<int, R::Z0>{},
                                        std::integral_constant<int, ac3>{},
                                        std::integral_constant<int, bc3 - d100>{});
            pA[x] += gab * vA;
            pB[x] += gab * vB;
          });
        });
      });
#pragma unroll
      for (int x = 0; x < 3; ++x) {
        GA[x] += pA[x];
        GB[x] += pB[x];
        double v = -(pA[x] + pB[x]);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) ACC[3 * atC + x] += v;
      }
    }
    // dA, dB of the pairs, lane by lane
    for (int j = 0; j < 64; ++j) {
      if (lane == j && valid) {
#pragma unroll
        for (int x = 0; x < 3; ++x) {
          ACC[3 * atA + x] += GA[x];
          ACC[3 * atB + x] += GB[x];
        }
      }
    }
  }
  __syncthreads();
  double *part = g.partial + int64_t(blockIdx.x) * 3 * g.natom;
  for (int x = lane; x < 3 * g.natom; x += 64) part[x] += ACC[x];
}

}  // namespace df3c

namespace df3c {

// ---------------------------------------------------------------------------
// Gradient engine (classes beyond the register engine): one workgroup per
// work item (shell pair, subset of the aux shells).  The HRRs of the four
// shifted classes are transposed onto G~ once per pair, giving twelve weight
// vectors over the targets e (shift s = A+, B+, A-, B-, direction x):
//   omega^{A+,x}_e = sum_ab G~_ab sum_i [a + 1_x + i = e] C(b,i) AB^{b-i}
//   omega^{B+,x}_e = sum_ab G~_ab sum_i [a + i = e] C(b+1_x,i) AB^{b+1_x-i}
//   omega^{A-,x}_e = sum_ab G~_ab a_x sum_i [a - 1_x + i = e] C(b,i) AB^{b-i}
//   omega^{B-,x}_e = sum_ab G~_ab b_x sum_i [a + i = e] C(b-1_x,i) AB^{b-1_x-i}
// (the HRR (ab|X) = sum_i C(b,i) AB^{b-i} X_{a+i} of every shifted block).
// Per primitive triplet, with the digested ket
//   Y_e = sum_u e!/(e-u)! H_u [e-u 0|0]^(LP),   e = max(l_a-1,0) .. l_a+l_b+1,
// the derivative integrals contracted with G~ and d are dot products,
//   dA_x = 2 zeta_a omega^{A+,x}.Y - omega^{A-,x}.Y,
//   dB_x = 2 zeta_b omega^{B+,x}.Y - omega^{B-,x}.Y,   dC_x = -(dA_x + dB_x),
// with dC on the primitive's own aux centre.  No per-aux-shell HRR remains, so
// chunks of primitive triplets span the aux shells of the subset (as in the
// J engine); the three lanes of the directions add the chunk's contributions
// in primitive order, so the atom arrays are filled in a fixed order.
// ---------------------------------------------------------------------------
template <int LP, int LA, int LB>
struct GEng {
  static constexpr int EA = LA > 0 ? LA - 1 : 0, EB = LA + LB + 1;
  using G = Geo<LP, EA, EB>;
  static constexpr int NA = ncart(LA), NB = ncart(LB), NCP = ncart(LP);
  static constexpr int NY = offT(EB + 1) - offT(EA);
  static constexpr int NU = offT(imin(LP, EB) + 1);   // H_u with |u| <= min(LP, EB)
  static constexpr int HU = PS_N + G::NV1 + G::NSW;    // record: scalars, VRR1, sW, H
  static constexpr int REC = HU + G::NSW;
  static constexpr int PCH = REC <= 200 ? 16 : 8;
  // LDS regions of the team (doubles)
  static constexpr int DP = PCH * REC;                 // d' per slot [PCH][NCP]
  static constexpr int ZW = DP + PCH * NCP;            // per slot: 2 zeta_a, 2 zeta_b, aux atom
  static constexpr int Y = ZW + 3 * PCH;               // [PCH][NY]
  static constexpr int T = Y + PCH * NY;               // dot products [PCH][12]
  static constexpr int OM = T + 12 * PCH;              // omega [12][NY]
  static constexpr int GT = OM + 12 * NY;              // G~ of the pair [NA][NB]
  static constexpr int PW = GT + NA * NB;              // AB powers [3][LB + 2]
  static constexpr int TEAM = PW + 3 * (LB + 2);       // doubles before the atom array
  // first and one-past-last flat target index of shift s (relative to level EA)
  static constexpr int lo(int s) {
    return offT(imax(s == 0 ? LA + 1 : s == 2 ? LA - 1 : LA, EA)) - offT(EA);
  }
  static constexpr int hi(int s) {
    const int top = s == 0 ? LA + 1 + LB : s == 1 ? LA + LB + 1 : s == 2 ? LA - 1 + LB : LA + LB - 1;
    return top < EA ? 0 : offT(top + 1) - offT(EA);
  }
};

template <int LP, int LA, int LB>
__global__ void __launch_bounds__(ENG_TS)
    __attribute__((amdgpu_waves_per_eu(DF3C_MIN_WAVES_WAVE))) k_grade(GradArgs g) {
  using E = GEng<LP, LA, LB>;
  using G = typename E::G;
  using SH = GenSolid<LP>;
  using TY = GenY<LP, E::EA, E::EB>;
  constexpr int TS = ENG_TS, PCH = E::PCH, REC = E::REC, NY = E::NY, NU = E::NU;
  constexpr int NA = E::NA, NB = E::NB, NCP = E::NCP;
  extern __shared__ double smem[];
  double *S = smem;
  double *ACC = S + E::TEAM;
  double *prims = S, *DP = S + E::DP, *ZW = S + E::ZW, *Yv = S + E::Y, *Tv = S + E::T;
  double *OM = S + E::OM, *GT = S + E::GT, *PW = S + E::PW;
  if (g.err && *g.err) return;
  const int tid = threadIdx.x;
  for (int x = tid; x < 3 * g.natom; x += TS) ACC[x] = 0.0;
  team_sync();

  const int64_t nblk = grad_items(g);  // one pair per block
  for (int64_t blk = blockIdx.x; blk < nblk * g.nsplit; blk += gridDim.x) {
    const int sub = int(blk / nblk);
    const int64_t q = g.plist ? g.plist[blk - sub * nblk] : blk - sub * nblk;
    int sa, sb;
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
    orient_pair<LA, LB>(g.orb, sa, sb);
    const int Ka = g.orb.nprim[sa], Kb = g.orb.nprim[sb];
    const int64_t oa = g.orb.prim_off[sa], ob = g.orb.prim_off[sb];
    const int atA = g.orb.atom[sa] - g.atom_base, atB = g.orb.atom[sb] - g.atom_base;
    double Ar[3], Br[3];
    for (int x = 0; x < 3; ++x) {
      Ar[x] = g.xyz[3 * atA + x];
      Br[x] = g.xyz[3 * atB + x];
    }
    const double AB2 = (Ar[0] - Br[0]) * (Ar[0] - Br[0]) + (Ar[1] - Br[1]) * (Ar[1] - Br[1]) +
                       (Ar[2] - Br[2]) * (Ar[2] - Br[2]);
    // G~ (both J blocks of an off-diagonal pair) and the powers of A - B
    {
      const int64_t ra = g.ao_off[sa], rb = g.ao_off[sb];
      for (int ab = tid; ab < NA * NB; ab += TS) {
        const int ia = ab / NB, ib = ab - ia * NB;
        double v = g.G[(ra + ia) * g.nao + rb + ib];
        if (sa != sb) v += g.G[(rb + ib) * g.nao + ra + ia];
        GT[ab] = v;
      }
      if (tid < 3) {
        const double d = Ar[tid] - Br[tid];
        double p = 1.0;
        for (int n = 0; n < LB + 2; ++n) {
          PW[tid * (LB + 2) + n] = p;
          p *= d;
        }
      }
    }
    team_sync();
    // omega from the generated terms: coefficient x G~_ab x AB^p per term
    for (int it = tid; it < 12 * NY; it += TS) {
      using TO = GenOmega<LA, LB>;
      double v = 0.0;
      for (int q = TO::o_start[it]; q < TO::o_start[it + 1]; ++q) {
        const uint32_t t = TO::o_t[q];
        v += double(t >> 24) * GT[t & 0xfffu] * PW[(t >> 20) & 0xfu] *
             PW[(LB + 2) + ((t >> 16) & 0xfu)] * PW[2 * (LB + 2) + ((t >> 12) & 0xfu)];
      }
      OM[it] = v;
    }
    team_sync();

    double GA = 0.0, GB = 0.0;  // lanes 0..2: direction x = tid
    const int Kab = Ka * Kb;
    // the pair's primitive triplets over the aux shells of its subset, in
    // (aux shell, p) order, cut into chunks of PCH; the cursor is uniform
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
      // d' of the aux shell of every slot
      for (int it = lt; it < npc * NCP; it += TS) {
        const int pp = it / NCP, c = it - pp * NCP;
        int ip = sl_ip[0];
#pragma unroll
        for (int qq = 1; qq < PCH; ++qq)
          if (pp == qq) ip = sl_ip[qq];
        const double *dP = g.d + g.aux_off[g.psh[ip]];
        double v;
        if (g.pure) {
          v = 0.0;
#pragma unroll
          for (int m = 0; m < G::NPURE; ++m) v += dP[m] * SH::dense[m * NCP + c];
        } else {
          v = dP[c];
        }
        DP[pp * NCP + c] = v;
      }
      // one lane per slot: record set-up, 2 zeta_a, 2 zeta_b and the aux atom
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
        const int atC = g.aux.atom[sP] - g.atom_base;
        const double Cr[3] = {g.xyz[3 * atC], g.xyz[3 * atC + 1], g.xyz[3 * atC + 2]};
        setup_prim<G, 0>(g.boys, prims + lt * REC, p, Kb, Kc, Ar, Br, Cr, AB2, g.orb.exps + oa,
                         g.orb.coefs + oa, g.orb.exps + ob, g.orb.coefs + ob, g.aux.exps + oc,
                         g.aux.coefs + oc);
        const int rest = p / Kc;
        ZW[lt * 3] = 2.0 * g.orb.exps[oa + rest / Kb];
        ZW[lt * 3 + 1] = 2.0 * g.orb.exps[ob + rest % Kb];
        ZW[lt * 3 + 2] = double(atC);
      }
      team_sync();
      vrr1<G, TS, PCH, REC>(prims, npc, lt);
      // H_u of the chunk (the digested ket, as in the J engine)
      for (int it = lt; it < npc * NU; it += TS) {
        const int u = it / npc, pp = it - u * npc;
        const double *SWp = prims + pp * REC + PS_N + G::NV1;
        const double *DPp = DP + pp * NCP;
        double h = 0.0;
#pragma unroll 4
        for (int qq = SH::jh_start[u]; qq < SH::jh_start[u + 1]; ++qq) {
          const uint32_t t = SH::jh_t[qq];
          h += double(t >> 16) * DPp[t & 0xffu] * SWp[(t >> 8) & 0xffu];
        }
        prims[pp * REC + E::HU + u] = h;
      }
      team_sync();
      // Y_e = sum_u e!/(e-u)! H_u V_{e-u} per slot
      for (int it = lt; it < npc * NY; it += TS) {
        const int pp = it / NY, ef = it - pp * NY;
        const double *R = prims + pp * REC;
        double v = 0.0;
#pragma unroll 4
        for (int qq = TY::y_start[ef]; qq < TY::y_start[ef + 1]; ++qq) {
          const uint32_t t = TY::y_t[qq];
          v += double(t >> 16) * R[E::HU + ((t >> 8) & 0xffu)] * R[PS_N + (t & 0xffu)];
        }
        Yv[pp * NY + ef] = v;
      }
      team_sync();
      // the twelve dot products per slot
      for (int it = lt; it < npc * 12; it += TS) {
        const int pp = it / 12, j = it - pp * 12, s = j / 3;
        const int e0 = s == 0 ? E::lo(0) : s == 1 ? E::lo(1) : s == 2 ? E::lo(2) : E::lo(3);
        const int e1 = s == 0 ? E::hi(0) : s == 1 ? E::hi(1) : s == 2 ? E::hi(2) : E::hi(3);
        const double *o = OM + j * NY, *y = Yv + pp * NY;
        double v = 0.0;
        for (int e = e0; e < e1; ++e) v += o[e] * y[e];
        Tv[it] = v;
      }
      team_sync();
      if (lt < 3) {
        for (int pp = 0; pp < npc; ++pp) {
          const double *t = Tv + pp * 12;
          const double dA = ZW[pp * 3] * t[lt] - t[6 + lt];
          const double dB = ZW[pp * 3 + 1] * t[3 + lt] - t[9 + lt];
          GA += dA;
          GB += dB;
          ACC[3 * int(ZW[pp * 3 + 2]) + lt] -= dA + dB;
        }
      }
      team_sync();
    }
    if (tid < 3) {
      ACC[3 * atA + tid] += GA;
      ACC[3 * atB + tid] += GB;
    }
    team_sync();
  }
  double *part = g.partial + int64_t(blockIdx.x) * 3 * g.natom;
  for (int x = tid; x < 3 * g.natom; x += TS) part[x] += ACC[x];
}

}  // namespace df3c

// Device building blocks of the gfx950 (ab|P) pipeline.
//
// One "team" of TS lanes (TS divides 64) evaluates one contracted shell
// triplet at a time; a workgroup is exactly one wavefront, so team-level
// synchronisation is a workgroup barrier of a single wave.  Intermediates live
// in the team's LDS slice between stages; every stage is lane-parallel over the
// items it produces (the paper's intra-shell-set parallelism, Section 2.2).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

#include "tables.hpp"

namespace df3c {

// ------------------------------------------------------------------ helpers
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  [&]<int... I>(std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
  }(std::make_integer_sequence<int, N>{});
}

__device__ __forceinline__ void team_sync() { __syncthreads(); }

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

struct ShellsDev {
  const int32_t *nprim;
  const int64_t *prim_off;
  const int32_t *atom;
  const double *exps;
  const double *coefs;
};

// ------------------------------------------------------------------- Boys
// F_m(T) = int_0^1 y^{2m} exp(-T y^2) dy (Appendix "Notation").  Section 2.5.2
// interpolates with 7th-order Chebyshev polynomials; here a 10-term Taylor
// expansion around the nearest node of a 1/8-spaced grid gives F_Mtop to
// ~1e-19 relative, followed by the (stable) downward recursion
//   F_m = (2T F_{m+1} + e^{-T}) / (2m + 1);
// for T >= BOYS_TMAX the asymptotic F_0 = sqrt(pi/T)/2 (erf(6) = 1 in FP64)
// and the (stable there) upward recursion F_{m+1} = ((2m+1)F_m - e^{-T})/(2T).
constexpr int BOYS_NTAY = 10;
constexpr int BOYS_MTOP_MAX = 17;
constexpr int BOYS_MTAB = BOYS_MTOP_MAX + BOYS_NTAY;  // columns of the table
constexpr double BOYS_DT = 0.125;
constexpr double BOYS_TMAX = 36.0;
constexpr int BOYS_NGRID = int(BOYS_TMAX / BOYS_DT) + 1;

// F[j] = F_{M0+j}(T), j = 0..NM-1; tab: BOYS_NGRID x BOYS_MTAB values F_m(i * BOYS_DT)
template <int M0, int NM>
__device__ __forceinline__ void boys(const double *__restrict__ tab, double T, double *F) {
  constexpr int MTOP = M0 + NM - 1;
  static_assert(MTOP <= BOYS_MTOP_MAX, "Boys order beyond the table");
  if (T < BOYS_TMAX) {
    const int i = min(max(int(T * (1.0 / BOYS_DT) + 0.5), 0), BOYS_NGRID - 1);
    const double md = double(i) * BOYS_DT - T;  // -(T - T_i)
    const double *row = tab + i * BOYS_MTAB + MTOP;
    double f = row[BOYS_NTAY - 1];
#pragma unroll
    for (int k = BOYS_NTAY - 2; k >= 0; --k) f = row[k] + f * md * (1.0 / double(k + 1));
    const double e = exp(-T);
    F[NM - 1] = f;
#pragma unroll
    for (int m = MTOP - 1; m >= M0; --m)
      F[m - M0] = (2.0 * T * F[m - M0 + 1] + e) * (1.0 / double(2 * m + 1));
  } else {
    const double e = exp(-T);
    const double r2t = 0.5 / T;
    double f = 0.5 * sqrt(3.14159265358979323846 / T);
#pragma unroll
    for (int m = 0; m < M0; ++m) f = (double(2 * m + 1) * f - e) * r2t;
    F[0] = f;
#pragma unroll
    for (int m = M0; m < MTOP; ++m) F[m - M0 + 1] = (double(2 * m + 1) * F[m - M0] - e) * r2t;
  }
}

// ---------------------------------------------------- per-primitive records
// scalars kept per primitive triplet in LDS
enum { PS_PAX = 0, PS_PAY, PS_PAZ, PS_RPX, PS_RPY, PS_RPZ, PS_I2G, PS_RG, PS_N };

// VRR1 over one chunk of primitives, 2-quantal stages in place (Section 2.5.3).
// prim(pp) points at the record of primitive pp: [PS_N scalars][T region][W region].
// On entry level 0 is stored (T[0] = m=LP, W[0..L-1] = m=LP+1..LP+L).
template <class G, int TS, int PCH, int REC>
__device__ __forceinline__ void vrr1(double *prims, int npc, int tid) {
  constexpr int L = G::L;
  using S = VStages<L>;
  static_for<S::nstage>([&](auto sc) {
    constexpr int s = decltype(sc)::value;
    constexpr int j = S::hi(s);
    constexpr bool twoq = S::two_q(s);
    constexpr int NIT = S::nitems(s);
    constexpr int IOFF = S::items_off(s);
    // input state: upper level hu, lower level hl (may be -1)
    constexpr int hu = twoq ? j - 2 : j - 1;
    constexpr int hl = hu - 1;
    constexpr int wl = (hl >= 0) ? ncart(hl) * (L - hl) : 0;  // lower input size
    constexpr int WIN_L = 0, WIN_U = wl;
    // output placement
    constexpr int WOUT_LO = 0;                                       // level j-1 (2-q)
    constexpr int WOUT_HI = twoq ? ncart(j - 1) * (L - j + 1) : L;   // level j
    constexpr int MAXIT = (NIT * PCH + TS - 1) / TS;
    using V = GenV<L>;

    double res[MAXIT];
    int dst[MAXIT];
    const int tot = NIT * npc;
#pragma unroll
    for (int q = 0; q < MAXIT; ++q) {
      const int it = tid + q * TS;
      dst[q] = -1;
      if (it < tot) {
        const int pp = it / NIT, x = it - pp * NIT;
        double *P = prims + pp * REC;
        const double *Tr = P + PS_N;
        const double *W = Tr + G::NT;
        const VI v = V::it[IOFF + x];
        const int m = v.m;
        // stored levels: value(level, comp, mm)
        auto up = [&](int c, int mm) -> double {
          return mm == 0 ? Tr[offT(hu) + c] : W[WIN_U + (mm - 1) * ncart(hu) + c];
        };
        auto lw = [&](int c, int mm) -> double {
          return mm == 0 ? Tr[offT(hl) + c] : W[WIN_L + (mm - 1) * ncart(hl) + c];
        };
        const double i2g = P[PS_I2G], rg = P[PS_RG];
        double val;
        if (v.q == 0) {
          const int i = v.i;
          val = P[PS_PAX + i] * up(v.a1, m) - P[PS_RPX + i] * up(v.a1, m + 1);
          if (v.a2 >= 0) val += double(v.f1) * i2g * (lw(v.a2, m) - rg * lw(v.a2, m + 1));
        } else {
          const int i = v.i, ip = v.ip;
          // x = e - 1_i (level j-1) at m and m+1, built in registers from the
          // stored levels j-2 (upper input) and j-3 (lower input)
          double X0 = P[PS_PAX + ip] * up(v.a1, m) - P[PS_RPX + ip] * up(v.a1, m + 1);
          double X1 = P[PS_PAX + ip] * up(v.a1, m + 1) - P[PS_RPX + ip] * up(v.a1, m + 2);
          if (v.a2 >= 0) {
            X0 += double(v.f1) * i2g * (lw(v.a2, m) - rg * lw(v.a2, m + 1));
            X1 += double(v.f1) * i2g * (lw(v.a2, m + 1) - rg * lw(v.a2, m + 2));
          }
          val = P[PS_PAX + i] * X0 - P[PS_RPX + i] * X1;
          if (v.y >= 0) val += double(v.f2) * i2g * (up(v.y, m) - rg * up(v.y, m + 1));
        }
        res[q] = val;
        const int lvl = (v.q == 1 || !twoq) ? j : j - 1;
        const int wout = (lvl == j) ? WOUT_HI : WOUT_LO;
        dst[q] = pp * REC + PS_N +
                 (m == 0 ? offT(lvl) + v.c : G::NT + wout + (m - 1) * ncart(lvl) + v.c);
      }
    }
    team_sync();
#pragma unroll
    for (int q = 0; q < MAXIT; ++q)
      if (dst[q] >= 0) prims[dst[q]] = res[q];
    team_sync();
  });
}

}  // namespace df3c

// Device building blocks of the gfx950 (ab|P) pipeline.
//
// One "team" of TS lanes evaluates one contracted shell triplet at a time
// (TS <= 64: several teams share one wavefront; TS = 128 / 256: a team spans
// 2 / 4 wavefronts); team synchronisation is a workgroup barrier.  Intermediates live
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

__device__ __forceinline__ bool wave_any(bool v) { return __any(v ? 1 : 0) != 0; }

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
  // both branches need e^{-T}: one evaluation, outside the (divergent) branch
  const double e = exp(-T);
  if (T < BOYS_TMAX) {
    const int i = min(max(int(T * (1.0 / BOYS_DT) + 0.5), 0), BOYS_NGRID - 1);
    const double md = double(i) * BOYS_DT - T;  // -(T - T_i)
    const double *row = tab + i * BOYS_MTAB + MTOP;
    double f = row[BOYS_NTAY - 1];
#pragma unroll
    for (int k = BOYS_NTAY - 2; k >= 0; --k) f = row[k] + f * md * (1.0 / double(k + 1));
    F[NM - 1] = f;
#pragma unroll
    for (int m = MTOP - 1; m >= M0; --m)
      F[m - M0] = (2.0 * T * F[m - M0 + 1] + e) * (1.0 / double(2 * m + 1));
  } else {
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
// vt0 / vt1 (optional): the table's item records staged in LDS by the
// kernel (words 0-3 and 4-5 of each 32-byte record), read there instead of
// from global memory.
template <class G, int TS, int PCH, int REC>
__device__ __forceinline__ void vrr1(double *prims, int npc, int tid, const uint4 *vt0 = nullptr,
                                     const uint2 *vt1 = nullptr) {
  constexpr int L = G::L;
  using S = VStages<L>;
  static_for<S::nstage>([&](auto sc) {
    constexpr int s = decltype(sc)::value;
    constexpr int NIT = S::nitems(s);
    constexpr int IOFF = S::items_off(s);
    constexpr int MAXIT = (NIT * PCH + TS - 1) / TS;
    using V = GenV<L>;

    static_assert(V::NT == G::NT && V::NW == G::NW, "generated VRR1 tables out of date");

    double res[MAXIT];
    int dst[MAXIT];
    const int tot = NIT * npc;
#pragma unroll
    for (int q = 0; q < MAXIT; ++q) {
      const int it = tid + q * TS;
      dst[q] = -1;
      if (it < tot) {
        const int pp = it / NIT, x = it - pp * NIT;
        const double *P = prims + pp * REC;
        const double *T = P + PS_N;
        // the 32-byte item record in two 16-byte loads; all fields are >= 0
        uint4 w0;
        uint2 w1;
        if (vt0) {
          w0 = vt0[IOFF + x];
          w1 = vt1[IOFF + x];
        } else {
          const uint4 *vp = reinterpret_cast<const uint4 *>(&V::ofs[IOFF + x]);
          w0 = vp[0];
          const uint4 t1 = vp[1];
          w1 = make_uint2(t1.x, t1.y);
        }
        const int u0 = w0.x & 0xffff, u1o = w0.x >> 16, u2 = w0.y & 0xffff, l0 = w0.y >> 16;
        const int l1o = w0.z & 0xffff, l2 = w0.z >> 16, y0 = w0.w & 0xffff, y1 = w0.w >> 16;
        const int od = w1.x & 0xffff, ax = w1.x >> 16, f1 = w1.y & 0xffff, f2 = w1.y >> 16;
        const int ip = (ax >> 2) & 3;
        const double i2g = P[PS_I2G], rg = P[PS_RG];
        const double pa = P[PS_PAX + ip], rp = P[PS_RPX + ip];
        const double c1 = double(f1) * i2g;
        const double u1 = T[u1o], l1 = T[l1o];
        double val = pa * T[u0] - rp * u1 + c1 * (T[l0] - rg * l1);
        if (ax & 16) {
          // 2-q: val is [x]^(m); [x]^(m+1), then the outer step along i
          const int i = ax & 3;
          const double x1 = pa * u1 - rp * T[u2] + c1 * (l1 - rg * T[l2]);
          val = P[PS_PAX + i] * val - P[PS_RPX + i] * x1 +
                double(f2) * i2g * (T[y0] - rg * T[y1]);
        }
        res[q] = val;
        dst[q] = pp * REC + PS_N + od;
      }
    }
    team_sync();
#pragma unroll
    for (int q = 0; q < MAXIT; ++q)
      if (dst[q] >= 0) prims[dst[q]] = res[q];
    team_sync();
  });
}

// Stage the VRR1 item records of level L into LDS (all threads of the
// workgroup; the caller synchronises): vt0[r] = words 0-3, vt1[r] = words 4-5.
template <int L>
__device__ __forceinline__ void stage_vrr1_table(uint4 *vt0, uint2 *vt1) {
  using V = GenV<L>;
  constexpr int N = VStages<L>::NITEMS;
  for (int r = threadIdx.x; r < N; r += blockDim.x) {
    const uint4 *vp = reinterpret_cast<const uint4 *>(&V::ofs[r]);
    vt0[r] = vp[0];
    const uint4 t1 = vp[1];
    vt1[r] = make_uint2(t1.x, t1.y);
  }
}

}  // namespace df3c

// Two-centre Coulomb metric V_PQ = (P|Q) of the auxiliary basis (the matrix
// of the density-fitting equations V d = gamma).
//
// (P|Q) is the three-centre integral with Q as the bra shell and a unit s
// function of exponent 0 on Q's centre as its partner: the bra pair reduces to
// Q itself (gamma = zeta_Q, P = Q, no Gaussian product factor), so the class
// (L_P, l_Q, 0) of the block pipeline (Boys, VRR1, contracted CVRR2, ket
// transform) gives (Q|P) with a Cartesian bra, and the bra is transformed to
// solid harmonics here.  One team per shell pair of a class with L_P >= l_Q;
// both triangles of V are written by the owner of the pair.
#pragma once
#include "kernels.hpp"

namespace df3c {

struct MetArgs {
  const double *boys;
  const double *xyz;
  ShellsDev aux;
  const int32_t *psh, *qsh;   // aux shells of l = LP and l = LQ
  int32_t np, nq, same;
  const int64_t *aux_off;     // function offset of each aux shell
  int64_t naux, npair;
  int32_t pure;
  double *V;                  // [naux][naux]
};

// the unit s partner of the bra: exponent 0, coefficient 1
static __device__ const double k_unit_s[2] = {0.0, 1.0};

template <int LP, int LQ, int TS, int PCH>
__global__ void __launch_bounds__(TS > 64 ? TS : 64)
    __attribute__((amdgpu_waves_per_eu(Cfg<LP, LQ, 0>::WPE))) k_metric(MetArgs g) {
  using G = Geo<LP, LQ, LQ>;
  using LY = Layout<LP, LQ, 0, PCH>;
  using SHQ = GenSolid<LQ>;
  constexpr int BLK = TS > 64 ? TS : 64;
  constexpr int TPB = BLK / TS;
  constexpr bool MF = (TS % 64 == 0) && PCH % 4 == 0;
  constexpr int NQS = MF ? 1 : (G::NPI + TS - 1) / TS;
  constexpr int NCQ = ncart(LQ);
  static_assert(G::NE == NCQ, "the metric bra is one level");
  extern __shared__ double smem[];
  const int team = threadIdx.x / TS, tid = threadIdx.x % TS;
  double *S = smem + team * LY::TOTAL;
  const double *EM = S + LY::EM;
  int slot[NQS];
  if constexpr (!MF) make_slots<LP, LQ, 0, TS>(slot, tid);
  const int np_out = g.pure ? npure(LP) : ncart(LP);
  const int nq_out = g.pure ? npure(LQ) : NCQ;

  for (int64_t base = int64_t(blockIdx.x) * TPB; base < g.npair; base += int64_t(gridDim.x) * TPB) {
    const int64_t q = base + team;
    const bool valid = q < g.npair;
    int sP = 0, sQ = 0;
    if (valid) {
      if (g.same) {
        int i = int((sqrt(8.0 * double(q) + 1.0) - 1.0) * 0.5);
        while (int64_t(i) * (i + 1) / 2 > q) --i;
        while (int64_t(i + 1) * (i + 2) / 2 <= q) ++i;
        const int j = int(q - int64_t(i) * (i + 1) / 2);
        sP = g.psh[i];
        sQ = g.qsh[j];
      } else {
        const int i = int(q / g.nq), j = int(q - int64_t(i) * g.nq);
        sP = g.psh[i];
        sQ = g.qsh[j];
      }
    }
    const int KQ = valid ? g.aux.nprim[sQ] : 0, KP = valid ? g.aux.nprim[sP] : 0;
    const int64_t oq = valid ? g.aux.prim_off[sQ] : 0, op = valid ? g.aux.prim_off[sP] : 0;
    double A[3] = {0, 0, 0}, C[3] = {0, 0, 0};
    if (valid) {
      const int aq = g.aux.atom[sQ], ap = g.aux.atom[sP];
      for (int x = 0; x < 3; ++x) {
        A[x] = g.xyz[3 * aq + x];
        C[x] = g.xyz[3 * ap + x];
      }
    }
    const int npmax = TS >= 64 ? KQ * KP : wave_max(KQ * KP);
    triplet_to_e0P<LP, LQ, 0, TS, PCH>(g.boys, S, tid, slot, npmax, A, A, C, KQ,
                                       g.aux.exps + oq, g.aux.coefs + oq, 1, k_unit_s,
                                       k_unit_s + 1, KP, g.aux.exps + op, g.aux.coefs + op,
                                       g.pure);
    if (valid) {
      const int64_t fP = g.aux_off[sP], fQ = g.aux_off[sQ];
      for (int it = tid; it < np_out * nq_out; it += TS) {
        const int mp = it / nq_out, mq = it - mp * nq_out;
        double v = 0.0;
        if (g.pure) {
#pragma unroll
          for (int e = 0; e < NCQ; ++e) v += SHQ::dense[mq * NCQ + e] * EM[mp * NCQ + e];
        } else {
          v = EM[mp * NCQ + mq];
        }
        // a diagonal shell block is written from its lower triangle only
        if (sP != sQ || mp >= mq) {
          g.V[(fP + mp) * g.naux + fQ + mq] = v;
          g.V[(fQ + mq) * g.naux + fP + mp] = v;
        }
      }
    }
    team_sync();
  }
}

}  // namespace df3c

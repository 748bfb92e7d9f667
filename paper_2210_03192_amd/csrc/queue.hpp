// Batched DF-J over many molecules with a device work queue.
//
// A work item is one orbital shell pair of one molecule for one class
// (L_P, l_a, l_b); the items of a class are numbered across all molecules
// (segments = molecules, prefix-summed item offsets).  One persistent launch
// per class serves all molecules: every workgroup repeatedly takes the next
// TPB x chunk items from an atomic counter until the queue is empty, so uneven
// molecules and contraction degrees balance dynamically.  The per-item work is
// the J pair kernel of kernels.hpp.
#pragma once
#include "kernels.hpp"

namespace df3c {

// one molecule's share of a class
struct JSeg {
  int64_t item0;      // first queue item of the segment
  int64_t npair;      // items (shell pairs) of the segment
  int64_t jbase;      // offset of the molecule's J block
  int64_t nao;        // molecule's AO count (J is nao x nao)
  int64_t ao_base;    // global AO offset of the molecule's first shell
  int32_t ash, bsh;   // offsets of the sorted shell lists (l = LA, l = LB)
  int32_t psh;        // offset of the sorted aux list (l = LP)
  int32_t na, nb, np, same;
  int32_t pad;        // molecule index (host-side bookkeeping)
};

struct JQArgs {
  JArgs a;            // shared fields; per-item fields are taken from the segment
  const int32_t *orb_sorted, *aux_sorted;
  double *Jall;
  const JSeg *seg;
  int32_t nseg;
  int32_t chunk;      // consecutive items per team and grab
  int64_t total;
  unsigned long long *counter;
};

// segment of an item: last s with seg[s].item0 <= item (binary search)
__device__ __forceinline__ int find_seg(const JSeg *seg, int nseg, int64_t item) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (seg[mid].item0 <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int LP, int LA, int LB, int TS, int PCH>
__global__ void __launch_bounds__(TS > 64 ? TS : 64)
    __attribute__((amdgpu_waves_per_eu(Cfg<LP, LA, LB>::WPEJ))) k_Jq(JQArgs q) {
  using JL = JLayout<LP, LA, LB, TS, PCH>;
  constexpr int BLK = TS > 64 ? TS : 64;
  constexpr int TPB = BLK / TS;
  constexpr bool REG = JL::REG;
  extern __shared__ double smem[];
  __shared__ unsigned long long s_base;
  // register engine: lane = sub (64 / nsub) + team, nsub lanes per item
  const int tpb = REG ? TPB / q.a.nsub : TPB;
  const int team = REG ? int(threadIdx.x) % tpb : int(threadIdx.x) / TS;
  const int sub = REG ? int(threadIdx.x) / tpb : 0;
  const int tid = threadIdx.x % TS;
  double *S = smem + (REG ? 0 : team * JL::TOTAL);
  if (q.a.err && *q.a.err) return;

  for (;;) {
    if (threadIdx.x == 0) s_base = atomicAdd(q.counter, (unsigned long long)(tpb * q.chunk));
    __syncthreads();
    const int64_t base = int64_t(s_base);
    __syncthreads();
    if (base >= q.total) break;  // uniform over the workgroup: every wave leaves together
    for (int j = 0; j < q.chunk; ++j) {
      const int64_t item = base + int64_t(team) * q.chunk + j;
      const bool valid = item < q.total;
      JArgs a = q.a;
      int sa = 0, sb = 0, np = 0;
      if (valid) {
        const JSeg &sg = q.seg[find_seg(q.seg, q.nseg, item)];
        const int64_t r = item - sg.item0;
        a.J = q.Jall + sg.jbase;
        a.nao = sg.nao;
        a.ao_base = sg.ao_base;
        a.psh = q.aux_sorted + sg.psh;
        a.arec = q.a.arec + int64_t(sg.psh) * AREC;
        np = sg.np;
        if (sg.same) {
          int i = int((sqrt(8.0 * double(r) + 1.0) - 1.0) * 0.5);
          while (int64_t(i) * (i + 1) / 2 > r) --i;
          while (int64_t(i + 1) * (i + 2) / 2 <= r) ++i;
          const int jj = int(r - int64_t(i) * (i + 1) / 2);
          sa = q.orb_sorted[sg.ash + i];
          sb = q.orb_sorted[sg.ash + jj];
        } else {
          const int i = int(r / sg.nb), jj = int(r - int64_t(i) * sg.nb);
          sa = q.orb_sorted[sg.ash + i];
          sb = q.orb_sorted[sg.bsh + jj];
        }
      }
      a.np = np;
      // the aux loop runs to the workgroup's largest np; shorter teams idle
      const int np_loop = TS >= 64 ? np : wave_max(np);
      j_pair<LP, LA, LB, TS, PCH>(a, S, tid, valid, sa, sb, np_loop, sub);
    }
  }
}

}  // namespace df3c

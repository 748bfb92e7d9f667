// The density-fitting solve V d = gamma (the fitting equations whose
// right-hand side is the adjoint digestion gamma = (P|ab) D and whose matrix is
// the two-centre metric V = (P|Q)): a blocked right-looking Cholesky
// factorisation V = L L^T in FP64 followed by the two triangular solves.
//
// V is row-major n x n and is overwritten: its lower triangle receives L and
// its upper triangle L^T (so both solves read rows).  Steps per block column
// k of width CB:
//   k_chol_diag    factor the diagonal block in LDS (one workgroup);
//   k_chol_panel   L21 = A21 L11^{-T}, one thread per row, L11 in LDS, and
//                  the transposed copy into the upper triangle;
//   k_chol_update  A22 -= L21 L21^T on the lower triangle, 64 x 64 output tiles
//                  (256 threads, 4 x 4 outputs each, L21 rows staged in LDS).
// The solves run block by block: k_trsv_block solves a block's triangle (one
// workgroup), k_trsv_update subtracts its contribution from every row still
// to be solved (one wavefront per row).
// A pivot below DBL_EPSILON x max_i V_ii (or NaN) stops the factorisation:
// bit 16 of the status word, and every later kernel does nothing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cstdint>
#include <mutex>

#include "../../include/df3c.h"

namespace df3c {
namespace {

constexpr int CB = 64;      // block column width
constexpr int UT = 64;      // output tile of the trailing update
constexpr int UK = 32;      // k extent staged in LDS per round of the update

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

__global__ void k_fit_init(int *err, double *dmax) {
  if (threadIdx.x < 8) err[threadIdx.x] = 0;
  if (threadIdx.x == 0) *dmax = 0.0;
}

// max_i V_ii (one workgroup, fixed reduction order); a non-positive or NaN
// diagonal element fails at once
__global__ void __launch_bounds__(256) k_diag_max(const double *V, int64_t n, double *dmax,
                                                 int *err) {
  __shared__ double m[256];
  double v = 0.0;
  bool bad = false;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double d = V[i * n + i];
    if (!(d > 0.0)) bad = true;
    v = fmax(v, d);
  }
  m[threadIdx.x] = v;
  if (bad) atomicOr(err, 16);
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) m[threadIdx.x] = fmax(m[threadIdx.x], m[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *dmax = m[0];
}

// Cholesky of the nb x nb diagonal block at (k, k), in place (lower).  Per
// column j: the pivot, the column scaled, then the rank-1 update of the
// trailing triangle with a fixed 16 x 16 thread grid (thread (ty, tx) owns the
// entries (i, c) with i = ty mod 16, c = tx mod 16), no index division.
__global__ void __launch_bounds__(256) k_chol_diag(double *V, int64_t n, int64_t k, int nb,
                                                  const double *dmax, int *err) {
  __shared__ double A[CB][CB + 1];
  __shared__ int fail;
  if (*err) return;
  const int t = threadIdx.x, ty = t >> 4, tx = t & 15;
  for (int x = t; x < nb * nb; x += 256) {
    const int i = x / nb, j = x - i * nb;
    A[i][j] = j <= i ? V[(k + i) * n + k + j] : 0.0;
  }
  if (t == 0) fail = 0;
  __syncthreads();
  const double tol = DBL_EPSILON * *dmax;
  for (int j = 0; j < nb; ++j) {
    // every thread takes the pivot itself (same value in every lane)
    const double p = A[j][j];
    const double piv = sqrt(fmax(p, tol));
    const double rpiv = 1.0 / piv;
    __syncthreads();
    if (t == 0) {
      if (!(p > tol)) fail = 1;
      A[j][j] = piv;
    }
    if (t > j && t < nb) A[t][j] *= rpiv;
    __syncthreads();
    // rank-1 update of the rest of the block's lower triangle
    for (int i = j + 1 + ty; i < nb; i += 16) {
      const double aij = A[i][j];
      for (int c = j + 1 + tx; c <= i; c += 16) A[i][c] -= aij * A[c][j];
    }
    __syncthreads();
  }
  for (int x = t; x < nb * nb; x += 256) {
    const int i = x / nb, j = x - i * nb;
    if (j <= i) {
      V[(k + i) * n + k + j] = A[i][j];
      V[(k + j) * n + k + i] = A[i][j];  // L^T in the upper triangle
    }
  }
  if (t == 0 && fail) atomicOr(err, 16);
}

// rows i >= k + nb: L21[i] = A21[i] L11^{-T} (forward substitution per row)
__global__ void __launch_bounds__(256) k_chol_panel(double *V, int64_t n, int64_t k, int nb,
                                                   const int *err) {
  __shared__ double L[CB][CB + 1];
  if (*err) return;
  const int t = threadIdx.x;
  for (int x = t; x < nb * nb; x += 256) {
    const int i = x / nb, j = x - i * nb;
    L[i][j] = j <= i ? V[(k + i) * n + k + j] : 0.0;
  }
  __syncthreads();
  for (int64_t r = k + nb + int64_t(blockIdx.x) * 256 + t; r < n; r += int64_t(gridDim.x) * 256) {
    double x[CB];
    double *row = V + r * n + k;
#pragma unroll
    for (int j = 0; j < CB; ++j) x[j] = j < nb ? row[j] : 0.0;
#pragma unroll
    for (int j = 0; j < CB; ++j) {
      if (j < nb) {
        double v = x[j];
#pragma unroll
        for (int q = 0; q < j; ++q) v -= x[q] * L[j][q];
        x[j] = v / L[j][j];
      }
    }
#pragma unroll
    for (int j = 0; j < CB; ++j)
      if (j < nb) {
        row[j] = x[j];
        V[(k + j) * n + r] = x[j];  // L^T in the upper triangle
      }
  }
}

// A22[i][j] -= sum_q L21[i][q] L21[j][q] for k + nb <= j <= i < n: tiles of
// the lower triangle, one per workgroup (tile (ti, tj), tj <= ti, from the
// workgroup index); 256 threads x 4 x 4 outputs; the rows of both tiles are
// staged UK columns at a time.  part 1: only the tiles of the first tile
// column (tj = 0, the next block column: the look-ahead); part 2: the others
// (tj >= 1); part 0: all.
__global__ void __launch_bounds__(256) k_chol_update(double *V, int64_t n, int64_t k, int nb,
                                                    int part, const int *err) {
  __shared__ double Ri[UT][UK + 1], Rj[UT][UK + 1];
  if (*err) return;
  const int64_t b = blockIdx.x;
  int64_t ti, tj;
  if (part == 1) {
    ti = b;
    tj = 0;
  } else {
    ti = int64_t((sqrt(8.0 * double(b) + 1.0) - 1.0) * 0.5);
    while (ti * (ti + 1) / 2 > b) --ti;
    while ((ti + 1) * (ti + 2) / 2 <= b) ++ti;
    tj = b - ti * (ti + 1) / 2;
    if (part == 2) {  // the triangle of tiles below and right of the first tile column
      ++ti;
      ++tj;
    }
  }
  const int64_t base = k + nb;
  const int64_t i0 = base + ti * UT, j0 = base + tj * UT;
  const int t = threadIdx.x, ty = t / 16, tx = t % 16;
  double acc[4][4] = {};
  for (int q0 = 0; q0 < nb; q0 += UK) {
    for (int x = t; x < UT * UK; x += 256) {
      const int r = x / UK, q = x % UK;
      const int64_t gi = i0 + r, gj = j0 + r;
      Ri[r][q] = (gi < n && q0 + q < nb) ? V[gi * n + k + q0 + q] : 0.0;
      Rj[r][q] = (gj < n && q0 + q < nb) ? V[gj * n + k + q0 + q] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int q = 0; q < UK; ++q) {
      double a[4], c[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = Ri[ty + 16 * u][q];
        c[u] = Rj[tx + 16 * u][q];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * c[v];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t gi = i0 + ty + 16 * u, gj = j0 + tx + 16 * v;
      if (gi < n && gj <= gi) V[gi * n + gj] -= acc[u][v];
    }
}

// One block of a triangular solve with the rows of V: lower (L y = b,
// blocks in increasing order) or upper (L^T x = y, blocks in decreasing
// order).  The contributions of the solved blocks are already subtracted
// (k_trsv_update after each block); one workgroup solves the nb x nb triangle
// in order.
__global__ void __launch_bounds__(256) k_trsv_block(const double *V, int64_t n, int64_t k,
                                                   int nb, int upper, double *x, const int *err) {
  __shared__ double r[CB];
  __shared__ double D[CB][CB + 1];
  if (*err) return;
  const int t = threadIdx.x;
  for (int e = t; e < nb * nb; e += 256) {
    const int i = e / nb, j = e - i * nb;
    D[i][j] = V[(k + i) * n + k + j];
  }
  if (t < nb) r[t] = x[k + t];
  __syncthreads();
  // column by column: the solved entry, then every later row subtracts its
  // share (lane i owns row i; the subtractions of row i come in column order)
  if (!upper) {
    for (int j = 0; j < nb; ++j) {
      if (t == j) r[j] /= D[j][j];
      __syncthreads();
      if (t > j && t < nb) r[t] -= D[t][j] * r[j];
      __syncthreads();
    }
  } else {
    for (int j = nb - 1; j >= 0; --j) {
      if (t == j) r[j] /= D[j][j];
      __syncthreads();
      if (t < j) r[t] -= D[t][j] * r[j];
      __syncthreads();
    }
  }
  if (t < nb) x[k + t] = r[t];
}

// Right-looking update of the triangular solves after block k (width nb) is
// solved: every row i still to be solved (lower: i >= k + nb; upper: i < k)
// subtracts sum_q V[i][k + q] x[k + q].  One wavefront per row at a time (the
// row's nb entries are contiguous, one per lane), summed by a fixed butterfly,
// so every x_i receives the blocks' contributions in the same order on every
// call.
__global__ void __launch_bounds__(256) k_trsv_update(const double *V, int64_t n, int64_t k,
                                                    int nb, int upper, double *x, const int *err) {
  if (*err) return;
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwave = (int64_t(gridDim.x) * blockDim.x) >> 6;
  const double xk = lane < nb ? x[k + lane] : 0.0;
  const int64_t r0 = upper ? 0 : k + nb, r1 = upper ? k : n;
  for (int64_t i = r0 + wave; i < r1; i += nwave) {
    double v = lane < nb ? V[i * n + k + lane] * xk : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) x[i] -= v;
  }
}

__global__ void k_copy_vec(const double *a, double *b, int64_t n, const int *err) {
  if (*err) return;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    b[i] = a[i];
}

}  // namespace
}  // namespace df3c

using namespace df3c;

namespace {
// the factorisation's look-ahead: a side stream (default priority) and two
// events per device, created on first use; the enqueue of a factorisation
// holds the lock (the events are shared)
struct FitSide {
  bool ready = false;
  hipStream_t side = nullptr;
  hipEvent_t panel = nullptr, rest = nullptr;
};
constexpr int FIT_MAX_DEV = 64;
FitSide g_fit[FIT_MAX_DEV];
std::mutex g_fit_mu;

int fit_side(FitSide **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= FIT_MAX_DEV) return DF3C_E_HIP;
  FitSide &f = g_fit[dev];
  if (!f.ready) {
    if (hipStreamCreateWithFlags(&f.side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&f.panel, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&f.rest, hipEventDisableTiming) != hipSuccess)
      return DF3C_E_HIP;
    f.ready = true;
  }
  *out = &f;
  return DF3C_OK;
}
}  // namespace

extern "C" {

size_t df3c_fit_solve_workspace(int64_t n) {
  (void)n;
  return align256(sizeof(int) * 8) + align256(sizeof(double));
}

int df3c_fit_solve(double *V, int64_t n, const double *rhs, double *x, void *ws, size_t ws_bytes,
                   uint32_t flags, void *stream) {
  if (flags & ~DF3C_ASYNC) return DF3C_E_ARG;
  if (n < 0 || (n > 0 && (!V || !rhs || !x))) return DF3C_E_ARG;
  if (n > (int64_t(1) << 31)) return DF3C_E_UNSUPPORTED;
  if (!ws || ws_bytes < df3c_fit_solve_workspace(n)) return DF3C_E_WORKSPACE;
  if (n == 0) return DF3C_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int *err = static_cast<int *>(ws);
  double *dmax = reinterpret_cast<double *>(static_cast<char *>(ws) + align256(sizeof(int) * 8));
  hipLaunchKernelGGL(k_fit_init, dim3(1), dim3(64), 0, s, err, dmax);
  hipLaunchKernelGGL(k_diag_max, dim3(1), dim3(256), 0, s, V, n, dmax, err);
  // Look-ahead: per block column k, the diagonal block, the panel and the
  // update of the next block column run on `stream`, the update of the rest
  // of the trailing matrix on a side stream, so the next diagonal block and
  // panel overlap it.  The next-column update of step k waits for the
  // rest-update of step k - 1 (both write that column); the rest-update of
  // step k waits for the panel of step k.  Every element still receives its
  // updates in step order.
  FitSide *fs = nullptr;
  if (int rc = fit_side(&fs)) return rc;
  {
    std::lock_guard<std::mutex> lk(g_fit_mu);
    bool pending = false;  // a rest-update has been recorded on fs->rest
    if (hipEventRecord(fs->rest, s) != hipSuccess) return DF3C_E_HIP;
    pending = true;
    for (int64_t k = 0; k < n; k += CB) {
      const int nb = int(std::min<int64_t>(CB, n - k));
      hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, s, V, n, k, nb, dmax, err);
      const int64_t m = n - k - nb;
      if (m <= 0) continue;
      const int gp = int(std::min<int64_t>((m + 255) / 256, 1024));
      hipLaunchKernelGGL(k_chol_panel, dim3(gp), dim3(256), 0, s, V, n, k, nb, err);
      if (hipEventRecord(fs->panel, s) != hipSuccess) return DF3C_E_HIP;
      const int64_t T = (m + UT - 1) / UT;
      // the next block column, after the previous rest-update
      if (pending && hipStreamWaitEvent(s, fs->rest, 0) != hipSuccess) return DF3C_E_HIP;
      hipLaunchKernelGGL(k_chol_update, dim3(unsigned(T)), dim3(256), 0, s, V, n, k, nb, 1, err);
      // the rest, on the side stream after this panel
      if (T > 1) {
        if (hipStreamWaitEvent(fs->side, fs->panel, 0) != hipSuccess) return DF3C_E_HIP;
        hipLaunchKernelGGL(k_chol_update, dim3(unsigned((T - 1) * T / 2)), dim3(256), 0,
                           fs->side, V, n, k, nb, 2, err);
        if (hipEventRecord(fs->rest, fs->side) != hipSuccess) return DF3C_E_HIP;
        pending = true;
      }
    }
    if (hipStreamWaitEvent(s, fs->rest, 0) != hipSuccess) return DF3C_E_HIP;
  }
  // x = rhs, then L y = x and L^T x = y in place
  if (x != rhs)
    hipLaunchKernelGGL(k_copy_vec, dim3(int(std::min<int64_t>((n + 255) / 256, 1024))), dim3(256),
                       0, s, rhs, x, n, err);
  // per block: solve its triangle, then update the rows still to be solved
  auto upd_grid = [](int64_t rows) {
    return int(std::max<int64_t>(1, std::min<int64_t>((rows + 3) / 4, 2048)));
  };
  for (int64_t k = 0; k < n; k += CB) {
    const int nb = int(std::min<int64_t>(CB, n - k));
    hipLaunchKernelGGL(k_trsv_block, dim3(1), dim3(256), 0, s, V, n, k, nb, 0, x, err);
    if (k + nb < n)
      hipLaunchKernelGGL(k_trsv_update, dim3(upd_grid(n - k - nb)), dim3(256), 0, s, V, n, k, nb,
                         0, x, err);
  }
  for (int64_t k = ((n - 1) / CB) * CB; k >= 0; k -= CB) {
    const int nb = int(std::min<int64_t>(CB, n - k));
    hipLaunchKernelGGL(k_trsv_block, dim3(1), dim3(256), 0, s, V, n, k, nb, 1, x, err);
    if (k > 0)
      hipLaunchKernelGGL(k_trsv_update, dim3(upd_grid(k)), dim3(256), 0, s, V, n, k, nb, 1, x,
                         err);
  }
  if (hipGetLastError() != hipSuccess) return DF3C_E_HIP;
  if (flags & DF3C_ASYNC) return DF3C_OK;
  int word = 0;
  if (hipMemcpyAsync(&word, err, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return DF3C_E_HIP;
  return word ? DF3C_E_NUMERIC : DF3C_OK;
}

}  // extern "C"

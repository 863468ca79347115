// gfx950 kernels of the solve (eq. kinv with the partition of eq. partition):
// U, V and Psi^T V sweeps, the X_RR^{-1} blocks, the border columns H and rows
// Psi^T, the reduced root system, and the refinement bookkeeping (residual
// norms, convergence flag, guarded accumulation).
#include "rs_device.h"

namespace rs {
namespace {

// ---- solve kernels -----------------------------------------------------------

// mode 0: U   c_R -= T^T c_S ; c_S -= E c_R
// mode 1: Psi^T V rows (columns of Psi)   c_R -= T^T c_S ; c_S -= F^T c_R
// mode 2: V   c_R -= F c_S ; c_S -= T c_R
// Each box's factors are read in the precision they are stored in (float
// copies when present, else float64); vectors and sums are float64.
template <typename T, typename TF>
__device__ __forceinline__ void sweep_box(const SolveBox& B, const TF* Tm, const TF* Em, const TF* Fm,
                                          const int* sidx, const int* ridx, T* c, int ncols, int mode,
                                          int kNC, T* smem) {
  const int k = B.k, r = B.r;
  const int q0 = blockIdx.y * kNC;
  const int nq = min(kNC, ncols - q0);
  T* cs = smem;
  T* cr = smem + (size_t)k * kNC;
  const int* S = sidx + B.s_off;
  const int* R = ridx + B.r_off;
  const int tid = threadIdx.x;
  for (int t = tid; t < k * kNC; t += kBlock) {
    const int s = t / kNC, q = t % kNC;
    cs[t] = q < nq ? c[(size_t)S[s] * ncols + q0 + q] : T(0);
  }
  for (int t = tid; t < r * kNC; t += kBlock) {
    const int i = t / kNC, q = t % kNC;
    cr[t] = q < nq ? c[(size_t)R[i] * ncols + q0 + q] : T(0);
  }
  __syncthreads();
  if (mode != 2) {
    for (int t = tid; t < r * kNC; t += kBlock) {
      const int i = t / kNC, q = t % kNC;
      T acc = 0;
      for (int s = 0; s < k; ++s) acc += Tm[(size_t)s * r + i] * cs[s * kNC + q];
      cr[t] -= acc;
    }
    __syncthreads();
    for (int t = tid; t < k * kNC; t += kBlock) {
      const int s = t / kNC, q = t % kNC;
      T acc = 0;
      if (mode == 0)
        for (int i = 0; i < r; ++i) acc += Em[(size_t)s * r + i] * cr[i * kNC + q];
      else
        for (int i = 0; i < r; ++i) acc += Fm[(size_t)i * k + s] * cr[i * kNC + q];
      cs[t] -= acc;
    }
  } else {
    for (int t = tid; t < r * kNC; t += kBlock) {
      const int i = t / kNC, q = t % kNC;
      T acc = 0;
      for (int s = 0; s < k; ++s) acc += Fm[(size_t)i * k + s] * cs[s * kNC + q];
      cr[t] -= acc;
    }
    __syncthreads();
    for (int t = tid; t < k * kNC; t += kBlock) {
      const int s = t / kNC, q = t % kNC;
      T acc = 0;
      for (int i = 0; i < r; ++i) acc += Tm[(size_t)s * r + i] * cr[i * kNC + q];
      cs[t] -= acc;
    }
  }
  __syncthreads();
  for (int t = tid; t < k * kNC; t += kBlock) {
    const int s = t / kNC, q = t % kNC;
    if (q < nq) c[(size_t)S[s] * ncols + q0 + q] = cs[t];
  }
  for (int t = tid; t < r * kNC; t += kBlock) {
    const int i = t / kNC, q = t % kNC;
    if (q < nq) c[(size_t)R[i] * ncols + q0 + q] = cr[t];
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_sweep(const SolveBox* boxes, const int* sidx,
                                                  const int* ridx, T* c, int ncols, int mode,
                                                  int kNC) {
  extern __shared__ double smem_d[];
  T* smem = reinterpret_cast<T*>(smem_d);
  const SolveBox& B = boxes[blockIdx.x];
  if (B.k == 0 || B.r == 0) return;
  if (B.Tf) sweep_box<T, float>(B, B.Tf, B.Ef, B.Ff, sidx, ridx, c, ncols, mode, kNC, smem);
  else sweep_box<T, double>(B, B.T, B.E, B.F, sidx, ridx, c, ncols, mode, kNC, smem);
}

// c_R <- X_RR^{-1} c_R
template <typename T, typename TF>
__device__ __forceinline__ void diag_box(const SolveBox& B, const TF* Xi, const int* ridx, T* c,
                                         int ncols, int kNC, T* smem) {
  const int r = B.r;
  const int q0 = blockIdx.y * kNC;
  const int nq = min(kNC, ncols - q0);
  T* in = smem;
  T* out = smem + (size_t)r * kNC;
  const int* R = ridx + B.r_off;
  for (int t = threadIdx.x; t < r * kNC; t += kBlock) {
    const int i = t / kNC, q = t % kNC;
    in[t] = q < nq ? c[(size_t)R[i] * ncols + q0 + q] : T(0);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < r * kNC; t += kBlock) {
    const int i = t / kNC, q = t % kNC;
    T acc = 0;
    for (int j = 0; j < r; ++j) acc += Xi[(size_t)i * r + j] * in[j * kNC + q];
    out[t] = acc;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < r * kNC; t += kBlock) {
    const int i = t / kNC, q = t % kNC;
    if (q < nq) c[(size_t)R[i] * ncols + q0 + q] = out[t];
  }
}

// The same product for boxes with r <= kDiagMaxR, through LDS: per 16
// columns, the K dimension goes in chunks of kDiagK rows of c_R (staged) and,
// for each 64-row tile of the box, the matching 64 x kDiagK tile of
// X_RR^{-1} (rows padded by one double against bank conflicts).  The thread
// (row ii of every tile, column group g) keeps 4 columns of up to
// kDiagMaxTiles rows in registers and writes them after the last read of c_R.
// Each output sums over j in order, as above.  21 KiB of LDS.
constexpr int kDiagTile = 64;
constexpr int kDiagK = 32;
constexpr int kDiagMaxTiles = 8;
constexpr int kDiagMaxR = kDiagTile * kDiagMaxTiles;                            // 512
constexpr int kDiagLds = (kDiagK * 16 + kDiagTile * (kDiagK + 1)) * 8;          // bytes
template <typename T, typename TF>
__device__ __forceinline__ void diag_box_tiled(const SolveBox& B, const TF* Xi, const int* ridx, T* c,
                                               int ncols, int kNC, double* smem) {
  const int r = B.r;
  const int q0 = blockIdx.y * kNC;
  const int nq = min(kNC, ncols - q0);
  const int* R = ridx + B.r_off;
  const int ntile = (r + kDiagTile - 1) / kDiagTile;
  double* sIn = smem;                      // kDiagK x 16
  double* sX = smem + kDiagK * 16;         // kDiagTile x (kDiagK + 1)
  const int ii = threadIdx.x % kDiagTile, g = threadIdx.x / kDiagTile;
  static_assert(kBlock == 4 * kDiagTile, "4 column groups of 4 cover 16 columns");
  for (int qa = 0; qa < nq; qa += 16) {
    const int na = min(16, nq - qa);
    double acc[kDiagMaxTiles][4];
#pragma unroll
    for (int t = 0; t < kDiagMaxTiles; ++t) acc[t][0] = acc[t][1] = acc[t][2] = acc[t][3] = 0.0;
    for (int k0 = 0; k0 < r; k0 += kDiagK) {
      const int kc = min(kDiagK, r - k0);
      __syncthreads();
      for (int e = threadIdx.x; e < kDiagK * 16; e += kBlock) {
        const int j = e / 16, k = e % 16;
        sIn[e] = (j < kc && k < na) ? (double)c[(size_t)R[k0 + j] * ncols + q0 + qa + k] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < kDiagMaxTiles; ++t) {
        if (t < ntile) {   // uniform over the block
          const int i0 = t * kDiagTile, nt = min(kDiagTile, r - i0);
          __syncthreads();
          for (int e = threadIdx.x; e < kDiagTile * kDiagK; e += kBlock) {
            const int rr = e / kDiagK, kk = e % kDiagK;
            sX[rr * (kDiagK + 1) + kk] = (rr < nt && kk < kc) ? (double)Xi[(size_t)(i0 + rr) * r + k0 + kk] : 0.0;
          }
          __syncthreads();
          if (ii < nt && 4 * g < na) {
            const double* xr = sX + ii * (kDiagK + 1);
            const double* vr = sIn + 4 * g;
            for (int kk = 0; kk < kc; ++kk) {
              const double x = xr[kk];
              const double4 v = *reinterpret_cast<const double4*>(vr + (size_t)kk * 16);
              acc[t][0] += x * v.x;
              acc[t][1] += x * v.y;
              acc[t][2] += x * v.z;
              acc[t][3] += x * v.w;
            }
          }
        }
      }
    }
    __syncthreads();   // every read of c_R for these columns is done
#pragma unroll
    for (int t = 0; t < kDiagMaxTiles; ++t) {
      const int i = t * kDiagTile + ii;
      if (t < ntile && i < r) {
        T* crow = c + (size_t)R[i] * ncols + q0 + qa + 4 * g;
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (4 * g + v < na) crow[v] = (T)acc[t][v];
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_diag(const SolveBox* boxes, const int* ridx, T* c,
                                                 int ncols, int kNC) {
  extern __shared__ __align__(16) double smem_d[];
  T* smem = reinterpret_cast<T*>(smem_d);
  const SolveBox& B = boxes[blockIdx.x];
  if (B.r == 0) return;
  if (B.r <= kDiagMaxR) {
    if (B.Xinvf) diag_box_tiled<T, float>(B, B.Xinvf, ridx, c, ncols, kNC, smem_d);
    else diag_box_tiled<T, double>(B, B.Xinv, ridx, c, ncols, kNC, smem_d);
  } else if (B.Xinvf) {
    diag_box<T, float>(B, B.Xinvf, ridx, c, ncols, kNC, smem);
  } else {
    diag_box<T, double>(B, B.Xinv, ridx, c, ncols, kNC, smem);
  }
}

// H (2N x 3p) and Psi (2N x 3p, i.e. Psi^T stored by columns), row-major.
// One thread per (node j, hole h), h fastest, so that a wavefront writes
// consecutive 3-column groups of the same rows (coalesced stores).
__global__ void k_assemble_H(Geo g, const double* hole_xy, int p, const int* curve_id,
                             double* H, double* Psi) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)g.N * p) return;
  const int j = (int)(t / p), h = (int)(t % p);
  const int p3 = 3 * p;
  const double xj = g.x[j], yj = g.y[j];
  const double rx = xj - hole_xy[2 * h], ry = yj - hole_xy[2 * h + 1];
  const double r2 = rx * rx + ry * ry;
  const double lg = -0.5 * log(r2);
  double* h0 = H + (size_t)(2 * j) * p3 + 3 * h;
  double* h1 = H + (size_t)(2 * j + 1) * p3 + 3 * h;
  h0[0] = kInv4Pi * (lg + rx * rx / r2);
  h0[1] = kInv4Pi * (rx * ry / r2);
  h1[0] = kInv4Pi * (ry * rx / r2);
  h1[1] = kInv4Pi * (lg + ry * ry / r2);
  h0[2] = kInv4Pi * (-ry) / r2;
  h1[2] = kInv4Pi * rx / r2;
  // Psi: the node's weight rows for its own hole, zero elsewhere
  const bool own = curve_id[j] == h + 1;
  const double w = own ? g.w[j] : 0.0;
  double* s0 = Psi + (size_t)(2 * j) * p3 + 3 * h;
  double* s1 = Psi + (size_t)(2 * j + 1) * p3 + 3 * h;
  s0[0] = w;
  s0[1] = 0.0;
  s0[2] = own ? -w * yj : 0.0;
  s1[0] = 0.0;
  s1[1] = w;
  s1[2] = own ? w * xj : 0.0;
}

// out[t] = scale * sum_p parts[p * stride + t], in two passes whose order is
// fixed (the result does not depend on timing).  Pass 1: block (tile, g) sums
// the parts g kPartsPerBlock .. (g + 1) kPartsPerBlock - 1 for the 64 outputs
// of its tile, wave w taking parts w, w + 4, ... of the range, the 4 wave sums
// added in order; the range sums go to scratch[g][t].  Pass 2 adds the range
// sums in order.
constexpr int kPartsPerBlock = 32;
__global__ __launch_bounds__(256) void k_sum_parts1(const double* parts, int nparts, long long stride,
                                                    int len, double* scratch) {
  __shared__ double sh[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int t = blockIdx.x * 64 + lane;
  const int p0 = blockIdx.y * kPartsPerBlock, p1 = min(nparts, p0 + kPartsPerBlock);
  double a = 0.0;
  if (t < len)
    for (int p = p0 + w; p < p1; p += 4) a += parts[(size_t)p * stride + t];
  sh[w][lane] = a;
  __syncthreads();
  if (w == 0 && t < len) scratch[(size_t)blockIdx.y * len + t] = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
}
__global__ void k_sum_parts2(const double* scratch, int ngroups, int len, double scale, double* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= len) return;
  double sum = 0.0;
  for (int g = 0; g < ngroups; ++g) sum += scratch[(size_t)g * len + t];
  out[t] = scale * sum;
}

constexpr int kBorderOuts = 12;      // outputs per thread of the unstaged border right-hand side
constexpr int kBorderLds = 24576;    // bytes of LDS for the staged rows of one block (several blocks per CU)

__host__ __device__ inline int round4(int v) { return (v + 3) & ~3; }

// Rows of a box staged in LDS per pass (3p and ncols padded to multiples of
// 4): a pass loads them with every thread of the block at once, so that many
// rows are in flight.  0 when a single row does not fit: the kernel then reads
// the rows from global memory directly (same summation order).
inline int border_tile(int p3, int ncols) {
  return std::min(32, kBorderLds / (8 * (round4(p3) + round4(ncols))));
}

// parts[box] (3p x ncols) = Ph_R^T c_R (accumulated in float64).  When the
// outputs are fewer than half the threads, the rows of R are split into
// nseg = kBlock / (3p ncols) interleaved segments (segment g takes rows
// g, g + nseg, ...), whose sums are added in segment order: the result
// depends on 3p and ncols only.  Otherwise the box's rows go through LDS in
// tiles and every thread accumulates a 4 x 4 block of outputs (4 consecutive
// h, 4 consecutive columns) in registers; with tile 0 every thread keeps
// kBorderOuts outputs (t, t + kBlock, ...) and reads global memory.  Each
// output sums the rows in order either way.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_border_rhs(const SolveBox* boxes, const int* ridx,
                                                       const T* Ph, int p3, const T* c, int ncols,
                                                       double* parts, int tile) {
  extern __shared__ __align__(16) double sh_rows[];
  __shared__ double seg[kBlock];
  const SolveBox& B = boxes[blockIdx.x];
  double* out = parts + (size_t)B.part * p3 * ncols;
  const int* R = ridx + B.r_off;
  const int nout = p3 * ncols;
  const int nseg = nout <= kBlock / 2 ? kBlock / nout : 1;
  if (nseg == 1 && tile > 0) {
    const int p3p = round4(p3), ncp = round4(ncols), nbq = ncp / 4, nblk = (p3p / 4) * nbq;
    double* sP = sh_rows;                        // tile x p3p
    double* sC = sh_rows + (size_t)tile * p3p;   // tile x ncp
    for (int b0 = 0; b0 < nblk; b0 += kBlock) {
      const int b = b0 + (int)threadIdx.x;
      const int h0 = 4 * (b / nbq), q0 = 4 * (b % nbq);
      double acc[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
      for (int i0 = 0; i0 < B.r; i0 += tile) {
        const int nt = min(tile, B.r - i0);
        __syncthreads();
        // one wavefront per row: coalesced, no index division
        for (int ii = threadIdx.x / 64; ii < nt; ii += kBlock / 64) {
          const size_t row = R[i0 + ii];
          for (int h = threadIdx.x % 64; h < p3p; h += 64)
            sP[ii * p3p + h] = h < p3 ? (double)Ph[row * p3 + h] : 0.0;
          for (int q = threadIdx.x % 64; q < ncp; q += 64)
            sC[ii * ncp + q] = q < ncols ? (double)c[row * ncols + q] : 0.0;
        }
        __syncthreads();
        if (b < nblk) {
          for (int ii = 0; ii < nt; ++ii) {
            const double4 pv = *reinterpret_cast<const double4*>(sP + (size_t)ii * p3p + h0);
            const double4 cv = *reinterpret_cast<const double4*>(sC + (size_t)ii * ncp + q0);
            const double pa[4] = {pv.x, pv.y, pv.z, pv.w}, ca[4] = {cv.x, cv.y, cv.z, cv.w};
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
              for (int v = 0; v < 4; ++v) acc[u][v] += pa[u] * ca[v];
          }
        }
      }
      if (b < nblk) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (h0 + u < p3 && q0 + v < ncols) out[(size_t)(h0 + u) * ncols + q0 + v] = acc[u][v];
      }
    }
    return;
  }
  if (nseg == 1) {
    for (int t0 = 0; t0 < nout; t0 += kBlock * kBorderOuts) {
      double acc[kBorderOuts];
      int hh[kBorderOuts], qq[kBorderOuts];
#pragma unroll
      for (int u = 0; u < kBorderOuts; ++u) {
        const int t = min(t0 + (int)threadIdx.x + u * kBlock, nout - 1);
        hh[u] = t / ncols;
        qq[u] = t % ncols;
        acc[u] = 0.0;
      }
      for (int i = 0; i < B.r; ++i) {
        const size_t r = R[i];
#pragma unroll
        for (int u = 0; u < kBorderOuts; ++u)
          acc[u] += (double)Ph[r * p3 + hh[u]] * (double)c[r * ncols + qq[u]];
      }
#pragma unroll
      for (int u = 0; u < kBorderOuts; ++u) {
        const int t = t0 + (int)threadIdx.x + u * kBlock;
        if (t < nout) out[t] = acc[u];
      }
    }
    return;
  }
  const int t = threadIdx.x, o = t % nout, g = t / nout;
  double acc = 0.0;
  if (g < nseg) {
    const int h = o / ncols, q = o % ncols;
    for (int i = g; i < B.r; i += nseg)
      acc += (double)Ph[(size_t)R[i] * p3 + h] * (double)c[(size_t)R[i] * ncols + q];
  }
  seg[t] = acc;
  __syncthreads();
  if (t < nout) {
    double sum = seg[t];
    for (int gg = 1; gg < nseg; ++gg) sum += seg[gg * nout + t];
    out[t] = sum;
  }
}

// c_R -= W lam.  The block stages lam (3p x 16 columns, zero-padded) in LDS
// and takes the box's rows of W in tiles of kFixRows rows by kFixK values of
// h (rows padded by one double against bank conflicts); the thread (row ii,
// column group g) accumulates 4 columns of row ii in registers, the sum over h
// in order.  With tile 0 (3p too large for LDS) the threads take the
// (row, column) pairs from global memory, in the same order over h.
constexpr int kFixCols = 16;
constexpr int kFixRows = kBlock / (kFixCols / 4);  // 64
constexpr int kFixK = 32;
template <typename T>
__global__ __launch_bounds__(kBlock) void k_border_fix(const SolveBox* boxes, const int* ridx,
                                                       int p3, const double* lam, T* c,
                                                       int ncols, int tile) {
  extern __shared__ __align__(16) double sh_rows[];
  const SolveBox& B = boxes[blockIdx.x];
  if (B.r == 0) return;
  const int* R = ridx + B.r_off;
  if (tile == 0) {
    for (int o = threadIdx.x; o < B.r * ncols; o += kBlock) {
      const int i = o / ncols, q = o % ncols;
      double acc = 0.0;
      if (B.Wf) {
        for (int h = 0; h < p3; ++h) acc += (double)B.Wf[(size_t)i * p3 + h] * lam[(size_t)h * ncols + q];
      } else {
        for (int h = 0; h < p3; ++h) acc += B.W[(size_t)i * p3 + h] * lam[(size_t)h * ncols + q];
      }
      c[(size_t)R[i] * ncols + q] -= (T)acc;
    }
    return;
  }
  double* sL = sh_rows;                              // 3p x kFixCols
  double* sW = sh_rows + (size_t)p3 * kFixCols;      // kFixRows x (kFixK + 1)
  const int ii = threadIdx.x % kFixRows, g = threadIdx.x / kFixRows;
  for (int q0 = 0; q0 < ncols; q0 += kFixCols) {
    const int nq = min(kFixCols, ncols - q0);
    __syncthreads();
    for (int e = threadIdx.x; e < p3 * kFixCols; e += kBlock) {
      const int h = e / kFixCols, k = e % kFixCols;
      sL[e] = k < nq ? lam[(size_t)h * ncols + q0 + k] : 0.0;
    }
    for (int i0 = 0; i0 < B.r; i0 += kFixRows) {
      const int nt = min(kFixRows, B.r - i0);
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < p3; k0 += kFixK) {
        const int kc = min(kFixK, p3 - k0);
        __syncthreads();
        for (int e = threadIdx.x; e < nt * kc; e += kBlock) {
          const int r = e / kc, kk = e % kc;
          const size_t src = (size_t)(i0 + r) * p3 + k0 + kk;
          sW[r * (kFixK + 1) + kk] = B.Wf ? (double)B.Wf[src] : B.W[src];
        }
        __syncthreads();
        if (ii < nt && 4 * g < nq) {
          const double* wr = sW + ii * (kFixK + 1);
          const double* lr = sL + (size_t)k0 * kFixCols + 4 * g;
          for (int kk = 0; kk < kc; ++kk) {
            const double w = wr[kk];
            const double4 lv = *reinterpret_cast<const double4*>(lr + (size_t)kk * kFixCols);
            acc[0] += w * lv.x;
            acc[1] += w * lv.y;
            acc[2] += w * lv.z;
            acc[3] += w * lv.w;
          }
        }
      }
      if (ii < nt) {
        T* crow = c + (size_t)R[i0 + ii] * ncols + q0 + 4 * g;
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (4 * g + v < nq) crow[v] -= (T)acc[v];
      }
    }
  }
}

// Z = [[X0, Hh(I0,:)], [Ph(I0,:)^T, -I - G]]
__global__ void k_assemble_Z(const double* X0, int n0, const double* Hh, const double* Ph,
                             const int* I0, int p3, const double* G, double* Z) {
  const int nz = n0 + p3;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nz * nz) return;
  const int i = (int)(t / nz), j = (int)(t % nz);
  double v;
  if (i < n0 && j < n0) v = X0[(size_t)i * n0 + j];
  else if (i < n0) v = Hh[(size_t)I0[i] * p3 + (j - n0)];
  else if (j < n0) v = Ph[(size_t)I0[j] * p3 + (i - n0)];
  else v = (i == j ? -1.0 : 0.0) - G[(size_t)(i - n0) * p3 + (j - n0)];
  Z[t] = v;
}

template <typename T>
__global__ void k_root_gather(const T* c, int ncols, const int* I0, int n0,
                              const double* rhs2, int p3, double* v) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (n0 + p3) * ncols) return;
  const int i = t / ncols, q = t % ncols;
  v[t] = i < n0 ? (double)c[(size_t)I0[i] * ncols + q] : rhs2[(size_t)(i - n0) * ncols + q];
}

// out = Zinv v (nz x ncols, rows layout): one wave per row of Zinv, lanes
// split the row (stride 64), 8 columns at a time, fixed-order wave sums.
__global__ __launch_bounds__(256) void k_dense_apply(const double* Zinv, int nz, const double* v,
                                                     int ncols, double* out) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= nz) return;   // uniform per wave
  const double* zr = Zinv + (size_t)i * nz;
  for (int q0 = 0; q0 < ncols; q0 += 8) {
    const int nq = min(8, ncols - q0);
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = 0.0;
    for (int j = lane; j < nz; j += 64) {
      const double z = zr[j];
      const double* vj = v + (size_t)j * ncols + q0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (u < nq) a[u] += z * vj[u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (u >= nq) break;
      const double sum = wave_sum(a[u]);
      if (lane == 0) out[(size_t)i * ncols + q0 + u] = sum;
    }
  }
}

template <typename T>
__global__ void k_root_scatter(const double* sol, int ncols, const int* I0, int n0, T* c) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n0 * ncols) return;
  const int i = t / ncols, q = t % ncols;
  c[(size_t)I0[i] * ncols + q] = (T)sol[t];
}

__global__ void k_fill(double* x, long long n, double v) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) x[t] = v;
}

// x += (double) d
template <typename TI>
__global__ void k_accumulate(const TI* d, long long n, double* x) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) x[t] += (double)d[t];
}

// Refinement control on the device (lets the refinement iterations run as a
// captured graph).  flag[0] = 1 once the certified residual is small enough,
// flag[1] counts the corrections applied, flag[2] = 1 when the next residual
// is updated with a float32 correction image, flag[3] = 1 once a correction
// image dropped a pair (the refinement then keeps to exact residuals).  Per
// iteration: k_accumulate_unless (reads the flags), operator apply, residual,
// then k_refine_flag (the only writer of flags 0-2: counts the correction the
// iteration applied, then tests the new residual).
//
// Certificate: after an exact residual the computed norm is the residual's
// norm (acc = 0); after an updated one the difference to the true residual is
// at most acc, the sum of the updates' rounding bounds bscale ||bt||_2, so
// column q passes when sqrt(colsq) + acc <= tol sqrt(fsq) (fsq = 0 counts as
// 1).  Updates continue (incr = 1) while acc stays within a quarter of the
// tolerance.
__global__ void k_refine_flag(const double* colsq, const double* fsq, const double* bsq, double* acc,
                              int ncols, double tol, int max_iters, int incr, double bscale, int* flag) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  if (flag[0] != 0 || flag[1] >= max_iters) return;   // the iteration was skipped
  flag[1] += 1;
  const bool upd = flag[2] == 1;
  const bool dropped = flag[3] != 0;
  bool next = incr != 0 && !dropped;
  double worst = 0.0;
  for (int q = 0; q < ncols; ++q) {
    const double fq = fsq[q] > 0.0 ? sqrt(fsq[q]) : 1.0;
    double a = 0.0;
    if (upd) a = dropped ? INFINITY : acc[q] + bscale * sqrt(bsq[q]);
    acc[q] = a;
    worst = fmax(worst, (sqrt(colsq[q]) + a) / fq);
    if (!(a <= 0.25 * tol * fq)) next = false;
  }
  flag[0] = worst <= tol ? 1 : 0;
  flag[2] = next ? 1 : 0;
}

// x += d unless refinement has converged or used up its iterations.
__global__ void k_accumulate_unless(const double* d, long long n, double* x, const int* flag,
                                    int max_iters) {
  if (flag[0] || flag[1] >= max_iters) return;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) x[t] += d[t];
}

__global__ void k_set_ints(int* p, int n, int v) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

// r = [f; 0] - y (or, when the refinement flags ask for an update, r = r - y
// with y the image of the correction) and the squared column norms of r and
// f, and for an update of the rounding bounds bt (one per node, both rows),
// in two passes of fixed order: block (c, q) takes rows c chunk .. (c + 1)
// chunk - 1 of column q and writes its sums to part[(q kResChunks + c) 3 +
// {0, 1, 2}]; the second pass adds each column's chunk sums in order.  A
// skipped refinement iteration leaves r and the norms as they are.
constexpr int kResChunks = 32;
__device__ __forceinline__ int residual_mode(const int* flag, int max_iters) {
  if (!flag) return 0;
  if (flag[0] != 0 || flag[1] >= max_iters) return -1;
  return flag[2] == 1 ? 1 : 0;
}
__global__ __launch_bounds__(kBlock) void k_residual1(const double* f, int nf, const double* y, int nrows,
                                                     int ncols, double* r, double* part, const int* flag,
                                                     int max_iters, const double* bt) {
  const int md = residual_mode(flag, max_iters);
  if (md < 0) return;
  constexpr int NW = kBlock / 64;
  __shared__ double red[NW];
  const int c = blockIdx.x, q = blockIdx.y;
  const int chunk = (nrows + kResChunks - 1) / kResChunks;
  const int i0 = c * chunk, i1 = min(nrows, i0 + chunk);
  double sr = 0.0, sf = 0.0, sb = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += kBlock) {
    const double fi = i < nf ? f[(size_t)i * ncols + q] : 0.0;
    const size_t k = (size_t)i * ncols + q;
    const double v = (md == 1 ? r[k] : fi) - y[k];
    r[k] = v;
    sr += v * v;
    sf += fi * fi;
    if (md == 1 && i < nf) {
      const double b = bt[(size_t)(i >> 1) * ncols + q];
      sb += b * b;
    }
  }
  sr = block_sum(sr, red);
  sf = block_sum(sf, red);
  sb = block_sum(sb, red);
  if (threadIdx.x == 0) {
    part[((size_t)q * kResChunks + c) * 3] = sr;
    part[((size_t)q * kResChunks + c) * 3 + 1] = sf;
    part[((size_t)q * kResChunks + c) * 3 + 2] = sb;
  }
}
__global__ void k_residual2(const double* part, int ncols, double* colsq, double* fsq, double* bsq,
                            const int* flag, int max_iters) {
  if (residual_mode(flag, max_iters) < 0) return;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ncols) return;
  double sr = 0.0, sf = 0.0, sb = 0.0;
  for (int c = 0; c < kResChunks; ++c) {
    sr += part[((size_t)q * kResChunks + c) * 3];
    sf += part[((size_t)q * kResChunks + c) * 3 + 1];
    sb += part[((size_t)q * kResChunks + c) * 3 + 2];
  }
  colsq[q] = sr;
  fsq[q] = sf;
  bsq[q] = sb;
}

// float copy of W (after the border stage) for the boxes whose solve reads
// float factors; boxes that keep float64 factors have no float W (Wf null)
__global__ void k_w_to_float(const SolveBox* boxes, int p3) {
  const SolveBox& B = boxes[blockIdx.x];
  if (!B.Wf) return;
  const int len = B.r * p3;
  for (int t = threadIdx.x; t < len; t += blockDim.x) B.Wf[t] = (float)B.W[t];
}

__global__ void k_to_rows(const double* f, int ld, int nrows, int ncols, double* c) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nrows * ncols) return;
  const int i = (int)(t / ncols), q = (int)(t % ncols);
  c[t] = f[(size_t)q * ld + i];
}

__global__ void k_from_rows(const double* c, int nrows, int ncols, double* x, int ld) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nrows * ncols) return;
  const int i = (int)(t / ncols), q = (int)(t % ncols);
  x[(size_t)q * ld + i] = c[t];
}

}  // namespace

// Columns per block of the sweep and diagonal kernels: at most kNC, within
// 64 KB of staged rows, and no more than the columns there are (the kernels'
// per-column work is not spent on padding).  When the boxes alone give fewer
// than kFillBlocks blocks (the upper levels), the columns are split further:
// a block's time is its rows x columns divided over 256 threads times the
// inner length, so narrower blocks finish sooner and run side by side.
constexpr int kFillBlocks = 512;
inline int chunk_cols(int rows, int ncols, int nbox) {
  int nc = kNC;
  while (nc > 1 && (size_t)rows * nc * sizeof(double) > 65536) nc >>= 1;
  nc = std::min(nc, std::max(ncols, 1));
  while (nc > 1 && (long long)nbox * blocks_for(ncols, nc) < kFillBlocks) nc >>= 1;
  return nc;
}

template <typename T>
void launch_sweep(const SolveBox* boxes, int nbox, const int* sidx, const int* ridx, T* c,
                  int ncols, int mode, int max_n, hipStream_t s) {
  if (nbox == 0 || ncols == 0) return;
  const int nc = chunk_cols(max_n, ncols, nbox);
  dim3 grid(nbox, blocks_for(ncols, nc));
  const size_t shm = (size_t)max_n * nc * sizeof(T);
  hipLaunchKernelGGL(k_sweep<T>, grid, dim3(kBlock), shm, s, boxes, sidx, ridx, c, ncols, mode, nc);
}
template void launch_sweep<double>(const SolveBox*, int, const int*, const int*, double*, int, int,
                                   int, hipStream_t);

template <typename T>
void launch_diag(const SolveBox* boxes, int nbox, const int* ridx, T* c, int ncols, int max_r,
                 hipStream_t s) {
  if (nbox == 0 || ncols == 0) return;
  // boxes beyond kDiagMaxR rows stage 2 r x nc values (the direct loop)
  const bool big = max_r > kDiagMaxR;
  const int nc = chunk_cols(big ? 2 * max_r : 0, ncols, nbox);
  dim3 grid(nbox, blocks_for(ncols, nc));
  const size_t shm = std::max(big ? (size_t)2 * max_r * nc * sizeof(T) : (size_t)0, (size_t)kDiagLds);
  hipLaunchKernelGGL(k_diag<T>, grid, dim3(kBlock), shm, s, boxes, ridx, c, ncols, nc);
}
template void launch_diag<double>(const SolveBox*, int, const int*, double*, int, int, hipStream_t);

void launch_assemble_H(Geo g, const double* hole_xy, int p, const int* curve_id, double* H,
                       double* Psi, hipStream_t s) {
  if (p == 0 || g.N == 0) return;
  hipLaunchKernelGGL(k_assemble_H, dim3(blocks_for((long long)g.N * p, kBlock)), dim3(kBlock), 0, s, g,
                     hole_xy, p, curve_id, H, Psi);
}

size_t sum_parts_scratch_doubles(int nparts, int len) {
  return (size_t)std::max(1, (nparts + kPartsPerBlock - 1) / kPartsPerBlock) * std::max(len, 1);
}

void launch_sum_parts(const double* parts, int nparts, long long stride, int len, double scale,
                      double* out, double* scratch, hipStream_t s) {
  if (len == 0) return;
  const int ng = std::max(1, (nparts + kPartsPerBlock - 1) / kPartsPerBlock);
  hipLaunchKernelGGL(k_sum_parts1, dim3(blocks_for(len, 64), ng), dim3(256), 0, s, parts, nparts, stride, len,
                     scratch);
  hipLaunchKernelGGL(k_sum_parts2, dim3(blocks_for(len, 256)), dim3(256), 0, s, scratch, ng, len, scale, out);
}

template <typename T>
void launch_border_rhs(const SolveBox* boxes, int nbox, const int* ridx, const T* Ph, int p3,
                       const T* c, int ncols, double* parts, hipStream_t s) {
  if (nbox == 0) return;
  const int tile = border_tile(p3, ncols);
  const size_t lds = (size_t)tile * (round4(p3) + round4(ncols)) * sizeof(double);
  hipLaunchKernelGGL(k_border_rhs<T>, dim3(nbox), dim3(kBlock), lds, s, boxes, ridx, Ph, p3, c, ncols,
                     parts, tile);
}
template void launch_border_rhs<double>(const SolveBox*, int, const int*, const double*, int,
                                        const double*, int, double*, hipStream_t);

template <typename T>
void launch_border_fix(const SolveBox* boxes, int nbox, const int* ridx, int p3, const double* lam,
                       T* c, int ncols, hipStream_t s) {
  if (nbox == 0) return;
  // lam's column block and a tile of W share 64 KiB of LDS; beyond that
  // (3p > 380) the kernel reads global memory
  const size_t lds = ((size_t)p3 * kFixCols + (size_t)kFixRows * (kFixK + 1)) * sizeof(double);
  const int tile = lds <= 65536 ? 1 : 0;
  hipLaunchKernelGGL(k_border_fix<T>, dim3(nbox), dim3(kBlock), tile ? lds : 0, s, boxes, ridx, p3, lam, c,
                     ncols, tile);
}
template void launch_border_fix<double>(const SolveBox*, int, const int*, int, const double*,
                                        double*, int, hipStream_t);

void launch_assemble_Z(const double* X0, int n0, const double* Hh, const double* Ph,
                       const int* I0, int p3, const double* G, double* Z, hipStream_t s) {
  const long long nz = n0 + p3;
  hipLaunchKernelGGL(k_assemble_Z, dim3(blocks_for(nz * nz, kBlock)), dim3(kBlock), 0, s, X0,
                     n0, Hh, Ph, I0, p3, G, Z);
}

template <typename T>
void launch_root_gather(const T* c, int ncols, const int* I0, int n0, const double* rhs2, int p3,
                        double* v, hipStream_t s) {
  hipLaunchKernelGGL(k_root_gather<T>, dim3(blocks_for((long long)(n0 + p3) * ncols, kBlock)),
                     dim3(kBlock), 0, s, c, ncols, I0, n0, rhs2, p3, v);
}
template void launch_root_gather<double>(const double*, int, const int*, int, const double*, int,
                                         double*, hipStream_t);

void launch_dense_apply(const double* Zinv, int nz, const double* v, int ncols, double* out,
                        hipStream_t s) {
  if (nz == 0 || ncols == 0) return;
  hipLaunchKernelGGL(k_dense_apply, dim3(blocks_for(nz, 4)), dim3(256), 0, s, Zinv, nz, v, ncols, out);
}

template <typename T>
void launch_root_scatter(const double* sol, int ncols, const int* I0, int n0, T* c, hipStream_t s) {
  hipLaunchKernelGGL(k_root_scatter<T>, dim3(blocks_for((long long)n0 * ncols, kBlock)),
                     dim3(kBlock), 0, s, sol, ncols, I0, n0, c);
}
template void launch_root_scatter<double>(const double*, int, const int*, int, double*, hipStream_t);

void launch_refine_flag(const double* colsq, const double* fsq, const double* bsq, double* acc, int ncols,
                        double tol, int max_iters, int incr, double bscale, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_refine_flag, dim3(1), dim3(64), 0, s, colsq, fsq, bsq, acc, ncols, tol, max_iters, incr,
                     bscale, flag);
}

void launch_accumulate_unless(const double* d, long long n, double* x, const int* flag, int max_iters,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_accumulate_unless, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, d, n, x,
                     flag, max_iters);
}

void launch_set_ints(int* p, int n, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_ints, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, p, n, v);
}

// Rows 2i + 1 (i < N) of a rows-layout block times `scale`: the Laplace Neumann
// kernel's uncoupled unknowns, whose diagonal entry lambda the solve divides by.
__global__ void k_scale_odd_rows(double* x, int N, int ncols, double scale) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)N * ncols) return;
  const long long i = t / ncols, q = t % ncols;
  x[(2 * i + 1) * ncols + q] *= scale;
}

void launch_scale_odd_rows(double* x, int N, int ncols, double scale, hipStream_t s) {
  const long long n = (long long)N * ncols;
  if (n) hipLaunchKernelGGL(k_scale_odd_rows, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, x, N, ncols, scale);
}

void launch_fill(double* x, long long n, double v, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, x, n, v);
}

void launch_accumulate(const double* d, long long n, double* x, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_accumulate<double>, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, d, n, x);
}

void launch_accumulate(const float* d, long long n, double* x, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_accumulate<float>, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, d, n, x);
}

size_t residual_scratch_doubles(int ncols) { return 3 * (size_t)kResChunks * std::max(ncols, 1); }

void launch_residual(const double* f, int nf, const double* y, int nrows, int ncols, double* r,
                     double* colsq, double* fsq, double* bsq, double* part, const int* flag, int max_iters,
                     const double* bt, hipStream_t s) {
  if (ncols == 0) return;
  hipLaunchKernelGGL(k_residual1, dim3(kResChunks, ncols), dim3(kBlock), 0, s, f, nf, y, nrows, ncols, r, part,
                     flag, max_iters, bt);
  hipLaunchKernelGGL(k_residual2, dim3(blocks_for(ncols, 64)), dim3(64), 0, s, part, ncols, colsq, fsq, bsq,
                     flag, max_iters);
}

void launch_w_to_float(const SolveBox* boxes, int nbox, int p3, hipStream_t s) {
  if (nbox) hipLaunchKernelGGL(k_w_to_float, dim3(nbox), dim3(kBlock), 0, s, boxes, p3);
}

void launch_to_rows(const double* f, int ld, int nrows, int ncols, double* c, hipStream_t s) {
  hipLaunchKernelGGL(k_to_rows, dim3(blocks_for((long long)nrows * ncols, kBlock)), dim3(kBlock),
                     0, s, f, ld, nrows, ncols, c);
}

void launch_from_rows(const double* c, int nrows, int ncols, double* x, int ld, hipStream_t s) {
  hipLaunchKernelGGL(k_from_rows, dim3(blocks_for((long long)nrows * ncols, kBlock)),
                     dim3(kBlock), 0, s, c, nrows, ncols, x, ld);
}

}  // namespace rs

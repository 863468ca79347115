// gfx950 kernels of the recursive-skeletonization factorization and solve
// (float64 path).
//
// Factorization of one level (Sections 2.2-2.7 of the paper):
//   k_assemble_M    the stacked ID matrix of every box: near field in both
//                   directions, proxy rows (eq. greens) and the two rows of
//                   the rank-one completion N (eq. null-spaceop)
//   k_cpqr          Householder QR with column pivoting to the ID tolerance
//                   (eq. lowrank): rank, pivot order and the leading rows of R
//   k_assemble_abb  the box's diagonal block in pivot order (children's X_SS
//                   on their own blocks, kernel entries elsewhere, eq.
//                   levelcompress)
//   k_eliminate     T = R11^{-1} R12, the ID transforms (eq. tmat), X_RR^{-1}
//                   with the conditioning guard, E, F and the Schur
//                   complement X_SS (eq. schurmat)
// Solve (eq. kinv, eq. partition):
//   k_sweep         U, V and Psi^T V sweeps, one launch per level
//   k_diag          X_RR^{-1} blocks
//   border/root     H, Psi^T, G, the reduced root system
// Residual:
//   k_apply_D / k_apply_psi   the exact float64 operator applied on the fly
#include "rs_internal.h"

#include <algorithm>
#include <cmath>

namespace rs {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kInvPi = 0.31830988618379067154;
constexpr double kInv4Pi = 0.07957747154594766788;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum over the block in a fixed order (deterministic); every thread gets it.
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = blockDim.x >> 6;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

__device__ double block_max(double v, double* red) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = red[0];
  const int nw = blockDim.x >> 6;
  for (int i = 1; i < nw; ++i) s = fmax(s, red[i]);
  return s;
}

// ---- kernel functions -----------------------------------------------------

// Stresslet double layer, eq. (stokesbie): w/pi ((x-y).n_y)/|x-y|^4 r_a r_b.
__device__ __forceinline__ double dl_entry(double rx, double ry, double nx, double ny,
                                           double w, int a, int b) {
  const double r2 = rx * rx + ry * ry;
  const double rn = rx * nx + ry * ny;
  const double coef = kInvPi * w * rn / (r2 * r2);
  return coef * (a ? ry : rx) * (b ? ry : rx);
}

// Stokeslet, (w/4pi) (-ln|r| delta_ab + r_a r_b / |r|^2).
__device__ __forceinline__ double sl_entry(double rx, double ry, double w, int a, int b) {
  const double r2 = rx * rx + ry * ry;
  double v = (a ? ry : rx) * (b ? ry : rx) / r2;
  if (a == b) v += -0.5 * log(r2);
  return kInv4Pi * w * v;
}

// Entry of lam I + D + N between unknown (ti, tc) (target node, component)
// and (sj, sc).  Coincident nodes use the curvature limit of D.
__device__ __forceinline__ double op_entry(const Geo& g, int ti, int tc, int sj, int sc,
                                           double lam) {
  double v;
  if (ti == sj) {
    const double tx = -g.ny[ti], ty = g.nx[ti];
    const double c = -(g.w[ti] * g.kap[ti]) / (2.0 * kPi);
    v = c * (tc ? ty : tx) * (sc ? ty : tx);
    if (tc == sc) v += lam;
  } else {
    v = dl_entry(g.x[ti] - g.x[sj], g.y[ti] - g.y[sj], g.nx[sj], g.ny[sj], g.w[sj], tc, sc);
  }
  const double nt = tc ? g.ny[ti] : g.nx[ti];
  const double ns = sc ? g.ny[sj] : g.nx[sj];
  return v + nt * (g.w[sj] * ns);
}

// ---- block-level dense helpers (row-major, global memory) ----------------

// C = beta*C0 + alpha*op(A) op(B); op(A) is M x K, op(B) K x N.  C0 may be C.
__device__ void wg_gemm(int M, int N, int K, double alpha, const double* A, int lda, bool tA,
                        const double* B, int ldb, bool tB, double beta, const double* C0,
                        int ldc0, double* C, int ldc) {
  const int tm = (M + 3) >> 2, tn = (N + 3) >> 2;
  for (int t = threadIdx.x; t < tm * tn; t += blockDim.x) {
    const int i0 = (t / tn) << 2, j0 = (t % tn) << 2;
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
    for (int kk = 0; kk < K; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + u;
        a[u] = (i < M) ? (tA ? A[(size_t)kk * lda + i] : A[(size_t)i * lda + kk]) : 0.0;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = j0 + v;
        b[v] = (j < N) ? (tB ? B[(size_t)j * ldb + kk] : B[(size_t)kk * ldb + j]) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u;
      if (i >= M) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = j0 + v;
        if (j >= N) continue;
        double val = alpha * acc[u][v];
        if (C0) val += beta * C0[(size_t)i * ldc0 + j];
        C[(size_t)i * ldc + j] = val;
      }
    }
  }
  __syncthreads();
}

// T (k x r, ld r) = R11^{-1} R12 with R11 = R[0:k,0:k], R12 = R[0:k,k:k+r] (ld ldr).
__device__ void wg_trsm_upper(const double* R, int ldr, int k, int r, double* T) {
  for (int c = threadIdx.x; c < r; c += blockDim.x) {
    for (int i = k - 1; i >= 0; --i) {
      double s = R[(size_t)i * ldr + k + c];
      for (int l = i + 1; l < k; ++l) s -= R[(size_t)i * ldr + l] * T[(size_t)l * r + c];
      T[(size_t)i * r + c] = s / R[(size_t)i * ldr + i];
    }
  }
  __syncthreads();
}

// Gauss-Jordan inverse with partial pivoting.  X (n x n, ld ldx) is kept;
// W is n x n work; Xi (ld ldi) receives X^{-1}.  Returns the reciprocal
// 1-norm condition number (0 if a pivot vanished), identical in all threads.
__device__ double wg_gj_inverse(const double* X, int n, int ldx, double* Xi, int ldi, double* W,
                                double* colbuf, double* red, int* ired) {
  const int tid = threadIdx.x, NT = blockDim.x;
  for (int t = tid; t < n * n; t += NT) {
    const int i = t / n, c = t % n;
    W[t] = X[(size_t)i * ldx + c];
    Xi[(size_t)i * ldi + c] = (i == c) ? 1.0 : 0.0;
  }
  double n1 = 0.0;
  for (int c = tid; c < n; c += NT) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += fabs(X[(size_t)i * ldx + c]);
    n1 = fmax(n1, s);
  }
  n1 = block_max(n1, red);
  __syncthreads();
  bool singular = false;
  for (int j = 0; j < n; ++j) {
    // pivot row: largest |W[i][j]|, i >= j; ties to the smaller row
    double best = -1.0;
    int bi = n;
    for (int i = j + tid; i < n; i += NT) {
      const double v = fabs(W[(size_t)i * n + j]);
      if (v > best) { best = v; bi = i; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    const int lane = tid & 63, wid = tid >> 6;
    __syncthreads();
    if (lane == 0) { red[wid] = best; ired[wid] = bi; }
    __syncthreads();
    best = red[0];
    bi = ired[0];
    for (int w = 1; w < (NT >> 6); ++w)
      if (red[w] > best || (red[w] == best && ired[w] < bi)) { best = red[w]; bi = ired[w]; }
    if (!(best > 0.0)) { singular = true; break; }
    if (bi != j) {
      for (int c = tid; c < n; c += NT) {
        double a = W[(size_t)j * n + c];
        W[(size_t)j * n + c] = W[(size_t)bi * n + c];
        W[(size_t)bi * n + c] = a;
        double b = Xi[(size_t)j * ldi + c];
        Xi[(size_t)j * ldi + c] = Xi[(size_t)bi * ldi + c];
        Xi[(size_t)bi * ldi + c] = b;
      }
    }
    __syncthreads();
    const double inv = 1.0 / W[(size_t)j * n + j];
    __syncthreads();
    for (int c = tid; c < n; c += NT) {
      W[(size_t)j * n + c] *= inv;
      Xi[(size_t)j * ldi + c] *= inv;
    }
    __syncthreads();
    for (int i = tid; i < n; i += NT) colbuf[i] = W[(size_t)i * n + j];
    __syncthreads();
    const int span = n - j;
    for (int t = tid; t < n * span; t += NT) {
      const int i = t / span, c = j + t % span;
      if (i == j) continue;
      const double f = colbuf[i];
      if (f != 0.0) W[(size_t)i * n + c] -= f * W[(size_t)j * n + c];
    }
    for (int t = tid; t < n * n; t += NT) {
      const int i = t / n, c = t % n;
      if (i == j) continue;
      const double f = colbuf[i];
      if (f != 0.0) Xi[(size_t)i * ldi + c] -= f * Xi[(size_t)j * ldi + c];
    }
    __syncthreads();
  }
  if (singular) return 0.0;
  double n2 = 0.0;
  for (int c = tid; c < n; c += NT) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += fabs(Xi[(size_t)i * ldi + c]);
    n2 = fmax(n2, s);
  }
  n2 = block_max(n2, red);
  __syncthreads();
  const double rc = 1.0 / (n1 * n2);
  return isfinite(rc) ? rc : 0.0;
}

// ---- factorization kernels -------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_assemble_M(const LevelBox* boxes, const int* dofs,
                                                       const int* fint, Geo g, int n_proxy,
                                                       double ratio) {
  const LevelBox& B = boxes[blockIdx.x];
  const int i = blockIdx.y * blockDim.x + threadIdx.x;
  const int m = B.m, n = B.n, nF = B.nF;
  if (i >= m || n == 0) return;
  const int* I = dofs + B.dof_off;
  const int np2 = 2 * n_proxy;
  const double rp = ratio * B.side;
  const double wp = 2.0 * kPi * rp / n_proxy;
  int type, f = 0, pa = 0;
  double px = 0, py = 0, pnx = 0, pny = 0;
  if (i < nF) {
    type = 0;
    f = fint[B.fint_off + i];
  } else if (i < 2 * nF) {
    type = 1;
    f = fint[B.fint_off + i - nF];
  } else if (i < 2 * nF + 3 * np2) {
    const int t = i - 2 * nF;
    type = 2 + t / np2;
    const int u = t % np2;
    const int pk = u >> 1;
    pa = u & 1;
    const double th = 2.0 * kPi * pk / n_proxy;
    pnx = cos(th);
    pny = sin(th);
    px = B.cx + rp * pnx;
    py = B.cy + rp * pny;
  } else {
    type = 5 + (i - 2 * nF - 3 * np2);
  }
  const int fj = f >> 1, fc = f & 1;
  for (int c = 0; c < n; ++c) {
    const int d = I[c];
    const int j = d >> 1, jc = d & 1;
    double v;
    switch (type) {
      case 0: v = op_entry(g, fj, fc, j, jc, 0.0); break;
      case 1: v = op_entry(g, j, jc, fj, fc, 0.0); break;
      case 2: v = dl_entry(px - g.x[j], py - g.y[j], g.nx[j], g.ny[j], g.w[j], pa, jc); break;
      case 3: v = dl_entry(g.x[j] - px, g.y[j] - py, pnx, pny, wp, jc, pa); break;
      case 4: v = sl_entry(g.x[j] - px, g.y[j] - py, wp, jc, pa); break;
      case 5: v = g.w[j] * (jc ? g.ny[j] : g.nx[j]); break;
      default: v = jc ? g.ny[j] : g.nx[j]; break;
    }
    B.M[(size_t)c * m + i] = v;
  }
}

// Pivoted Householder QR of M_B (m x n, column-major), one block per box.
// Pivot: largest remaining column norm (recomputed exactly after every
// step), ties to the column that came first in I_B.  Runs until the first
// step with |R_jj| <= tol |R_11| plus `extra` further steps (head-room for
// the X_RR guard).  Writes perm (pivot order of positions in I_B), the
// tolerance rank k and the number of R rows kept, R in pivot order.
// The Householder vector lives in LDS; each trailing column is read once
// into registers (rows lane + 64 u), updated and written back, and its new
// norm is formed in the same pass.
constexpr int kQRThreads = 512;
constexpr int kQRRows = 32;             // rows per lane held in registers (m <= 2048)

__global__ __launch_bounds__(kQRThreads) void k_cpqr(const LevelBox* boxes, double tol, int extra,
                                                     int* perm_out, int* k_out, int* kx_out) {
  extern __shared__ double smem[];
  const LevelBox& B = boxes[blockIdx.x];
  const int m = B.m, n = B.n;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  constexpr int NW = kQRThreads / 64;
  __shared__ double red[NW];
  __shared__ double bval[NW];
  __shared__ int bperm[NW];
  __shared__ int bpos[NW];
  if (n == 0) {
    if (tid == 0) { k_out[blockIdx.x] = 0; kx_out[blockIdx.x] = 0; }
    return;
  }
  double* nrm = smem;              // n
  double* rdiag = smem + n;        // n
  double* vsh = smem + 2 * n;      // m
  int* pv = (int*)(smem + 2 * n + m);  // n
  double* A = B.M;
  const bool regs = m <= 64 * kQRRows;
  for (int c = wid; c < n; c += NW) {
    const double* col = A + (size_t)c * m;
    double sum = 0.0;
    for (int i = lane; i < m; i += 64) {
      const double a = col[i];
      sum += a * a;
    }
    sum = wave_sum(sum);
    if (lane == 0) { nrm[c] = sum; pv[c] = c; }
  }
  __syncthreads();
  const int steps = min(m, n);
  int limit = steps;
  int kk = -1;
  double r00 = 0.0;
  int j = 0;
  for (; j < limit; ++j) {
    double best = -1.0;
    int bp = 1 << 30, bq = -1;
    for (int c = j + tid; c < n; c += kQRThreads) {
      const double v = nrm[c];
      const int p = pv[c];
      if (v > best || (v == best && p < bp)) { best = v; bp = p; bq = c; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o, 64);
      const int op = __shfl_xor(bp, o, 64);
      const int oq = __shfl_xor(bq, o, 64);
      if (ov > best || (ov == best && op < bp)) { best = ov; bp = op; bq = oq; }
    }
    if (lane == 0) { bval[wid] = best; bperm[wid] = bp; bpos[wid] = bq; }
    __syncthreads();
    if (tid == 0) {
      double bv = bval[0];
      int bpp = bperm[0], bqq = bpos[0];
      for (int w = 1; w < NW; ++w)
        if (bval[w] > bv || (bval[w] == bv && bperm[w] < bpp)) { bv = bval[w]; bpp = bperm[w]; bqq = bpos[w]; }
      if (bqq != j) {
        const double t = nrm[j]; nrm[j] = nrm[bqq]; nrm[bqq] = t;
        const int u = pv[j]; pv[j] = pv[bqq]; pv[bqq] = u;
      }
    }
    __syncthreads();
    const double* x = A + (size_t)pv[j] * m;
    double sum = 0.0;
    for (int i = j + 1 + tid; i < m; i += kQRThreads) {
      const double a = x[i];
      vsh[i] = a;
      sum += a * a;
    }
    sum = block_sum(sum, red);
    const double alpha = x[j];
    double beta, tau;
    if (sum == 0.0) {
      beta = alpha;
      tau = 0.0;
    } else {
      beta = -copysign(sqrt(alpha * alpha + sum), alpha);
      tau = (beta - alpha) / beta;
      const double scal = 1.0 / (alpha - beta);
      for (int i = j + 1 + tid; i < m; i += kQRThreads) vsh[i] *= scal;
    }
    if (tid == 0) rdiag[j] = beta;
    __syncthreads();
    const double rjj = fabs(beta);
    if (j == 0) r00 = rjj;
    if (kk < 0 && !(rjj > tol * r00)) {
      kk = j;
      limit = min(steps, j + 1 + extra);
    }
    if (regs) {
      for (int c = j + 1 + wid; c < n; c += NW) {
        double* y = A + (size_t)pv[c] * m;
        const double yj = y[j];
        double yr[kQRRows];
        double ws = 0.0;
#pragma unroll
        for (int u = 0; u < kQRRows; ++u) {
          const int i = lane + 64 * u;
          yr[u] = (i > j && i < m) ? y[i] : 0.0;
          ws += (i > j && i < m) ? vsh[i] * yr[u] : 0.0;
        }
        ws = wave_sum(ws) + yj;
        const double tw = tau * ws;
        double ns = 0.0;
#pragma unroll
        for (int u = 0; u < kQRRows; ++u) {
          const int i = lane + 64 * u;
          if (i > j && i < m) {
            const double v = yr[u] - tw * vsh[i];
            y[i] = v;
            ns += v * v;
          }
        }
        ns = wave_sum(ns);
        if (lane == 0) {
          y[j] = yj - tw;
          nrm[c] = ns;
        }
      }
    } else {
      for (int c = j + 1 + wid; c < n; c += NW) {
        double* y = A + (size_t)pv[c] * m;
        const double yj = y[j];
        double ws = 0.0;
        for (int i = j + 1 + lane; i < m; i += 64) ws += vsh[i] * y[i];
        ws = wave_sum(ws) + yj;
        const double tw = tau * ws;
        double ns = 0.0;
        for (int i = j + 1 + lane; i < m; i += 64) {
          const double v = y[i] - tw * vsh[i];
          y[i] = v;
          ns += v * v;
        }
        ns = wave_sum(ns);
        if (lane == 0) {
          y[j] = yj - tw;
          nrm[c] = ns;
        }
      }
    }
    __syncthreads();
  }
  const int kx = j;
  if (kk < 0) kk = kx;
  for (int t = tid; t < kx * n; t += kQRThreads) {
    const int r = t / n, c = t % n;
    double v;
    if (c < r) v = 0.0;
    else if (c == r) v = rdiag[r];
    else v = A[(size_t)pv[c] * m + r];
    B.R[t] = v;
  }
  for (int c = tid; c < n; c += kQRThreads) perm_out[B.dof_off + c] = pv[c];
  if (tid == 0) { k_out[blockIdx.x] = kk; kx_out[blockIdx.x] = kx; }
}

__global__ __launch_bounds__(kBlock) void k_assemble_abb(const LevelBox* boxes, const int* dofs,
                                                         const int* perm, const ChildSrc* src,
                                                         Geo g, double lam) {
  const LevelBox& B = boxes[blockIdx.x];
  const int n = B.n;
  const int t = blockIdx.y * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  const int i = t / n, j = t % n;
  const int pi = perm ? perm[B.dof_off + i] : i;
  const int pj = perm ? perm[B.dof_off + j] : j;
  if (B.src_off >= 0) {
    const ChildSrc& si = src[B.src_off + pi];
    const ChildSrc& sj = src[B.src_off + pj];
    if (si.child == sj.child) {
      B.Ap[t] = si.xss[(size_t)si.idx * si.ld + sj.idx];
      return;
    }
  }
  const int di = dofs[B.dof_off + pi], dj = dofs[B.dof_off + pj];
  B.Ap[t] = op_entry(g, di >> 1, di & 1, dj >> 1, dj & 1, lam);
}

__global__ __launch_bounds__(kBlock) void k_eliminate(const LevelBox* boxes, int* k_io,
                                                      const int* kx_in, double rcond_min,
                                                      int* status) {
  extern __shared__ double smem[];
  constexpr int NW = kBlock / 64;
  __shared__ double red[NW];
  __shared__ int ired[NW];
  const LevelBox& B = boxes[blockIdx.x];
  const int n = B.n;
  if (n == 0) return;
  int k = k_io[blockIdx.x];
  const int kx = kx_in[blockIdx.x];
  int st = 0;
  const double* Ap = B.Ap;
  while (true) {
    const int r = n - k;
    double* T = B.T;
    wg_trsm_upper(B.R, n, k, r, T);
    if (r == 0) {
      for (int t = threadIdx.x; t < k * k; t += kBlock) {
        const int i = t / k, c = t % k;
        B.Xss[t] = Ap[(size_t)i * n + c];
      }
      break;
    }
    double* Xsr = B.scr;
    double* Xrs = Xsr + (size_t)k * r;
    double* Xrr = Xrs + (size_t)r * k;
    double* Wk = Xrr + (size_t)r * r;
    wg_gemm(k, r, k, -1.0, Ap, n, false, T, r, false, 1.0, Ap + k, n, Xsr, r);
    wg_gemm(r, k, k, -1.0, T, r, true, Ap, n, false, 1.0, Ap + (size_t)k * n, n, Xrs, k);
    wg_gemm(r, r, k, -1.0, Ap + (size_t)k * n, n, false, T, r, false, 1.0,
            Ap + (size_t)k * n + k, n, Xrr, r);
    wg_gemm(r, r, k, -1.0, T, r, true, Xsr, r, false, 1.0, Xrr, r, Xrr, r);
    const double rc = wg_gj_inverse(Xrr, r, r, B.Xinv, r, Wk, smem, red, ired);
    if (!(rc >= rcond_min)) {
      if (k < kx) {
        ++k;
        continue;
      }
      st = 1;
    }
    wg_gemm(k, r, r, 1.0, Xsr, r, false, B.Xinv, r, false, 0.0, nullptr, 0, B.E, r);
    wg_gemm(r, k, r, 1.0, B.Xinv, r, false, Xrs, k, false, 0.0, nullptr, 0, B.F, k);
    wg_gemm(k, k, r, -1.0, Xsr, r, false, B.F, k, false, 1.0, Ap, n, B.Xss, k);
    break;
  }
  if (threadIdx.x == 0) {
    k_io[blockIdx.x] = k;
    status[blockIdx.x] = st;
  }
}

__global__ __launch_bounds__(kBlock) void k_gj_inverse(double* A, int n, int lda, double* Ainv,
                                                       double* work, double* rcond_out,
                                                       int* status) {
  extern __shared__ double smem[];
  constexpr int NW = kBlock / 64;
  __shared__ double red[NW];
  __shared__ int ired[NW];
  const double rc = wg_gj_inverse(A, n, lda, Ainv, n, work, smem, red, ired);
  if (threadIdx.x == 0) {
    *rcond_out = rc;
    *status = rc > 0.0 ? 0 : 1;
  }
}

// ---- blocked in-place Gauss-Jordan inverse (root system) ----------------------
// A (n x n, row-major) is overwritten by the inverse of P A, where P is the
// row permutation chosen by partial pivoting (recorded in rowperm); a final
// column scatter yields A^{-1}.  Per block of b pivot columns K:
//   panel:  LU with partial pivoting of A[k0:n, K] picks the pivot rows and
//           gives D^{-1} for the pivot block D (after the row swaps);
//   swap:   the b row interchanges over all columns, copy of the column block;
//   rows:   R = D^{-1} A[K, :];
//   update: A[K,K] = D^{-1}, A[K,~K] = R, A[~K,K] = -A[~K,K] D^{-1},
//           A[~K,~K] -= A[~K,K] R.
constexpr int kGJB = 32;

__global__ __launch_bounds__(kBlock) void k_gjb_panel(const double* A, int n, int k0, int bb,
                                                      double* W, int* piv, double* Dinv,
                                                      int* status) {
  constexpr int NW = kBlock / 64;
  __shared__ double red[NW];
  __shared__ int ired[NW];
  __shared__ double lu[kGJB][kGJB + 1];
  __shared__ double inv[kGJB][kGJB + 1];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int h = n - k0;
  for (int t = tid; t < h * bb; t += kBlock) {
    const int i = t / bb, c = t % bb;
    W[t] = A[(size_t)(k0 + i) * n + k0 + c];
  }
  __syncthreads();
  bool singular = false;
  for (int j = 0; j < bb; ++j) {
    double best = -1.0;
    int bi = h;
    for (int i = j + tid; i < h; i += kBlock) {
      const double v = fabs(W[(size_t)i * bb + j]);
      if (v > best) { best = v; bi = i; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if (lane == 0) { red[wid] = best; ired[wid] = bi; }
    __syncthreads();
    best = red[0];
    bi = ired[0];
    for (int w = 1; w < NW; ++w)
      if (red[w] > best || (red[w] == best && ired[w] < bi)) { best = red[w]; bi = ired[w]; }
    __syncthreads();
    if (!(best > 0.0)) { singular = true; break; }
    if (tid == 0) piv[j] = bi;
    if (bi != j)
      for (int c = tid; c < bb; c += kBlock) {
        const double a = W[(size_t)j * bb + c];
        W[(size_t)j * bb + c] = W[(size_t)bi * bb + c];
        W[(size_t)bi * bb + c] = a;
      }
    __syncthreads();
    const double d = W[(size_t)j * bb + j];
    for (int i = j + 1 + tid; i < h; i += kBlock) W[(size_t)i * bb + j] /= d;
    __syncthreads();
    const int rest = bb - j - 1;
    if (rest > 0)
      for (int t = tid; t < (h - j - 1) * rest; t += kBlock) {
        const int i = j + 1 + t / rest, c = j + 1 + t % rest;
        W[(size_t)i * bb + c] -= W[(size_t)i * bb + j] * W[(size_t)j * bb + c];
      }
    __syncthreads();
  }
  if (singular) {
    if (tid == 0) *status = 1;
    return;
  }
  // D = L U (first bb rows of W); D^{-1} = U^{-1} L^{-1}
  for (int t = tid; t < bb * bb; t += kBlock) lu[t / bb][t % bb] = W[t];
  __syncthreads();
  // columns of L^{-1} (unit lower) then U^{-1} applied: one thread per column
  if (tid < bb) {
    const int c = tid;
    double y[kGJB];
    for (int i = 0; i < bb; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int l = 0; l < i; ++l) s -= lu[i][l] * y[l];
      y[i] = s;
    }
    for (int i = bb - 1; i >= 0; --i) {
      double s = y[i];
      for (int l = i + 1; l < bb; ++l) s -= lu[i][l] * y[l];
      y[i] = s / lu[i][i];
    }
    for (int i = 0; i < bb; ++i) inv[i][c] = y[i];
  }
  __syncthreads();
  for (int t = tid; t < bb * bb; t += kBlock) Dinv[t] = inv[t / bb][t % bb];
}

// Row interchanges of this block over all columns; copy of the column block.
__global__ void k_gjb_swap(double* A, int n, int k0, int bb, const int* piv, int* rowperm,
                           double* Cpanel) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) {
    for (int j = 0; j < bb; ++j) {
      const int r = k0 + piv[j];
      if (r != k0 + j) {
        const double a = A[(size_t)(k0 + j) * n + c];
        A[(size_t)(k0 + j) * n + c] = A[(size_t)r * n + c];
        A[(size_t)r * n + c] = a;
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int j = 0; j < bb; ++j) {
      const int r = k0 + piv[j];
      const int t = rowperm[k0 + j];
      rowperm[k0 + j] = rowperm[r];
      rowperm[r] = t;
    }
  }
}

__global__ void k_gjb_copycol(const double* A, int n, int k0, int bb, double* Cpanel) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * bb) return;
  const int i = t / bb, c = t % bb;
  Cpanel[t] = A[(size_t)i * n + k0 + c];
}

// R = D^{-1} A[K, :]
__global__ void k_gjb_rows(const double* A, int n, int k0, int bb, const double* Dinv, double* R) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= bb * n) return;
  const int i = t / n, c = t % n;
  double s = 0.0;
  for (int l = 0; l < bb; ++l) s += Dinv[i * bb + l] * A[(size_t)(k0 + l) * n + c];
  R[t] = s;
}

__global__ void k_gjb_update(double* A, int n, int k0, int bb, const double* Dinv,
                             const double* R, const double* Cpanel) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * n) return;
  const int i = (int)(t / n), c = (int)(t % n);
  const bool ik = i >= k0 && i < k0 + bb;
  const bool ck = c >= k0 && c < k0 + bb;
  double v;
  if (ik) {
    v = ck ? Dinv[(i - k0) * bb + (c - k0)] : R[(size_t)(i - k0) * n + c];
  } else if (ck) {
    double s = 0.0;
    for (int l = 0; l < bb; ++l) s += Cpanel[(size_t)i * bb + l] * Dinv[l * bb + (c - k0)];
    v = -s;
  } else {
    double s = 0.0;
    for (int l = 0; l < bb; ++l) s += Cpanel[(size_t)i * bb + l] * R[(size_t)l * n + c];
    v = A[t] - s;
  }
  A[t] = v;
}

// out[:, rowperm[i]] = A[:, i]  (undo the row permutation of the input)
__global__ void k_gjb_unpermute(const double* A, int n, const int* rowperm, double* out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * n) return;
  const int i = (int)(t / n), c = (int)(t % n);
  out[(size_t)i * n + rowperm[c]] = A[t];
}

__global__ void k_iota(int* v, int n, int* zero) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) v[t] = t;
  if (t == 0) *zero = 0;
}

// ---- solve kernels -----------------------------------------------------------

// mode 0: U   c_R -= T^T c_S ; c_S -= E c_R
// mode 1: Psi^T V rows (columns of Psi)   c_R -= T^T c_S ; c_S -= F^T c_R
// mode 2: V   c_R -= F c_S ; c_S -= T c_R
__global__ __launch_bounds__(kBlock) void k_sweep(const SolveBox* boxes, const int* sidx,
                                                  const int* ridx, double* c, int ncols,
                                                  int mode, int kNC) {
  extern __shared__ double smem[];
  const SolveBox& B = boxes[blockIdx.x];
  const int k = B.k, r = B.r;
  if (k == 0 || r == 0) return;
  const int q0 = blockIdx.y * kNC;
  const int nq = min(kNC, ncols - q0);
  double* cs = smem;
  double* cr = smem + (size_t)k * kNC;
  const int* S = sidx + B.s_off;
  const int* R = ridx + B.r_off;
  const int tid = threadIdx.x;
  for (int t = tid; t < k * kNC; t += kBlock) {
    const int s = t / kNC, q = t % kNC;
    cs[t] = q < nq ? c[(size_t)S[s] * ncols + q0 + q] : 0.0;
  }
  for (int t = tid; t < r * kNC; t += kBlock) {
    const int i = t / kNC, q = t % kNC;
    cr[t] = q < nq ? c[(size_t)R[i] * ncols + q0 + q] : 0.0;
  }
  __syncthreads();
  if (mode != 2) {
    for (int t = tid; t < r * kNC; t += kBlock) {
      const int i = t / kNC, q = t % kNC;
      double acc = 0.0;
      for (int s = 0; s < k; ++s) acc += B.T[(size_t)s * r + i] * cs[s * kNC + q];
      cr[t] -= acc;
    }
    __syncthreads();
    for (int t = tid; t < k * kNC; t += kBlock) {
      const int s = t / kNC, q = t % kNC;
      double acc = 0.0;
      if (mode == 0)
        for (int i = 0; i < r; ++i) acc += B.E[(size_t)s * r + i] * cr[i * kNC + q];
      else
        for (int i = 0; i < r; ++i) acc += B.F[(size_t)i * k + s] * cr[i * kNC + q];
      cs[t] -= acc;
    }
  } else {
    for (int t = tid; t < r * kNC; t += kBlock) {
      const int i = t / kNC, q = t % kNC;
      double acc = 0.0;
      for (int s = 0; s < k; ++s) acc += B.F[(size_t)i * k + s] * cs[s * kNC + q];
      cr[t] -= acc;
    }
    __syncthreads();
    for (int t = tid; t < k * kNC; t += kBlock) {
      const int s = t / kNC, q = t % kNC;
      double acc = 0.0;
      for (int i = 0; i < r; ++i) acc += B.T[(size_t)s * r + i] * cr[i * kNC + q];
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

// c_R <- X_RR^{-1} c_R
__global__ __launch_bounds__(kBlock) void k_diag(const SolveBox* boxes, const int* ridx,
                                                 double* c, int ncols, int kNC) {
  extern __shared__ double smem[];
  const SolveBox& B = boxes[blockIdx.x];
  const int r = B.r;
  if (r == 0) return;
  const int q0 = blockIdx.y * kNC;
  const int nq = min(kNC, ncols - q0);
  double* in = smem;
  double* out = smem + (size_t)r * kNC;
  const int* R = ridx + B.r_off;
  for (int t = threadIdx.x; t < r * kNC; t += kBlock) {
    const int i = t / kNC, q = t % kNC;
    in[t] = q < nq ? c[(size_t)R[i] * ncols + q0 + q] : 0.0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < r * kNC; t += kBlock) {
    const int i = t / kNC, q = t % kNC;
    double acc = 0.0;
    for (int j = 0; j < r; ++j) acc += B.Xinv[(size_t)i * r + j] * in[j * kNC + q];
    out[t] = acc;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < r * kNC; t += kBlock) {
    const int i = t / kNC, q = t % kNC;
    if (q < nq) c[(size_t)R[i] * ncols + q0 + q] = out[t];
  }
}

// H (2N x 3p) and Psi (2N x 3p, i.e. Psi^T stored by columns), row-major.
__global__ void k_assemble_H(Geo g, const double* hole_xy, int p, const int* curve_id,
                             double* H, double* Psi) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= g.N) return;
  const int p3 = 3 * p;
  const double xj = g.x[j], yj = g.y[j];
  for (int h = 0; h < p; ++h) {
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
  }
  for (int t = 0; t < p3; ++t) {
    Psi[(size_t)(2 * j) * p3 + t] = 0.0;
    Psi[(size_t)(2 * j + 1) * p3 + t] = 0.0;
  }
  const int cid = curve_id[j];
  if (cid > 0) {
    const int h = cid - 1;
    const double w = g.w[j];
    Psi[(size_t)(2 * j) * p3 + 3 * h + 0] = w;
    Psi[(size_t)(2 * j + 1) * p3 + 3 * h + 1] = w;
    Psi[(size_t)(2 * j) * p3 + 3 * h + 2] = -w * yj;
    Psi[(size_t)(2 * j + 1) * p3 + 3 * h + 2] = w * xj;
  }
}

// Per box: W = X_RR^{-1} Hh_R (r x 3p) and Gpart = Ph_R^T W (3p x 3p).
__global__ __launch_bounds__(kBlock) void k_border_box(const SolveBox* boxes, const int* ridx,
                                                       const double* Hh, const double* Ph,
                                                       int p3, double* Gpart, double* scratch,
                                                       long long scr_stride) {
  const SolveBox& B = boxes[blockIdx.x];
  const int r = B.r;
  double* G = Gpart + (size_t)B.part * p3 * p3;
  if (r == 0) {
    for (int t = threadIdx.x; t < p3 * p3; t += kBlock) G[t] = 0.0;
    return;
  }
  double* hr = scratch + (size_t)blockIdx.x * scr_stride;
  double* pr = hr + (size_t)r * p3;
  const int* R = ridx + B.r_off;
  for (int t = threadIdx.x; t < r * p3; t += kBlock) {
    const int i = t / p3, h = t % p3;
    hr[t] = Hh[(size_t)R[i] * p3 + h];
    pr[t] = Ph[(size_t)R[i] * p3 + h];
  }
  __syncthreads();
  wg_gemm(r, p3, r, 1.0, B.Xinv, r, false, hr, p3, false, 0.0, nullptr, 0, B.W, p3);
  wg_gemm(p3, p3, r, 1.0, pr, p3, true, B.W, p3, false, 0.0, nullptr, 0, G, p3);
}

__global__ void k_sum_parts(const double* parts, int nparts, long long stride, int len,
                            double scale, double* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= len) return;
  double s = 0.0;
  for (int p = 0; p < nparts; ++p) s += parts[(size_t)p * stride + t];
  out[t] = scale * s;
}

// parts[box] (3p x ncols) = Ph_R^T c_R
__global__ __launch_bounds__(kBlock) void k_border_rhs(const SolveBox* boxes, const int* ridx,
                                                       const double* Ph, int p3,
                                                       const double* c, int ncols,
                                                       double* parts) {
  const SolveBox& B = boxes[blockIdx.x];
  double* out = parts + (size_t)B.part * p3 * ncols;
  const int* R = ridx + B.r_off;
  for (int t = threadIdx.x; t < p3 * ncols; t += kBlock) {
    const int h = t / ncols, q = t % ncols;
    double acc = 0.0;
    for (int i = 0; i < B.r; ++i) acc += Ph[(size_t)R[i] * p3 + h] * c[(size_t)R[i] * ncols + q];
    out[t] = acc;
  }
}

// c_R -= W lam
__global__ __launch_bounds__(kBlock) void k_border_fix(const SolveBox* boxes, const int* ridx,
                                                       int p3, const double* lam, double* c,
                                                       int ncols) {
  const SolveBox& B = boxes[blockIdx.x];
  const int* R = ridx + B.r_off;
  for (int t = threadIdx.x; t < B.r * ncols; t += kBlock) {
    const int i = t / ncols, q = t % ncols;
    double acc = 0.0;
    for (int h = 0; h < p3; ++h) acc += B.W[(size_t)i * p3 + h] * lam[(size_t)h * ncols + q];
    c[(size_t)R[i] * ncols + q] -= acc;
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

__global__ void k_root_gather(const double* c, int ncols, const int* I0, int n0,
                              const double* rhs2, int p3, double* v) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (n0 + p3) * ncols) return;
  const int i = t / ncols, q = t % ncols;
  v[t] = i < n0 ? c[(size_t)I0[i] * ncols + q] : rhs2[(size_t)(i - n0) * ncols + q];
}

__global__ void k_dense_apply(const double* Zinv, int nz, const double* v, int ncols,
                              double* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nz * ncols) return;
  const int i = t / ncols, q = t % ncols;
  double acc = 0.0;
  for (int j = 0; j < nz; ++j) acc += Zinv[(size_t)i * nz + j] * v[(size_t)j * ncols + q];
  out[t] = acc;
}

__global__ void k_root_scatter(const double* sol, int ncols, const int* I0, int n0, double* c) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n0 * ncols) return;
  const int i = t / ncols, q = t % ncols;
  c[(size_t)I0[i] * ncols + q] = sol[t];
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

// ---- exact float64 operator (refinement residual) ---------------------------
// y = A x with A = [[lam I + D + N, H], [Psi^T, -I]]; x, y row layout
// [(2N + 3p)][ncols].  One thread per target node, sources staged through LDS,
// kApplyCols columns per block.
constexpr int kApplyCols = 8;
constexpr int kApplyTile = 256;

__global__ __launch_bounds__(kApplyTile) void k_apply_D(Geo g, const double* hole_xy, int p,
                                                        double lam, const double* x,
                                                        int ncols, double* y) {
  __shared__ double sx[kApplyTile], sy[kApplyTile], snx[kApplyTile], sny[kApplyTile],
      sw[kApplyTile];
  __shared__ double sm[kApplyTile][2 * kApplyCols];
  const int N = g.N;
  const int i = blockIdx.x * kApplyTile + threadIdx.x;
  const int q0 = blockIdx.y * kApplyCols;
  const int nq = min(kApplyCols, ncols - q0);
  const int ldx = ncols;
  const bool live = i < N;
  const double xi = live ? g.x[i] : 0.0, yi = live ? g.y[i] : 0.0;
  const double nxi = live ? g.nx[i] : 0.0, nyi = live ? g.ny[i] : 0.0;
  double ax[kApplyCols], ay[kApplyCols];
#pragma unroll
  for (int q = 0; q < kApplyCols; ++q) { ax[q] = 0.0; ay[q] = 0.0; }
  for (int j0 = 0; j0 < N; j0 += kApplyTile) {
    const int j = j0 + threadIdx.x;
    __syncthreads();
    if (j < N) {
      sx[threadIdx.x] = g.x[j];
      sy[threadIdx.x] = g.y[j];
      snx[threadIdx.x] = g.nx[j];
      sny[threadIdx.x] = g.ny[j];
      sw[threadIdx.x] = g.w[j];
#pragma unroll
      for (int q = 0; q < kApplyCols; ++q) {
        sm[threadIdx.x][2 * q] = q < nq ? x[(size_t)(2 * j) * ldx + q0 + q] : 0.0;
        sm[threadIdx.x][2 * q + 1] = q < nq ? x[(size_t)(2 * j + 1) * ldx + q0 + q] : 0.0;
      }
    }
    __syncthreads();
    const int cnt = min(kApplyTile, N - j0);
    if (!live) continue;
    for (int jj = 0; jj < cnt; ++jj) {
      const int js = j0 + jj;
      double bxx, bxy, byx, byy;
      const double wn_x = sw[jj] * snx[jj], wn_y = sw[jj] * sny[jj];
      if (js == i) {
        const double tx = -nyi, ty = nxi;
        const double c = -(g.w[i] * g.kap[i]) / (2.0 * kPi);
        bxx = c * tx * tx + lam;
        bxy = c * tx * ty;
        byx = bxy;
        byy = c * ty * ty + lam;
      } else {
        const double rx = xi - sx[jj], ry = yi - sy[jj];
        const double r2 = rx * rx + ry * ry;
        const double rn = rx * snx[jj] + ry * sny[jj];
        const double coef = kInvPi * sw[jj] * rn / (r2 * r2);
        bxx = coef * rx * rx;
        bxy = coef * rx * ry;
        byx = bxy;
        byy = coef * ry * ry;
      }
      bxx += nxi * wn_x;
      bxy += nxi * wn_y;
      byx += nyi * wn_x;
      byy += nyi * wn_y;
#pragma unroll
      for (int q = 0; q < kApplyCols; ++q) {
        const double mx = sm[jj][2 * q], my = sm[jj][2 * q + 1];
        ax[q] += bxx * mx + bxy * my;
        ay[q] += byx * mx + byy * my;
      }
    }
  }
  if (!live) return;
  const int p3 = 3 * p;
  const size_t base = (size_t)2 * N;
  for (int h = 0; h < p; ++h) {
    const double rx = xi - hole_xy[2 * h], ry = yi - hole_xy[2 * h + 1];
    const double r2 = rx * rx + ry * ry;
    const double lg = -0.5 * log(r2);
    const double sxx = kInv4Pi * (lg + rx * rx / r2), sxy = kInv4Pi * (rx * ry / r2);
    const double syy = kInv4Pi * (lg + ry * ry / r2);
    const double rotx = kInv4Pi * (-ry) / r2, roty = kInv4Pi * rx / r2;
    for (int q = 0; q < nq; ++q) {
      const double a1 = x[(base + 3 * h) * ldx + q0 + q];
      const double a2 = x[(base + 3 * h + 1) * ldx + q0 + q];
      const double b = x[(base + 3 * h + 2) * ldx + q0 + q];
      ax[q] += sxx * a1 + sxy * a2 + rotx * b;
      ay[q] += sxy * a1 + syy * a2 + roty * b;
    }
  }
  (void)p3;
  for (int q = 0; q < nq; ++q) {
    y[(size_t)(2 * i) * ldx + q0 + q] = ax[q];
    y[(size_t)(2 * i + 1) * ldx + q0 + q] = ay[q];
  }
}

// Rows of Psi^T x - lambda: one block per (hole, mode), fixed-order sums.
__global__ __launch_bounds__(kBlock) void k_apply_psi(Geo g, const int* curve_id, int p,
                                                      const double* x, int ncols, double* y) {
  constexpr int NW = kBlock / 64;
  __shared__ double red[NW];
  const int h = blockIdx.x / 3, mode = blockIdx.x % 3;
  const size_t base = (size_t)2 * g.N;
  for (int q = 0; q < ncols; ++q) {
    double s = 0.0;
    for (int j = threadIdx.x; j < g.N; j += kBlock) {
      if (curve_id[j] != h + 1) continue;
      const double w = g.w[j];
      const double mx = x[(size_t)(2 * j) * ncols + q], my = x[(size_t)(2 * j + 1) * ncols + q];
      if (mode == 0) s += w * mx;
      else if (mode == 1) s += w * my;
      else s += w * (-g.y[j] * mx + g.x[j] * my);
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
      const size_t row = base + 3 * h + mode;
      y[row * ncols + q] = s - x[row * ncols + q];
    }
  }
}

inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// ---- launchers ---------------------------------------------------------------

void launch_assemble_M(const LevelBox* boxes, int nbox, int max_m, const int* dofs,
                       const int* fint, Geo g, int n_proxy, double ratio, hipStream_t s) {
  if (nbox == 0 || max_m == 0) return;
  dim3 grid(nbox, blocks_for(max_m, kBlock));
  hipLaunchKernelGGL(k_assemble_M, grid, dim3(kBlock), 0, s, boxes, dofs, fint, g, n_proxy, ratio);
}

size_t cpqr_lds_bytes(int max_m, int max_n) {
  return (size_t)max_n * (2 * sizeof(double) + sizeof(int)) + (size_t)max_m * sizeof(double) + 16;
}

void launch_cpqr(const LevelBox* boxes, int nbox, double tol, int extra, int* perm,
                 int* k_out, int* kx_out, int max_m, int max_n, hipStream_t s) {
  if (nbox == 0) return;
  hipLaunchKernelGGL(k_cpqr, dim3(nbox), dim3(kQRThreads), cpqr_lds_bytes(max_m, max_n), s, boxes,
                     tol, extra, perm, k_out, kx_out);
}

void launch_assemble_abb(const LevelBox* boxes, int nbox, int max_n, const int* dofs,
                         const int* perm, const ChildSrc* src, Geo g, double lam,
                         hipStream_t s) {
  if (nbox == 0 || max_n == 0) return;
  dim3 grid(nbox, blocks_for((long long)max_n * max_n, kBlock));
  hipLaunchKernelGGL(k_assemble_abb, grid, dim3(kBlock), 0, s, boxes, dofs, perm, src, g, lam);
}

void launch_eliminate(const LevelBox* boxes, int nbox, int* k_io, const int* kx,
                      double rcond_min, int* status, int max_n, hipStream_t s) {
  if (nbox == 0) return;
  const size_t shm = (size_t)(max_n + 1) * sizeof(double);
  hipLaunchKernelGGL(k_eliminate, dim3(nbox), dim3(kBlock), shm, s, boxes, k_io, kx, rcond_min,
                     status);
}

void launch_gj_inverse(double* A, int n, int lda, double* Ainv, double* work,
                       double* rcond_out, int* status, hipStream_t s) {
  const size_t shm = (size_t)(n + 1) * sizeof(double);
  hipLaunchKernelGGL(k_gj_inverse, dim3(1), dim3(kBlock), shm, s, A, n, lda, Ainv, work,
                     rcond_out, status);
}

// Right-hand-side columns per block so that `rows` rows fit in 64 KiB of LDS.
inline int chunk_cols(int rows) {
  int nc = kNC;
  while (nc > 1 && (size_t)rows * nc * sizeof(double) > 65536) nc >>= 1;
  return nc;
}

// Inverse of A (n x n) into Ainv; A is destroyed.  work: >= n*kGJB + kGJB*n +
// n*kGJB + kGJB*kGJB doubles; iwork: >= n + kGJB ints.
void launch_gj_blocked(double* A, int n, double* Ainv, double* work, int* iwork, int* status,
                       hipStream_t s) {
  double* W = work;                        // (n x kGJB)
  double* R = W + (size_t)n * kGJB;        // (kGJB x n)
  double* Cp = R + (size_t)kGJB * n;       // (n x kGJB)
  double* Dinv = Cp + (size_t)n * kGJB;    // kGJB x kGJB
  int* rowperm = iwork;
  int* piv = iwork + n;
  hipLaunchKernelGGL(k_iota, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, rowperm, n, status);
  const long long nn = (long long)n * n;
  for (int k0 = 0; k0 < n; k0 += kGJB) {
    const int bb = std::min(kGJB, n - k0);
    hipLaunchKernelGGL(k_gjb_panel, dim3(1), dim3(kBlock), 0, s, A, n, k0, bb, W, piv, Dinv, status);
    hipLaunchKernelGGL(k_gjb_swap, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, A, n, k0, bb,
                       piv, rowperm, Cp);
    hipLaunchKernelGGL(k_gjb_copycol, dim3(blocks_for((long long)n * bb, kBlock)), dim3(kBlock), 0,
                       s, A, n, k0, bb, Cp);
    hipLaunchKernelGGL(k_gjb_rows, dim3(blocks_for((long long)bb * n, kBlock)), dim3(kBlock), 0, s,
                       A, n, k0, bb, Dinv, R);
    hipLaunchKernelGGL(k_gjb_update, dim3(blocks_for(nn, kBlock)), dim3(kBlock), 0, s, A, n, k0, bb,
                       Dinv, R, Cp);
  }
  hipLaunchKernelGGL(k_gjb_unpermute, dim3(blocks_for(nn, kBlock)), dim3(kBlock), 0, s, A, n,
                     rowperm, Ainv);
}

void launch_sweep(const SolveBox* boxes, int nbox, const int* sidx, const int* ridx, double* c,
                  int ncols, int mode, int max_n, hipStream_t s) {
  if (nbox == 0 || ncols == 0) return;
  const int nc = chunk_cols(max_n);
  dim3 grid(nbox, blocks_for(ncols, nc));
  const size_t shm = (size_t)max_n * nc * sizeof(double);
  hipLaunchKernelGGL(k_sweep, grid, dim3(kBlock), shm, s, boxes, sidx, ridx, c, ncols, mode, nc);
}

void launch_diag(const SolveBox* boxes, int nbox, const int* ridx, double* c, int ncols,
                 int max_r, hipStream_t s) {
  if (nbox == 0 || ncols == 0) return;
  const int nc = chunk_cols(2 * max_r);
  dim3 grid(nbox, blocks_for(ncols, nc));
  const size_t shm = (size_t)2 * max_r * nc * sizeof(double);
  hipLaunchKernelGGL(k_diag, grid, dim3(kBlock), shm, s, boxes, ridx, c, ncols, nc);
}

void launch_assemble_H(Geo g, const double* hole_xy, int p, const int* curve_id, double* H,
                       double* Psi, hipStream_t s) {
  hipLaunchKernelGGL(k_assemble_H, dim3(blocks_for(g.N, kBlock)), dim3(kBlock), 0, s, g,
                     hole_xy, p, curve_id, H, Psi);
}

void launch_border_box(const SolveBox* boxes, int nbox, const int* ridx, const double* Hh,
                       const double* Ph, int p3, double* Gpart, double* scratch,
                       long long scr_stride, hipStream_t s) {
  if (nbox == 0) return;
  hipLaunchKernelGGL(k_border_box, dim3(nbox), dim3(kBlock), 0, s, boxes, ridx, Hh, Ph, p3,
                     Gpart, scratch, scr_stride);
}

void launch_sum_parts(const double* parts, int nparts, long long stride, int len, double scale,
                      double* out, hipStream_t s) {
  if (len == 0) return;
  hipLaunchKernelGGL(k_sum_parts, dim3(blocks_for(len, kBlock)), dim3(kBlock), 0, s, parts,
                     nparts, stride, len, scale, out);
}

void launch_border_rhs(const SolveBox* boxes, int nbox, const int* ridx, const double* Ph,
                       int p3, const double* c, int ncols, double* parts, hipStream_t s) {
  if (nbox == 0) return;
  hipLaunchKernelGGL(k_border_rhs, dim3(nbox), dim3(kBlock), 0, s, boxes, ridx, Ph, p3, c,
                     ncols, parts);
}

void launch_border_fix(const SolveBox* boxes, int nbox, const int* ridx, int p3,
                       const double* lam, double* c, int ncols, hipStream_t s) {
  if (nbox == 0) return;
  hipLaunchKernelGGL(k_border_fix, dim3(nbox), dim3(kBlock), 0, s, boxes, ridx, p3, lam, c,
                     ncols);
}

void launch_assemble_Z(const double* X0, int n0, const double* Hh, const double* Ph,
                       const int* I0, int p3, const double* G, double* Z, hipStream_t s) {
  const long long nz = n0 + p3;
  hipLaunchKernelGGL(k_assemble_Z, dim3(blocks_for(nz * nz, kBlock)), dim3(kBlock), 0, s, X0,
                     n0, Hh, Ph, I0, p3, G, Z);
}

void launch_root_gather(const double* c, int ncols, const int* I0, int n0, const double* rhs2,
                        int p3, double* v, hipStream_t s) {
  hipLaunchKernelGGL(k_root_gather, dim3(blocks_for((long long)(n0 + p3) * ncols, kBlock)),
                     dim3(kBlock), 0, s, c, ncols, I0, n0, rhs2, p3, v);
}

void launch_dense_apply(const double* Zinv, int nz, const double* v, int ncols, double* out,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_dense_apply, dim3(blocks_for((long long)nz * ncols, 64)), dim3(64), 0, s,
                     Zinv, nz, v, ncols, out);
}

void launch_root_scatter(const double* sol, int ncols, const int* I0, int n0, double* c,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_root_scatter, dim3(blocks_for((long long)n0 * ncols, kBlock)),
                     dim3(kBlock), 0, s, sol, ncols, I0, n0, c);
}

void launch_to_rows(const double* f, int ld, int nrows, int ncols, double* c, hipStream_t s) {
  hipLaunchKernelGGL(k_to_rows, dim3(blocks_for((long long)nrows * ncols, kBlock)), dim3(kBlock),
                     0, s, f, ld, nrows, ncols, c);
}

void launch_from_rows(const double* c, int nrows, int ncols, double* x, int ld, hipStream_t s) {
  hipLaunchKernelGGL(k_from_rows, dim3(blocks_for((long long)nrows * ncols, kBlock)),
                     dim3(kBlock), 0, s, c, nrows, ncols, x, ld);
}

void launch_apply_operator(Geo g, const int* curve_id, const double* hole_xy, int p, double lam,
                           const double* x, int ncols, double* y, double* hole_parts,
                           hipStream_t s) {
  (void)hole_parts;
  dim3 grid(blocks_for(g.N, kApplyTile), blocks_for(ncols, kApplyCols));
  hipLaunchKernelGGL(k_apply_D, grid, dim3(kApplyTile), 0, s, g, hole_xy, p, lam, x, ncols, y);
  if (p > 0)
    hipLaunchKernelGGL(k_apply_psi, dim3(3 * p), dim3(kBlock), 0, s, g, curve_id, p, x, ncols, y);
}

}  // namespace rs

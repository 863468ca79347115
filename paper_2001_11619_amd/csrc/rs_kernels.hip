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

// Wave reductions through DPP row permutations and lane reads (no permute
// traffic through LDS).  Every lane receives the same value; the order is
// fixed: a butterfly inside each 16-lane row, then (row0 + row1) + (row2 + row3).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ double lane_f64(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
constexpr int kDppXor1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppMirror = 0x140;

__device__ __forceinline__ double wave_sum_fast(double v) {
  v += dpp_f64<kDppXor1>(v);
  v += dpp_f64<kDppXor2>(v);
  v += dpp_f64<kDppHalfMirror>(v);
  v += dpp_f64<kDppMirror>(v);
  return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

// Pivot comparison key of a squared column norm: its leading 20 mantissa
// bits (the low 32 bits of the pattern cleared).  Columns whose norms agree
// to that precision are tied and the first column of I_B wins, so the choice
// does not depend on rounding in the norms (mirror-symmetric node pairs give
// such ties).
__device__ __forceinline__ double pivot_key(double sq) { return __hiloint2double(__double2hiint(sq), 0); }

// (value, index) maximum with ties to the smaller index.
__device__ __forceinline__ void arg_better(double& bv, int& bi, double v, int i) {
  if (v > bv || (v == bv && i < bi)) { bv = v; bi = i; }
}
template <int CTRL>
__device__ __forceinline__ void argmax_step(double& bv, int& bi) {
  const double ov = dpp_f64<CTRL>(bv);
  const int oi = dpp_i32<CTRL>(bi);
  arg_better(bv, bi, ov, oi);
}
// Wave-wide argmax; the result is uniform (read from lanes 0, 16, 32, 48).
__device__ __forceinline__ void wave_argmax(double& bv, int& bi) {
  argmax_step<kDppXor1>(bv, bi);
  argmax_step<kDppXor2>(bv, bi);
  argmax_step<kDppHalfMirror>(bv, bi);
  argmax_step<kDppMirror>(bv, bi);
  double rv = lane_f64(bv, 0);
  int ri = __builtin_amdgcn_readlane(bi, 0);
#pragma unroll
  for (int r = 16; r < 64; r += 16) arg_better(rv, ri, lane_f64(bv, r), __builtin_amdgcn_readlane(bi, r));
  bv = rv;
  bi = ri;
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

__global__ __launch_bounds__(kBlock) void k_assemble_M(const LevelBox* boxes, int n_proxy,
                                                       double ratio) {
  const LevelBox& B = boxes[blockIdx.x];
  const int i = blockIdx.y * blockDim.x + threadIdx.x;
  const int m = B.m, n = B.n, nF = B.nF;
  if (i >= m || n == 0) return;
  const int* I = B.dofs;
  const Geo& g = B.geo;
  const int np2 = 2 * n_proxy;
  const double rp = ratio * B.side;
  const double wp = 2.0 * kPi * rp / n_proxy;
  int type, f = 0, pa = 0;
  double px = 0, py = 0, pnx = 0, pny = 0;
  if (i < nF) {
    type = 0;
    f = B.fint[i];
  } else if (i < 2 * nF) {
    type = 1;
    f = B.fint[i - nF];
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

// Pivoted Householder QR of M_B (m x n, column-major).
// Pivot: largest remaining column norm (recomputed exactly after every
// step, compared through pivot_key), ties to the column that came first in
// I_B.  Runs until the first
// step with |R_jj| <= tol |R_11| plus `extra` further steps (head-room for
// the X_RR guard).  Writes perm (pivot order of positions in I_B), the
// tolerance rank k and the number of R rows kept, R in pivot order.
//
// A box is worked on by G workgroups (G = 1 for the many small boxes of the
// lower levels; the few large boxes near the root get many).  Workgroup g
// owns the physical columns q with q % G == g for the whole factorization.
// Each step: local pivot candidates -> box barrier -> the owner of the pivot
// column forms the Householder vector and publishes it -> box barrier -> every
// workgroup reflects its own columns and recomputes their norms.  Cross-
// workgroup data goes through agent-scope atomics; barrier waits are bounded
// (a timed-out wait flags an error and the kernel drains).
constexpr int kQRThreads = 512;
constexpr int kQRRows = 24;             // rows per lane held in registers (m <= 1536)
constexpr unsigned kSpinLimit = 1u << 22;

__device__ __forceinline__ void st_relaxed(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_relaxed(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_relaxed(const int* p) {
  return __hip_atomic_load(const_cast<int*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barriers over the G workgroups of one box.  `count` is this workgroup's
// number of completed box barriers; `dead` turns every later wait into a no-op
// once a wait has timed out (the kernel then drains and the host reports it).
//
// box_barrier_x: for exchanges whose data is written and read only with
// agent-scope atomics (coherent across the device): every wave waits for its
// own memory operations to complete, then one thread per workgroup counts in.
// box_barrier_full: additionally an agent-scope release / acquire fence, for
// phases that share ordinary global-memory matrices.
__device__ __forceinline__ void box_wait(unsigned* bar, int G, unsigned& count, int* dead,
                                         int* err) {
  if (threadIdx.x == 0 && !*dead) {
    ++count;
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned target = count * (unsigned)G;
    unsigned spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit) {
        *dead = 1;
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
}

__device__ void box_barrier_x(unsigned* bar, int G, unsigned& count, int* dead, int* err) {
  if (G > 1) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    box_wait(bar, G, count, dead, err);
  }
  __syncthreads();
}

__device__ void box_barrier_full(unsigned* bar, int G, unsigned& count, int* dead, int* err) {
  if (G > 1) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    box_wait(bar, G, count, dead, err);
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

__global__ __launch_bounds__(kQRThreads) void k_cpqr(const LevelBox* boxes, const int* list, int G,
                                                     double tol, int extra, int* k_out, int* kx_out,
                                                     int* err) {
  extern __shared__ double smem[];
  const int bidx = list[blockIdx.x / G], g = blockIdx.x % G;
  const LevelBox& B = boxes[bidx];
  const int m = B.m, n = B.n;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  constexpr int NW = kQRThreads / 64;
  __shared__ double red[NW];
  __shared__ double bval[NW];
  __shared__ int bphys[NW];
  __shared__ int s_q;
  __shared__ double s_hh[2];
  __shared__ int s_dead;
  if (n == 0) {
    if (tid == 0 && g == 0) { k_out[B.slot] = 0; kx_out[B.slot] = 0; }
    return;
  }
  double* nrm = smem;                        // n, by physical column
  double* rdiag = smem + n;                  // n
  double* vsh = smem + 2 * n;                // m
  int* pv = (int*)(smem + 2 * n + m);        // n: physical column at each position
  int* ipv = pv + n;                         // n: position of each physical column
  int* own = ipv + n;                        // columns owned by this workgroup
  unsigned char* done = (unsigned char*)(own + n);   // n
  const int nown = (n - g + G - 1) / G;
  double* A = B.M;
  const bool regs = m <= 64 * kQRRows;
  unsigned nbar = 0;
  if (tid == 0) s_dead = 0;
  for (int c = tid; c < n; c += kQRThreads) { pv[c] = c; ipv[c] = c; done[c] = 0; }
  for (int t = tid; t < nown; t += kQRThreads) own[t] = g + t * G;
  for (int t = wid; t < nown; t += NW) {
    const int c = g + t * G;
    const double* col = A + (size_t)c * m;
    double sum = 0.0;
    for (int i = lane; i < m; i += 64) {
      const double a = col[i];
      sum += a * a;
    }
    sum = wave_sum(sum);
    if (lane == 0) nrm[c] = sum;
  }
  __syncthreads();
  const int steps = min(m, n);
  int limit = steps;
  int kk = -1;
  double r00 = 0.0;
  int j = 0;
  for (; j < limit; ++j) {
    // local pivot candidate among owned, not yet pivoted columns
    double best = -1.0;
    int bq = 1 << 30;
    for (int t = tid; t < nown; t += kQRThreads) {
      const int q = own[t];
      if (done[q]) continue;
      const double v = pivot_key(nrm[q]);
      if (v > best || (v == best && q < bq)) { best = v; bq = q; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o, 64);
      const int oq = __shfl_xor(bq, o, 64);
      if (ov > best || (ov == best && oq < bq)) { best = ov; bq = oq; }
    }
    if (lane == 0) { bval[wid] = best; bphys[wid] = bq; }
    __syncthreads();
    if (tid == 0) {
      for (int w = 1; w < NW; ++w)
        if (bval[w] > best || (bval[w] == best && bphys[w] < bq)) { best = bval[w]; bq = bphys[w]; }
      if (G > 1) {
        const int par = j & 1;
        st_relaxed(B.cval + par * G + g, best);
        st_relaxed(B.cphys + par * G + g, bq);
      } else {
        s_q = bq;
      }
    }
    if (G > 1) {
      box_barrier_x(B.bar, G, nbar, &s_dead, err);
      if (tid == 0) {
        const int par = j & 1;
        double bb = -1.0;
        int qq = 1 << 30;
        for (int h = 0; h < G; ++h) {
          const double v = ld_relaxed(B.cval + par * G + h);
          const int q = ld_relaxed(B.cphys + par * G + h);
          if (v > bb || (v == bb && q < qq)) { bb = v; qq = q; }
        }
        s_q = qq;
      }
    }
    __syncthreads();
    const int q = s_q;
    if (q >= n) {   // no finite candidate (non-finite entries in M_B): flag and stop
      if (tid == 0) __hip_atomic_store(err + 2, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    if (tid == 0) {
      const int p = ipv[q];
      const int u = pv[j];
      pv[j] = q; pv[p] = u;
      ipv[q] = j; ipv[u] = p;
      done[q] = 1;
    }
    // Householder vector of the pivot column, formed by its owner
    if (q % G == g) {
      const double* x = A + (size_t)q * m;
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
        for (int i = j + 1 + tid; i < m; i += kQRThreads) {
          const double v = vsh[i] * scal;
          vsh[i] = v;
          if (G > 1) st_relaxed(B.vbuf + i, v);
        }
      }
      if (tid == 0) {
        s_hh[0] = beta;
        s_hh[1] = tau;
        if (G > 1) { st_relaxed(B.hh, beta); st_relaxed(B.hh + 1, tau); }
      }
    }
    if (G > 1) {
      box_barrier_x(B.bar, G, nbar, &s_dead, err);
      if (q % G != g) {
        for (int i = j + 1 + tid; i < m; i += kQRThreads) vsh[i] = ld_relaxed(B.vbuf + i);
        if (tid == 0) { s_hh[0] = ld_relaxed(B.hh); s_hh[1] = ld_relaxed(B.hh + 1); }
      }
    }
    __syncthreads();
    const double beta = s_hh[0], tau = s_hh[1];
    if (tid == 0) rdiag[j] = beta;
    const double rjj = fabs(beta);
    if (j == 0) r00 = rjj;
    if (kk < 0 && !(rjj > tol * r00)) {
      kk = j;
      limit = min(steps, j + 1 + extra);
    }
    // reflect the owned columns that are still to be pivoted; in the register
    // path each wave carries two columns at once so their loads overlap
    if (regs) {
      // compact list of this step's live owned columns, dealt two per wave
      for (int t = wid; 2 * t < nown; t += NW) {
        const int c0 = own[2 * t];
        const int c1 = 2 * t + 1 < nown ? own[2 * t + 1] : -1;
        const bool a0 = !done[c0];
        const bool a1 = c1 >= 0 && !done[c1];
        if (!a0 && !a1) continue;
        double* y0 = A + (size_t)c0 * m;
        double* y1 = A + (size_t)(a1 ? c1 : c0) * m;
        const double yj0 = y0[j], yj1 = y1[j];
        double r0[kQRRows], r1[kQRRows];
        double w0 = 0.0, w1 = 0.0;
#pragma unroll
        for (int u = 0; u < kQRRows; ++u) {
          const int i = lane + 64 * u;
          const bool in = i > j && i < m;
          r0[u] = (in && a0) ? y0[i] : 0.0;
          r1[u] = (in && a1) ? y1[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kQRRows; ++u) {
          const int i = lane + 64 * u;
          const double v = (i > j && i < m) ? vsh[i] : 0.0;
          w0 += v * r0[u];
          w1 += v * r1[u];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          w0 += __shfl_xor(w0, o, 64);
          w1 += __shfl_xor(w1, o, 64);
        }
        const double tw0 = tau * (w0 + yj0), tw1 = tau * (w1 + yj1);
        double n0 = 0.0, n1 = 0.0;
#pragma unroll
        for (int u = 0; u < kQRRows; ++u) {
          const int i = lane + 64 * u;
          if (i > j && i < m) {
            const double v = vsh[i];
            const double z0 = r0[u] - tw0 * v;
            const double z1 = r1[u] - tw1 * v;
            if (a0) y0[i] = z0;
            if (a1) y1[i] = z1;
            n0 += z0 * z0;
            n1 += z1 * z1;
          }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          n0 += __shfl_xor(n0, o, 64);
          n1 += __shfl_xor(n1, o, 64);
        }
        if (lane == 0) {
          if (a0) { y0[j] = yj0 - tw0; nrm[c0] = n0; }
          if (a1) { y1[j] = yj1 - tw1; nrm[c1] = n1; }
        }
      }
    } else {
      for (int t = wid; t < nown; t += NW) {
        const int c = own[t];
        if (done[c]) continue;
        double* y = A + (size_t)c * m;
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
        if (lane == 0) { y[j] = yj - tw; nrm[c] = ns; }
      }
    }
    __syncthreads();
  }
  const int kx = j;
  if (kk < 0) kk = kx;
  // R rows in pivot order: each workgroup writes the entries of its columns
  for (int t = tid; t < kx * n; t += kQRThreads) {
    const int r = t / n, c = t % n;
    if (c <= r) {
      if (g == 0) B.R[t] = (c == r) ? rdiag[r] : 0.0;
    } else if (pv[c] % G == g) {
      B.R[t] = A[(size_t)pv[c] * m + r];
    }
  }
  if (g == 0) {
    for (int c = tid; c < n; c += kQRThreads) B.perm[c] = pv[c];
    if (tid == 0) { k_out[B.slot] = kk; kx_out[B.slot] = kx; }
  }
}

__global__ void k_zero_bars(const LevelBox* boxes, int nbox, int* err, int nerr) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nbox && boxes[t].bar) *boxes[t].bar = 0u;
  if (t < nerr) err[t] = 0;
}

// ---- register-resident pivoted QR ------------------------------------------
// The same factorization as k_cpqr (largest remaining column norm, ties to
// the first column of I_B, stop at |R_jj| <= tol |R_11| plus `extra` steps),
// with M_B held in registers for all steps instead of being re-read from
// memory at every step.  Layout: the box's columns are dealt to G workgroups
// (column c to workgroup c % G), inside a workgroup to its 16 waves and then
// to CPW register slots per wave; lane l of a wave holds rows l + 64 u,
// u < RU, of each of its columns (rows >= m are zero).  Every dot product and
// norm of a column is summed by its wave in a fixed order, so the result does
// not depend on G, on CPW or on RU.  Work item = (box, g, G, RU).
// Householder vector of column x at step j (rows j..m-1), formed by the one
// wave holding the column: v (v_i = 0 above j, v_j = 1) into vsh, (beta, tau)
// into hh; with vbuf/hhg non-null also into those (agent-scope stores, for
// the other workgroups of the box).  x_j becomes R_jj = beta.
template <int RU>
__device__ __forceinline__ void reg_householder(double (&x)[RU], const int j, const int m,
                                                const int lane, double* vsh, double* hh,
                                                double* vbuf, double* hhg) {
  const int uj = j >> 6, lj = j & 63;
  double xj = 0.0, sum = 0.0;
#pragma unroll
  for (int u = 0; u < RU; ++u) {
    if (u == uj) {
      xj = x[u];
      if (lane > lj) sum += x[u] * x[u];
    } else if (u > uj) {
      sum += x[u] * x[u];
    }
  }
  const double alpha = lane_f64(xj, lj);
  sum = wave_sum_fast(sum);
  double beta, tau, scal = 0.0;
  if (sum == 0.0) {
    beta = alpha;
    tau = 0.0;
  } else {
    beta = -copysign(sqrt(alpha * alpha + sum), alpha);
    tau = (beta - alpha) / beta;
    scal = 1.0 / (alpha - beta);
  }
#pragma unroll
  for (int u = 0; u < RU; ++u) {
    const int i = lane + 64 * u;
    double v;
    if (u < uj) v = 0.0;
    else if (u > uj) v = x[u] * scal;
    else v = lane < lj ? 0.0 : (lane == lj ? 1.0 : x[u] * scal);
    vsh[i] = v;
    if (vbuf && i < m) st_relaxed(vbuf + i, v);
    if (u == uj && lane == lj) x[u] = beta;
  }
  if (lane == 0) {
    hh[0] = beta;
    hh[1] = tau;
    if (hhg) { st_relaxed(hhg, beta); st_relaxed(hhg + 1, tau); }
  }
}

// ---- register-resident pivoted QR ------------------------------------------
// The same factorization as k_cpqr (largest remaining column norm, ties to
// the first column of I_B, stop at |R_jj| <= tol |R_11| plus `extra` steps),
// of the matrix B.Mq (mq rows: M_B itself, or the triangular factor of its
// row reduction, which has the same pivots, ranks and R up to row signs),
// held in registers for all steps.  Layout: the box's columns are dealt to G
// workgroups (column c to workgroup c % G), inside a workgroup to its waves
// and then to CPW register slots per wave; lane l of a wave holds rows
// l + 64 u, u < RU, of each of its columns (rows >= mq are zero).  Every dot
// product and norm of a column is summed by its wave in a fixed order, so the
// result does not depend on G, on CPW or on RU.  Work item = (box, g, G, RU).
template <int RU>
__device__ __forceinline__ void cpqr_reg_box(const LevelBox& B, const int G, const int g,
                                             const double tol, const int extra, int* k_out,
                                             int* kx_out, int* err, double* dyn, double* s_hh,
                                             int* s_dead, double* wv, int* wi) {
  constexpr int CPW = rq_cols_per_wave(RU);
  const int m = B.mq, n = B.n;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  double* vsh = dyn;                                    // 64 RU: Householder vector
  int* pv = reinterpret_cast<int*>(vsh + 64 * RU);      // n: physical column at each position
  int* ipv = pv + n;                                    // n: position of each physical column
  const double* Mc = B.Mq;
  double a[CPW][RU];
#pragma unroll
  for (int sl = 0; sl < CPW; ++sl) {
    const int c = g + G * (wid + kRQWaves * sl);
    if (c < n) {
      const double* src = Mc + (size_t)c * m;
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int i = lane + 64 * u;
        a[sl][u] = i < m ? src[i] : 0.0;
      }
    } else {
#pragma unroll
      for (int u = 0; u < RU; ++u) a[sl][u] = 0.0;
    }
  }
  // column norms (uniform across the wave) and this wave's pivot candidate
  unsigned long long dm = 0;           // slots whose column has been pivoted
  {
    double bv = -1.0;
    int bi = 1 << 30;
#pragma unroll
    for (int sl = 0; sl < CPW; ++sl) {
      const int c = g + G * (wid + kRQWaves * sl);
      if (c < n) {
        double t = 0.0;
#pragma unroll
        for (int u = 0; u < RU; ++u) t += a[sl][u] * a[sl][u];
        arg_better(bv, bi, pivot_key(wave_sum_fast(t)), c);
      }
    }
    if (lane == 0) { wv[wid] = bv; wi[wid] = bi; }
  }
  for (int c = tid; c < n; c += kRQThreads) { pv[c] = c; ipv[c] = c; }
  if (tid == 0) *s_dead = 0;
  __syncthreads();
  const int steps = min(m, n);
  int limit = steps;
  int kk = -1;
  double r00 = 0.0;
  unsigned nbar = 0;
  int j = 0;
  for (; j < limit; ++j) {
    // pivot: the workgroup's best candidate, then (G > 1) the box's
    double best = -1.0;
    int bq = 1 << 30;
    if (lane < kRQWaves) { best = wv[lane]; bq = wi[lane]; }
    wave_argmax(best, bq);
    if (G > 1) {
      const int par = j & 1;
      if (tid == 0) {
        st_relaxed(B.cval + par * G + g, best);
        st_relaxed(B.cphys + par * G + g, bq);
      }
      box_barrier_x(B.bar, G, nbar, s_dead, err);
      best = -1.0;
      bq = 1 << 30;
      if (lane < G) {
        best = ld_relaxed(B.cval + par * G + lane);
        bq = ld_relaxed(B.cphys + par * G + lane);
      }
      wave_argmax(best, bq);
    }
    const int q = __builtin_amdgcn_readfirstlane(bq);
    if (q >= n) {   // no finite candidate (non-finite entries in M_B): flag and stop
      if (tid == 0) __hip_atomic_store(err + 2, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    const bool mine = (q % G) == g;
    const int qo = q / G;
    if (mine && wid == qo % kRQWaves) {
      const int os = qo / kRQWaves;
#pragma unroll
      for (int sl = 0; sl < CPW; ++sl)
        if (sl == os)
          reg_householder<RU>(a[sl], j, m, lane, vsh, s_hh, G > 1 ? B.vbuf : nullptr,
                              G > 1 ? B.hh : nullptr);
    }
    if (G > 1) {
      box_barrier_x(B.bar, G, nbar, s_dead, err);
      if (!mine) {
        for (int i = tid; i < 64 * RU; i += kRQThreads) vsh[i] = i < m ? ld_relaxed(B.vbuf + i) : 0.0;
        if (tid == 0) { s_hh[0] = ld_relaxed(B.hh); s_hh[1] = ld_relaxed(B.hh + 1); }
      }
    }
    __syncthreads();
    const double beta = s_hh[0], tau = s_hh[1];
    const double rjj = fabs(beta);
    if (j == 0) r00 = rjj;
    if (kk < 0 && !(rjj > tol * r00)) {
      kk = j;
      limit = min(steps, j + 1 + extra);
    }
    if (tid == 0) {
      const int p = ipv[q];
      const int u = pv[j];
      pv[j] = q; pv[p] = u;
      ipv[q] = j; ipv[u] = p;
    }
    // reflect the live columns of this wave; recompute their norms below row j
#pragma unroll
    for (int sl = 0; sl < CPW; ++sl)
      if (g + G * (wid + kRQWaves * sl) == q) dm |= 1ull << sl;
    const int uj = j >> 6, lj = j & 63;
    double v[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u) v[u] = u < uj ? 0.0 : vsh[lane + 64 * u];
    double bv = -1.0;
    int bi = 1 << 30;
#pragma unroll
    for (int sl = 0; sl < CPW; ++sl) {
      const int c = g + G * (wid + kRQWaves * sl);
      if (c < n && !((dm >> sl) & 1)) {
        double t = 0.0;
#pragma unroll
        for (int u = 0; u < RU; ++u) t += v[u] * a[sl][u];
        const double tw = tau * wave_sum_fast(t);
        t = 0.0;
#pragma unroll
        for (int u = 0; u < RU; ++u) {
          a[sl][u] -= tw * v[u];   // v is zero above row j: those rows stay
          if (u > uj || (u == uj && lane > lj)) t += a[sl][u] * a[sl][u];
        }
        arg_better(bv, bi, pivot_key(wave_sum_fast(t)), c);
      }
    }
    if (lane == 0) { wv[wid] = bv; wi[wid] = bi; }
    __syncthreads();
  }
  const int kx = j;
  if (kk < 0) kk = kx;
  // rows 0..kx-1 of R in pivot order: each wave writes its columns
#pragma unroll
  for (int sl = 0; sl < CPW; ++sl) {
    const int c = g + G * (wid + kRQWaves * sl);
    if (c >= n) continue;
    const int p = ipv[c];
    double* dst = B.R + p;
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int r = lane + 64 * u;
      if (r < kx) dst[(size_t)r * n] = r <= p ? a[sl][u] : 0.0;
    }
  }
  if (g == 0) {
    for (int c = tid; c < n; c += kRQThreads) B.perm[c] = pv[c];
    if (tid == 0) { k_out[B.slot] = kk; kx_out[B.slot] = kx; }
  }
}

// ---- 16-lane column layout --------------------------------------------------
// Used by the row reduction and by the pivoted QR of matrices of at most 256
// rows: a column lives in one 16-lane row of a wave (4 columns per wave and
// register slot); lane p of that row holds rows p + 16 u, u < RU.  A column's
// dot product is then a 16-lane reduction (4 DPP steps, done for the 4
// columns of a wave at once).  Column of (wave w, slot s, lane group r):
// 4 (w + 8 s) + r.
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_f64<kDppXor1>(v);
  v += dpp_f64<kDppXor2>(v);
  v += dpp_f64<kDppHalfMirror>(v);
  v += dpp_f64<kDppMirror>(v);
  return v;
}

// Householder vector at step j of the column x held by lane group og of the
// calling wave: v into vsh (rows 0..16 RU-1, zero above j, one at j), (beta,
// tau) into hh; x_j becomes R_jj = beta.
template <int RU>
__device__ __forceinline__ void r16_householder(double (&x)[RU], const int j, const int og,
                                                const int p, const int rg, double* vsh, double* hh) {
  const int uj = j >> 4, pj = j & 15;
  double xj = 0.0, s0 = 0.0, s1 = 0.0;
#pragma unroll
  for (int u = 0; u < RU; ++u) {
    double& acc = (u & 1) ? s1 : s0;
    if (u == uj) {
      xj = x[u];
      if (p > pj) acc += x[u] * x[u];
    } else if (u > uj) {
      acc += x[u] * x[u];
    }
  }
  const double sum = row16_sum(s0 + s1);
  const double alpha = lane_f64(xj, 16 * og + pj);
  const double s2 = lane_f64(sum, 16 * og);
  double beta, tau, scal = 0.0;
  if (s2 == 0.0) {
    beta = alpha;
    tau = 0.0;
  } else {
    beta = -copysign(sqrt(alpha * alpha + s2), alpha);
    const double d = alpha - beta;
    const double rcp = 1.0 / (beta * d);
    tau = -d * d * rcp;          // (beta - alpha) / beta
    scal = beta * rcp;           // 1 / (alpha - beta)
  }
  if (rg == og) {
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      double v;
      if (u < uj) v = 0.0;
      else if (u > uj) v = x[u] * scal;
      else v = p < pj ? 0.0 : (p == pj ? 1.0 : x[u] * scal);
      vsh[p + 16 * u] = v;
      if (u == uj && p == pj) x[u] = beta;
    }
  }
  if ((threadIdx.x & 63) == 0) { hh[0] = beta; hh[1] = tau; }
}

// ---- row reduction of tall ID matrices (unpivoted block Householder QR) ----
// One task = one block of rows (at most 16 RU) of an n-column matrix: its
// triangular factor (n rows, zeros below the diagonal) is written to dst.
// Blocks of M_B first, then blocks of stacked factors, until the stack has at
// most 256 rows.  One barrier per step: the Householder vector of step j + 1
// goes to the other of two buffers.
template <int RU, int NS>
__device__ __forceinline__ void tsqr16_block(const QRTask& T, double* vsh2, double* hh2) {
  const int rows = T.rows, n = T.n;
  const int lane = threadIdx.x & 63, p = lane & 15, rg = lane >> 4;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  double a[NS][RU];
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int c = 4 * (wid + kRQWaves * sl) + rg;
    const double* src = T.src + (size_t)(c < n ? c : 0) * T.ld;
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int i = p + 16 * u;
      a[sl][u] = (c < n && i < rows) ? src[i] : 0.0;
    }
  }
  const int steps = min(rows, n);
  for (int j = 0; j < steps; ++j) {
    double* vsh = vsh2 + (j & 1) * 16 * RU;
    double* hh = hh2 + 2 * (j & 1);
    const int sj = j >> 2;
    if (wid == sj % kRQWaves) {
      const int os = sj / kRQWaves;
#pragma unroll
      for (int sl = 0; sl < NS; ++sl)
        if (sl == os) r16_householder<RU>(a[sl], j, j & 3, p, rg, vsh, hh);
    }
    __syncthreads();
    const double tau = hh[1];
    // the slots' dependent chains are interleaved; a column that is done or
    // absent gets tw = 0 and is left as it is
    double v[RU], t[NS];
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) t[sl] = 0.0;
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      v[u] = vsh[p + 16 * u];
#pragma unroll
      for (int sl = 0; sl < NS; ++sl) t[sl] += v[u] * a[sl][u];
    }
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      const int c = 4 * (wid + kRQWaves * sl) + rg;
      const double dot = row16_sum(t[sl]);
      t[sl] = (c > j && c < n) ? tau * dot : 0.0;
    }
#pragma unroll
    for (int u = 0; u < RU; ++u)
#pragma unroll
      for (int sl = 0; sl < NS; ++sl) a[sl][u] -= t[sl] * v[u];
  }
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int c = 4 * (wid + kRQWaves * sl) + rg;
    if (c >= n) continue;
    double* dst = T.dst + (size_t)c * T.ldd;
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int r = p + 16 * u;
      if (r < n) dst[r] = r <= c ? a[sl][u] : 0.0;
    }
  }
}

// ---- pivoted QR in the 16-lane layout (one workgroup per box) ---------------
// The factorization of cpqr_reg_box (same pivot rule, stopping rule and
// outputs) of B.Mq (at most 256 rows), for boxes whose columns fit one
// workgroup.
template <int RU, int NS>
__device__ __forceinline__ void cpqr16_box(const LevelBox& B, const double tol, const int extra,
                                           int* k_out, int* kx_out, int* err, double* dyn,
                                           double* s_hh, double* wv, int* wi) {
  const int m = B.mq, n = B.n;
  const int tid = threadIdx.x, lane = tid & 63, p = lane & 15, rg = lane >> 4;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  double* vsh = dyn;                                    // 16 RU
  int* pv = reinterpret_cast<int*>(vsh + 16 * RU);      // n: physical column at each position
  int* ipv = pv + n;                                    // n: position of each physical column
  double a[NS][RU];
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int c = 4 * (wid + kRQWaves * sl) + rg;
    const double* src = B.Mq + (size_t)(c < n ? c : 0) * m;
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int i = p + 16 * u;
      a[sl][u] = (c < n && i < m) ? src[i] : 0.0;
    }
  }
  // the wave's pivot candidate: best of its lane groups (uniform within a group)
  auto publish = [&](double bv, int bi) {
    double rv = lane_f64(bv, 0);
    int ri = __builtin_amdgcn_readlane(bi, 0);
#pragma unroll
    for (int r = 16; r < 64; r += 16) arg_better(rv, ri, lane_f64(bv, r), __builtin_amdgcn_readlane(bi, r));
    if (lane == 0) { wv[wid] = rv; wi[wid] = ri; }
  };
  double t[NS];
  {
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) t[sl] = 0.0;
#pragma unroll
    for (int u = 0; u < RU; ++u)
#pragma unroll
      for (int sl = 0; sl < NS; ++sl) t[sl] += a[sl][u] * a[sl][u];
    double bv = -1.0;
    int bi = 1 << 30;
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      const int c = 4 * (wid + kRQWaves * sl) + rg;
      const double nn = row16_sum(t[sl]);
      if (c < n) arg_better(bv, bi, pivot_key(nn), c);
    }
    publish(bv, bi);
  }
  for (int c = tid; c < n; c += kRQThreads) { pv[c] = c; ipv[c] = c; }
  __syncthreads();
  unsigned dm = 0;                     // this lane group's slots whose column is pivoted
  const int steps = min(m, n);
  int limit = steps;
  int kk = -1;
  double r00 = 0.0;
  int j = 0;
  for (; j < limit; ++j) {
    double best = -1.0;
    int bq = 1 << 30;
    if (lane < kRQWaves) { best = wv[lane]; bq = wi[lane]; }
    wave_argmax(best, bq);
    const int q = __builtin_amdgcn_readfirstlane(bq);
    if (q >= n) {   // no finite candidate (non-finite entries in M_B): flag and stop
      if (tid == 0) __hip_atomic_store(err + 2, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    const int sq = q >> 2;
    if (wid == sq % kRQWaves) {
      const int os = sq / kRQWaves;
#pragma unroll
      for (int sl = 0; sl < NS; ++sl)
        if (sl == os) r16_householder<RU>(a[sl], j, q & 3, p, rg, vsh, s_hh);
    }
    __syncthreads();
    const double beta = s_hh[0], tau = s_hh[1];
    const double rjj = fabs(beta);
    if (j == 0) r00 = rjj;
    if (kk < 0 && !(rjj > tol * r00)) {
      kk = j;
      limit = min(steps, j + 1 + extra);
    }
    if (tid == 0) {
      const int pp = ipv[q];
      const int u = pv[j];
      pv[j] = q; pv[pp] = u;
      ipv[q] = j; ipv[u] = pp;
    }
    const int uj = j >> 4, pj = j & 15;
    double v[RU];
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      if (4 * (wid + kRQWaves * sl) + rg == q) dm |= 1u << sl;
      t[sl] = 0.0;
    }
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      v[u] = vsh[p + 16 * u];
#pragma unroll
      for (int sl = 0; sl < NS; ++sl) t[sl] += v[u] * a[sl][u];
    }
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      const int c = 4 * (wid + kRQWaves * sl) + rg;
      const double dot = row16_sum(t[sl]);
      t[sl] = (c < n && !((dm >> sl) & 1)) ? tau * dot : 0.0;
    }
#pragma unroll
    for (int u = 0; u < RU; ++u)
#pragma unroll
      for (int sl = 0; sl < NS; ++sl) a[sl][u] -= t[sl] * v[u];   // v is zero above row j
    // norms below row j, and this wave's next candidate
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) t[sl] = 0.0;
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      if (u > uj) {
#pragma unroll
        for (int sl = 0; sl < NS; ++sl) t[sl] += a[sl][u] * a[sl][u];
      } else if (u == uj) {
#pragma unroll
        for (int sl = 0; sl < NS; ++sl) t[sl] += p > pj ? a[sl][u] * a[sl][u] : 0.0;
      }
    }
    double bv = -1.0;
    int bi = 1 << 30;
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      const int c = 4 * (wid + kRQWaves * sl) + rg;
      const double nn = row16_sum(t[sl]);
      if (c < n && !((dm >> sl) & 1)) arg_better(bv, bi, pivot_key(nn), c);
    }
    publish(bv, bi);
    __syncthreads();
  }
  const int kx = j;
  if (kk < 0) kk = kx;
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int c = 4 * (wid + kRQWaves * sl) + rg;
    if (c >= n) continue;
    const int pp = ipv[c];
    double* dst = B.R + pp;
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int r = p + 16 * u;
      if (r < kx) dst[(size_t)r * n] = r <= pp ? a[sl][u] : 0.0;
    }
  }
  for (int c = tid; c < n; c += kRQThreads) B.perm[c] = pv[c];
  if (tid == 0) { k_out[B.slot] = kk; kx_out[B.slot] = kx; }
}

#define RS_R16_CASES(CALL) \
  case 17: CALL(2, 1); break; \
  case 18: CALL(2, 2); break; \
  case 19: CALL(2, 3); break; \
  case 20: CALL(2, 4); break; \
  case 33: CALL(4, 1); break; \
  case 34: CALL(4, 2); break; \
  case 35: CALL(4, 3); break; \
  case 36: CALL(4, 4); break; \
  case 49: CALL(6, 1); break; \
  case 50: CALL(6, 2); break; \
  case 51: CALL(6, 3); break; \
  case 52: CALL(6, 4); break; \
  case 65: CALL(8, 1); break; \
  case 66: CALL(8, 2); break; \
  case 67: CALL(8, 3); break; \
  case 68: CALL(8, 4); break; \
  case 81: CALL(10, 1); break; \
  case 82: CALL(10, 2); break; \
  case 83: CALL(10, 3); break; \
  case 84: CALL(10, 4); break; \
  case 97: CALL(12, 1); break; \
  case 98: CALL(12, 2); break; \
  case 99: CALL(12, 3); break; \
  case 100: CALL(12, 4); break; \
  case 113: CALL(14, 1); break; \
  case 114: CALL(14, 2); break; \
  case 115: CALL(14, 3); break; \
  case 116: CALL(14, 4); break; \
  case 129: CALL(16, 1); break; \
  case 130: CALL(16, 2); break; \
  case 131: CALL(16, 3); break; \
  case 132: CALL(16, 4); break; \
  default: break;

__global__ __launch_bounds__(kRQThreads) void k_tsqr(const QRTask* tasks) {
  __shared__ double vsh2[2 * 16 * kR16MaxRU];
  __shared__ double hh2[4];
  const QRTask& T = tasks[blockIdx.x];
#define RS_TSQR(R, S) tsqr16_block<R, S>(T, vsh2, hh2)
  switch (T.ru * 8 + (T.n + 31) / 32) { RS_R16_CASES(RS_TSQR) }
#undef RS_TSQR
}

__global__ __launch_bounds__(kRQThreads) void k_cpqr16(const LevelBox* boxes, const int4* work,
                                                       double tol, int extra, int* k_out, int* kx_out,
                                                       int* err) {
  __shared__ double dyn[16 * kR16MaxRU + kR16MaxCols];   // v, then pv / ipv as ints
  __shared__ double s_hh[2];
  __shared__ double wv[kRQWaves];
  __shared__ int wi[kRQWaves];
  const int4 w = work[blockIdx.x];
  const LevelBox& B = boxes[w.x];
#define RS_CPQR16(R, S) cpqr16_box<R, S>(B, tol, extra, k_out, kx_out, err, dyn, s_hh, wv, wi)
  switch (w.w * 8 + (B.n + 31) / 32) { RS_R16_CASES(RS_CPQR16) }
#undef RS_CPQR16
}

#define RS_RU_CASES(CALL)   \
  case 2: CALL(2); break;   \
  case 4: CALL(4); break;   \
  case 6: CALL(6); break;   \
  case 8: CALL(8); break;   \
  case 10: CALL(10); break; \
  case 12: CALL(12); break; \
  case 14: CALL(14); break; \
  case 16: CALL(16); break; \
  case 18: CALL(18); break; \
  case 20: CALL(20); break; \
  case 22: CALL(22); break; \
  default: CALL(24); break;


__global__ __launch_bounds__(kRQThreads) void k_cpqr_reg(const LevelBox* boxes, const int4* work,
                                                         double tol, int extra, int* k_out,
                                                         int* kx_out, int* err) {
  extern __shared__ double dyn[];
  __shared__ double s_hh[2];
  __shared__ double wv[kRQWaves];
  __shared__ int wi[kRQWaves];
  __shared__ int s_dead;
  const int4 w = work[blockIdx.x];
  const LevelBox& B = boxes[w.x];
  if (B.n == 0) {
    if (threadIdx.x == 0 && w.y == 0) { k_out[B.slot] = 0; kx_out[B.slot] = 0; }
    return;
  }
#define RS_CPQR(R) cpqr_reg_box<R>(B, w.z, w.y, tol, extra, k_out, kx_out, err, dyn, s_hh, &s_dead, wv, wi)
  switch (w.w) { RS_RU_CASES(RS_CPQR) }
#undef RS_CPQR
}

__global__ __launch_bounds__(kBlock) void k_assemble_abb(const LevelBox* boxes, double lam,
                                                         int use_perm) {
  const LevelBox& B = boxes[blockIdx.x];
  const int n = B.n;
  const int t = blockIdx.y * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  const int i = t / n, j = t % n;
  const int pi = use_perm ? B.perm[i] : i;
  const int pj = use_perm ? B.perm[j] : j;
  if (B.src) {
    const ChildSrc& si = B.src[pi];
    const ChildSrc& sj = B.src[pj];
    if (si.child == sj.child) {
      B.Ap[t] = si.xss[(size_t)si.idx * si.ld + sj.idx];
      return;
    }
  }
  const int di = B.dofs[pi], dj = B.dofs[pj];
  B.Ap[t] = op_entry(B.geo, di >> 1, di & 1, dj >> 1, dj & 1, lam);
}

// ---- elimination of the redundant unknowns (G workgroups per box) -----------

// C = beta*C0 + alpha*op(A) op(B), 4x4 tiles dealt cyclically over the
// G*blockDim threads of a box; no barrier inside.
__device__ void coop_gemm(int g, int G, int M, int N, int K, double alpha, const double* A,
                          int lda, bool tA, const double* B, int ldb, bool tB, double beta,
                          const double* C0, int ldc0, double* C, int ldc) {
  const int tm = (M + 3) >> 2, tn = (N + 3) >> 2;
  const int stride = G * blockDim.x;
  for (int t = g * blockDim.x + threadIdx.x; t < tm * tn; t += stride) {
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
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

// C = beta*C0 + alpha*op(A) op(B) on FP64 matrix cores.  32 x 32 blocks of C
// are dealt to the G workgroups of the box; in a block each of the 4 waves
// owns a 16 x 16 tile and accumulates v_mfma_f64_16x16x4 products over K
// chunks of 16 staged through LDS (zero padded at the edges).  Operand lanes:
// A[l % 16][l / 16], B[l / 16][l % 16]; result lane l, register q holds
// row 4 q + l / 16, column l % 16 of the tile.  C0 may alias C.
constexpr int kTB = 32;   // block edge
constexpr int kTK = 16;   // K chunk

__device__ void mfma_gemm(int g, int G, int M, int N, int K, double alpha, const double* A,
                          int lda, bool tA, const double* B, int ldb, bool tB, double beta,
                          const double* C0, int ldc0, double* C, int ldc, double* sA, double* sB) {
  const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
  const int bm = (M + kTB - 1) / kTB, bn = (N + kTB - 1) / kTB;
  const int wr = (wid >> 1) * 16, wc = (wid & 1) * 16;
  for (int blk = g; blk < bm * bn; blk += G) {
    const int i0 = (blk / bn) * kTB, j0 = (blk % bn) * kTB;
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += kTK) {
      for (int t = tid; t < kTB * kTK; t += blockDim.x) {
        const int ii = t / kTK, kk = t % kTK;
        const int gi = i0 + ii, gk = k0 + kk;
        sA[ii * (kTK + 1) + kk] =
            (gi < M && gk < K) ? (tA ? A[(size_t)gk * lda + gi] : A[(size_t)gi * lda + gk]) : 0.0;
        const int kb = t / kTB, jj = t % kTB;
        const int gk2 = k0 + kb, gj = j0 + jj;
        sB[kb * (kTB + 1) + jj] =
            (gk2 < K && gj < N) ? (tB ? B[(size_t)gj * ldb + gk2] : B[(size_t)gk2 * ldb + gj]) : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < kTK; kk += 4) {
        const double a = sA[(wr + (lane & 15)) * (kTK + 1) + kk + (lane >> 4)];
        const double b = sB[(kk + (lane >> 4)) * (kTB + 1) + wc + (lane & 15)];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
      }
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int gi = i0 + wr + 4 * q + (lane >> 4), gj = j0 + wc + (lane & 15);
      if (gi < M && gj < N) {
        double v = alpha * acc[q];
        if (C0) v += beta * C0[(size_t)gi * ldc0 + gj];
        C[(size_t)gi * ldc + gj] = v;
      }
    }
  }
}

// In-place Gauss-Jordan sweep with partial pivoting of X (r x r) held in
// LDS (W, row-major); the inverse of X goes to Xi (global, ld r).  One
// workgroup.  Returns the reciprocal 1-norm condition number (0 if a pivot
// vanished), identical in all threads.
constexpr int kLdsGJMax = 128;   // X_RR up to this edge is inverted by one workgroup (registers)
constexpr size_t kTSolveMax = 12288;   // T (k x r) up to this size is solved in LDS

// Gauss-Jordan inverse of X (r x r, row-major, r <= kLdsGJMax) by one
// workgroup with partial pivoting by exchange steps: step j pivots on the
// largest |W[i][j]| over the rows not used yet, and row i and column j trade
// places; the finished tableau W holds X^{-1} with X^{-1}[j][p_c] = W[p_j][c].
// A 16 x 16 thread grid keeps rows ty + 16 a, columns tx + 16 b of W in
// registers for the whole sweep; per step the pivot row and column go
// through LDS.  The pivot is compared on a 64-bit key (|W| with its low 8
// mantissa bits replaced by 255 - i, ties within 2^-44 to the smaller row)
// that the holders of column j + 1 fold into LDS with an atomic max during
// step j.  The update is one FMA per element (the multipliers absorb the
// pivot row and column).  Column 1-norms for rcond_1 are summed in a fixed
// order.  Two barriers per step.  Returns rcond_1 (0 if singular).
// LDS: gj_lds_doubles(r) doubles at `sh`.
__device__ __forceinline__ unsigned long long gj_key(double v, int i) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(fabs(v));
  return (b & ~0xFFull) | (unsigned long long)(255 - i);
}

__host__ __device__ constexpr size_t gj_lds_doubles(int r) { return 18 * (size_t)r + 4 + (size_t)r; }

__device__ double reg_gj(const double* X, int r, double* Xi, double* sh, double* red) {
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  constexpr int MB = (kLdsGJMax + 15) / 16;
  const int mb = (r + 15) >> 4;
  double* rowbuf = sh;                       // r: pivot row
  double* colbuf = rowbuf + r;               // r: pivot column
  double* part = colbuf + r;                 // 16 r: column-sum partials
  unsigned long long* keys = reinterpret_cast<unsigned long long*>(part + 16 * (size_t)r);   // 2
  int* pv = reinterpret_cast<int*>(keys + 2);        // r
  int* ipv = pv + r;                                  // r
  double w[MB][MB];
#pragma unroll
  for (int a = 0; a < MB; ++a) {
    if (a >= mb) break;
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      if (b >= mb) break;
      const int i = ty + 16 * a, c = tx + 16 * b;
      w[a][b] = (i < r && c < r) ? X[(size_t)i * r + c] : 0.0;
    }
  }
  if (tid < 2) keys[tid] = 0ull;
  // largest column 1-norm: per-thread partial sums, then 16 partials per column in order
  auto colnorm = [&]() {
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      if (b >= mb) break;
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < MB; ++a) {
        if (a >= mb) break;
        s += fabs(w[a][b]);
      }
      const int c = tx + 16 * b;
      if (c < r) part[ty * r + c] = s;
    }
    __syncthreads();
    double nm = 0.0;
    for (int c = tid; c < r; c += kBlock) {
      double s = 0.0;
      for (int t = 0; t < 16; ++t) s += part[t * r + c];
      nm = fmax(nm, s);
    }
    return block_max(nm, red);
  };
  const double n1 = colnorm();
  if (tx == 0)
#pragma unroll
    for (int a = 0; a < MB; ++a) {
      if (a >= mb) break;
      const int i = ty + 16 * a;
      if (i < r) atomicMax(&keys[0], gj_key(w[a][0], i));
    }
  __syncthreads();
  unsigned used = 0;             // bit a: row ty + 16 a is a pivot row already
  for (int j = 0; j < r; ++j) {
    const unsigned long long key = keys[j & 1];
    const int bi = 255 - (int)(key & 0xFF);
    const int ab = bi >> 4, bj = j >> 4;
    if (ty == (bi & 15))
#pragma unroll
      for (int a = 0; a < MB; ++a)
        if (a == ab)
#pragma unroll
          for (int b = 0; b < MB; ++b) {
            if (b >= mb) break;
            const int c = tx + 16 * b;
            if (c < r) rowbuf[c] = w[a][b];
          }
    if (tx == (j & 15))
#pragma unroll
      for (int b = 0; b < MB; ++b)
        if (b == bj)
#pragma unroll
          for (int a = 0; a < MB; ++a) {
            if (a >= mb) break;
            const int i = ty + 16 * a;
            if (i < r) colbuf[i] = w[a][b];
          }
    if (tid == 0) { keys[(j + 1) & 1] = 0ull; pv[j] = bi; }
    __syncthreads();
    const double pvt = colbuf[bi];
    if (!(pvt != 0.0)) return 0.0;          // uniform: every thread read the same key
    if ((bi & 15) == ty) used |= 1u << ab;
    const double inv = 1.0 / pvt;
    double pr[MB], pc[MB];
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      if (b >= mb) break;
      const int c = tx + 16 * b;
      pr[b] = c < r ? (c == j ? inv : rowbuf[c] * inv) : 0.0;
      const int i = ty + 16 * b;
      pc[b] = i < r ? (i == bi ? -1.0 : colbuf[i]) : 0.0;
    }
    const int bn = (j + 1) >> 4;
    double cand[MB];
#pragma unroll
    for (int a = 0; a < MB; ++a) {
      if (a >= mb) break;
      const bool prow = ty + 16 * a == bi;
      cand[a] = 0.0;
#pragma unroll
      for (int b = 0; b < MB; ++b) {
        if (b >= mb) break;
        const double w0 = (prow || tx + 16 * b == j) ? 0.0 : w[a][b];
        w[a][b] = w0 - pc[a] * pr[b];
        if (b == bn) cand[a] = w[a][b];
      }
    }
    if (tx == ((j + 1) & 15) && j + 1 < r)
#pragma unroll
      for (int a = 0; a < MB; ++a) {
        if (a >= mb) break;
        const int i = ty + 16 * a;
        if (i < r && !((used >> a) & 1)) atomicMax(&keys[(j + 1) & 1], gj_key(cand[a], i));
      }
    __syncthreads();
  }
  // X^{-1}[j][p_c] = W[p_j][c]
  for (int j = tid; j < r; j += kBlock) ipv[pv[j]] = j;
  __syncthreads();
#pragma unroll
  for (int a = 0; a < MB; ++a) {
    if (a >= mb) break;
    const int i = ty + 16 * a;
    if (i >= r) continue;
    const int row = ipv[i];
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      if (b >= mb) break;
      const int c = tx + 16 * b;
      if (c < r) Xi[(size_t)row * r + pv[c]] = w[a][b];
    }
  }
  // column c of W is column p_c of X^{-1} with its rows permuted
  const double n2 = colnorm();
  const double rc = 1.0 / (n1 * n2);
  return isfinite(rc) ? rc : 0.0;
}

// T = R11^{-1} R12 (k x r, row-major) by back substitution on all columns at
// once, T staged in LDS (k r doubles): step i removes row i's contribution
// from the rows above it; one barrier per step.  R: k x n rows of R, pivot order.
__device__ void lds_tsolve(const double* R, int n, int k, int r, double* Tl, double* T) {
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  for (int l = ty; l < k; l += 16)
    for (int c = tx; c < r; c += 16) Tl[l * r + c] = R[(size_t)l * n + k + c];
  __syncthreads();
  for (int i = k - 1; i > 0; --i) {
    const double d = R[(size_t)i * n + i];
    for (int c = tx; c < r; c += 16) {
      const double x = Tl[i * r + c] / d;
      for (int l = ty; l < i; l += 16) Tl[l * r + c] -= R[(size_t)l * n + i] * x;
    }
    __syncthreads();
  }
  for (int l = ty; l < k; l += 16) {
    const double d = R[(size_t)l * n + l];
    for (int c = tx; c < r; c += 16) T[(size_t)l * r + c] = Tl[l * r + c] / d;
  }
  __syncthreads();
}

__device__ double lds_gj(const double* X, int r, double* W, double* Xi, double* rowj, double* colj,
                         int* rowperm, double* red, int* ired) {
  const int tid = threadIdx.x, NT = blockDim.x, lane = tid & 63, wid = tid >> 6;
  for (int t = tid; t < r * r; t += NT) W[t] = X[t];
  for (int c = tid; c < r; c += NT) rowperm[c] = c;
  __syncthreads();
  double n1 = 0.0;
  for (int c = tid; c < r; c += NT) {
    double sum = 0.0;
    for (int i = 0; i < r; ++i) sum += fabs(W[i * r + c]);
    n1 = fmax(n1, sum);
  }
  n1 = block_max(n1, red);
  bool singular = false;
  for (int j = 0; j < r; ++j) {
    double best = -1.0;
    int bi = r;
    for (int i = j + tid; i < r; i += NT) {
      const double v = fabs(W[i * r + j]);
      if (v > best) { best = v; bi = i; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    __syncthreads();
    if (lane == 0) { red[wid] = best; ired[wid] = bi; }
    __syncthreads();
    best = red[0];
    bi = ired[0];
    for (int w = 1; w < (NT >> 6); ++w)
      if (red[w] > best || (red[w] == best && ired[w] < bi)) { best = red[w]; bi = ired[w]; }
    if (!(best > 0.0)) { singular = true; break; }
    // row interchange, then copies of the pivot row and column
    for (int c = tid; c < r; c += NT) {
      double a = W[j * r + c];
      double b = W[bi * r + c];
      if (bi != j) {
        W[j * r + c] = b;
        W[bi * r + c] = a;
        a = b;
      }
      rowj[c] = a;
    }
    if (tid == 0 && bi != j) {
      const int t = rowperm[j];
      rowperm[j] = rowperm[bi];
      rowperm[bi] = t;
    }
    __syncthreads();
    for (int i = tid; i < r; i += NT) colj[i] = W[i * r + j];
    __syncthreads();
    const double inv = 1.0 / rowj[j];
    for (int t = tid; t < r * r; t += NT) {
      const int i = t / r, c = t % r;
      double v;
      if (i == j) v = (c == j) ? inv : rowj[c] * inv;
      else if (c == j) v = -colj[i] * inv;
      else v = W[t] - colj[i] * (rowj[c] * inv);
      W[t] = v;
    }
    __syncthreads();
  }
  if (singular) return 0.0;
  for (int t = tid; t < r * r; t += NT) {
    const int i = t / r, c = t % r;
    Xi[(size_t)i * r + rowperm[c]] = W[t];
  }
  __syncthreads();
  double n2 = 0.0;
  for (int c = tid; c < r; c += NT) {
    double sum = 0.0;
    for (int i = 0; i < r; ++i) sum += fabs(Xi[(size_t)i * r + c]);
    n2 = fmax(n2, sum);
  }
  n2 = block_max(n2, red);
  const double rc = 1.0 / (n1 * n2);
  return isfinite(rc) ? rc : 0.0;
}

// Largest column 1-norm of X (n x n, ld ldx) over the box, identical in all workgroups.
__device__ double coop_norm1(int g, int G, const double* X, int n, int ldx, double* red,
                             const LevelBox& B, unsigned& nbar, int* dead, int* err) {
  double v = 0.0;
  for (int c = g * blockDim.x + threadIdx.x; c < n; c += G * blockDim.x) {
    double sum = 0.0;
    for (int i = 0; i < n; ++i) sum += fabs(X[(size_t)i * ldx + c]);
    v = fmax(v, sum);
  }
  v = block_max(v, red);
  if (G == 1) return v;
  if (threadIdx.x == 0) st_relaxed(B.cval + g, v);
  box_barrier_x(B.bar, G, nbar, dead, err);
  double m = 0.0;
  for (int h = 0; h < G; ++h) m = fmax(m, ld_relaxed(B.cval + h));
  box_barrier_x(B.bar, G, nbar, dead, err);   // slots are reused afterwards
  return m;
}

constexpr int kGJP = 32;   // pivot block of the in-place Gauss-Jordan

// X_RR^{-1} of the box (blocked in-place Gauss-Jordan with partial pivoting,
// panels of kGJP columns): W holds X_RR on entry and is destroyed; Xi receives
// the inverse.  Returns false (uniformly) if a pivot vanished.
__device__ bool coop_gj(int g, int G, double* W, int r, double* Xi, double* Pn, double* Rb,
                        double* Cp, double* Dinv, int* piv, int* rowperm, int* flag, double* red,
                        int* ired, const LevelBox& B, unsigned& nbar, int* dead, int* err) {
  const int NT = blockDim.x, tid = threadIdx.x;
  const int gt = g * NT + tid, GT = G * NT;
  for (int c = gt; c < r; c += GT) rowperm[c] = c;
  __shared__ double lu[kGJP][kGJP + 1];
  __shared__ double inv[kGJP][kGJP + 1];
  for (int k0 = 0; k0 < r; k0 += kGJP) {
    const int bb = min(kGJP, r - k0);
    const int h = r - k0;
    if (g == 0) {
      // panel: LU with partial pivoting of W[k0:r, k0:k0+bb] (private copy Pn)
      for (int t = tid; t < h * bb; t += NT) {
        const int i = t / bb, c = t % bb;
        Pn[t] = W[(size_t)(k0 + i) * r + k0 + c];
      }
      __syncthreads();
      bool singular = false;
      for (int j = 0; j < bb; ++j) {
        double best = -1.0;
        int bi = h;
        for (int i = j + tid; i < h; i += NT) {
          const double v = fabs(Pn[(size_t)i * bb + j]);
          if (v > best) { best = v; bi = i; }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          const double ov = __shfl_xor(best, o, 64);
          const int oi = __shfl_xor(bi, o, 64);
          if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
        }
        const int lane = tid & 63, wid = tid >> 6;
        if (lane == 0) { red[wid] = best; ired[wid] = bi; }
        __syncthreads();
        best = red[0];
        bi = ired[0];
        for (int w = 1; w < (NT >> 6); ++w)
          if (red[w] > best || (red[w] == best && ired[w] < bi)) { best = red[w]; bi = ired[w]; }
        __syncthreads();
        if (!(best > 0.0)) { singular = true; break; }
        if (tid == 0) piv[j] = bi;
        if (bi != j)
          for (int c = tid; c < bb; c += NT) {
            const double a = Pn[(size_t)j * bb + c];
            Pn[(size_t)j * bb + c] = Pn[(size_t)bi * bb + c];
            Pn[(size_t)bi * bb + c] = a;
          }
        __syncthreads();
        const double d = Pn[(size_t)j * bb + j];
        for (int i = j + 1 + tid; i < h; i += NT) Pn[(size_t)i * bb + j] /= d;
        __syncthreads();
        const int rest = bb - j - 1;
        if (rest > 0)
          for (int t = tid; t < (h - j - 1) * rest; t += NT) {
            const int i = j + 1 + t / rest, c = j + 1 + t % rest;
            Pn[(size_t)i * bb + c] -= Pn[(size_t)i * bb + j] * Pn[(size_t)j * bb + c];
          }
        __syncthreads();
      }
      if (singular) {
        if (tid == 0) *flag = 1;
      } else {
        for (int t = tid; t < bb * bb; t += NT) lu[t / bb][t % bb] = Pn[t];
        __syncthreads();
        if (tid < bb) {
          const int c = tid;
          double y[kGJP];
          for (int i = 0; i < bb; ++i) {
            double sum = (i == c) ? 1.0 : 0.0;
            for (int l = 0; l < i; ++l) sum -= lu[i][l] * y[l];
            y[i] = sum;
          }
          for (int i = bb - 1; i >= 0; --i) {
            double sum = y[i];
            for (int l = i + 1; l < bb; ++l) sum -= lu[i][l] * y[l];
            y[i] = sum / lu[i][i];
          }
          for (int i = 0; i < bb; ++i) inv[i][c] = y[i];
        }
        __syncthreads();
        for (int t = tid; t < bb * bb; t += NT) Dinv[t] = inv[t / bb][t % bb];
      }
    }
    box_barrier_full(B.bar, G, nbar, dead, err);
    if (*(volatile int*)flag) return false;
    // row interchanges over all columns; the owner of a panel column copies it
    for (int c = gt; c < r; c += GT) {
      for (int j = 0; j < bb; ++j) {
        const int rr = k0 + piv[j];
        if (rr != k0 + j) {
          const double a = W[(size_t)(k0 + j) * r + c];
          W[(size_t)(k0 + j) * r + c] = W[(size_t)rr * r + c];
          W[(size_t)rr * r + c] = a;
        }
      }
    }
    if (g == 0 && tid == 0)
      for (int j = 0; j < bb; ++j) {
        const int rr = k0 + piv[j];
        const int t = rowperm[k0 + j];
        rowperm[k0 + j] = rowperm[rr];
        rowperm[rr] = t;
      }
    box_barrier_full(B.bar, G, nbar, dead, err);
    for (int t = gt; t < r * bb; t += GT) {
      const int i = t / bb, l = t % bb;
      Cp[t] = W[(size_t)i * r + k0 + l];
    }
    for (int t = gt; t < bb * r; t += GT) {
      const int i = t / r, c = t % r;
      double sum = 0.0;
      for (int l = 0; l < bb; ++l) sum += Dinv[i * bb + l] * W[(size_t)(k0 + l) * r + c];
      Rb[t] = sum;
    }
    box_barrier_full(B.bar, G, nbar, dead, err);
    for (int t = gt; t < r * r; t += GT) {
      const int i = t / r, c = t % r;
      const bool ik = i >= k0 && i < k0 + bb;
      const bool ck = c >= k0 && c < k0 + bb;
      double v;
      if (ik) {
        v = ck ? Dinv[(i - k0) * bb + (c - k0)] : Rb[(size_t)(i - k0) * r + c];
      } else if (ck) {
        double sum = 0.0;
        for (int l = 0; l < bb; ++l) sum += Cp[(size_t)i * bb + l] * Dinv[l * bb + (c - k0)];
        v = -sum;
      } else {
        double sum = 0.0;
        for (int l = 0; l < bb; ++l) sum += Cp[(size_t)i * bb + l] * Rb[(size_t)l * r + c];
        v = W[t] - sum;
      }
      W[t] = v;
    }
    box_barrier_full(B.bar, G, nbar, dead, err);
  }
  for (int t = gt; t < r * r; t += GT) {
    const int i = t / r, c = t % r;
    Xi[(size_t)i * r + rowperm[c]] = W[t];
  }
  box_barrier_full(B.bar, G, nbar, dead, err);
  return true;
}

// Per box (G workgroups): T = R11^{-1} R12; X_SR, X_RS, X_RR (eq. tmat);
// X_RR^{-1} with the rcond guard (move the next pivot to S while
// rcond_1(X_RR) < rcond_min); E, F and the Schur complement X_SS (eq. schurmat).
__global__ __launch_bounds__(kBlock) void k_eliminate(const LevelBox* boxes, int G, int* k_io,
                                                      const int* kx_in, double rcond_min,
                                                      int* status, double* rc_out, int* err) {
  extern __shared__ double smem_e[];
  constexpr int NW = kBlock / 64;
  __shared__ double red[NW];
  __shared__ int ired[NW];
  __shared__ int s_dead;
  __shared__ double sA[kTB * (kTK + 1)];
  __shared__ double sB[kTK * (kTB + 1)];
  const int bidx = blockIdx.x / G, g = blockIdx.x % G;
  const LevelBox& B = boxes[bidx];
  const int n = B.n;
  if (n == 0) return;
  if (threadIdx.x == 0) s_dead = 0;
  __syncthreads();
  unsigned nbar = 0;
  int k = k_io[B.slot];
  const int kx = kx_in[B.slot];
  int st = 0;
  double rc_final = 1.0;          // rcond_1 of the accepted X_RR (1 when r = 0)
  const double* Ap = B.Ap;
  const int gt = g * kBlock + threadIdx.x, GT = G * kBlock;
  while (true) {
    const int r = n - k;
    double* T = B.T;
    // the route depends on k and r only (not on the launch)
    if ((size_t)k * r <= kTSolveMax) {
      if (g == 0) lds_tsolve(B.R, n, k, r, smem_e, T);
    } else {
      for (int c = gt; c < r; c += GT) {
        for (int i = k - 1; i >= 0; --i) {
          double sum = B.R[(size_t)i * n + k + c];
          for (int l = i + 1; l < k; ++l) sum -= B.R[(size_t)i * n + l] * T[(size_t)l * r + c];
          T[(size_t)i * r + c] = sum / B.R[(size_t)i * n + i];
        }
      }
    }
    box_barrier_full(B.bar, G, nbar, &s_dead, err);
    if (r == 0) {
      for (int t = gt; t < k * k; t += GT) {
        const int i = t / k, c = t % k;
        B.Xss[t] = Ap[(size_t)i * n + c];
      }
      break;
    }
    double* Xsr = B.scr;
    double* Xrs = Xsr + (size_t)k * r;
    double* Xrr = Xrs + (size_t)r * k;
    double* W = Xrr + (size_t)r * r;
    double* Pn = W + (size_t)r * r;
    double* Rb = Pn + (size_t)r * kGJP;
    double* Cp = Rb + (size_t)kGJP * r;
    double* Dinv = Cp + (size_t)r * kGJP;
    int* piv = reinterpret_cast<int*>(Dinv + kGJP * kGJP);
    int* rowperm = piv + kGJP;
    int* flag = rowperm + r + 1;
    mfma_gemm(g, G, k, r, k, -1.0, Ap, n, false, T, r, false, 1.0, Ap + k, n, Xsr, r, sA, sB);
    mfma_gemm(g, G, r, k, k, -1.0, T, r, true, Ap, n, false, 1.0, Ap + (size_t)k * n, n, Xrs, k, sA, sB);
    mfma_gemm(g, G, r, r, k, -1.0, Ap + (size_t)k * n, n, false, T, r, false, 1.0,
              Ap + (size_t)k * n + k, n, Xrr, r, sA, sB);
    if (g == 0 && threadIdx.x == 0) *flag = 0;
    box_barrier_full(B.bar, G, nbar, &s_dead, err);
    // X_RR -= T^T X_SR
    mfma_gemm(g, G, r, r, k, -1.0, T, r, true, Xsr, r, false, 1.0, Xrr, r, W, r, sA, sB);
    box_barrier_full(B.bar, G, nbar, &s_dead, err);
    double rc = 0.0;
    // the inversion algorithm depends on r only (not on G), so a box factors
    // identically whatever launch it is part of
    if (r <= kLdsGJMax) {
      if (g == 0) {
        rc = reg_gj(W, r, B.Xinv, smem_e, red);
        if (G > 1 && threadIdx.x == 0) st_relaxed(B.cval, rc);
      }
      if (G > 1) {
        box_barrier_full(B.bar, G, nbar, &s_dead, err);
        rc = ld_relaxed(B.cval);
      }
    } else {
      const double n1 = coop_norm1(g, G, W, r, r, red, B, nbar, &s_dead, err);
      const bool ok = coop_gj(g, G, W, r, B.Xinv, Pn, Rb, Cp, Dinv, piv, rowperm, flag, red, ired,
                              B, nbar, &s_dead, err);
      if (ok) {
        const double n2 = coop_norm1(g, G, B.Xinv, r, r, red, B, nbar, &s_dead, err);
        rc = 1.0 / (n1 * n2);
        if (!isfinite(rc)) rc = 0.0;
      }
    }
    if (!(rc >= rcond_min)) {
      if (k < kx) {
        ++k;
        box_barrier_full(B.bar, G, nbar, &s_dead, err);
        continue;
      }
      st = 1;
    }
    rc_final = rc;
    box_barrier_full(B.bar, G, nbar, &s_dead, err);
    mfma_gemm(g, G, k, r, r, 1.0, Xsr, r, false, B.Xinv, r, false, 0.0, nullptr, 0, B.E, r, sA, sB);
    mfma_gemm(g, G, r, k, r, 1.0, B.Xinv, r, false, Xrs, k, false, 0.0, nullptr, 0, B.F, k, sA, sB);
    box_barrier_full(B.bar, G, nbar, &s_dead, err);
    mfma_gemm(g, G, k, k, r, -1.0, Xsr, r, false, B.F, k, false, 1.0, Ap, n, B.Xss, k, sA, sB);
    break;
  }
  if (g == 0 && threadIdx.x == 0) {
    k_io[B.slot] = k;
    status[B.slot] = st;
    rc_out[B.slot] = rc_final;
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
// A panel without a nonzero pivot sets *status; every kernel of the sequence
// returns at once when *status is set, so no pivot index of a failed panel is
// ever used (the panel also leaves its unused entries as the identity).
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
  if (*(volatile const int*)status) return;
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
    if (!(best > 0.0)) {
      for (int jj = j + tid; jj < bb; jj += kBlock) piv[jj] = jj;
      singular = true;
      break;
    }
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
                           const int* status) {
  if (*(volatile const int*)status) return;
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

__global__ void k_gjb_copycol(const double* A, int n, int k0, int bb, double* Cpanel,
                              const int* status) {
  if (*(volatile const int*)status) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * bb) return;
  const int i = t / bb, c = t % bb;
  Cpanel[t] = A[(size_t)i * n + k0 + c];
}

// R = D^{-1} A[K, :]
__global__ void k_gjb_rows(const double* A, int n, int k0, int bb, const double* Dinv, double* R,
                           const int* status) {
  if (*(volatile const int*)status) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= bb * n) return;
  const int i = t / n, c = t % n;
  double s = 0.0;
  for (int l = 0; l < bb; ++l) s += Dinv[i * bb + l] * A[(size_t)(k0 + l) * n + c];
  R[t] = s;
}

__global__ void k_gjb_update(double* A, int n, int k0, int bb, const double* Dinv,
                             const double* R, const double* Cpanel, const int* status) {
  if (*(volatile const int*)status) return;
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

template <typename T>
__global__ __launch_bounds__(kBlock) void k_diag(const SolveBox* boxes, const int* ridx, T* c,
                                                 int ncols, int kNC) {
  extern __shared__ double smem_d[];
  T* smem = reinterpret_cast<T*>(smem_d);
  const SolveBox& B = boxes[blockIdx.x];
  if (B.r == 0) return;
  if (B.Xinvf) diag_box<T, float>(B, B.Xinvf, ridx, c, ncols, kNC, smem);
  else diag_box<T, double>(B, B.Xinv, ridx, c, ncols, kNC, smem);
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

// parts[box] (3p x ncols) = Ph_R^T c_R (accumulated in float64)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_border_rhs(const SolveBox* boxes, const int* ridx,
                                                       const T* Ph, int p3, const T* c, int ncols,
                                                       double* parts) {
  const SolveBox& B = boxes[blockIdx.x];
  double* out = parts + (size_t)B.part * p3 * ncols;
  const int* R = ridx + B.r_off;
  for (int t = threadIdx.x; t < p3 * ncols; t += kBlock) {
    const int h = t / ncols, q = t % ncols;
    double acc = 0.0;
    for (int i = 0; i < B.r; ++i)
      acc += (double)Ph[(size_t)R[i] * p3 + h] * (double)c[(size_t)R[i] * ncols + q];
    out[t] = acc;
  }
}

// c_R -= W lam
template <typename T>
__global__ __launch_bounds__(kBlock) void k_border_fix(const SolveBox* boxes, const int* ridx,
                                                       int p3, const double* lam, T* c,
                                                       int ncols) {
  const SolveBox& B = boxes[blockIdx.x];
  const int* R = ridx + B.r_off;
  for (int t = threadIdx.x; t < B.r * ncols; t += kBlock) {
    const int i = t / ncols, q = t % ncols;
    double acc = 0.0;
    if (B.Wf)
      for (int h = 0; h < p3; ++h) acc += (double)B.Wf[(size_t)i * p3 + h] * lam[(size_t)h * ncols + q];
    else
      for (int h = 0; h < p3; ++h) acc += B.W[(size_t)i * p3 + h] * lam[(size_t)h * ncols + q];
    c[(size_t)R[i] * ncols + q] -= (T)acc;
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

__global__ void k_dense_apply(const double* Zinv, int nz, const double* v, int ncols,
                              double* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nz * ncols) return;
  const int i = t / ncols, q = t % ncols;
  double acc = 0.0;
  for (int j = 0; j < nz; ++j) acc += Zinv[(size_t)i * nz + j] * v[(size_t)j * ncols + q];
  out[t] = acc;
}

template <typename T>
__global__ void k_root_scatter(const double* sol, int ncols, const int* I0, int n0, T* c) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n0 * ncols) return;
  const int i = t / ncols, q = t % ncols;
  c[(size_t)I0[i] * ncols + q] = (T)sol[t];
}

// y = (T) x  (element count n)
template <typename TO, typename TI>
__global__ void k_convert(const TI* x, long long n, TO* y) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[t] = (TO)x[t];
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
// captured graph).  flag[0] = 1 once max_q sqrt(colsq[q] / fsq[q]) <= tol
// (fsq = 0 counts as 1); flag[1] counts the corrections applied.  Per
// iteration: k_accumulate_unless (reads the flags), operator apply, residual,
// then k_refine_flag (the only writer: counts the correction the iteration
// applied, then tests the new residual).
__global__ void k_refine_flag(const double* colsq, const double* fsq, int ncols, double tol,
                              int max_iters, int* flag) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  if (flag[0] == 0 && flag[1] < max_iters) flag[1] += 1;
  double worst = 0.0;
  for (int q = 0; q < ncols; ++q) {
    const double fq = fsq[q] > 0.0 ? fsq[q] : 1.0;
    worst = fmax(worst, sqrt(colsq[q] / fq));
  }
  flag[0] = worst <= tol ? 1 : 0;
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

// r = [f; 0] - y  (rows layout, f has nf rows); colsq[q] = ||r_q||^2 and fsq[q] = ||f_q||^2,
// one block per column, fixed-order sums.
__global__ __launch_bounds__(kBlock) void k_residual(const double* f, int nf, const double* y,
                                                    int nrows, int ncols, double* r,
                                                    double* colsq, double* fsq) {
  constexpr int NW = kBlock / 64;
  __shared__ double red[NW];
  const int q = blockIdx.x;
  double sr = 0.0, sf = 0.0;
  for (int i = threadIdx.x; i < nrows; i += kBlock) {
    const double fi = i < nf ? f[(size_t)i * ncols + q] : 0.0;
    const double v = fi - y[(size_t)i * ncols + q];
    r[(size_t)i * ncols + q] = v;
    sr += v * v;
    sf += fi * fi;
  }
  sr = block_sum(sr, red);
  sf = block_sum(sf, red);
  if (threadIdx.x == 0) { colsq[q] = sr; fsq[q] = sf; }
}

// float copies of the factor blocks of every box of a level (sizes from the final ranks)
__global__ void k_factor_to_float(const LevelBox* boxes, const int* k_final) {
  const LevelBox& B = boxes[blockIdx.x];
  const int n = B.n;
  if (n == 0) return;
  const int k = k_final[B.slot], r = n - k;
  const int kr = k * r, rr = r * r;
  for (int t = threadIdx.x; t < kr; t += blockDim.x) {
    B.Tf[t] = (float)B.T[t];
    B.Ef[t] = (float)B.E[t];
    B.Ff[t] = (float)B.F[t];
  }
  for (int t = threadIdx.x; t < rr; t += blockDim.x) B.Xinvf[t] = (float)B.Xinv[t];
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

// ---- exact float64 operator (refinement residual) ---------------------------
// y = A x with A = [[lam I + D + N, H], [Psi^T, -I]]; x, y row layout
// [(2N + 3p)][ncols].  Blocks tile (targets) x (source chunks) x (column
// chunks); each block writes the partial sums of its source chunk, and a
// second kernel adds the chunks in a fixed order (deterministic).
constexpr int kApplyCols = 8;
constexpr int kApplyTile = 256;

__global__ __launch_bounds__(kApplyTile) void k_apply_D(Geo g, double lam, const double* x,
                                                        int ncols, int chunk, double* part) {
  __shared__ double sx[kApplyTile], sy[kApplyTile], snx[kApplyTile], sny[kApplyTile],
      sw[kApplyTile];
  __shared__ double sm[kApplyTile][2 * kApplyCols];
  const int N = g.N;
  const int i = blockIdx.x * kApplyTile + threadIdx.x;
  const int js0 = blockIdx.y * chunk, js1 = min(N, js0 + chunk);
  const int q0 = blockIdx.z * kApplyCols;
  const int nq = min(kApplyCols, ncols - q0);
  const bool live = i < N;
  const double xi = live ? g.x[i] : 0.0, yi = live ? g.y[i] : 0.0;
  const double nxi = live ? g.nx[i] : 0.0, nyi = live ? g.ny[i] : 0.0;
  double ax[kApplyCols], ay[kApplyCols];
#pragma unroll
  for (int q = 0; q < kApplyCols; ++q) { ax[q] = 0.0; ay[q] = 0.0; }
  for (int j0 = js0; j0 < js1; j0 += kApplyTile) {
    const int j = j0 + threadIdx.x;
    __syncthreads();
    if (j < js1) {
      sx[threadIdx.x] = g.x[j];
      sy[threadIdx.x] = g.y[j];
      snx[threadIdx.x] = g.nx[j];
      sny[threadIdx.x] = g.ny[j];
      sw[threadIdx.x] = g.w[j];
#pragma unroll
      for (int q = 0; q < kApplyCols; ++q) {
        sm[threadIdx.x][2 * q] = q < nq ? x[(size_t)(2 * j) * ncols + q0 + q] : 0.0;
        sm[threadIdx.x][2 * q + 1] = q < nq ? x[(size_t)(2 * j + 1) * ncols + q0 + q] : 0.0;
      }
    }
    __syncthreads();
    const int cnt = min(kApplyTile, js1 - j0);
    if (!live) continue;
    for (int jj = 0; jj < cnt; ++jj) {
      const int js = j0 + jj;
      double bxx, bxy, byy;
      const double wn_x = sw[jj] * snx[jj], wn_y = sw[jj] * sny[jj];
      if (js == i) {
        const double tx = -nyi, ty = nxi;
        const double c = -(g.w[i] * g.kap[i]) / (2.0 * kPi);
        bxx = c * tx * tx + lam;
        bxy = c * tx * ty;
        byy = c * ty * ty + lam;
      } else {
        const double rx = xi - sx[jj], ry = yi - sy[jj];
        const double r2 = rx * rx + ry * ry;
        const double rn = rx * snx[jj] + ry * sny[jj];
        const double coef = kInvPi * sw[jj] * rn / (r2 * r2);
        bxx = coef * rx * rx;
        bxy = coef * rx * ry;
        byy = coef * ry * ry;
      }
      const double byx = bxy + nyi * wn_x;
      bxx += nxi * wn_x;
      bxy += nxi * wn_y;
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
  double* out = part + (size_t)blockIdx.y * 2 * N * ncols;
  for (int q = 0; q < nq; ++q) {
    out[(size_t)(2 * i) * ncols + q0 + q] = ax[q];
    out[(size_t)(2 * i + 1) * ncols + q0 + q] = ay[q];
  }
}

// y[2N rows] = sum over source chunks (fixed order) + H lambda
__global__ void k_apply_sum(Geo g, const double* hole_xy, int p, const double* x, int ncols,
                            const double* part, int nchunk, double* y) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int N = g.N;
  if (t >= (long long)N * ncols) return;
  const int i = (int)(t / ncols), q = (int)(t % ncols);
  const size_t stride = (size_t)2 * N * ncols;
  double ax = 0.0, ay = 0.0;
  for (int c = 0; c < nchunk; ++c) {
    ax += part[c * stride + (size_t)(2 * i) * ncols + q];
    ay += part[c * stride + (size_t)(2 * i + 1) * ncols + q];
  }
  const double xi = g.x[i], yi = g.y[i];
  const size_t base = (size_t)2 * N;
  for (int h = 0; h < p; ++h) {
    const double rx = xi - hole_xy[2 * h], ry = yi - hole_xy[2 * h + 1];
    const double r2 = rx * rx + ry * ry;
    const double lg = -0.5 * log(r2);
    const double sxx = kInv4Pi * (lg + rx * rx / r2), sxy = kInv4Pi * (rx * ry / r2);
    const double syy = kInv4Pi * (lg + ry * ry / r2);
    const double rotx = kInv4Pi * (-ry) / r2, roty = kInv4Pi * rx / r2;
    const double a1 = x[(base + 3 * h) * ncols + q];
    const double a2 = x[(base + 3 * h + 1) * ncols + q];
    const double b = x[(base + 3 * h + 2) * ncols + q];
    ax += sxx * a1 + sxy * a2 + rotx * b;
    ay += sxy * a1 + syy * a2 + roty * b;
  }
  y[(size_t)(2 * i) * ncols + q] = ax;
  y[(size_t)(2 * i + 1) * ncols + q] = ay;
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

void launch_assemble_M(const LevelBox* boxes, int nbox, int max_m, int n_proxy, double ratio,
                       hipStream_t s) {
  if (nbox == 0 || max_m == 0) return;
  dim3 grid(nbox, blocks_for(max_m, kBlock));
  hipLaunchKernelGGL(k_assemble_M, grid, dim3(kBlock), 0, s, boxes, n_proxy, ratio);
}

size_t cpqr_lds_bytes(int max_m, int max_n) {
  return (size_t)max_n * (2 * sizeof(double) + 4 * sizeof(int) + 1) + (size_t)max_m * sizeof(double) + 64;
}

// Workgroups per resident CU for the pivoted-QR kernel with `lds` bytes of LDS.
int cpqr_blocks_per_cu(size_t lds) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_cpqr, kQRThreads, lds) != hipSuccess) return 0;
  return nb;
}

void launch_zero_bars(const LevelBox* boxes, int nbox, int* err, hipStream_t s) {
  if (nbox == 0) return;
  hipLaunchKernelGGL(k_zero_bars, dim3(blocks_for(std::max(nbox, 3), kBlock)), dim3(kBlock), 0, s, boxes,
                     nbox, err, 3);
}

hipError_t launch_cpqr(const LevelBox* boxes, const int* list, int nbox, int G, double tol, int extra,
                       int* k_out, int* kx_out, int* err, int max_m, int max_n, hipStream_t s) {
  if (nbox == 0) return hipSuccess;
  const size_t lds = cpqr_lds_bytes(max_m, max_n);
  if (G <= 1) {
    hipLaunchKernelGGL(k_cpqr, dim3(nbox), dim3(kQRThreads), lds, s, boxes, list, 1, tol, extra,
                       k_out, kx_out, err);
    return hipGetLastError();
  }
  void* args[] = {(void*)&boxes, (void*)&list, (void*)&G, (void*)&tol, (void*)&extra,
                  (void*)&k_out, (void*)&kx_out, (void*)&err};
  return hipLaunchCooperativeKernel((const void*)k_cpqr, dim3(nbox * G), dim3(kQRThreads), args,
                                    (unsigned)lds, s);
}

size_t cpqr_reg_lds_bytes(int max_ru, int max_n) {
  return (size_t)(64 * max_ru) * sizeof(double) + 2 * (size_t)max_n * sizeof(int) + 64;
}

void launch_tsqr(const QRTask* tasks, int ntask, hipStream_t s) {
  if (ntask == 0) return;
  hipLaunchKernelGGL(k_tsqr, dim3(ntask), dim3(kRQThreads), 0, s, tasks);
}

hipError_t launch_cpqr16(const LevelBox* boxes, const int4* work, int nbox, double tol, int extra,
                         int* k_out, int* kx_out, int* err, hipStream_t s) {
  if (nbox == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cpqr16, dim3(nbox), dim3(kRQThreads), 0, s, boxes, work, tol, extra, k_out,
                     kx_out, err);
  return hipGetLastError();
}

int cpqr_reg_blocks_per_cu(size_t lds) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_cpqr_reg, kRQThreads, lds) != hipSuccess) return 0;
  return nb;
}

hipError_t launch_cpqr_reg(const LevelBox* boxes, const int4* work, int nblocks, bool coop, double tol,
                           int extra, int* k_out, int* kx_out, int* err, size_t lds, hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  if (!coop) {
    hipLaunchKernelGGL(k_cpqr_reg, dim3(nblocks), dim3(kRQThreads), lds, s, boxes, work, tol, extra,
                       k_out, kx_out, err);
    return hipGetLastError();
  }
  void* args[] = {(void*)&boxes, (void*)&work, (void*)&tol, (void*)&extra,
                  (void*)&k_out, (void*)&kx_out, (void*)&err};
  return hipLaunchCooperativeKernel((const void*)k_cpqr_reg, dim3(nblocks), dim3(kRQThreads), args,
                                    (unsigned)lds, s);
}

void launch_assemble_abb(const LevelBox* boxes, int nbox, int max_n, double lam, bool use_perm,
                         hipStream_t s) {
  if (nbox == 0 || max_n == 0) return;
  dim3 grid(nbox, blocks_for((long long)max_n * max_n, kBlock));
  hipLaunchKernelGGL(k_assemble_abb, grid, dim3(kBlock), 0, s, boxes, lam, use_perm ? 1 : 0);
}

size_t eliminate_lds_bytes(int max_n) {
  const int r = std::min(max_n, kLdsGJMax);
  const size_t gj = gj_lds_doubles(r) * sizeof(double);
  const size_t ts = std::min<size_t>((size_t)max_n * max_n / 4, kTSolveMax) * sizeof(double);
  return std::max(gj, ts) + 64;
}

int eliminate_blocks_per_cu(int max_n) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_eliminate, kBlock,
                                                   eliminate_lds_bytes(max_n)) != hipSuccess)
    return 0;
  return nb;
}

hipError_t launch_eliminate(const LevelBox* boxes, int nbox, int G, int* k_io, const int* kx,
                            double rcond_min, int* status, double* rc_out, int* err, int max_n,
                            hipStream_t s) {
  if (nbox == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_bars, dim3(blocks_for(nbox, kBlock)), dim3(kBlock), 0, s, boxes, nbox, err, 1);
  const size_t lds = eliminate_lds_bytes(max_n);
  if (lds > 65536) {
    hipFuncAttributes fa;
    hipError_t e = hipFuncGetAttributes(&fa, (const void*)k_eliminate);
    if (e != hipSuccess) return e;
    if (fa.maxDynamicSharedSizeBytes < (int)lds) {
      e = hipFuncSetAttribute((const void*)k_eliminate, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
      if (e != hipSuccess) return e;
    }
  }
  if (G <= 1) {
    hipLaunchKernelGGL(k_eliminate, dim3(nbox), dim3(kBlock), lds, s, boxes, 1, k_io, kx, rcond_min,
                       status, rc_out, err);
    return hipGetLastError();
  }
  void* args[] = {(void*)&boxes, (void*)&G, (void*)&k_io, (void*)&kx, (void*)&rcond_min,
                  (void*)&status, (void*)&rc_out, (void*)&err};
  return hipLaunchCooperativeKernel((const void*)k_eliminate, dim3(nbox * G), dim3(kBlock), args,
                                    (unsigned)lds, s);
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
                       piv, rowperm, status);
    hipLaunchKernelGGL(k_gjb_copycol, dim3(blocks_for((long long)n * bb, kBlock)), dim3(kBlock), 0,
                       s, A, n, k0, bb, Cp, status);
    hipLaunchKernelGGL(k_gjb_rows, dim3(blocks_for((long long)bb * n, kBlock)), dim3(kBlock), 0, s,
                       A, n, k0, bb, Dinv, R, status);
    hipLaunchKernelGGL(k_gjb_update, dim3(blocks_for(nn, kBlock)), dim3(kBlock), 0, s, A, n, k0, bb,
                       Dinv, R, Cp, status);
  }
  hipLaunchKernelGGL(k_gjb_unpermute, dim3(blocks_for(nn, kBlock)), dim3(kBlock), 0, s, A, n,
                     rowperm, Ainv);
}

template <typename T>
void launch_sweep(const SolveBox* boxes, int nbox, const int* sidx, const int* ridx, T* c,
                  int ncols, int mode, int max_n, hipStream_t s) {
  if (nbox == 0 || ncols == 0) return;
  const int nc = chunk_cols(max_n);
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
  const int nc = chunk_cols(2 * max_r);
  dim3 grid(nbox, blocks_for(ncols, nc));
  const size_t shm = (size_t)2 * max_r * nc * sizeof(T);
  hipLaunchKernelGGL(k_diag<T>, grid, dim3(kBlock), shm, s, boxes, ridx, c, ncols, nc);
}
template void launch_diag<double>(const SolveBox*, int, const int*, double*, int, int, hipStream_t);

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

template <typename T>
void launch_border_rhs(const SolveBox* boxes, int nbox, const int* ridx, const T* Ph, int p3,
                       const T* c, int ncols, double* parts, hipStream_t s) {
  if (nbox == 0) return;
  hipLaunchKernelGGL(k_border_rhs<T>, dim3(nbox), dim3(kBlock), 0, s, boxes, ridx, Ph, p3, c, ncols,
                     parts);
}
template void launch_border_rhs<double>(const SolveBox*, int, const int*, const double*, int,
                                        const double*, int, double*, hipStream_t);

template <typename T>
void launch_border_fix(const SolveBox* boxes, int nbox, const int* ridx, int p3, const double* lam,
                       T* c, int ncols, hipStream_t s) {
  if (nbox == 0) return;
  hipLaunchKernelGGL(k_border_fix<T>, dim3(nbox), dim3(kBlock), 0, s, boxes, ridx, p3, lam, c, ncols);
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
  hipLaunchKernelGGL(k_dense_apply, dim3(blocks_for((long long)nz * ncols, 64)), dim3(64), 0, s,
                     Zinv, nz, v, ncols, out);
}

template <typename T>
void launch_root_scatter(const double* sol, int ncols, const int* I0, int n0, T* c, hipStream_t s) {
  hipLaunchKernelGGL(k_root_scatter<T>, dim3(blocks_for((long long)n0 * ncols, kBlock)),
                     dim3(kBlock), 0, s, sol, ncols, I0, n0, c);
}
template void launch_root_scatter<double>(const double*, int, const int*, int, double*, hipStream_t);

void launch_to_float(const double* x, long long n, float* y, hipStream_t s) {
  if (n) hipLaunchKernelGGL((k_convert<float, double>), dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, x, n, y);
}
void launch_to_double(const float* x, long long n, double* y, hipStream_t s) {
  if (n) hipLaunchKernelGGL((k_convert<double, float>), dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, x, n, y);
}
void launch_refine_flag(const double* colsq, const double* fsq, int ncols, double tol, int max_iters,
                        int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_refine_flag, dim3(1), dim3(64), 0, s, colsq, fsq, ncols, tol, max_iters, flag);
}

void launch_accumulate_unless(const double* d, long long n, double* x, const int* flag, int max_iters,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_accumulate_unless, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, d, n, x,
                     flag, max_iters);
}

void launch_set_ints(int* p, int n, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_ints, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, p, n, v);
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
void launch_residual(const double* f, int nf, const double* y, int nrows, int ncols, double* r,
                     double* colsq, double* fsq, hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3(ncols), dim3(kBlock), 0, s, f, nf, y, nrows, ncols, r, colsq, fsq);
}
void launch_factor_to_float(const LevelBox* boxes, int nbox, const int* k_final, hipStream_t s) {
  if (nbox) hipLaunchKernelGGL(k_factor_to_float, dim3(nbox), dim3(kBlock), 0, s, boxes, k_final);
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

// Source chunk length so that targets x chunks gives about 2048 blocks.
int apply_chunk(int N) {
  const int tiles = (N + kApplyTile - 1) / kApplyTile;
  const int want = std::max(1, 2048 / std::max(1, tiles));
  int chunk = (N + want - 1) / want;
  chunk = ((chunk + kApplyTile - 1) / kApplyTile) * kApplyTile;
  return std::max(chunk, kApplyTile);
}

size_t apply_scratch_doubles(int N, int ncols) {
  const int chunk = apply_chunk(N);
  const int nchunk = (N + chunk - 1) / chunk;
  return (size_t)nchunk * 2 * N * ncols;
}

void launch_apply_operator(Geo g, const int* curve_id, const double* hole_xy, int p, double lam,
                           const double* x, int ncols, double* y, double* part, hipStream_t s) {
  const int chunk = apply_chunk(g.N);
  const int nchunk = (g.N + chunk - 1) / chunk;
  dim3 grid(blocks_for(g.N, kApplyTile), nchunk, blocks_for(ncols, kApplyCols));
  hipLaunchKernelGGL(k_apply_D, grid, dim3(kApplyTile), 0, s, g, lam, x, ncols, chunk, part);
  hipLaunchKernelGGL(k_apply_sum, dim3(blocks_for((long long)g.N * ncols, kBlock)), dim3(kBlock), 0, s,
                     g, hole_xy, p, x, ncols, part, nchunk, y);
  if (p > 0)
    hipLaunchKernelGGL(k_apply_psi, dim3(3 * p), dim3(kBlock), 0, s, g, curve_id, p, x, ncols, y);
}

}  // namespace rs

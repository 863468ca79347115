#pragma once
// Device-side helpers shared by the gfx950 kernels of the solver: wave and
// block reductions, pivot keys, the Stokes kernel entries, a workgroup GEMM,
// box barriers of cooperative launches and small launch helpers.  Everything
// has internal linkage; each kernel source includes this header once.
#include "rs_internal.h"

#include <algorithm>
#include <cmath>

namespace rs {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kInvPi = 0.31830988618379067154;
constexpr double kInv4Pi = 0.07957747154594766788;
constexpr double kInv2Pi = 0.15915494309189533577;

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

// ---- the Laplace Neumann kernel (Section 4.4.1) ------------------------------
// Operator lam I - D + N with D the adjoint double layer (normal at the
// target) and N mu = the integral of mu.  Its density lives in component 0 of
// each node; component 1 is an uncoupled unknown with the row lam x (kept so
// that vectors have the Stokes path's two-per-node layout; it joins no box).

// -D between distinct points: (1/2pi) ((x - y) . n_x) / |x - y|^2 w_y.
__device__ __forceinline__ double lap_dl(double rx, double ry, double nx, double ny, double w) {
  return kInv2Pi * w * (rx * nx + ry * ny) / (rx * rx + ry * ry);
}

// Entry of lam I - D + N; the coincident limit of -D is kappa w / (4 pi).
__device__ __forceinline__ double lap_op_entry(const Geo& g, int ti, int tc, int sj, int sc,
                                               double lam) {
  if (tc | sc) return (ti == sj && tc == sc) ? lam : 0.0;
  if (ti == sj) return lam + kInv4Pi * g.kap[ti] * g.w[ti] + g.w[ti];
  return lap_dl(g.x[ti] - g.x[sj], g.y[ti] - g.y[sj], g.nx[ti], g.ny[ti], g.w[sj]) + g.w[sj];
}

// Entry of lam I + D + N between unknown (ti, tc) (target node, component)
// and (sj, sc).  Coincident nodes use the curvature limit of D.
__device__ __forceinline__ double op_entry(const Geo& g, int ti, int tc, int sj, int sc,
                                           double lam) {
  if (g.kernel == 1) return lap_op_entry(g, ti, tc, sj, sc, lam);
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

// ---- the same entries in float32 (the float32 bulk form) -------------------
// Positions enter as box-local offsets: (x - c_B) rounded to float, with c_B
// the compressed box's centre, so that a difference of two nearby nodes keeps
// float32's relative precision whatever the domain's size.
__device__ __forceinline__ float dl_entry_f(float rx, float ry, float nx, float ny, float w, int a,
                                            int b) {
  const float r2 = rx * rx + ry * ry;
  const float rn = rx * nx + ry * ny;
  const float coef = (float)kInvPi * w * rn / (r2 * r2);
  return coef * (a ? ry : rx) * (b ? ry : rx);
}

__device__ __forceinline__ float sl_entry_f(float rx, float ry, float w, int a, int b) {
  const float r2 = rx * rx + ry * ry;
  float v = (a ? ry : rx) * (b ? ry : rx) / r2;
  if (a == b) v += -0.5f * logf(r2);
  return (float)kInv4Pi * w * v;
}

// The Laplace Neumann entries in float32 (box-local offsets, as below).
__device__ __forceinline__ float lap_dl_f(float rx, float ry, float nx, float ny, float w) {
  return (float)kInv2Pi * w * (rx * nx + ry * ny) / (rx * rx + ry * ry);
}

__device__ __forceinline__ float lap_op_entry_f(const Geo& g, int ti, int tc, int sj, int sc, double lam,
                                                double cx, double cy) {
  if (tc | sc) return (ti == sj && tc == sc) ? (float)lam : 0.0f;
  if (ti == sj) return (float)lam + (float)kInv4Pi * (float)g.kap[ti] * (float)g.w[ti] + (float)g.w[ti];
  const float rx = (float)(g.x[ti] - cx) - (float)(g.x[sj] - cx);
  const float ry = (float)(g.y[ti] - cy) - (float)(g.y[sj] - cy);
  return lap_dl_f(rx, ry, (float)g.nx[ti], (float)g.ny[ti], (float)g.w[sj]) + (float)g.w[sj];
}

// op_entry in float32; (cx, cy) = the box centre the offsets are taken from.
__device__ __forceinline__ float op_entry_f(const Geo& g, int ti, int tc, int sj, int sc, double lam,
                                            double cx, double cy) {
  if (g.kernel == 1) return lap_op_entry_f(g, ti, tc, sj, sc, lam, cx, cy);
  float v;
  if (ti == sj) {
    const float tx = (float)-g.ny[ti], ty = (float)g.nx[ti];
    const float c = -((float)g.w[ti] * (float)g.kap[ti]) / (2.0f * (float)kPi);
    v = c * (tc ? ty : tx) * (sc ? ty : tx);
    if (tc == sc) v += (float)lam;
  } else {
    const float rx = (float)(g.x[ti] - cx) - (float)(g.x[sj] - cx);
    const float ry = (float)(g.y[ti] - cy) - (float)(g.y[sj] - cy);
    v = dl_entry_f(rx, ry, (float)g.nx[sj], (float)g.ny[sj], (float)g.w[sj], tc, sc);
  }
  const float nt = (float)(tc ? g.ny[ti] : g.nx[ti]);
  const float ns = (float)(sc ? g.ny[sj] : g.nx[sj]);
  return v + nt * ((float)g.w[sj] * ns);
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

__global__ void k_zero_bars(const LevelBox* boxes, int nbox, int* err, int nerr) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nbox && boxes[t].bar) *boxes[t].bar = 0u;
  if (t < nerr) err[t] = 0;
}

inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace
}  // namespace rs

// gfx950 kernels applying the exact float64 operator of the augmented system
// (eq. backwardeq), the residual of iterative refinement.
#include "rs_device.h"

#include <cstdio>
#include <mutex>
#include <type_traits>

namespace rs {
namespace {

// ---- exact float64 operator (refinement residual) ---------------------------
// y = A x with A = [[lam I + D + N, H], [Psi^T, -I]]; x, y row layout
// [(2N + 3p)][ncols].  The O(N^2) part is the double layer D between distinct
// nodes; the diagonal (curvature limit and lam), the rank-one completion N
// (n_i sum_j w_j n_j . x_j) and the border columns are O(N) and are added by
// k_apply_sum.  Blocks tile (targets) x (source chunks) x (column chunks);
// each block writes the partial sums of its source chunk and k_apply_sum adds
// the chunks in a fixed order (deterministic).
//
// A thread holds T targets and NC right-hand-side columns in registers; every
// source staged in LDS (position, w n / pi, its NC column values) serves the T
// targets, so LDS traffic per pair falls as 1 / T.  (NC, T) is chosen per
// problem shape by the host's autotuner.
constexpr int kApplyThreads = 256;   // threads per block = sources per LDS tile

// 1 / d from the hardware reciprocal and one Newton step (relative error
// about one ulp).
__device__ __forceinline__ double recip(double d) {
  const double y0 = __builtin_amdgcn_rcp(d);
  const double e = fma(-d, y0, 1.0);
  return fma(y0, e, y0);
}

// A floor added to |r|^4 so that a coincident pair (a target's own node,
// r = 0) needs no branch: its |r|^4 + floor has a finite reciprocal and its
// r . n is zero, so it contributes exactly zero.  For every other pair |r|^4
// exceeds the floor by more than 2^53 and the sum rounds to |r|^4 itself.
constexpr double kR4Floor = 1e-300;

// Packed source weights: w n / pi (the double layer's prefactor folded in).
__device__ __forceinline__ double2 source_wn(double w, double nx, double ny) {
  const double wp = w * kInvPi;
  return make_double2(wp * nx, wp * ny);
}

// Add one source's double-layer block to NC columns of a target at (xi, yi):
// the 2 x 2 block c r r^T, c = (r . w n / pi) / |r|^4, r = target - source,
// formed once and applied to every column as two chains of two FMAs (32
// independent accumulators keep the FP64 pipeline full).
template <int NC>
__device__ __forceinline__ void pair_add(double xi, double yi, double px, double py, double wnx, double wny,
                                         const double* mv, double* ax, double* ay) {
  const double rx = xi - px, ry = yi - py;
  const double r2 = fma(rx, rx, ry * ry);
  const double rn = fma(rx, wnx, ry * wny);
  const double c = rn * recip(fma(r2, r2, kR4Floor));
  const double crx = c * rx;
  const double bxx = crx * rx, bxy = crx * ry, byy = c * ry * ry;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    ax[q] = fma(bxx, mv[2 * q], fma(bxy, mv[2 * q + 1], ax[q]));
    ay[q] = fma(bxy, mv[2 * q], fma(byy, mv[2 * q + 1], ay[q]));
  }
}

// What a refinement iteration's apply does, from the refinement flags (null
// outside refinement): flag[0] converged, flag[1] iterations done, flag[2] = 1
// when the iteration updates the residual with a float32 image of the
// correction.  -1: nothing (converged or out of iterations); 0: the exact
// float64 apply of x; 1: the float32 correction image (A dx).
__device__ __forceinline__ int apply_mode(const int* flag, int max_iters) {
  if (!flag) return 0;
  if (flag[0] != 0 || flag[1] >= max_iters) return -1;
  return flag[2] == 1 ? 1 : 0;
}

// Targets (tx, ty), nt of them: the boundary nodes themselves for the
// operator apply, arbitrary points for the evaluation of the velocity.
template <int NC, int T>
__global__ __launch_bounds__(kApplyThreads) void k_apply_pairs(Geo g, const double* __restrict__ tx,
                                                               const double* __restrict__ ty, int nt,
                                                               const double* __restrict__ x,
                                                               int ncols, int chunk,
                                                               double* __restrict__ part,
                                                               const int* skip, int max_iters) {
  if (apply_mode(skip, max_iters) != 0) return;
  __shared__ double2 sxy[kApplyThreads];
  __shared__ double2 swn[kApplyThreads];
  __shared__ double sm[kApplyThreads * 2 * NC];
  const int N = g.N, tid = threadIdx.x;
  const int ib = blockIdx.x * (kApplyThreads * T) + tid;
  const int js0 = blockIdx.y * chunk, js1 = min(N, js0 + chunk);
  const int q0 = blockIdx.z * NC;
  const int nq = min(NC, ncols - q0);
  double xi[T], yi[T];
  double ax[T][NC], ay[T][NC];
#pragma unroll
  for (int u = 0; u < T; ++u) {
    const int i = ib + u * kApplyThreads;
    xi[u] = i < nt ? tx[i] : 0.0;
    yi[u] = i < nt ? ty[i] : 0.0;
#pragma unroll
    for (int q = 0; q < NC; ++q) { ax[u][q] = 0.0; ay[u][q] = 0.0; }
  }
  for (int j0 = js0; j0 < js1; j0 += kApplyThreads) {
    const int j = j0 + tid;
    __syncthreads();
    if (j < js1) {
      const double w = g.w[j];
      sxy[tid] = make_double2(g.x[j], g.y[j]);
      swn[tid] = source_wn(w, g.nx[j], g.ny[j]);
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        sm[tid * 2 * NC + 2 * q] = q < nq ? x[(size_t)(2 * j) * ncols + q0 + q] : 0.0;
        sm[tid * 2 * NC + 2 * q + 1] = q < nq ? x[(size_t)(2 * j + 1) * ncols + q0 + q] : 0.0;
      }
    }
    __syncthreads();
    const int cnt = min(kApplyThreads, js1 - j0);
    for (int jj = 0; jj < cnt; ++jj) {
      const double2 p = sxy[jj];
      const double2 wn = swn[jj];
      double mv[2 * NC];
#pragma unroll
      for (int t = 0; t < 2 * NC; ++t) mv[t] = sm[jj * 2 * NC + t];
#pragma unroll
      for (int u = 0; u < T; ++u) pair_add<NC>(xi[u], yi[u], p.x, p.y, wn.x, wn.y, mv, ax[u], ay[u]);
    }
  }
  double* out = part + (size_t)blockIdx.y * 2 * nt * ncols;
#pragma unroll
  for (int u = 0; u < T; ++u) {
    const int i = ib + u * kApplyThreads;
    if (i >= nt) continue;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      if (q < nq) {
        out[(size_t)(2 * i) * ncols + q0 + q] = ax[u][q];
        out[(size_t)(2 * i + 1) * ncols + q0 + q] = ay[u][q];
      }
    }
  }
}

// The same pair sums with the sources read by uniform (scalar) loads instead
// of LDS: src4 packs (x, y, w n_x / pi, w n_y / pi) per node; each wave walks the sources
// of its chunk in order, every lane holding T targets.  Same arithmetic and
// order per target as k_apply_pairs (bitwise the same result).
template <int NC, int T>
__global__ __launch_bounds__(kApplyThreads) void k_apply_pairs_s(const double4* __restrict__ src4,
                                                                 const double* __restrict__ tx,
                                                                 const double* __restrict__ ty, int nt,
                                                                 int N, const double* __restrict__ x,
                                                                 int ncols, int chunk,
                                                                 double* __restrict__ part,
                                                                 const int* __restrict__ skip,
                                                                 int max_iters) {
  if (apply_mode(skip, max_iters) != 0) return;
  const int tid = threadIdx.x;
  const int ib = blockIdx.x * (kApplyThreads * T) + tid;
  const int js0 = blockIdx.y * chunk, js1 = min(N, js0 + chunk);
  const int q0 = blockIdx.z * NC;
  const int nq = min(NC, ncols - q0);
  double xi[T], yi[T];
  double ax[T][NC], ay[T][NC];
#pragma unroll
  for (int u = 0; u < T; ++u) {
    const int i = ib + u * kApplyThreads;
    xi[u] = i < nt ? tx[i] : 0.0;
    yi[u] = i < nt ? ty[i] : 0.0;
#pragma unroll
    for (int q = 0; q < NC; ++q) { ax[u][q] = 0.0; ay[u][q] = 0.0; }
  }
  // full column chunks read without per-column checks
  auto sweep = [&](auto full) {
    for (int js = js0; js < js1; ++js) {
      const double4 sp = src4[js];
      double mv[2 * NC];
      const double* xr0 = x + (size_t)(2 * js) * ncols + q0;
      const double* xr1 = xr0 + ncols;
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        if (decltype(full)::value) {
          mv[2 * q] = xr0[q];
          mv[2 * q + 1] = xr1[q];
        } else {
          mv[2 * q] = q < nq ? xr0[q] : 0.0;
          mv[2 * q + 1] = q < nq ? xr1[q] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < T; ++u) pair_add<NC>(xi[u], yi[u], sp.x, sp.y, sp.z, sp.w, mv, ax[u], ay[u]);
    }
  };
  if (nq == NC) sweep(std::true_type{});
  else sweep(std::false_type{});
  double* out = part + (size_t)blockIdx.y * 2 * nt * ncols;
#pragma unroll
  for (int u = 0; u < T; ++u) {
    const int i = ib + u * kApplyThreads;
    if (i >= nt) continue;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      if (q < nq) {
        out[(size_t)(2 * i) * ncols + q0 + q] = ax[u][q];
        out[(size_t)(2 * i + 1) * ncols + q0 + q] = ay[u][q];
      }
    }
  }
}

// ---- the Laplace Neumann operator (Section 4.4.1) -----------------------------
// Pair sums of -D mu (the adjoint double layer, normal at the target) at the
// boundary nodes, EVAL = 0, or of S mu and d(S mu)/dx at arbitrary targets,
// EVAL = 1.  The density is component 0 of each node's pair of unknowns.  A
// thread holds one target and NC columns; a block stages 256 sources (position,
// w / 2pi, NC density values) in LDS.  Grid and chunking as for the Stokes
// pairs: per source chunk the partial sums go to rows 2i (and 2i + 1 for the
// x-derivative) of that chunk's slice of `part`, added in a fixed order by the
// O(N) kernels.
template <int NC, int EVAL>
__global__ __launch_bounds__(kApplyThreads) void k_lap_pairs(Geo g, const double* __restrict__ tx,
                                                             const double* __restrict__ ty, int nt,
                                                             const double* __restrict__ x, int ncols,
                                                             int chunk, double* __restrict__ part,
                                                             const int* skip, int max_iters) {
  if (apply_mode(skip, max_iters) != 0) return;
  __shared__ double2 sxy[kApplyThreads];
  __shared__ double sw[kApplyThreads];
  __shared__ double sm[kApplyThreads * NC];
  const int N = g.N, tid = threadIdx.x;
  const int i = blockIdx.x * kApplyThreads + tid;
  const int js0 = blockIdx.y * chunk, js1 = min(N, js0 + chunk);
  const int q0 = blockIdx.z * NC;
  const int nq = min(NC, ncols - q0);
  const double xi = i < nt ? tx[i] : 0.0, yi = i < nt ? ty[i] : 0.0;
  const double nxi = (!EVAL && i < nt) ? g.nx[i] : 0.0, nyi = (!EVAL && i < nt) ? g.ny[i] : 0.0;
  double a[NC], b[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) { a[q] = 0.0; b[q] = 0.0; }
  for (int j0 = js0; j0 < js1; j0 += kApplyThreads) {
    const int j = j0 + tid;
    __syncthreads();
    if (j < js1) {
      sxy[tid] = make_double2(g.x[j], g.y[j]);
      sw[tid] = kInv2Pi * g.w[j];
#pragma unroll
      for (int q = 0; q < NC; ++q) sm[tid * NC + q] = q < nq ? x[(size_t)(2 * j) * ncols + q0 + q] : 0.0;
    }
    __syncthreads();
    const int cnt = min(kApplyThreads, js1 - j0);
    for (int jj = 0; jj < cnt; ++jj) {
      const double2 p = sxy[jj];
      const double rx = xi - p.x, ry = yi - p.y;
      // the floor makes a target's own node (r = 0, r . n = 0) contribute
      // exactly zero without a branch; every other pair's |r|^2 exceeds it
      // by far more than 2^53
      const double r2 = fma(rx, rx, fma(ry, ry, kR4Floor));
      const double ir2 = recip(r2);
      if (EVAL) {
        const double cu = -0.5 * sw[jj] * log(r2);
        const double cx = -sw[jj] * rx * ir2;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
          a[q] = fma(cu, sm[jj * NC + q], a[q]);
          b[q] = fma(cx, sm[jj * NC + q], b[q]);
        }
      } else {
        const double c = fma(rx, nxi, ry * nyi) * ir2 * sw[jj];
#pragma unroll
        for (int q = 0; q < NC; ++q) a[q] = fma(c, sm[jj * NC + q], a[q]);
      }
    }
  }
  if (i >= nt) return;
  double* out = part + (size_t)blockIdx.y * 2 * nt * ncols;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    if (q < nq) {
      out[(size_t)(2 * i) * ncols + q0 + q] = a[q];
      if (EVAL) out[(size_t)(2 * i + 1) * ncols + q0 + q] = b[q];
    }
  }
}

// src4[j] = (x_j, y_j, w_j n_xj / pi, w_j n_yj / pi)
__global__ void k_pack_sources(Geo g, double4* src4) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= g.N) return;
  const double2 wn = source_wn(g.w[j], g.nx[j], g.ny[j]);
  src4[j] = make_double4(g.x[j], g.y[j], wn.x, wn.y);
}

// Threads per block of the two node reductions below (k_apply_nsum,
// k_apply_psi): they have few blocks, so a wide block keeps the
// per-thread loop over the nodes short.
constexpr int kNodeSumThreads = 1024;

// The rank-one term's scalar of column q, sum_j w_j (n_j . x_j), in
// kNsumParts node ranges: block (q, b) sums range b into nsum[q kNsumParts + b]
// and k_apply_sum adds the ranges in order (fixed-order sums).
constexpr int kNsumParts = 8;
// The O(N) kernels below take x (the exact apply) and xc (the correction, read
// when the refinement flags ask for its image).
__global__ __launch_bounds__(kNodeSumThreads) void k_apply_nsum(Geo g, const double* x, const double* xc,
                                                                int ncols, double* nsum, const int* skip,
                                                                int max_iters) {
  const int md = apply_mode(skip, max_iters);
  if (md < 0) return;
  if (md == 1) x = xc;
  constexpr int NW = kNodeSumThreads / 64;
  __shared__ double red[NW];
  const int q = blockIdx.x, b = blockIdx.y;
  const int len = (g.N + kNsumParts - 1) / kNsumParts;
  const int j1 = min(g.N, (b + 1) * len);
  double s = 0.0;
  if (g.kernel == 1) {   // Laplace: N mu = sum_j w_j mu_j
    for (int j = b * len + threadIdx.x; j < j1; j += kNodeSumThreads) s += g.w[j] * x[(size_t)(2 * j) * ncols + q];
  } else {
    for (int j = b * len + threadIdx.x; j < j1; j += kNodeSumThreads)
      s += g.w[j] * (g.nx[j] * x[(size_t)(2 * j) * ncols + q] + g.ny[j] * x[(size_t)(2 * j + 1) * ncols + q]);
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) nsum[q * kNsumParts + b] = s;
}

// The Stokes form of k_apply_sum with p > 0 holes (see there); called by the
// whole block, so every thread reaches the barriers.
constexpr int kSumCoefs = 320;   // (node, hole) coefficient sets per chunk
__device__ __forceinline__ void apply_sum_stokes(const Geo& g, double lam, const double* hole_xy, int p,
                                                 const double* x, int ncols, const double* part, int nchunk,
                                                 const double* nsum, const float* bpart, double* bt, double* y) {
  __shared__ double coef[kSumCoefs * 5];
  const int N = g.N;
  const long long t0 = (long long)blockIdx.x * kBlock;
  const long long t = t0 + threadIdx.x;
  const bool live = t < (long long)N * ncols;
  const int i = live ? (int)(t / ncols) : 0, q = (int)(t % ncols);
  // nodes of this block's (node, column) range: at most kBlock of them
  const int i_lo = (int)(t0 / ncols);
  const int i_hi = (int)min((long long)N - 1, (t0 + kBlock - 1) / ncols);
  const int nn = i_hi - i_lo + 1;
  const int hcap = max(1, kSumCoefs / nn);
  const size_t stride = (size_t)2 * N * ncols;
  double ax = 0.0, ay = 0.0;
  if (live) {
    for (int c = 0; c < nchunk; ++c) {
      ax += part[c * stride + (size_t)(2 * i) * ncols + q];
      ay += part[c * stride + (size_t)(2 * i + 1) * ncols + q];
    }
    if (bpart) {
      double b = 0.0;
      for (int c = 0; c < nchunk; ++c) b += (double)bpart[((size_t)c * N + i) * ncols + q];
      bt[(size_t)i * ncols + q] = b;
    }
    const double mx = x[(size_t)(2 * i) * ncols + q], my = x[(size_t)(2 * i + 1) * ncols + q];
    const double nxi = g.nx[i], nyi = g.ny[i];
    {
      const double tx = -nyi, ty = nxi;
      const double cs = -(g.w[i] * g.kap[i]) / (2.0 * kPi);
      ax += (cs * tx * tx + lam) * mx + cs * tx * ty * my;
      ay += cs * tx * ty * mx + (cs * ty * ty + lam) * my;
    }
    double ns = 0.0;
    for (int b = 0; b < kNsumParts; ++b) ns += nsum[q * kNsumParts + b];
    ax += nxi * ns;
    ay += nyi * ns;
  }
  const size_t base = (size_t)2 * N;
  for (int h0 = 0; h0 < p; h0 += hcap) {
    const int hn = min(hcap, p - h0);
    __syncthreads();
    for (int e = threadIdx.x; e < nn * hn; e += kBlock) {
      const int node = i_lo + e / hn, h = h0 + e % hn;
      const double rx = g.x[node] - hole_xy[2 * h], ry = g.y[node] - hole_xy[2 * h + 1];
      const double r2 = rx * rx + ry * ry;
      const double lg = -0.5 * log(r2);
      double* cf = coef + 5 * e;
      cf[0] = kInv4Pi * (lg + rx * rx / r2);
      cf[1] = kInv4Pi * (rx * ry / r2);
      cf[2] = kInv4Pi * (lg + ry * ry / r2);
      cf[3] = kInv4Pi * (-ry) / r2;
      cf[4] = kInv4Pi * rx / r2;
    }
    __syncthreads();
    if (live) {
      const double* cfi = coef + 5 * (size_t)(i - i_lo) * hn;
      for (int u = 0; u < hn; ++u) {
        const int h = h0 + u;
        const double* cf = cfi + 5 * u;
        const double a1 = x[(base + 3 * h) * ncols + q];
        const double a2 = x[(base + 3 * h + 1) * ncols + q];
        const double b = x[(base + 3 * h + 2) * ncols + q];
        ax += cf[0] * a1 + cf[1] * a2 + cf[3] * b;
        ay += cf[1] * a1 + cf[2] * a2 + cf[4] * b;
      }
    }
  }
  if (live) {
    y[(size_t)(2 * i) * ncols + q] = ax;
    y[(size_t)(2 * i + 1) * ncols + q] = ay;
  }
}

// y[2N rows] = sum over source chunks (fixed order) + the diagonal (lam and
// the curvature limit of D) + the rank-one term + H lambda
// For a correction image it also adds the rounding bounds of the chunks
// (bpart, float) into bt (per node and column).
// With holes, the Stokeslet and rotlet coefficients of H (per node and hole,
// the same for every column) are formed once per block in LDS, a chunk of
// holes at a time, and every (node, column) thread adds the holes in order.
__global__ __launch_bounds__(kBlock) void k_apply_sum(Geo g, double lam, const double* hole_xy, int p, const double* x,
                            const double* xc, int ncols, const double* part, int nchunk, const double* nsum,
                            const float* bpart, double* bt, double* y, const int* skip, int max_iters) {
  const int md = apply_mode(skip, max_iters);
  if (md < 0) return;
  if (md == 1) x = xc;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int N = g.N;
  if (g.kernel == 0 && p > 0) {
    apply_sum_stokes(g, lam, hole_xy, p, x, ncols, part, nchunk, nsum, md == 1 ? bpart : nullptr, bt, y);
    return;
  }
  if (t >= (long long)N * ncols) return;
  const int i = (int)(t / ncols), q = (int)(t % ncols);
  const size_t stride = (size_t)2 * N * ncols;
  if (g.kernel == 1) {
    // Laplace: chunks of -D mu, the coincident limit kappa w / 4pi, lam and
    // N mu; the second unknown of the node has the row lam x
    double a = 0.0;
    for (int c = 0; c < nchunk; ++c) a += part[c * stride + (size_t)(2 * i) * ncols + q];
    double ns = 0.0;
    for (int b = 0; b < kNsumParts; ++b) ns += nsum[q * kNsumParts + b];
    const double mu = x[(size_t)(2 * i) * ncols + q];
    a += (lam + kInv4Pi * g.kap[i] * g.w[i]) * mu + ns;
    y[(size_t)(2 * i) * ncols + q] = a;
    y[(size_t)(2 * i + 1) * ncols + q] = lam * x[(size_t)(2 * i + 1) * ncols + q];
    return;
  }
  double ax = 0.0, ay = 0.0;
  for (int c = 0; c < nchunk; ++c) {
    ax += part[c * stride + (size_t)(2 * i) * ncols + q];
    ay += part[c * stride + (size_t)(2 * i + 1) * ncols + q];
  }
  if (md == 1 && bpart) {
    double b = 0.0;
    for (int c = 0; c < nchunk; ++c) b += (double)bpart[((size_t)c * N + i) * ncols + q];
    bt[(size_t)i * ncols + q] = b;
  }
  const double mx = x[(size_t)(2 * i) * ncols + q], my = x[(size_t)(2 * i + 1) * ncols + q];
  const double nxi = g.nx[i], nyi = g.ny[i];
  {
    const double tx = -nyi, ty = nxi;
    const double cs = -(g.w[i] * g.kap[i]) / (2.0 * kPi);
    ax += (cs * tx * tx + lam) * mx + cs * tx * ty * my;
    ay += cs * tx * ty * mx + (cs * ty * ty + lam) * my;
  }
  double ns = 0.0;
  for (int b = 0; b < kNsumParts; ++b) ns += nsum[q * kNsumParts + b];
  ax += nxi * ns;
  ay += nyi * ns;
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

// Velocity at targets: u[2 t + a] = sum over source chunks (fixed order) of
// the double-layer sums + (H lambda)(target): the Stokeslet and rotlet of
// every hole (eq. forwardeq).  x holds [mu; lambda] in the rows layout.
__global__ void k_eval_sum(Geo g, const double* tx, const double* ty, int nt, const double* hole_xy,
                           int p, const double* x, int ncols, const double* part, int nchunk,
                           double* u) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)nt * ncols) return;
  const int i = (int)(t / ncols), q = (int)(t % ncols);
  const size_t stride = (size_t)2 * nt * ncols;
  double ax = 0.0, ay = 0.0;
  for (int c = 0; c < nchunk; ++c) {
    ax += part[c * stride + (size_t)(2 * i) * ncols + q];
    ay += part[c * stride + (size_t)(2 * i + 1) * ncols + q];
  }
  const double xi = tx[i], yi = ty[i];
  const size_t base = (size_t)2 * g.N;
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
  u[(size_t)(2 * i) * ncols + q] = ax;
  u[(size_t)(2 * i + 1) * ncols + q] = ay;
}

// Rows of Psi^T x - lambda.  Block (h, column chunk) scans the nodes once for
// the three modes of hole h and kPsiCols columns; each output is the same
// fixed-order sum as with one block per output (thread-strided over the
// nodes, then the block sum).
constexpr int kPsiCols = 8;
__global__ __launch_bounds__(kNodeSumThreads) void k_apply_psi(Geo g, const int* curve_id, int p,
                                                               const double* x, const double* xc, int ncols,
                                                               double* y, const int* skip, int max_iters) {
  const int md = apply_mode(skip, max_iters);
  if (md < 0) return;
  if (md == 1) x = xc;
  constexpr int NW = kNodeSumThreads / 64;
  __shared__ double red[NW];
  const int h = blockIdx.x;
  const int q0 = blockIdx.y * kPsiCols, nq = min(kPsiCols, ncols - q0);
  const size_t base = (size_t)2 * g.N;
  double s[3][kPsiCols];
#pragma unroll
  for (int k = 0; k < kPsiCols; ++k) s[0][k] = s[1][k] = s[2][k] = 0.0;
  for (int j = threadIdx.x; j < g.N; j += kNodeSumThreads) {
    if (curve_id[j] != h + 1) continue;
    const double w = g.w[j], xj = g.x[j], yj = g.y[j];
    const double* x0 = x + (size_t)(2 * j) * ncols + q0;
    const double* x1 = x + (size_t)(2 * j + 1) * ncols + q0;
#pragma unroll
    for (int k = 0; k < kPsiCols; ++k) {
      if (k < nq) {
        const double mx = x0[k], my = x1[k];
        s[0][k] += w * mx;
        s[1][k] += w * my;
        s[2][k] += w * (-yj * mx + xj * my);
      }
    }
  }
#pragma unroll
  for (int mode = 0; mode < 3; ++mode) {
#pragma unroll
    for (int k = 0; k < kPsiCols; ++k) {
      if (k < nq) {   // uniform over the block
        const double v = block_sum(s[mode][k], red);
        if (threadIdx.x == 0) {
          const size_t row = base + 3 * h + mode;
          y[row * ncols + q0 + k] = v - x[row * ncols + q0 + k];
        }
      }
    }
  }
}

// ---- float32 image of a refinement correction --------------------------------
// Once the residual r = [f; 0] - A x is known exactly, the next one follows
// from the correction dx alone: r' = r - A dx.  dx is small (about |r| relative
// to x), so A dx is needed only to a relative accuracy of about
// refine_tol / |r|, which float32 arithmetic meets.  Its double-layer pair
// sums (the O(N^2) part) run on the FP32 matrix cores: a wave holds 16
// targets x 16 columns, and per step of 4 sources every lane forms one pair's
// 2 x 2 block (target lane % 16, source lane / 16) in float32, which feeds
// four v_mfma_f32_16x16x4f32 (y_x += K_xx d_x + K_xy d_y, y_y += K_xy d_x +
// K_yy d_y) with d as the B operand (source lane / 16, column lane % 16).  The
// float32 accumulators are added into float64 ones every kCorrFlush sources.
// The O(N) terms stay float64.
//
// Rounding bound.  The offsets r and r . (w n / pi) are formed in float64 and
// rounded once, so every entry of the block is its exact value times
// (1 + delta) with |delta| <= 17.25 u (u = 2^-24: the two roundings of r and
// the one of r . wn, then r^2, r^4 with its floor (u / 4), the reciprocal
// (2 u), and the three products of an entry, to first order), up to float64
// rounding of the offsets.
// Rounding d and the product cost u each, and accumulating a window of
// kCorrFlush sources (2 kCorrFlush products per row) in float32 at most
// 2 kCorrFlush u times the sum of the terms' magnitudes.  So per target t and
// column q the float32 sum is off by at most (19.25 + 2 kCorrFlush) u
// sum_s e_ts max(|dx_s,q|, |dy_s,q|), e_ts the larger row sum of |K_ts|.  The
// kernel accumulates, per tile of kCorrTile sources, sum_s e_ts times the
// tile's largest |d| of column q; the host scales by kCorrBoundScale u >=
// (19.25 + 2 kCorrFlush) u, and the refinement test adds the bound's 2-norm to
// the residual's, so a converged residual is certified.
constexpr int kCorrThreads = 256;                      // 4 waves
constexpr int kCorrGroups = 2;                         // 16-target groups per wave
constexpr int kCorrTargets = 4 * 16 * kCorrGroups;     // targets per block
constexpr int kCorrTile = 64;                          // sources per LDS tile (16 steps of 4)
constexpr int kCorrFlush = 16;                         // sources per float32 accumulation window
// A distinct pair with |r|^2 below 2^-50 (nodes closer than 2^-25) is out of
// the float32 kernel's range: flag[3] is set and the refinement returns to
// exact residuals (rs_apply_f32 reports an error).  kR4Floor32 is added to
// every |r|^4 (the smallest normal float).
constexpr unsigned kR2MinBits = 0x26800000u;   // bits of 2^-50
constexpr float kR4Floor32 = 0x1p-126f;
typedef float corr_f4 __attribute__((ext_vector_type(4)));

// dx (rows layout, 2N x ncols, float64) to float32 in column blocks of 16
// ([cb][2N][16], columns past ncols zero), and per tile of kCorrTile sources
// the largest |d| of each column over both components ([cb][tile][16]).
__global__ __launch_bounds__(256) void k_corr_prep(const double* x, int N, int ncols, float* d32,
                                                   float* dmax, const int* flag, int max_iters) {
  if (apply_mode(flag, max_iters) != 1) return;
  __shared__ float red[16][16];
  const int tile = blockIdx.x, cb = blockIdx.y;
  const int j = threadIdx.x & 15, sub = threadIdx.x >> 4;
  const int q = cb * 16 + j;
  const int ntile = (N + kCorrTile - 1) / kCorrTile;
  float m = 0.0f;
  for (int u = sub; u < kCorrTile; u += 16) {
    const int sidx = tile * kCorrTile + u;
    if (sidx >= N) break;
    float vx = 0.0f, vy = 0.0f;
    if (q < ncols) {
      vx = (float)x[(size_t)(2 * sidx) * ncols + q];
      vy = (float)x[(size_t)(2 * sidx + 1) * ncols + q];
    }
    d32[((size_t)cb * 2 * N + 2 * sidx) * 16 + j] = vx;
    d32[((size_t)cb * 2 * N + 2 * sidx + 1) * 16 + j] = vy;
    m = fmaxf(m, fmaxf(fabsf(vx), fabsf(vy)));
  }
  red[sub][j] = m;
  __syncthreads();
  if (threadIdx.x < 16) {
    float mm = 0.0f;
    for (int u = 0; u < 16; ++u) mm = fmaxf(mm, red[u][threadIdx.x]);
    dmax[((size_t)cb * ntile + tile) * 16 + threadIdx.x] = mm;
  }
}

// Pair sums of the correction image over one source chunk: grid = (target
// blocks of kCorrTargets, source chunks, column blocks of 16).  part: float64
// partials in the exact apply's layout; bpart: float32 bound partials
// [chunk][N][ncols]; flag[3] is set when a pair had to be dropped.
__global__ __launch_bounds__(kCorrThreads) void k_apply_pairs32(const double4* __restrict__ src4, int N,
                                                                const float* __restrict__ d32,
                                                                const float* __restrict__ dmax, int ncols,
                                                                int chunk, double* __restrict__ part,
                                                                float* __restrict__ bpart, int* flag,
                                                                int max_iters) {
  if (apply_mode(flag, max_iters) != 1) return;
  __shared__ double2 sxy[kCorrTile];
  __shared__ double2 swn[kCorrTile];
  __shared__ float sd[kCorrTile * 32];   // [source][component][16 columns]
  __shared__ float sdm[16];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int cb = blockIdx.z;
  const int js0 = blockIdx.y * chunk, js1 = min(N, js0 + chunk);
  const int ntile = (N + kCorrTile - 1) / kCorrTile;
  const int tbase = blockIdx.x * kCorrTargets + wid * 16 * kCorrGroups;
  double xt[kCorrGroups], yt[kCorrGroups];
  corr_f4 cx[kCorrGroups], cy[kCorrGroups];
  double ax[kCorrGroups][4], ay[kCorrGroups][4];
  float bnd[kCorrGroups][4], sacc[kCorrGroups];
#pragma unroll
  for (int g = 0; g < kCorrGroups; ++g) {
    const double4 tp = src4[min(tbase + 16 * g + r16, N - 1)];
    xt[g] = tp.x;
    yt[g] = tp.y;
    cx[g] = corr_f4{0.0f, 0.0f, 0.0f, 0.0f};
    cy[g] = cx[g];
    sacc[g] = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) { ax[g][i] = 0.0; ay[g][i] = 0.0; bnd[g][i] = 0.0f; }
  }
  bool dropped = false;
  const float* dblk = d32 + (size_t)cb * 2 * N * 16;
  for (int j0 = js0; j0 < js1; j0 += kCorrTile) {
    const int nsrc = min(kCorrTile, js1 - j0);
    __syncthreads();
    if (tid < kCorrTile) {
      if (tid < nsrc) {
        const double4 sp = src4[j0 + tid];
        sxy[tid] = make_double2(sp.x, sp.y);
        swn[tid] = make_double2(sp.z, sp.w);
      } else {
        // padding: no weight, far away (its |r|^2 overflows, its terms are 0)
        sxy[tid] = make_double2(1e30, 1e30);
        swn[tid] = make_double2(0.0, 0.0);
      }
    }
    for (int e = tid; e < kCorrTile * 32; e += kCorrThreads)
      sd[e] = (e >> 5) < nsrc ? dblk[(size_t)(2 * j0) * 16 + e] : 0.0f;
    if (tid < 16) sdm[tid] = dmax[((size_t)cb * ntile + j0 / kCorrTile) * 16 + tid];
    __syncthreads();
#pragma unroll 1
    for (int u0 = 0; u0 < kCorrTile / 4; u0 += kCorrFlush / 4) {
      for (int u = u0; u < u0 + kCorrFlush / 4; ++u) {
        const int sl = 4 * u + kq;
        const double2 pp = sxy[sl];
        const double2 wn = swn[sl];
        const float bx = sd[sl * 32 + r16], by = sd[sl * 32 + 16 + r16];
#pragma unroll
        for (int g = 0; g < kCorrGroups; ++g) {
          const double rxd = xt[g] - pp.x, ryd = yt[g] - pp.y;
          const float rx = (float)rxd, ry = (float)ryd;
          const float rn = (float)fma(rxd, wn.x, ryd * wn.y);
          const float r2 = fmaf(rx, rx, ry * ry);
          // 0 < r2 < 2^-50: two distinct nodes too close for float32
          dropped |= (unsigned)__float_as_uint(r2) - 1u < kR2MinBits - 1u;
          // the floor keeps the coincident pair (r = 0, r . wn = 0 exactly)
          // and padding (wn = 0) finite and zero; for every other pair it
          // changes |r|^4 by at most 2^-26 relative
          const float inv = __builtin_amdgcn_rcpf(fmaf(r2, r2, kR4Floor32));
          const float c = rn * inv;
          const float crx = c * rx, cry = c * ry;
          const float kxx = crx * rx, kxy = crx * ry, kyy = cry * ry;
          sacc[g] += fmaxf(fabsf(kxx) + fabsf(kxy), fabsf(kxy) + fabsf(kyy));
          cx[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(kxx, bx, cx[g], 0, 0, 0);
          cx[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(kxy, by, cx[g], 0, 0, 0);
          cy[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(kxy, bx, cy[g], 0, 0, 0);
          cy[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(kyy, by, cy[g], 0, 0, 0);
        }
      }
      // window end: float32 sums into float64
#pragma unroll
      for (int g = 0; g < kCorrGroups; ++g) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          ax[g][i] += (double)cx[g][i];
          ay[g][i] += (double)cy[g][i];
        }
        cx[g] = corr_f4{0.0f, 0.0f, 0.0f, 0.0f};
        cy[g] = cx[g];
      }
    }
    // tile end: bound of the tile
    const float dm = sdm[r16];
#pragma unroll
    for (int g = 0; g < kCorrGroups; ++g) {
      float st = sacc[g];
      st += __shfl_xor(st, 16);
      st += __shfl_xor(st, 32);
      sacc[g] = 0.0f;
      // result lane l, register i holds target 4 (l / 16) + i, column l % 16
#pragma unroll
      for (int i = 0; i < 4; ++i) bnd[g][i] = fmaf(__shfl(st, 4 * kq + i), dm, bnd[g][i]);
    }
  }
  if (dropped) flag[3] = 1;
  const int q = cb * 16 + r16;
  if (q >= ncols) return;
  double* out = part + (size_t)blockIdx.y * 2 * N * ncols;
  float* bout = bpart + (size_t)blockIdx.y * N * ncols;
#pragma unroll
  for (int g = 0; g < kCorrGroups; ++g)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int t = tbase + 16 * g + 4 * kq + i;
      if (t < N) {
        out[(size_t)(2 * t) * ncols + q] = ax[g][i];
        out[(size_t)(2 * t + 1) * ncols + q] = ay[g][i];
        bout[(size_t)t * ncols + q] = bnd[g][i];
      }
    }
}

}  // namespace

// Apply configurations (columns per pass NC, targets per thread T) the
// autotuner chooses from.
namespace {
// sc = 1: sources by uniform loads (k_apply_pairs_s), 0: staged in LDS.
struct ApplyShape { int nc, t, sc; };
constexpr ApplyShape kApplyShapes[] = {{4, 2, 0}, {4, 4, 0}, {8, 1, 0}, {8, 2, 0}, {8, 4, 0}, {16, 1, 0},
                                       {16, 2, 0}, {4, 4, 1}, {8, 2, 1}, {8, 4, 1}, {16, 1, 1}, {16, 2, 1}};
constexpr int kNumApplyShapes = (int)(sizeof(kApplyShapes) / sizeof(kApplyShapes[0]));

// Source chunks: about 4096 blocks of one-target threads.  The partition
// depends on N only, so every shape sums the pairs of a target in the same
// order and all shapes give bitwise the same result.
int apply_chunk_len(int N) {
  const int tiles = (N + kApplyThreads - 1) / kApplyThreads;
  const int nch = std::max(1, std::min(tiles, (4096 + tiles - 1) / std::max(1, tiles)));
  const int chunk = (N + nch - 1) / nch;
  return ((chunk + kApplyThreads - 1) / kApplyThreads) * kApplyThreads;
}
}  // namespace

// The double-layer pair sums of one shape; grid = (target tiles, chunks,
// column chunks).  src4: scratch of 4N doubles (32-byte aligned) for the
// packed sources of the uniform-load variants.
static void launch_pairs(Geo g, double4* src4, const double* tx, const double* ty, int nt, const double* x,
                         int ncols, int chunk, double* part, const int* skip, int max_iters, int cfg,
                         dim3 grid, hipStream_t s) {
  const ApplyShape sh = kApplyShapes[cfg];
  if (sh.sc) hipLaunchKernelGGL(k_pack_sources, dim3(blocks_for(g.N, kBlock)), dim3(kBlock), 0, s, g, src4);
#define RS_APPLY(NC, T)                                                                             \
  if (!sh.sc && sh.nc == NC && sh.t == T)                                                           \
    hipLaunchKernelGGL((k_apply_pairs<NC, T>), grid, dim3(kApplyThreads), 0, s, g, tx, ty, nt, x, ncols, \
                       chunk, part, skip, max_iters);
#define RS_APPLY_S(NC, T)                                                                           \
  if (sh.sc && sh.nc == NC && sh.t == T)                                                            \
    hipLaunchKernelGGL((k_apply_pairs_s<NC, T>), grid, dim3(kApplyThreads), 0, s, src4, tx, ty, nt, g.N, \
                       x, ncols, chunk, part, skip, max_iters);
  RS_APPLY(4, 2) RS_APPLY(4, 4) RS_APPLY(8, 1) RS_APPLY(8, 2) RS_APPLY(8, 4) RS_APPLY(16, 1)
  RS_APPLY(16, 2)
  RS_APPLY_S(4, 4) RS_APPLY_S(8, 2) RS_APPLY_S(8, 4) RS_APPLY_S(16, 1) RS_APPLY_S(16, 2)
#undef RS_APPLY
#undef RS_APPLY_S
}

// The Laplace pair sums (EVAL: potential and x-derivative at arbitrary
// targets); the column block follows ncols, the partition into source chunks
// is the Stokes one.
static void launch_lap_pairs(Geo g, const double* tx, const double* ty, int nt, const double* x, int ncols,
                             int chunk, double* part, const int* skip, int max_iters, bool eval, hipStream_t s) {
  const int nc = ncols <= 1 ? 1 : (ncols <= 4 ? 4 : (ncols <= 8 ? 8 : 16));
  dim3 grid(blocks_for(nt, kApplyThreads), (g.N + chunk - 1) / chunk, blocks_for(ncols, nc));
#define RS_LAP(NC)                                                                                    \
  if (nc == NC) {                                                                                     \
    if (eval)                                                                                         \
      hipLaunchKernelGGL((k_lap_pairs<NC, 1>), grid, dim3(kApplyThreads), 0, s, g, tx, ty, nt, x, ncols, \
                         chunk, part, skip, max_iters);                                               \
    else                                                                                              \
      hipLaunchKernelGGL((k_lap_pairs<NC, 0>), grid, dim3(kApplyThreads), 0, s, g, tx, ty, nt, x, ncols, \
                         chunk, part, skip, max_iters);                                               \
  }
  RS_LAP(1) RS_LAP(4) RS_LAP(8) RS_LAP(16)
#undef RS_LAP
}

// Offset (in doubles, a multiple of 4) of the packed sources in a scratch
// whose first `used` doubles hold partial sums.
static size_t src4_offset(size_t used) { return (used + 3) / 4 * 4; }

int apply_config_count() { return kNumApplyShapes; }

bool apply_config_valid(int cfg, int ncols) {
  if (cfg < 0 || cfg >= kNumApplyShapes) return false;
  int want = 4;
  while (want < ncols && want < 16) want *= 2;
  return kApplyShapes[cfg].nc <= want;
}

int apply_default_config(int ncols) {
  return ncols <= 4 ? 0 : (ncols <= 8 ? 3 : 6);
}

void apply_config_name(int cfg, char* buf, int len) {
  if (cfg < 0 || cfg >= kNumApplyShapes) { std::snprintf(buf, len, "?"); return; }
  std::snprintf(buf, len, "nc%d_t%d", kApplyShapes[cfg].nc, kApplyShapes[cfg].t);
}

size_t apply_scratch_doubles(int N, int ncols) {
  const int len = apply_chunk_len(N);
  const int nch = (N + len - 1) / len;
  return src4_offset((size_t)nch * 2 * N * ncols + (size_t)kNsumParts * ncols) + 4 * (size_t)N;
}

namespace {
// Layout of the correction image's scratch (bytes): d32, dmax, bpart (float),
// then bt (double, N x ncols).
struct CorrLayout {
  size_t d32, dmax, bpart, bt, total;
};
CorrLayout corr_layout(int N, int ncols) {
  const int len = apply_chunk_len(N);
  const size_t nch = (size_t)((N + len - 1) / len);
  const size_t ncb = (size_t)((ncols + 15) / 16);
  const size_t ntile = (size_t)((N + kCorrTile - 1) / kCorrTile);
  CorrLayout L;
  L.d32 = 0;
  L.dmax = L.d32 + ncb * 2 * N * 16 * sizeof(float);
  L.bpart = L.dmax + ncb * ntile * 16 * sizeof(float);
  L.bt = (L.bpart + nch * N * ncols * sizeof(float) + 255) / 256 * 256;
  L.total = L.bt + (size_t)N * ncols * sizeof(double);
  return L;
}

// The O(N) terms and the sum of the chunk partials (both modes).
void apply_tail(Geo g, const int* curve_id, const double* hole_xy, int p, double lam, const double* x,
                const double* xc, int ncols, double* y, double* part, int nchunk, const float* bpart,
                double* bt, const int* flag, int max_iters, hipStream_t s) {
  double* nsum = part + (size_t)nchunk * 2 * g.N * ncols;
  hipLaunchKernelGGL(k_apply_nsum, dim3(ncols, kNsumParts), dim3(kNodeSumThreads), 0, s, g, x, xc, ncols, nsum,
                     flag, max_iters);
  hipLaunchKernelGGL(k_apply_sum, dim3(blocks_for((long long)g.N * ncols, kBlock)), dim3(kBlock), 0, s,
                     g, lam, hole_xy, p, x, xc, ncols, part, nchunk, nsum, bpart, bt, y, flag, max_iters);
  if (p > 0)
    hipLaunchKernelGGL(k_apply_psi, dim3(p, blocks_for(ncols, kPsiCols)), dim3(kNodeSumThreads), 0, s, g, curve_id, p, x, xc,
                       ncols, y, flag, max_iters);
}

double4* apply_src4(double* part, int N, int ncols) {
  const int chunk = apply_chunk_len(N);
  const int nchunk = (N + chunk - 1) / chunk;
  return reinterpret_cast<double4*>(part + src4_offset((size_t)nchunk * 2 * N * ncols + (size_t)kNsumParts * ncols));
}
}  // namespace

void launch_apply_operator(Geo g, const int* curve_id, const double* hole_xy, int p, double lam,
                           const double* x, int ncols, double* y, double* part, const int* skip,
                           int max_iters, int cfg, hipStream_t s) {
  if (ncols <= 0 || g.N <= 0) return;
  if (!apply_config_valid(cfg, ncols)) cfg = apply_default_config(ncols);
  const ApplyShape sh = kApplyShapes[cfg];
  const int chunk = apply_chunk_len(g.N);
  const int nchunk = (g.N + chunk - 1) / chunk;
  dim3 grid(blocks_for(g.N, kApplyThreads * sh.t), nchunk, blocks_for(ncols, sh.nc));
  if (g.kernel == 1)
    launch_lap_pairs(g, g.x, g.y, g.N, x, ncols, chunk, part, skip, max_iters, false, s);
  else
    launch_pairs(g, apply_src4(part, g.N, ncols), g.x, g.y, g.N, x, ncols, chunk, part, skip, max_iters, cfg,
                 grid, s);
  apply_tail(g, curve_id, hole_xy, p, lam, x, x, ncols, y, part, nchunk, nullptr, nullptr, skip, max_iters, s);
}

size_t corr_scratch_bytes(int N, int ncols) { return corr_layout(N, ncols).total; }

// The bound of the correction image's pair sums: kCorrBoundScale u times the
// per-node sums of e_ts max |d| (u = 2^-24).  (19.25 + 2 kCorrFlush) u = 51.25 u
// is derived above; 64 leaves room.
constexpr double kCorrBoundScale = 64.0;
static_assert(kCorrBoundScale >= 19.25 + 2 * kCorrFlush, "bound scale below the derived constant");
double corr_bound_scale() { return kCorrBoundScale * 0x1p-24; }

double* corr_bound_rows(void* corr, int N, int ncols) {
  return reinterpret_cast<double*>(static_cast<char*>(corr) + corr_layout(N, ncols).bt);
}

void launch_apply_refine(Geo g, const int* curve_id, const double* hole_xy, int p, double lam, const double* x,
                         const double* dx, int ncols, double* y, double* part, void* corr, int* flag,
                         int max_iters, int cfg, int which, hipStream_t s) {
  if (ncols <= 0 || g.N <= 0) return;
  if (!apply_config_valid(cfg, ncols)) cfg = apply_default_config(ncols);
  const int chunk = apply_chunk_len(g.N);
  const int nchunk = (g.N + chunk - 1) / chunk;
  double4* src4 = apply_src4(part, g.N, ncols);
  if (g.kernel == 1) {   // the Laplace path has no float32 image: exact residuals only
    which = 0;
    corr = nullptr;
  }
  if (which != 1) {
    const ApplyShape sh = kApplyShapes[cfg];
    dim3 grid(blocks_for(g.N, kApplyThreads * sh.t), nchunk, blocks_for(ncols, sh.nc));
    if (g.kernel == 1)
      launch_lap_pairs(g, g.x, g.y, g.N, x, ncols, chunk, part, flag, max_iters, false, s);
    else
      launch_pairs(g, src4, g.x, g.y, g.N, x, ncols, chunk, part, flag, max_iters, cfg, grid, s);
  }
  float *d32 = nullptr, *dmax = nullptr, *bpart = nullptr;
  double* bt = nullptr;
  if (corr) {
    const CorrLayout L = corr_layout(g.N, ncols);
    char* cb = static_cast<char*>(corr);
    d32 = reinterpret_cast<float*>(cb + L.d32);
    dmax = reinterpret_cast<float*>(cb + L.dmax);
    bpart = reinterpret_cast<float*>(cb + L.bpart);
    bt = reinterpret_cast<double*>(cb + L.bt);
  } else {
    which = 0;   // no scratch: the exact apply only
  }
  if (which != 0) {
    const int ncb = (ncols + 15) / 16;
    const int ntile = (g.N + kCorrTile - 1) / kCorrTile;
    hipLaunchKernelGGL(k_pack_sources, dim3(blocks_for(g.N, kBlock)), dim3(kBlock), 0, s, g, src4);
    hipLaunchKernelGGL(k_corr_prep, dim3(ntile, ncb), dim3(256), 0, s, dx, g.N, ncols, d32, dmax, flag,
                       max_iters);
    hipLaunchKernelGGL(k_apply_pairs32, dim3(blocks_for(g.N, kCorrTargets), nchunk, ncb), dim3(kCorrThreads), 0,
                       s, src4, g.N, d32, dmax, ncols, chunk, part, bpart, flag, max_iters);
  }
  apply_tail(g, curve_id, hole_xy, p, lam, x, dx, ncols, y, part, nchunk, bpart, bt, flag, max_iters, s);
}

// ---- fixed device scratch of the allocation-free apply ------------------------
// rs_apply_dev_noalloc keeps its row-layout copies of x and y and the apply's
// partial sums in this array instead of memory it allocates.  Each device the
// library runs on holds its own copy for the life of the process; its device
// address is looked up once per device (in host code the name `scratch` is a
// host-side stand-in, never a device address) and only that address is passed
// to kernels.
namespace {
constexpr size_t kNoAllocScratchDoubles = (size_t)8 << 20;   // 64 MiB per device
__device__ __align__(256) double scratch[kNoAllocScratchDoubles];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

size_t noalloc_scratch_doubles() { return kNoAllocScratchDoubles; }

hipError_t noalloc_scratch(int device, double** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

size_t eval_scratch_doubles(int N, int nt, int ncols) {
  const int len = apply_chunk_len(N);
  const int nch = (N + len - 1) / len;
  return src4_offset((size_t)nch * 2 * nt * ncols) + 4 * (size_t)N;
}

void launch_evaluate(Geo g, const double* hole_xy, int p, const double* tx, const double* ty, int nt,
                     const double* x, int ncols, double* u, double* part, int cfg, hipStream_t s) {
  if (nt == 0 || ncols == 0) return;
  if (!apply_config_valid(cfg, ncols)) cfg = apply_default_config(ncols);
  const ApplyShape sh = kApplyShapes[cfg];
  const int chunk = apply_chunk_len(g.N);
  const int nchunk = (g.N + chunk - 1) / chunk;
  double4* src4 = reinterpret_cast<double4*>(part + src4_offset((size_t)nchunk * 2 * nt * ncols));
  dim3 grid(blocks_for(nt, kApplyThreads * sh.t), nchunk, blocks_for(ncols, sh.nc));
  if (g.kernel == 1)
    launch_lap_pairs(g, tx, ty, nt, x, ncols, chunk, part, nullptr, 0, true, s);
  else
    launch_pairs(g, src4, tx, ty, nt, x, ncols, chunk, part, nullptr, 0, cfg, grid, s);
  hipLaunchKernelGGL(k_eval_sum, dim3(blocks_for((long long)nt * ncols, kBlock)), dim3(kBlock), 0, s, g,
                     tx, ty, nt, hole_xy, p, x, ncols, part, nchunk, u);
}

}  // namespace rs

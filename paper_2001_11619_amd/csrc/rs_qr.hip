// gfx950 pivoted QR of the ID matrices M_B (Section 2.4's interpolative
// decomposition, eq. lowrank): rank to the relative tolerance, pivot order and
// the leading rows of R.  Routes: memory-resident Householder (k_cpqr), the
// register-resident kernel (k_cpqr_reg, one or several workgroups per box),
// unpivoted row reduction of tall matrices (k_tsqr) and the 16-lane single-
// workgroup kernel for the reduced factors (k_cpqr16).
#include "rs_device.h"

namespace rs {
namespace {

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
    if (lane == 0) {
      nrm[c] = sum;
      // a non-finite column would never win a pivot comparison and be left
      // out silently: flag it (the host reports non-finite entries)
      if (!isfinite(sum)) __hip_atomic_store(err + 2, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
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
        const double nn = wave_sum_fast(t);
        // a non-finite column would never win a pivot comparison: flag it
        if (!isfinite(nn) && lane == 0) __hip_atomic_store(err + 2, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        arg_better(bv, bi, pivot_key(nn), c);
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
// tau) into hh and R_jj = beta into rdg[j] (x itself is left as it is: the
// column is not read again).  One wave runs this while the others
// wait, so the column is first spread over all 64 lanes of the wave (through
// vsh, in wave order): each lane then holds at most 4 rows (row lane + 64 q),
// and the norm, the reflector and v are short per-lane loops; the squared
// norm below row j is a full-wave sum in a fixed order.
template <int RU>
__device__ __forceinline__ void r16_householder(const double (&x)[RU], const int j, const int og,
                                                const int p, const int rg, double* vsh, double* hh,
                                                double* rdg) {
  constexpr int Q = (RU + 3) / 4;          // rows per lane after the spread
  constexpr int M = 16 * RU;
  const int lane = threadIdx.x & 63;
  if (rg == og)
#pragma unroll
    for (int u = 0; u < RU; ++u) vsh[p + 16 * u] = x[u];
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  double y[Q];
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int row = lane + 64 * q;
    y[q] = row < M ? vsh[row] : 0.0;
    const double yv = row > j ? y[q] : 0.0;
    acc += yv * yv;
  }
  // x_j sits in lane j % 64 at position q = j / 64 (uniform)
  const int qj = j >> 6;
  double yj = y[0];
#pragma unroll
  for (int q = 1; q < Q; ++q) yj = (qj == q) ? y[q] : yj;
  const double alpha = lane_f64(yj, j & 63);
  const double s2 = wave_sum_fast(acc);
  double beta, tau, scal = 0.0;
  if (s2 == 0.0) {
    beta = alpha;
    tau = 0.0;
  } else {
    // two divisions, not one reciprocal of beta (alpha - beta): in a
    // rank-deficient block of rows the rounding residue below the diagonal
    // shrinks from step to step, and once s2 is subnormal that product
    // underflows and its reciprocal overflows (tau = inf, then NaN).  Each
    // quotient here stays finite: |alpha - beta| >= |beta| >= sqrt(s2) > 0.
    beta = -copysign(sqrt(alpha * alpha + s2), alpha);
    tau = (beta - alpha) / beta;
    scal = 1.0 / (alpha - beta);
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int row = lane + 64 * q;
    if (row < M) vsh[row] = row < j ? 0.0 : (row == j ? 1.0 : y[q] * scal);
  }
  if (lane == 0) { hh[0] = beta; hh[1] = tau; rdg[j] = beta; }
}

// ---- row reduction of tall ID matrices (unpivoted block Householder QR) ----
// One task = one block of rows (at most 16 RU) of an n-column matrix: its
// triangular factor (n rows, zeros below the diagonal) is written to dst.
// Blocks of M_B first, then blocks of stacked factors, until the stack has at
// most 256 rows.  One barrier per step: the Householder vector of step j + 1
// goes to the other of two buffers.
//
// The reflector of step j applied to the register slots S0.. of the wave:
// the slots before S0 hold finished columns only, whose multipliers are zero,
// so the result is that of the full update.
template <int RU, int NS, int S0>
__device__ __forceinline__ void tsqr16_apply(double (&a)[NS][RU], const double* vsh, const int p,
                                             const double tau, const int j, const int n,
                                             const int wid, const int rg) {
  double v[RU], t[NS];
#pragma unroll
  for (int sl = S0; sl < NS; ++sl) t[sl] = 0.0;
#pragma unroll
  for (int u = 0; u < RU; ++u) {
    v[u] = vsh[p + 16 * u];
#pragma unroll
    for (int sl = S0; sl < NS; ++sl) t[sl] += v[u] * a[sl][u];
  }
#pragma unroll
  for (int sl = S0; sl < NS; ++sl) {
    const int c = 4 * (wid + kRQWaves * sl) + rg;
    const double dot = row16_sum(t[sl]);
    t[sl] = (c > j && c < n) ? tau * dot : 0.0;
  }
#pragma unroll
  for (int u = 0; u < RU; ++u)
#pragma unroll
    for (int sl = S0; sl < NS; ++sl) a[sl][u] -= t[sl] * v[u];
}

template <int RU, int NS>
__device__ __forceinline__ void tsqr16_block(const QRTask& T, double* vsh2, double* hh2, double* rdg) {
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
        if (sl == os) r16_householder<RU>(a[sl], j, j & 3, p, rg, vsh, hh, rdg);
    }
    __syncthreads();
    const double tau = hh[1];
    // slot sl of this wave holds columns 4 (wid + 8 sl) .. + 3: the first slot
    // with a column right of j
    const int d = j - 3 - 4 * wid;
    const int s0 = d < 0 ? 0 : d / (4 * kRQWaves) + 1;
    switch (s0) {
      case 0: tsqr16_apply<RU, NS, 0>(a, vsh, p, tau, j, n, wid, rg); break;
      case 1: if constexpr (NS > 1) tsqr16_apply<RU, NS, 1>(a, vsh, p, tau, j, n, wid, rg); break;
      case 2: if constexpr (NS > 2) tsqr16_apply<RU, NS, 2>(a, vsh, p, tau, j, n, wid, rg); break;
      case 3: if constexpr (NS > 3) tsqr16_apply<RU, NS, 3>(a, vsh, p, tau, j, n, wid, rg); break;
      default: break;
    }
  }
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int c = 4 * (wid + kRQWaves * sl) + rg;
    if (c >= n) continue;
    double* dst = T.dst + (size_t)c * T.ldd;
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int r = p + 16 * u;
      if (r < n) dst[r] = r < c ? a[sl][u] : (r == c ? (c < steps ? rdg[c] : a[sl][u]) : 0.0);
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
                                           double* s_hh, double* wv, int* wi, double* rdg) {
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
      // a non-finite column would never win a pivot comparison: flag it
      if (c < n && !isfinite(nn) && p == 0)
        __hip_atomic_store(err + 2, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
        if (sl == os) r16_householder<RU>(a[sl], j, q & 3, p, rg, vsh, s_hh, rdg);
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
      if (r < kx) dst[(size_t)r * n] = r < pp ? a[sl][u] : (r == pp ? rdg[pp] : 0.0);
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
  __shared__ double rdg[kR16MaxN];
  const QRTask& T = tasks[blockIdx.x];
#define RS_TSQR(R, S) tsqr16_block<R, S>(T, vsh2, hh2, rdg)
  switch (T.ru * 8 + (T.n + 31) / 32) { RS_R16_CASES(RS_TSQR) }
#undef RS_TSQR
}

__global__ __launch_bounds__(kRQThreads) void k_cpqr16(const LevelBox* boxes, const int4* work,
                                                       double tol, int extra, int* k_out, int* kx_out,
                                                       int* err) {
  __shared__ double dyn[16 * kR16MaxRU + kR16MaxCols];   // v, then pv / ipv as ints
  __shared__ double rdg[kR16MaxN];                        // R_jj
  __shared__ double s_hh[2];
  __shared__ double wv[kRQWaves];
  __shared__ int wi[kRQWaves];
  const int4 w = work[blockIdx.x];
  const LevelBox& B = boxes[w.x];
#define RS_CPQR16(R, S) cpqr16_box<R, S>(B, tol, extra, k_out, kx_out, err, dyn, s_hh, wv, wi, rdg)
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
  case 24: CALL(24); break; \
  case 26: CALL(26); break; \
  case 28: CALL(28); break; \
  case 30: CALL(30); break; \
  case 32: CALL(32); break; \
  case 34: CALL(34); break; \
  case 36: CALL(36); break; \
  case 38: CALL(38); break; \
  default: CALL(40); break;

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

}  // namespace

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

}  // namespace rs

// gfx950 kernels of one level of the factorization around the pivoted QR
// (Sections 2.2-2.7): the stacked ID matrix M_B (eq. greens, eq. null-spaceop),
// the diagonal block A_BB in pivot order, the elimination of the redundant
// unknowns (T, eq. tmat; X_RR^{-1} with the conditioning guard; E, F and the
// Schur complement, eq. schurmat), the blocked Gauss-Jordan inverse of the root
// system (eq. partition) and the float copies of the factors.
#include "rs_device.h"

#include <type_traits>

namespace rs {
namespace {

// ---- factorization kernels -------------------------------------------------

// Thread per row of M_B; the box's columns (source node geometry and
// component) are staged in LDS 256 at a time, so the loop over columns reads
// no global memory.  F32: the float32 bulk form, every entry computed in
// float32 from box-local offsets (stored as doubles, exactly).
template <bool F32>
__global__ __launch_bounds__(kBlock) void k_assemble_M(const LevelBox* boxes, int n_proxy,
                                                       double ratio) {
  __shared__ double sx[kBlock], sy[kBlock], snx[kBlock], sny[kBlock], sw[kBlock];
  __shared__ float sxf[kBlock], syf[kBlock];
  __shared__ int sj[kBlock];
  const LevelBox& B = boxes[blockIdx.x];
  const int i = blockIdx.y * blockDim.x + threadIdx.x;
  const int m = B.m, n = B.n, nF = B.nF;
  if (n == 0 || blockIdx.y * blockDim.x >= m) return;   // uniform per block
  const bool live = i < m;
  const int* I = B.dofs;
  const Geo& g = B.geo;
  const int np2 = 2 * n_proxy;
  // proxy row blocks: D(P,B), D(B,P)^T and S(B,P)^T; the Laplace kernel has no
  // Stokeslet block
  const int npb = g.kernel == 1 ? 2 : 3;
  const double rp = ratio * B.side;
  // target-side proxy rows and the target-side rank-one row carry the scale
  // of one boundary interaction: the box's largest node weight
  const double wp = B.wscale;
  int type = 6, f = 0, pa = 0;
  double px = 0, py = 0, pnx = 0, pny = 0;
  if (!live) {
    type = 6;
  } else if (i < nF) {
    type = 0;
    f = B.fint[i];
  } else if (i < 2 * nF) {
    type = 1;
    f = B.fint[i - nF];
  } else if (i < 2 * nF + npb * np2) {
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
    type = 5 + (i - 2 * nF - npb * np2);
  }
  const int fj = f >> 1, fc = f & 1;
  double fx = 0, fy = 0, fnx = 0, fny = 0, fw = 0;
  if (type <= 1) {
    fx = g.x[fj];
    fy = g.y[fj];
    fnx = g.nx[fj];
    fny = g.ny[fj];
    fw = g.w[fj];
  }
  const double fn_c = fc ? fny : fnx;
  for (int c0 = 0; c0 < n; c0 += kBlock) {
    const int cnt = min(kBlock, n - c0);
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
      const int d = I[c0 + threadIdx.x];
      const int j = d >> 1;
      sj[threadIdx.x] = d;
      sx[threadIdx.x] = g.x[j];
      sy[threadIdx.x] = g.y[j];
      if (F32) {
        sxf[threadIdx.x] = (float)(g.x[j] - B.cx);
        syf[threadIdx.x] = (float)(g.y[j] - B.cy);
      }
      snx[threadIdx.x] = g.nx[j];
      sny[threadIdx.x] = g.ny[j];
      sw[threadIdx.x] = g.w[j];
    }
    __syncthreads();
    if (!live) continue;
    double* col = B.M + (size_t)c0 * m + i;
    if (g.kernel == 1) {
      // Laplace Neumann (Section 4.4.1): near-field rows from the operator;
      // source side, the potential and normal flux on the proxy circle of the
      // box's charges plus their total (the rank-one row); target side, the
      // normal derivative at the nodes of a proxy charge and a proxy dipole,
      // plus the constant row of N.  (The uncoupled second unknown of a node
      // joins no box; were one passed, its column would be zero.)
      if (F32) {
        // float32 entries from box-local offsets (the proxy point's is exact)
        const float rxf = type <= 1 ? (float)(fx - B.cx) : (float)(rp * pnx);
        const float ryf = type <= 1 ? (float)(fy - B.cy) : (float)(rp * pny);
        const float fnxf = (float)fnx, fnyf = (float)fny, fwf = (float)fw, wpf = (float)wp;
        const float pnxf = (float)pnx, pnyf = (float)pny;
        for (int cc = 0; cc < cnt; ++cc) {
          const int d = sj[cc];
          const int j = d >> 1, jc = d & 1;
          const float xj = sxf[cc], yj = syf[cc], nxj = (float)snx[cc], nyj = (float)sny[cc], wj = (float)sw[cc];
          float v = 0.0f;
          if (type == 0) {
            if (fj == j) v = lap_op_entry_f(g, fj, fc, j, jc, 0.0, B.cx, B.cy);
            else if (!(fc | jc)) v = lap_dl_f(rxf - xj, ryf - yj, fnxf, fnyf, wj) + wj;
          } else if (type == 1) {
            if (fj == j) v = lap_op_entry_f(g, j, jc, fj, fc, 0.0, B.cx, B.cy);
            else if (!(fc | jc)) v = lap_dl_f(xj - rxf, yj - ryf, nxj, nyj, fwf) + fwf;
          } else if (jc == 0) {
            if (type == 2) {
              const float rx = rxf - xj, ry = ryf - yj;
              const float r2 = rx * rx + ry * ry;
              v = pa ? (float)kInv2Pi * wj * (rx * pnxf + ry * pnyf) / r2 : -(float)kInv4Pi * wj * logf(r2);
            } else if (type == 3) {
              const float rx = xj - rxf, ry = yj - ryf;
              const float r2 = rx * rx + ry * ry;
              const float rnj = rx * nxj + ry * nyj;
              if (!pa) {
                v = (float)kInv2Pi * wpf * rnj / r2;
              } else {
                const float rnp = rx * pnxf + ry * pnyf;
                v = (float)kInv2Pi * wpf * ((nxj * pnxf + nyj * pnyf) - 2.0f * rnp * rnj / r2) / r2;
              }
            } else if (type == 5) {
              v = wj;
            } else if (type == 6) {
              v = (float)B.wscale;
            }
          }
          col[(size_t)cc * m] = (double)v;
        }
        continue;
      }
      for (int cc = 0; cc < cnt; ++cc) {
        const int d = sj[cc];
        const int j = d >> 1, jc = d & 1;
        double v = 0.0;
        if (type == 0) {
          v = lap_op_entry(g, fj, fc, j, jc, 0.0);
        } else if (type == 1) {
          v = lap_op_entry(g, j, jc, fj, fc, 0.0);
        } else if (jc == 0) {
          const double xj = sx[cc], yj = sy[cc], wj = sw[cc];
          if (type == 2) {
            const double rx = px - xj, ry = py - yj;
            const double r2 = rx * rx + ry * ry;
            v = pa ? kInv2Pi * wj * (rx * pnx + ry * pny) / r2 : -kInv4Pi * wj * log(r2);
          } else if (type == 3) {
            const double rx = xj - px, ry = yj - py;
            const double r2 = rx * rx + ry * ry;
            const double rnj = rx * snx[cc] + ry * sny[cc];
            if (!pa) {
              v = kInv2Pi * wp * rnj / r2;
            } else {
              const double rnp = rx * pnx + ry * pny;
              v = kInv2Pi * wp * ((snx[cc] * pnx + sny[cc] * pny) - 2.0 * rnp * rnj / r2) / r2;
            }
          } else if (type == 5) {
            v = wj;
          } else if (type == 6) {
            v = B.wscale;
          }
        }
        col[(size_t)cc * m] = v;
      }
      continue;
    }
    if (F32) {
      // row point as a box-local float offset (the proxy point's is exact)
      const float rxf = type <= 1 ? (float)(fx - B.cx) : (float)(rp * pnx);
      const float ryf = type <= 1 ? (float)(fy - B.cy) : (float)(rp * pny);
      const float fnxf = (float)fnx, fnyf = (float)fny, fwf = (float)fw, wpf = (float)wp;
      const float pnxf = (float)pnx, pnyf = (float)pny, fn_cf = (float)fn_c, wsf = (float)B.wscale;
      for (int cc = 0; cc < cnt; ++cc) {
        const int d = sj[cc];
        const int j = d >> 1, jc = d & 1;
        const float xj = sxf[cc], yj = syf[cc], nxj = (float)snx[cc], nyj = (float)sny[cc], wj = (float)sw[cc];
        const float nj_c = jc ? nyj : nxj;
        float v;
        switch (type) {
          case 0:
            if (fj == j) v = op_entry_f(g, fj, fc, j, jc, 0.0, B.cx, B.cy);
            else v = dl_entry_f(rxf - xj, ryf - yj, nxj, nyj, wj, fc, jc) + fn_cf * (wj * nj_c);
            break;
          case 1:
            if (fj == j) v = op_entry_f(g, j, jc, fj, fc, 0.0, B.cx, B.cy);
            else v = dl_entry_f(xj - rxf, yj - ryf, fnxf, fnyf, fwf, jc, fc) + nj_c * (fwf * fn_cf);
            break;
          case 2: v = dl_entry_f(rxf - xj, ryf - yj, nxj, nyj, wj, pa, jc); break;
          case 3: v = dl_entry_f(xj - rxf, yj - ryf, pnxf, pnyf, wpf, jc, pa); break;
          case 4: v = sl_entry_f(xj - rxf, yj - ryf, wpf, jc, pa); break;
          case 5: v = wj * nj_c; break;
          default: v = wsf * nj_c; break;
        }
        col[(size_t)cc * m] = (double)v;
      }
      continue;
    }
    for (int cc = 0; cc < cnt; ++cc) {
      const int d = sj[cc];
      const int j = d >> 1, jc = d & 1;
      const double xj = sx[cc], yj = sy[cc], nxj = snx[cc], nyj = sny[cc], wj = sw[cc];
      const double nj_c = jc ? nyj : nxj;
      double v;
      switch (type) {
        case 0:   // target: near-field unknown f, source: column unknown (op_entry)
          if (fj == j) v = op_entry(g, fj, fc, j, jc, 0.0);
          else v = dl_entry(fx - xj, fy - yj, nxj, nyj, wj, fc, jc) + fn_c * (wj * nj_c);
          break;
        case 1:   // target: column unknown, source: near-field unknown f
          if (fj == j) v = op_entry(g, j, jc, fj, fc, 0.0);
          else v = dl_entry(xj - fx, yj - fy, fnx, fny, fw, jc, fc) + nj_c * (fw * fn_c);
          break;
        case 2: v = dl_entry(px - xj, py - yj, nxj, nyj, wj, pa, jc); break;
        case 3: v = dl_entry(xj - px, yj - py, pnx, pny, wp, jc, pa); break;
        case 4: v = sl_entry(xj - px, yj - py, wp, jc, pa); break;
        case 5: v = wj * nj_c; break;
        default: v = B.wscale * nj_c; break;
      }
      col[(size_t)cc * m] = v;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_assemble_abb(const LevelBox* boxes, double lam,
                                                         int use_perm, int f32) {
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
  B.Ap[t] = f32 ? (double)op_entry_f(B.geo, di >> 1, di & 1, dj >> 1, dj & 1, lam, B.cx, B.cy)
                : op_entry(B.geo, di >> 1, di & 1, dj >> 1, dj & 1, lam);
}

// ---- elimination of the redundant unknowns (G workgroups per box) -----------

typedef double dbl4 __attribute__((ext_vector_type(4)));

// C = beta*C0 + alpha*op(A) op(B) on FP64 matrix cores.  The 16 x 16 tiles
// of C are dealt to the waves of the G workgroups of the box; a wave
// accumulates v_mfma_f64_16x16x4 products over K in groups of 4 with its
// operands read straight from memory (the factors were just written and sit
// in L2): no LDS staging and no workgroup barrier, and the loads of the next
// 8 groups are issued before the products of the current ones.  Operand
// lanes: A[l % 16][l / 16], B[l / 16][l % 16]; result lane l, register q
// holds row 4 q + l / 16, column l % 16 of the tile.  Every tile is summed
// in the same order whatever G is.  C0 may alias C (each element is read
// before it is written, by the same lane).
//
// F32 (the float32 bulk form): the operands are rounded to float32 on load
// and multiplied on FP32 matrix cores (v_mfma_f32_16x16x4f32) with float32
// accumulation; beta*C0 + alpha*product is formed in float32 and stored as a
// double (exactly).  Same operand lanes; result lane l, register q holds row
// 4 (l / 16) + q.
typedef float flt4 __attribute__((ext_vector_type(4)));

template <bool F32>
__device__ void mfma_gemm_t(int g, int G, int M, int N, int K, double alpha, const double* A,
                            int lda, bool tA, const double* B, int ldb, bool tB, double beta,
                            const double* C0, int ldc0, double* C, int ldc) {
  using E = typename std::conditional<F32, float, double>::type;
  using V4 = typename std::conditional<F32, flt4, dbl4>::type;
  const int lane = threadIdx.x & 63;
  const int NW = blockDim.x >> 6, wid = threadIdx.x >> 6;
  const int tm = (M + 15) >> 4, tn = (N + 15) >> 4;
  const int r16 = lane & 15, kq = lane >> 4;
  const long long sa = tA ? lda : 1, sb = tB ? 1 : ldb;
  const int kg = (K + 3) >> 2;                  // groups of 4 along K
  constexpr int PF = 8;                         // groups per prefetch chunk
  for (int t = g * NW + wid; t < tm * tn; t += G * NW) {
    const int i0 = (t / tn) << 4, j0 = (t % tn) << 4;
    const int gi = i0 + r16, gj = j0 + r16;
    const double* pa = tA ? A + gi : A + (size_t)gi * lda;
    const double* pb = tB ? B + (size_t)gj * ldb : B + gj;
    const bool va = gi < M, vb = gj < N;
    E an[PF], bn[PF];
    auto load = [&](int q0) {
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int k = 4 * (q0 + u) + kq;
        an[u] = (va && k < K) ? (E)pa[k * sa] : (E)0;
        bn[u] = (vb && k < K) ? (E)pb[k * sb] : (E)0;
      }
    };
    V4 acc = {0, 0, 0, 0};
    load(0);
    for (int q0 = 0; q0 < kg; q0 += PF) {
      E ac[PF], bc[PF];
#pragma unroll
      for (int u = 0; u < PF; ++u) { ac[u] = an[u]; bc[u] = bn[u]; }
      if (q0 + PF < kg) load(q0 + PF);
#pragma unroll
      for (int u = 0; u < PF; ++u)
        if (q0 + u < kg) {
          if constexpr (F32)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ac[u], bc[u], acc, 0, 0, 0);
          else
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ac[u], bc[u], acc, 0, 0, 0);
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ri = F32 ? i0 + 4 * kq + q : i0 + 4 * q + kq, cj = j0 + r16;
      if (ri < M && cj < N) {
        E v = (E)alpha * acc[q];
        if (C0) v += (E)beta * (E)C0[(size_t)ri * ldc0 + cj];
        C[(size_t)ri * ldc + cj] = (double)v;
      }
    }
  }
}

__device__ __forceinline__ void mfma_gemm(int g, int G, int M, int N, int K, double alpha, const double* A,
                                          int lda, bool tA, const double* B, int ldb, bool tB, double beta,
                                          const double* C0, int ldc0, double* C, int ldc, bool f32 = false) {
  if (f32)
    mfma_gemm_t<true>(g, G, M, N, K, alpha, A, lda, tA, B, ldb, tB, beta, C0, ldc0, C, ldc);
  else
    mfma_gemm_t<false>(g, G, M, N, K, alpha, A, lda, tA, B, ldb, tB, beta, C0, ldc0, C, ldc);
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
// A 16 x 16 thread grid keeps rows ty + 16 a, columns tx + 16 b (a, b < MB,
// MB = ceil(r / 16) fixed at compile time) of W in registers for the whole
// sweep; padding rows and columns hold zeros and stay zero.  Per step the
// holders of the pivot row and column copy them to LDS and clear them, and
// every element then takes one FMA (the multipliers absorb the pivot row and
// column).  The pivot row and the column block are uniform over the
// workgroup, so choosing the registers that hold them costs scalar branches,
// not per-element selects.  The pivot is compared on a 64-bit key (|W| with
// its low 8 mantissa bits replaced by 255 - i, ties within 2^-44 to the
// smaller row) that the holders of column j + 1 fold into LDS with one atomic
// max each (over their own rows first) during step j.  Column 1-norms for rcond_1 are summed in a fixed order.
// Two barriers per step.  Returns rcond_1 (0 if singular).
// LDS: gj_lds_doubles(r) doubles at `sh`.
__device__ __forceinline__ unsigned long long gj_key(double v, int i) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(fabs(v));
  return (b & ~0xFFull) | (unsigned long long)(255 - i);
}

__host__ __device__ constexpr size_t gj_lds_doubles(int r) { return 18 * (size_t)r + 4 + (size_t)r; }

template <int MB>
__device__ __noinline__ double reg_gj_t(const double* X, int r, double* Xi, double* sh, double* red) {
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  double* rowbuf = sh;                       // r: pivot row
  double* colbuf = rowbuf + r;               // r: pivot column
  double* part = colbuf + r;                 // 16 r: column-sum partials
  unsigned long long* keys = reinterpret_cast<unsigned long long*>(part + 16 * (size_t)r);   // 2
  int* pv = reinterpret_cast<int*>(keys + 2);        // r
  int* ipv = pv + r;                                  // r
  double w[MB][MB];
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      const int i = ty + 16 * a, c = tx + 16 * b;
      w[a][b] = (i < r && c < r) ? X[(size_t)i * r + c] : 0.0;
    }
  if (tid < 2) keys[tid] = 0ull;
  // largest column 1-norm: per-thread partial sums, then 16 partials per column in order
  auto colnorm = [&]() {
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < MB; ++a) s += fabs(w[a][b]);
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
      const int i = ty + 16 * a;
      if (i < r) atomicMax(&keys[0], gj_key(w[a][0], i));
    }
  __syncthreads();
  unsigned used = 0;             // bit a: row ty + 16 a is a pivot row already
  for (int j = 0; j < r; ++j) {
    const unsigned long long key = keys[j & 1];
    const int bi = __builtin_amdgcn_readfirstlane(255 - (int)(key & 0xFF));
    const int ab = bi >> 4, bj = j >> 4;
    // copy the pivot column and row to LDS, then clear them in the tableau
    // (bj, ab uniform: one scalar branch selects the register block)
    const bool ccol = tx == (j & 15), crow = ty == (bi & 15);
    switch (bj) {
#define RS_GJ_COL(B)                                                   \
      case B:                                                          \
        if constexpr (B < MB) {                                        \
          if (ccol) {                                                  \
            _Pragma("unroll") for (int a = 0; a < MB; ++a) {           \
              const int i = ty + 16 * a;                               \
              if (i < r) colbuf[i] = w[a][B];                          \
            }                                                          \
          }                                                            \
        }                                                              \
        break;
      RS_GJ_COL(0) RS_GJ_COL(1) RS_GJ_COL(2) RS_GJ_COL(3)
      RS_GJ_COL(4) RS_GJ_COL(5) RS_GJ_COL(6) RS_GJ_COL(7)
#undef RS_GJ_COL
    }
    switch (ab) {
#define RS_GJ_ROW(A)                                                   \
      case A:                                                          \
        if constexpr (A < MB) {                                        \
          if (crow) {                                                  \
            _Pragma("unroll") for (int b = 0; b < MB; ++b) {           \
              const int c = tx + 16 * b;                               \
              if (c < r) rowbuf[c] = w[A][b];                          \
              w[A][b] = 0.0;                                           \
            }                                                          \
          }                                                            \
        }                                                              \
        break;
      RS_GJ_ROW(0) RS_GJ_ROW(1) RS_GJ_ROW(2) RS_GJ_ROW(3)
      RS_GJ_ROW(4) RS_GJ_ROW(5) RS_GJ_ROW(6) RS_GJ_ROW(7)
#undef RS_GJ_ROW
    }
    switch (bj) {
#define RS_GJ_CLR(B)                                                   \
      case B:                                                          \
        if constexpr (B < MB) {                                        \
          if (ccol) {                                                  \
            _Pragma("unroll") for (int a = 0; a < MB; ++a) w[a][B] = 0.0; \
          }                                                            \
        }                                                              \
        break;
      RS_GJ_CLR(0) RS_GJ_CLR(1) RS_GJ_CLR(2) RS_GJ_CLR(3)
      RS_GJ_CLR(4) RS_GJ_CLR(5) RS_GJ_CLR(6) RS_GJ_CLR(7)
#undef RS_GJ_CLR
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
      const int c = tx + 16 * b;
      pr[b] = c < r ? (c == j ? inv : rowbuf[c] * inv) : 0.0;
      const int i = ty + 16 * b;
      pc[b] = i < r ? (i == bi ? -1.0 : colbuf[i]) : 0.0;
    }
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
      for (int b = 0; b < MB; ++b) w[a][b] = fma(-pc[a], pr[b], w[a][b]);
    const int bn = (j + 1) >> 4;
    const bool cnext = tx == ((j + 1) & 15);
    if (j + 1 < r) switch (bn) {
#define RS_GJ_KEY(B)                                                   \
      case B:                                                          \
        if constexpr (B < MB) {                                        \
          if (cnext) {                                                 \
            unsigned long long best = 0ull;                            \
            _Pragma("unroll") for (int a = 0; a < MB; ++a) {           \
              const int i = ty + 16 * a;                               \
              if (i < r && !((used >> a) & 1))                         \
                best = max(best, gj_key(w[a][B], i));                  \
            }                                                          \
            atomicMax(&keys[(j + 1) & 1], best);                       \
          }                                                            \
        }                                                              \
        break;
      RS_GJ_KEY(0) RS_GJ_KEY(1) RS_GJ_KEY(2) RS_GJ_KEY(3)
      RS_GJ_KEY(4) RS_GJ_KEY(5) RS_GJ_KEY(6) RS_GJ_KEY(7)
#undef RS_GJ_KEY
    }
    __syncthreads();
  }
  // X^{-1}[j][p_c] = W[p_j][c]
  for (int j = tid; j < r; j += kBlock) ipv[pv[j]] = j;
  __syncthreads();
#pragma unroll
  for (int a = 0; a < MB; ++a) {
    const int i = ty + 16 * a;
    if (i >= r) continue;
    const int row = ipv[i];
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      const int c = tx + 16 * b;
      if (c < r) Xi[(size_t)row * r + pv[c]] = w[a][b];
    }
  }
  // column c of W is column p_c of X^{-1} with its rows permuted
  const double n2 = colnorm();
  const double rc = 1.0 / (n1 * n2);
  return isfinite(rc) ? rc : 0.0;
}

__device__ double reg_gj(const double* X, int r, double* Xi, double* sh, double* red) {
  static_assert(kLdsGJMax == 128, "reg_gj dispatches MB = 1 .. 8");
  switch ((r + 15) >> 4) {
    case 1: return reg_gj_t<1>(X, r, Xi, sh, red);
    case 2: return reg_gj_t<2>(X, r, Xi, sh, red);
    case 3: return reg_gj_t<3>(X, r, Xi, sh, red);
    case 4: return reg_gj_t<4>(X, r, Xi, sh, red);
    case 5: return reg_gj_t<5>(X, r, Xi, sh, red);
    case 6: return reg_gj_t<6>(X, r, Xi, sh, red);
    case 7: return reg_gj_t<7>(X, r, Xi, sh, red);
    default: return reg_gj_t<8>(X, r, Xi, sh, red);
  }
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
                                                      int* status, double* rc_out, int* err, int f32,
                                                      double f32_rcond) {
  extern __shared__ double smem_e[];
  constexpr int NW = kBlock / 64;
  __shared__ double red[NW];
  __shared__ int ired[NW];
  __shared__ int s_dead;
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
  // float32 bulk form: a box whose X_RR comes out with rcond_1 below
  // f32_rcond (which would amplify float32 rounding by its inverse) is
  // eliminated again with float64 products
  bool fgo = f32 != 0;
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
    const bool fg = fgo;   // the Schur-complement products in float32 (float32 bulk form)
    mfma_gemm(g, G, k, r, k, -1.0, Ap, n, false, T, r, false, 1.0, Ap + k, n, Xsr, r, fg);
    mfma_gemm(g, G, r, k, k, -1.0, T, r, true, Ap, n, false, 1.0, Ap + (size_t)k * n, n, Xrs, k, fg);
    mfma_gemm(g, G, r, r, k, -1.0, Ap + (size_t)k * n, n, false, T, r, false, 1.0,
              Ap + (size_t)k * n + k, n, Xrr, r, fg);
    if (g == 0 && threadIdx.x == 0) *flag = 0;
    box_barrier_full(B.bar, G, nbar, &s_dead, err);
    // X_RR -= T^T X_SR
    mfma_gemm(g, G, r, r, k, -1.0, T, r, true, Xsr, r, false, 1.0, Xrr, r, W, r, fg);
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
    if (fgo && !(rc >= f32_rcond)) {
      fgo = false;
      box_barrier_full(B.bar, G, nbar, &s_dead, err);
      continue;
    }
    rc_final = rc;
    box_barrier_full(B.bar, G, nbar, &s_dead, err);
    mfma_gemm(g, G, k, r, r, 1.0, Xsr, r, false, B.Xinv, r, false, 0.0, nullptr, 0, B.E, r, fg);
    mfma_gemm(g, G, r, k, r, 1.0, B.Xinv, r, false, Xrs, k, false, 0.0, nullptr, 0, B.F, k, fg);
    box_barrier_full(B.bar, G, nbar, &s_dead, err);
    mfma_gemm(g, G, k, k, r, -1.0, Xsr, r, false, B.F, k, false, 1.0, Ap, n, B.Xss, k, fg);
    break;
  }
  if (g == 0 && threadIdx.x == 0) {
    k_io[B.slot] = k;
    status[B.slot] = st;
    rc_out[B.slot] = rc_final;
  }
}

// ---- border of the root system (eq. partition) -----------------------------
// W_B = X_RR^{-1} (U H)_R of every box (r x 3p) as an LDS-tiled float64 GEMM.
// Block (box, y) owns the output tile of rows 64 ty .. and columns 64 tx ..
// (y = ty * ntx + tx; tiles beyond the box's r exit at once); the K dimension
// (r) goes in chunks of 32: a 64 x 32 tile of X_RR^{-1} and the 32 gathered
// rows of (U H) over the tile's 64 columns are staged in LDS, and each thread
// accumulates a 4 x 4 block of W in registers, the sum over k in order.
constexpr int kBWT = 64;   // output tile edge
constexpr int kBWK = 32;   // K chunk
__global__ __launch_bounds__(kBlock) void k_border_w(const SolveBox* boxes, const int* ridx,
                                                     const double* Hh, int p3, int ntx) {
  __shared__ double sa[kBWT][kBWK + 1];
  __shared__ __align__(16) double sb[kBWK][kBWT];
  const SolveBox& B = boxes[blockIdx.x];
  const int r = B.r;
  const int ty = blockIdx.y / ntx, tx = blockIdx.y % ntx;
  const int i0 = ty * kBWT, h0 = tx * kBWT;
  if (i0 >= r) return;   // uniform over the block
  const int* R = ridx + B.r_off;
  const double* Xi = B.Xinv;
  const int tid = threadIdx.x;
  const int ri = (tid >> 4) * 4, cj = (tid & 15) * 4;
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int k0 = 0; k0 < r; k0 += kBWK) {
    const int kc = min(kBWK, r - k0);
    __syncthreads();
    for (int e = tid; e < kBWT * kBWK; e += kBlock) {
      const int row = e / kBWK, kk = e % kBWK;
      sa[row][kk] = (i0 + row < r && kk < kc) ? Xi[(size_t)(i0 + row) * r + k0 + kk] : 0.0;
    }
    for (int e = tid; e < kBWK * kBWT; e += kBlock) {
      const int kk = e / kBWT, col = e % kBWT;
      sb[kk][col] = (kk < kc && h0 + col < p3) ? Hh[(size_t)R[k0 + kk] * p3 + h0 + col] : 0.0;
    }
    __syncthreads();
    for (int kk = 0; kk < kc; ++kk) {
      const double4 bv = *reinterpret_cast<const double4*>(&sb[kk][cj]);
      const double bb[4] = {bv.x, bv.y, bv.z, bv.w};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double av = sa[ri + u][kk];
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(av, bb[v], acc[u][v]);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = i0 + ri + u;
    if (i >= r) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (h0 + cj + v < p3) B.W[(size_t)i * p3 + h0 + cj + v] = acc[u][v];
  }
}

// Gpart[chunk] = sum over the rows i of the chunk of Ph[R_i]^T W[i], where the
// R lists of all boxes are concatenated (ridx) and W holds the boxes' W blocks
// in the same order: G = sum_B (Psi^T V)_R W_B as one gathered product.  A
// block owns a 64 x 64 tile of G and a chunk of rows; each thread a 4 x 4
// sub-tile; rows are staged 32 at a time in LDS; the chunks are added by
// k_sum_parts in a fixed order.
constexpr int kBGT = 64;
__global__ __launch_bounds__(kBlock) void k_border_g(const int* ridx, int total_r, const double* Ph,
                                                     const double* W, int p3, int chunk,
                                                     double* Gpart) {
  // unpadded rows: a thread reads its 4 consecutive entries as two 16-byte
  // loads (the 4 values of ra in a wavefront are broadcasts, the 16 of rb
  // one contiguous span)
  __shared__ __align__(16) double sp[32][kBGT];
  __shared__ __align__(16) double sw[32][kBGT];
  const int tiles = (p3 + kBGT - 1) / kBGT;
  const int a0 = (blockIdx.x / tiles) * kBGT, b0 = (blockIdx.x % tiles) * kBGT;
  const int i0 = blockIdx.y * chunk, i1 = min(total_r, i0 + chunk);
  const int tid = threadIdx.x;
  const int ra = (tid >> 4) * 4, rb = (tid & 15) * 4;
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int r0 = i0; r0 < i1; r0 += 32) {
    const int cnt = min(32, i1 - r0);
    __syncthreads();
    for (int t = tid; t < 32 * kBGT; t += kBlock) {
      const int i = t / kBGT, cc = t % kBGT;
      double pv = 0.0, wv = 0.0;
      if (i < cnt) {
        const int row = r0 + i;
        if (a0 + cc < p3) pv = Ph[(size_t)ridx[row] * p3 + a0 + cc];
        if (b0 + cc < p3) wv = W[(size_t)row * p3 + b0 + cc];
      }
      sp[i][cc] = pv;
      sw[i][cc] = wv;
    }
    __syncthreads();
    for (int i = 0; i < cnt; ++i) {
      const double4 pv = *reinterpret_cast<const double4*>(&sp[i][ra]);
      const double4 wv = *reinterpret_cast<const double4*>(&sw[i][rb]);
      const double pa[4] = {pv.x, pv.y, pv.z, pv.w}, wb[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(pa[u], wb[v], acc[u][v]);
    }
  }
  double* G = Gpart + (size_t)blockIdx.y * p3 * p3;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = a0 + ra + u, b = b0 + rb + v;
      if (a < p3 && b < p3) G[(size_t)a * p3 + b] = acc[u][v];
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
// threads of the panel kernel: every step of the panel is a pass over its
// rows, so the panel's time is its column count times one pass
constexpr int kPanelThreads = 1024;
static_assert(kPanelThreads % kGJB == 0, "the panel update deals rows to kPanelThreads / kGJB lanes");

// The panel (h x bb) is factored in LDS when it fits (in_lds != 0, dynamic
// LDS of h * bb doubles), else in the global work array W.
constexpr size_t kPanelLdsBytes = 136 * 1024;

// D^{-1} = U^{-1} L^{-1} for the pivot block D = L U of a panel (lu holds L
// below the diagonal, unit diagonal implied, and U on and above it; bb <=
// kGJB).  Thread c < bb builds column c in registers: x = L^{-1} e_c by forward
// substitution, then U^{-1} x by back substitution, with the rows of lu read
// by broadcast from LDS.  Kept in registers, the substitutions are chains of
// FMAs; built in LDS, every step waited for the previous step's store.
__device__ __forceinline__ void pivot_block_inverse(const double (*lu)[kGJB + 1], const int bb, double* Dinv) {
  const int c = threadIdx.x;
  if (c >= bb) return;
  double x[kGJB];
#pragma unroll
  for (int i = 0; i < kGJB; ++i) {
    double s = (i == c) ? 1.0 : 0.0;
    if (i < bb) {
#pragma unroll
      for (int l = 0; l < i; ++l) s -= lu[i][l] * x[l];
    }
    x[i] = s;
  }
#pragma unroll
  for (int i = kGJB - 1; i >= 0; --i) {
    if (i < bb) {
      double s = x[i];
#pragma unroll
      for (int l = i + 1; l < kGJB; ++l)
        if (l < bb) s -= lu[i][l] * x[l];
      x[i] = s / lu[i][i];
    }
  }
#pragma unroll
  for (int i = 0; i < kGJB; ++i)
    if (i < bb) Dinv[i * bb + c] = x[i];
}

__global__ __launch_bounds__(kPanelThreads) void k_gjb_panel(const double* A, int n, int k0, int bb,
                                                              double* Wg, int* piv, double* Dinv,
                                                              int* status, int in_lds) {
  extern __shared__ double wsh[];
  constexpr int NW = kPanelThreads / 64;
  __shared__ double red[NW];
  __shared__ int ired[NW];
  __shared__ double lu[kGJB][kGJB + 1];
  __shared__ int spiv[kGJB];   // pivot rows, written out once at the end (see k_gjb_panel_reg)
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (*(volatile const int*)status) return;
  double* W = in_lds ? wsh : Wg;
  // rows of W are ldw apart: one more than bb in LDS, so that the passes down
  // a column (pivot search, scaling) hit distinct banks
  const int ldw = in_lds ? bb + 1 : bb;
  const int h = n - k0;
  for (int t = tid; t < h * bb; t += kPanelThreads) {
    const int i = t / bb, c = t % bb;
    W[(size_t)i * ldw + c] = A[(size_t)(k0 + i) * n + k0 + c];
  }
  __syncthreads();
  bool singular = false;
  // The pivot of column j + 1 is found during step j's update: the threads
  // that update column j + 1 fold a 64-bit key (|W| with its low 16 bits
  // replaced by 65535 - row: the larger value, ties to the smaller row) into
  // pkey with an atomic max.  Panels taller than 65535 rows search each column
  // instead.  The update forms each multiplier as W[i][j] / d on the fly (one
  // reciprocal per step, kept in dsc); the L columns are scaled once at the end
  // (a per-column factor, so the later row swaps commute with it).  Two
  // barriers per step.
  __shared__ unsigned long long pkey[2];
  __shared__ double dsc[kGJB];
  const bool fused = h <= 0xFFFF;
  const int cc = tid & (kGJB - 1), rl = tid / kGJB;
  if (tid < 2) pkey[tid] = 0ull;
  for (int j = 0; j < bb; ++j) {
    double best = -1.0;
    int bi = h;
    if (j == 0 || !fused) {
      for (int i = j + tid; i < h; i += kPanelThreads) {
        const double v = fabs(W[(size_t)i * ldw + j]);
        if (v > best) { best = v; bi = i; }
      }
      wave_argmax(best, bi);
      if (lane == 0) { red[wid] = best; ired[wid] = bi; }
      __syncthreads();
      best = red[0];
      bi = ired[0];
      for (int w = 1; w < NW; ++w)
        if (red[w] > best || (red[w] == best && ired[w] < bi)) { best = red[w]; bi = ired[w]; }
      __syncthreads();
    } else {
      const unsigned long long key = pkey[j & 1];
      best = (key >> 16) ? 1.0 : 0.0;        // a candidate with a nonzero value
      bi = 0xFFFF - (int)(key & 0xFFFF);
    }
    if (!(best > 0.0)) {
      for (int jj = tid; jj < bb; jj += kPanelThreads) piv[jj] = jj < j ? spiv[jj] : jj;
      singular = true;
      break;
    }
    // pkey[(j + 1) & 1] was last read at the start of step j - 1
    if (tid == 0) { spiv[j] = bi; pkey[(j + 1) & 1] = 0ull; }
    if (bi != j)
      for (int c = tid; c < bb; c += kPanelThreads) {
        const double a = W[(size_t)j * ldw + c];
        W[(size_t)j * ldw + c] = W[(size_t)bi * ldw + c];
        W[(size_t)bi * ldw + c] = a;
      }
    __syncthreads();
    const double rd = 1.0 / W[(size_t)j * ldw + j];
    if (tid == 0) dsc[j] = rd;
    // trailing update of the panel: thread (row lane tid / 32, column j + 1 +
    // tid % 32) takes every (kPanelThreads / 32)-th row, with its entry of row
    // j in a register; rows go in batches of 8 (all reads, then all writes),
    // so the LDS round trips of a batch overlap
    if (cc < bb - j - 1) {
      constexpr int RL = kPanelThreads / kGJB, RB = 8;
      const int c = j + 1 + cc;
      const double ujc = W[(size_t)j * ldw + c];
      unsigned long long kmax = 0ull;
      for (int i0 = j + 1 + rl; i0 < h; i0 += RB * RL) {
        double wij[RB], wic[RB];
#pragma unroll
        for (int u = 0; u < RB; ++u) {
          const int i = i0 + u * RL;
          wij[u] = i < h ? W[(size_t)i * ldw + j] : 0.0;
          wic[u] = i < h ? W[(size_t)i * ldw + c] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < RB; ++u) {
          const int i = i0 + u * RL;
          if (i < h) {
            const double v = wic[u] - (wij[u] * rd) * ujc;
            W[(size_t)i * ldw + c] = v;
            if (cc == 0 && fused) {
              const unsigned long long kb =
                  ((unsigned long long)__double_as_longlong(fabs(v)) & ~0xFFFFull) | (unsigned long long)(0xFFFF - i);
              kmax = kmax > kb ? kmax : kb;
            }
          }
        }
      }
      if (cc == 0 && fused && kmax) atomicMax(&pkey[(j + 1) & 1], kmax);
    }
    __syncthreads();
  }
  if (!singular) {
    // scale the L columns by their pivots' reciprocals
    for (int c = cc; c < bb; c += kGJB)
      for (int i = c + 1 + rl; i < h; i += kPanelThreads / kGJB) W[(size_t)i * ldw + c] *= dsc[c];
    __syncthreads();
  }
  if (singular) {
    if (tid == 0) *status = 1;
    return;
  }
  // D = L U (first bb rows of W); D^{-1} = U^{-1} L^{-1}
  for (int t = tid; t < bb * bb; t += kPanelThreads) lu[t / bb][t % bb] = W[(size_t)(t / bb) * ldw + t % bb];
  __syncthreads();
  pivot_block_inverse(lu, bb, Dinv);
  for (int t = tid; t < bb; t += kPanelThreads) piv[t] = spiv[t];
}

// The panel with its rows in registers: thread t holds rows t + NT u (u < RU)
// of the h x bb panel (h <= NT RU, bb <= kGJB), so a step reads its
// multipliers from its own registers.  A row is kept rotated: after step j its
// registers hold columns j + 1, j + 2, ... followed by its multipliers for
// columns 0 .. j, so the column of a step is always register 0, the update of
// the remaining columns is also the shift (one FMA per register), and a row
// interchange carries the multipliers along.  One barrier per step: every
// wave publishes its best candidate row (the largest |W[i][j]| over its rows
// i >= j, ties to the smaller row) with its value, and the row to be
// displaced (row j) is published too; after the barrier every thread picks
// the pivot among the candidates and reads the pivot row from LDS, rows j and
// the pivot's trade places, and every row below j takes W[i][c] -= l W[j][c]
// for c > j with l = W[i][j] / W[j][j].  The pivot row is final at its step
// and records its L and U entries in LDS.  Outputs as the LDS panel: the
// pivot rows and D^{-1} of the pivot block D = L U.
template <int NT, int RU>
__global__ __launch_bounds__(NT) void k_gjb_panel_reg(const double* A, int n, int k0, int bb, int* piv,
                                                       double* Dinv, int* status) {
  constexpr int NW = NT / 64;
  __shared__ double cval[2][NW];
  __shared__ int cidx[2][NW];
  __shared__ double cand[2][NW][kGJB];   // each wave's candidate row (by step parity)
  __shared__ double srow[2][kGJB];        // row j before the interchange
  __shared__ double lu[kGJB][kGJB + 1];
  __shared__ int spiv[kGJB];              // pivot rows, written out at the end
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (*(volatile const int*)status) return;
  const int h = n - k0;
  double W[RU][kGJB];
#pragma unroll
  for (int u = 0; u < RU; ++u) {
    const int i = tid + NT * u;
#pragma unroll
    for (int c = 0; c < kGJB; ++c) W[u][c] = (i < h && c < bb) ? A[(size_t)(k0 + i) * n + k0 + c] : 0.0;
  }
  for (int j = 0; j < bb; ++j) {
    const int par = j & 1;
    // this wave's candidate
    double best = -1.0;
    int bi = h;
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int i = tid + NT * u;
      if (i >= j && i < h) arg_better(best, bi, fabs(W[u][0]), i);
    }
    wave_argmax(best, bi);
    if (bi < h && tid == bi % NT) {
      // the winner publishes its row
      const int ub = bi / NT;
#pragma unroll
      for (int u = 0; u < RU; ++u)
        if (u == ub)
#pragma unroll
          for (int c = 0; c < kGJB; ++c) cand[par][wid][c] = W[u][c];
    }
    if (lane == 0) { cval[par][wid] = best; cidx[par][wid] = bi; }
    if (tid == j % NT) {
#pragma unroll
      for (int u = 0; u < RU; ++u)
        if (u == j / NT)
#pragma unroll
          for (int c = 0; c < kGJB; ++c) srow[par][c] = W[u][c];
    }
    __syncthreads();
    // the pivot among the waves' candidates: lane w of every wave takes wave
    // w's, and the wave-wide argmax gives all threads the same pivot
    best = lane < NW ? cval[par][lane] : -1.0;
    bi = lane < NW ? cidx[par][lane] : h;
    wave_argmax(best, bi);
    if (!(best > 0.0)) {
      for (int jj = tid; jj < bb; jj += NT) piv[jj] = jj < j ? spiv[jj] : jj;
      if (tid == 0) *status = 1;
      return;   // uniform: every thread saw the same candidates
    }
    const double* prow = cand[par][(bi % NT) >> 6];   // published by the wave holding row bi
    if (tid == 0) spiv[j] = bi;
    // rows j and bi trade places (the pivot row is prow, row j is srow)
    if (bi != j) {
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        if (tid + NT * u == bi)
#pragma unroll
          for (int c = 0; c < kGJB; ++c) W[u][c] = srow[par][c];
        if (tid + NT * u == j)
#pragma unroll
          for (int c = 0; c < kGJB; ++c) W[u][c] = prow[c];
      }
    }
    // the pivot row is U's row j (columns j .. bb - 1) and L's row j
    // (multipliers for columns 0 .. j - 1)
    if (tid < bb - j) lu[j][j + tid] = prow[tid];
    if (tid < j) lu[j][tid] = prow[kGJB - j + tid];
    const double rp = 1.0 / prow[0];
    const int live = kGJB - j;   // registers 1 .. live - 1 are columns, the rest multipliers
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int i = tid + NT * u;
      if (i > j && i < h) {
        const double l = W[u][0] * rp;
#pragma unroll
        for (int c = 1; c < kGJB; ++c) W[u][c - 1] = fma(-l, c < live ? prow[c] : 0.0, W[u][c]);
        W[u][kGJB - 1] = l;
      }
    }
    // the next step publishes into the other parity; this step's reads end
    // before the next step's barrier
  }
  __syncthreads();
  pivot_block_inverse(lu, bb, Dinv);
  for (int t = tid; t < bb; t += NT) piv[t] = spiv[t];
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

// The same update with the rank-bb products on FP64 matrix cores: one wave
// per 16 x 16 tile of A, acc = Cpanel[tile rows, :] (R or D^{-1})[:, tile
// columns] in bb / 4 v_mfma_f64_16x16x4f64 (K padded with zeros), then the
// element cases of the scalar kernel above.
__global__ __launch_bounds__(kBlock) void k_gjb_update_mfma(double* A, int n, int k0, int bb, const double* Dinv,
                                                           const double* R, const double* Cpanel,
                                                           const int* status) {
  if (*(volatile const int*)status) return;
  const int lane = threadIdx.x & 63;
  const int tn = (n + 15) >> 4;
  const int t = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (t >= tn * tn) return;
  const int i0 = (t / tn) << 4, j0 = (t % tn) << 4;
  const int r16 = lane & 15, kq = lane >> 4;
  const int ia = i0 + r16, jb = j0 + r16;
  const bool bk = jb >= k0 && jb < k0 + bb;
  dbl4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int l0 = 0; l0 < bb; l0 += 4) {
    const int l = l0 + kq;
    const double a = (ia < n && l < bb) ? Cpanel[(size_t)ia * bb + l] : 0.0;
    const double b = (jb < n && l < bb) ? (bk ? Dinv[l * bb + (jb - k0)] : R[(size_t)l * n + jb]) : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = i0 + 4 * q + kq, c = j0 + r16;   // result lane layout of the f64 MFMA
    if (i >= n || c >= n) continue;
    const bool ik = i >= k0 && i < k0 + bb, ck = c >= k0 && c < k0 + bb;
    double v;
    if (ik) v = ck ? Dinv[(i - k0) * bb + (c - k0)] : R[(size_t)(i - k0) * n + c];
    else if (ck) v = -acc[q];
    else v = A[(size_t)i * n + c] - acc[q];
    A[(size_t)i * n + c] = v;
  }
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

}  // namespace

void launch_assemble_M(const LevelBox* boxes, int nbox, int max_m, int n_proxy, double ratio, bool f32,
                       hipStream_t s) {
  if (nbox == 0 || max_m == 0) return;
  dim3 grid(nbox, blocks_for(max_m, kBlock));
  if (f32)
    hipLaunchKernelGGL(k_assemble_M<true>, grid, dim3(kBlock), 0, s, boxes, n_proxy, ratio);
  else
    hipLaunchKernelGGL(k_assemble_M<false>, grid, dim3(kBlock), 0, s, boxes, n_proxy, ratio);
}

void launch_assemble_abb(const LevelBox* boxes, int nbox, int max_n, double lam, bool use_perm, bool f32,
                         hipStream_t s) {
  if (nbox == 0 || max_n == 0) return;
  dim3 grid(nbox, blocks_for((long long)max_n * max_n, kBlock));
  hipLaunchKernelGGL(k_assemble_abb, grid, dim3(kBlock), 0, s, boxes, lam, use_perm ? 1 : 0, f32 ? 1 : 0);
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
                            bool f32, double f32_rcond, hipStream_t s) {
  int f32i = f32 ? 1 : 0;
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
                       status, rc_out, err, f32i, f32_rcond);
    return hipGetLastError();
  }
  void* args[] = {(void*)&boxes, (void*)&G,      (void*)&k_io, (void*)&kx, (void*)&rcond_min,
                  (void*)&status, (void*)&rc_out, (void*)&err,  (void*)&f32i, (void*)&f32_rcond};
  return hipLaunchCooperativeKernel((const void*)k_eliminate, dim3(nbox * G), dim3(kBlock), args,
                                    (unsigned)lds, s);
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
  for (int k0 = 0; k0 < n;) {
    // a panel is worked on in LDS: one taller than the LDS budget at kGJB
    // columns is narrowed until it fits (down to 8 columns; taller panels
    // stay in global memory); the blocking depends on n only
    const int h = n - k0;
    int bb = std::min(kGJB, h);
    // rows in registers: full-width panels.  The fewest waves that hold the
    // rows: a step's barrier and candidate exchange cost less with fewer
    // waves, and below 1024 threads the registers hold the whole step without
    // spilling.  The pivot rule and every row's arithmetic do not depend on
    // the thread count, so the results are bitwise the same.
    if (h <= 256) {
      hipLaunchKernelGGL((k_gjb_panel_reg<256, 1>), dim3(1), dim3(256), 0, s, A, n, k0, bb, piv, Dinv, status);
    } else if (h <= 512) {
      hipLaunchKernelGGL((k_gjb_panel_reg<512, 1>), dim3(1), dim3(512), 0, s, A, n, k0, bb, piv, Dinv, status);
    } else if (h <= 1024) {
      hipLaunchKernelGGL((k_gjb_panel_reg<512, 2>), dim3(1), dim3(512), 0, s, A, n, k0, bb, piv, Dinv, status);
    } else if (h <= 1536) {
      hipLaunchKernelGGL((k_gjb_panel_reg<512, 3>), dim3(1), dim3(512), 0, s, A, n, k0, bb, piv, Dinv, status);
    } else {
      while (bb > 8 && (size_t)h * (bb + 1) * sizeof(double) > kPanelLdsBytes) --bb;
      const size_t pbytes = (size_t)h * (bb + 1) * sizeof(double);
      const int in_lds = pbytes <= kPanelLdsBytes ? 1 : 0;
      hipLaunchKernelGGL(k_gjb_panel, dim3(1), dim3(kPanelThreads), in_lds ? pbytes : 0, s, A, n, k0, bb, W,
                         piv, Dinv, status, in_lds);
    }
    hipLaunchKernelGGL(k_gjb_swap, dim3(blocks_for(n, kBlock)), dim3(kBlock), 0, s, A, n, k0, bb,
                       piv, rowperm, status);
    hipLaunchKernelGGL(k_gjb_copycol, dim3(blocks_for((long long)n * bb, kBlock)), dim3(kBlock), 0,
                       s, A, n, k0, bb, Cp, status);
    hipLaunchKernelGGL(k_gjb_rows, dim3(blocks_for((long long)bb * n, kBlock)), dim3(kBlock), 0, s,
                       A, n, k0, bb, Dinv, R, status);
    const long long tiles = (long long)((n + 15) / 16) * ((n + 15) / 16);
    hipLaunchKernelGGL(k_gjb_update_mfma, dim3(blocks_for(tiles, kBlock / 64)), dim3(kBlock), 0, s, A, n, k0,
                       bb, Dinv, R, Cp, status);
    k0 += bb;
  }
  hipLaunchKernelGGL(k_gjb_unpermute, dim3(blocks_for(nn, kBlock)), dim3(kBlock), 0, s, A, n,
                     rowperm, Ainv);
}

void launch_factor_to_float(const LevelBox* boxes, int nbox, const int* k_final, hipStream_t s) {
  if (nbox) hipLaunchKernelGGL(k_factor_to_float, dim3(nbox), dim3(kBlock), 0, s, boxes, k_final);
}

void launch_border_w(const SolveBox* boxes, int nbox, const int* ridx, const double* Hh, int p3, int max_r,
                     hipStream_t s) {
  if (nbox == 0 || p3 == 0 || max_r <= 0) return;
  const int ntx = (p3 + kBWT - 1) / kBWT, nty = (max_r + kBWT - 1) / kBWT;
  hipLaunchKernelGGL(k_border_w, dim3(nbox, ntx * nty), dim3(kBlock), 0, s, boxes, ridx, Hh, p3, ntx);
}

int border_g_chunks(int total_r, int p3) {
  const int tiles = (p3 + kBGT - 1) / kBGT;
  const int want = std::max(1, 2048 / std::max(1, tiles * tiles));
  const int most = std::max(1, (total_r + 255) / 256);
  return std::min(want, most);
}

void launch_border_g(const int* ridx, int total_r, const double* Ph, const double* W, int p3, int nchunk,
                     double* Gpart, hipStream_t s) {
  if (p3 == 0) return;
  const int tiles = (p3 + kBGT - 1) / kBGT;
  const int chunk = std::max(1, (total_r + nchunk - 1) / nchunk);
  hipLaunchKernelGGL(k_border_g, dim3(tiles * tiles, nchunk), dim3(kBlock), 0, s, ridx, total_r, Ph, W, p3,
                     chunk, Gpart);
}

}  // namespace rs

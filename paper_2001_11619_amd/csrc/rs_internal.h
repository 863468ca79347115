// Internal types shared by the host driver and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace rs {

// Node geometry in structure-of-arrays form (device pointers, float64).
struct Geo {
  const double* x;
  const double* y;
  const double* nx;
  const double* ny;
  const double* w;
  const double* kap;
  int N;
  int kernel;   // 0: Stokes (Section 3.1), 1: Laplace Neumann (Section 4.4.1)
};

// One box compressed at a level.  Device pointers point into per-level
// workspaces and into the persistent factor arena.
struct ChildSrc;

struct LevelBox {
  double cx, cy, side;
  double wscale;  // largest quadrature weight of the box's active nodes: the weight of its
                  // target-side proxy rows and the factor of its target-side rank-one row
  int n;          // active unknowns |I_B|
  int m;          // rows of the ID matrix M_B
  int nF;         // |F_int|
  int slot;       // index of the box in the level's full descriptor list (rank outputs)
  Geo geo;                 // geometry of the box's boundary (per context)
  const int* dofs;         // I_B (n), ascending
  const int* fint;         // F_int (nF)
  const ChildSrc* src;     // per position of I_B: where its child's X_SS is (null for a leaf)
  int* perm;               // pivot order output (n)
  double* M;      // m x n, column-major (ld = m)
  const double* Mq;  // matrix the pivoted QR factors: M, or its row-reduced factor
  int mq;            // its rows (leading dimension)
  int mq_pad;
  double* R;      // kcap x n, row-major, pivot order
  double* Ap;     // n x n, row-major, A_BB in pivot order
  double* scr;    // scratch for the elimination: 3 n^2 + 128 n + 2048
  double* T;      // k x r  (capacity n^2/4 + n)
  double* E;      // k x r
  double* F;      // r x k
  double* Xinv;   // r x r  (capacity n^2)
  double* Xss;    // k x k  (capacity n^2)
  float* Tf;      // float copies for the mixed-precision solve (or null)
  float* Ef;
  float* Ff;
  float* Xinvf;
  // cooperation of several workgroups on one box (pivoted QR, elimination)
  unsigned* bar;  // box barrier counter
  double* hh;     // beta, tau of the current step
  double* cval;   // 2 x G pivot candidates (value)
  int* cphys;     // 2 x G pivot candidates (column)
  double* vbuf;   // m: current Householder vector
};

// Where the parent's diagonal block finds a child's skeleton block.
struct ChildSrc {
  const double* xss;   // child's X_SS (k_c x k_c, row-major)
  int idx;             // position of this unknown in the child's skeleton order
  int ld;              // k_c
  int child;           // child box id (positions with equal ids share X_SS)
  int pad;
};

// One compressed box as seen by the solve sweeps.
struct SolveBox {
  int k, r;
  int s_off, r_off;      // offsets of S and R in the solve index lists
  int part;              // slot of this box in per-box partial buffers
  int pad;
  const double* T;
  const double* E;
  const double* F;
  const double* Xinv;
  double* W;             // r x 3p: X_RR^{-1} (U H)_R (bordered root only)
  const float* Tf;       // float copies (mixed precision); null where the box's
                         // solve reads its float64 factors (Ef, Ff, Xinvf, Wf too)
  const float* Ef;
  const float* Ff;
  const float* Xinvf;
  float* Wf;
};

constexpr int kBlock = 256;
constexpr int kNC = 16;        // right-hand-side columns per sweep block

// ---- launchers (rs_qr.hip, rs_factor.hip, rs_solve.hip, rs_apply.hip) ----
// f32: the float32 bulk form (entries computed in float32 from box-local
// offsets; the Schur-complement products on FP32 matrix cores)
void launch_assemble_M(const LevelBox* boxes, int nbox, int max_m, int n_proxy, double ratio, bool f32,
                       hipStream_t s);
// Register-resident pivoted QR: a 1024-thread workgroup holds RU rows per
// lane (RU even, 64 RU >= m) of CPW columns per wave.
constexpr int kRQThreads = 512;
constexpr int kRQWaves = kRQThreads / 64;
constexpr int kRQBudget = 88;         // doubles per lane: CPW columns of RU rows plus v
constexpr int kRQMaxRU = 40;           // m <= 2560 (one column per wave from RU = 24 on)
__host__ __device__ constexpr int rq_cols_per_wave(int ru) {
  return kRQBudget / ru - 1 < 20 ? kRQBudget / ru - 1 : 20;
}
__host__ __device__ constexpr int rq_row_class(int m) {
  const int ru = (m + 63) / 64;
  return ru < 2 ? 2 : ru + (ru & 1);
}
size_t cpqr_reg_lds_bytes(int max_ru, int max_n);
// One block of the row reduction (unpivoted QR of rows x n, n-row factor out).
struct QRTask {
  const double* src;   // first row of the block, column-major, leading dimension ld
  double* dst;         // triangular factor, n rows, column-major, leading dimension ldd
  int ld, ldd;
  int rows, n;
  int ru, pad;         // rows per lane of the 16-lane layout: 16 ru >= max(rows, n)
};
void launch_tsqr(const QRTask* tasks, int ntask, hipStream_t s);
// 16-lane layout (row reduction, pivoted QR of at most 256 rows): 32 columns
// per register slot and workgroup, rows per lane RU = r16_row_class(rows).
constexpr int kR16MaxRU = 16;
constexpr int kR16MaxCols = 128;       // LDS room for the column bookkeeping (2 ints each)
__host__ __device__ constexpr int r16_row_class(int rows) {
  const int ru = (rows + 15) / 16;
  return ru < 2 ? 2 : ru + (ru & 1);
}
// columns one workgroup holds in the 16-lane kernels (at most 4 slots of 32)
constexpr int kR16MaxN = 128;
hipError_t launch_cpqr16(const LevelBox* boxes, const int4* work, int nbox, double tol, int extra,
                         int* k_out, int* kx_out, int* err, hipStream_t s);
int cpqr_reg_blocks_per_cu(size_t lds);
// work[b] = (box, g, G, RU) for block b; coop: cooperative launch (G > 1 boxes)
hipError_t launch_cpqr_reg(const LevelBox* boxes, const int4* work, int nblocks, bool coop, double tol,
                           int extra, int* k_out, int* kx_out, int* err, size_t lds, hipStream_t s);
void launch_zero_bars(const LevelBox* boxes, int nbox, int* err, hipStream_t s);
size_t cpqr_lds_bytes(int max_m, int max_n);
int cpqr_blocks_per_cu(size_t lds);
hipError_t launch_cpqr(const LevelBox* boxes, const int* list, int nbox, int G, double tol, int extra,
                       int* k_out, int* kx_out, int* err, int max_m, int max_n, hipStream_t s);
void launch_assemble_abb(const LevelBox* boxes, int nbox, int max_n, double lam, bool use_perm, bool f32,
                         hipStream_t s);
int eliminate_blocks_per_cu(int max_n);
hipError_t launch_eliminate(const LevelBox* boxes, int nbox, int G, int* k_io, const int* kx,
                            double rcond_min, int* status, double* rc_out, int* err, int max_n,
                            bool f32, double f32_rcond, hipStream_t s);
void launch_gj_blocked(double* A, int n, double* Ainv, double* work, int* iwork, int* status,
                       hipStream_t s);
template <typename T>
void launch_sweep(const SolveBox* boxes, int nbox, const int* sidx, const int* ridx, T* c,
                  int ncols, int mode, int max_n, hipStream_t s);
template <typename T>
void launch_diag(const SolveBox* boxes, int nbox, const int* ridx, T* c, int ncols, int max_r,
                 hipStream_t s);
void launch_assemble_H(Geo g, const double* hole_xy, int p, const int* curve_id,
                       double* H, double* Psi, hipStream_t s);
// Border of the root system: W_B = X_RR^{-1} (U H)_R per box (max_r >= every
// box's r), then G parts over chunks of the concatenated R lists
// (nchunk = border_g_chunks, Gpart: nchunk x p3 x p3).
void launch_border_w(const SolveBox* boxes, int nbox, const int* ridx, const double* Hh, int p3, int max_r,
                     hipStream_t s);
int border_g_chunks(int total_r, int p3);
void launch_border_g(const int* ridx, int total_r, const double* Ph, const double* W, int p3, int nchunk,
                     double* Gpart, hipStream_t s);
// scratch: sum_parts_scratch_doubles(nparts, len) doubles
size_t sum_parts_scratch_doubles(int nparts, int len);
void launch_sum_parts(const double* parts, int nparts, long long stride, int len,
                      double scale, double* out, double* scratch, hipStream_t s);
template <typename T>
void launch_border_rhs(const SolveBox* boxes, int nbox, const int* ridx, const T* Ph, int p3,
                       const T* c, int ncols, double* parts, hipStream_t s);
template <typename T>
void launch_border_fix(const SolveBox* boxes, int nbox, const int* ridx, int p3, const double* lam,
                       T* c, int ncols, hipStream_t s);
void launch_assemble_Z(const double* X0, int n0, const double* Hh, const double* Ph,
                       const int* I0, int p3, const double* G, double* Z, hipStream_t s);
template <typename T>
void launch_root_gather(const T* c, int ncols, const int* I0, int n0, const double* rhs2, int p3,
                        double* v, hipStream_t s);
void launch_dense_apply(const double* Zinv, int nz, const double* v, int ncols, double* out,
                        hipStream_t s);
template <typename T>
void launch_root_scatter(const double* sol, int ncols, const int* I0, int n0, T* c, hipStream_t s);
void launch_fill(double* x, long long n, double v, hipStream_t s);
void launch_scale_odd_rows(double* x, int N, int ncols, double scale, hipStream_t s);
// flag: 4 ints (converged, iterations, next residual updated, a pair dropped);
// acc: per column, the accumulated rounding bound of updated residuals
void launch_refine_flag(const double* colsq, const double* fsq, const double* bsq, double* acc, int ncols,
                        double tol, int max_iters, int incr, double bscale, int* flag, hipStream_t s);
void launch_accumulate_unless(const double* d, long long n, double* x, const int* flag, int max_iters,
                              hipStream_t s);
void launch_set_ints(int* p, int n, int v, hipStream_t s);
void launch_accumulate(const double* d, long long n, double* x, hipStream_t s);
void launch_accumulate(const float* d, long long n, double* x, hipStream_t s);
// part: residual_scratch_doubles(ncols) doubles; flag (nullable): refinement
// flags (an updated residual r - y when flag[2] = 1, bt its rounding bounds
// per node); bsq receives the squared column norms of the bounds
size_t residual_scratch_doubles(int ncols);
void launch_residual(const double* f, int nf, const double* y, int nrows, int ncols, double* r,
                     double* colsq, double* fsq, double* bsq, double* part, const int* flag, int max_iters,
                     const double* bt, hipStream_t s);
void launch_factor_to_float(const LevelBox* boxes, int nbox, const int* k_final, hipStream_t s);
void launch_w_to_float(const SolveBox* boxes, int nbox, int p3, hipStream_t s);
void launch_to_rows(const double* f, int ld, int nrows, int ncols, double* c, hipStream_t s);
void launch_from_rows(const double* c, int nrows, int ncols, double* x, int ld, hipStream_t s);
// Exact operator apply (refinement residual).  cfg selects one of
// apply_config_count() kernel shapes (columns per pass, targets per thread);
// skip (nullable) holds the refinement flags: the apply is skipped once they
// say converged or exhausted.
size_t apply_scratch_doubles(int N, int ncols);
// the fixed per-device array of the allocation-free apply: its size in
// doubles, and its device address on `device` (which must be current;
// looked up on the first call per device)
size_t noalloc_scratch_doubles();
hipError_t noalloc_scratch(int device, double** out);
int apply_config_count();
bool apply_config_valid(int cfg, int ncols);
int apply_default_config(int ncols);
void apply_config_name(int cfg, char* buf, int len);
void launch_apply_operator(Geo g, const int* curve_id, const double* hole_xy, int p,
                           double lam, const double* x, int ncols, double* y,
                           double* part, const int* skip, int max_iters, int cfg, hipStream_t s);
// The apply of one refinement iteration: the exact float64 apply of x, or the
// float32 image of the correction dx (flag[2] = 1), chosen on the device; which
// = -1 launches both (graph capture), 0 or 1 only that one.  corr:
// corr_scratch_bytes(N, ncols) bytes; corr_bound_rows(corr, ...) the
// per-node rounding bounds of the last image (N x ncols doubles), to be
// scaled by corr_bound_scale().
size_t corr_scratch_bytes(int N, int ncols);
double* corr_bound_rows(void* corr, int N, int ncols);
double corr_bound_scale();
void launch_apply_refine(Geo g, const int* curve_id, const double* hole_xy, int p, double lam, const double* x,
                         const double* dx, int ncols, double* y, double* part, void* corr, int* flag,
                         int max_iters, int cfg, int which, hipStream_t s);
// Velocity u = D mu + H lambda at nt target points (tx, ty); x, u rows layout
// ((2N + 3p) x ncols and 2 nt x ncols); part: eval_scratch_doubles(N, nt, ncols).
size_t eval_scratch_doubles(int N, int nt, int ncols);
void launch_evaluate(Geo g, const double* hole_xy, int p, const double* tx, const double* ty, int nt,
                     const double* x, int ncols, double* u, double* part, int cfg, hipStream_t s);

}  // namespace rs

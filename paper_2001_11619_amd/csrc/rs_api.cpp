// Host driver and C ABI of the recursive-skeletonization solver.
//
// The host owns the quadtree (Section 2.3), the per-level bookkeeping of
// active unknowns and near fields (Section 2.7: every box of a level reads
// the level-start active set), and the launch sequence; every arithmetic step
// of the factorization and solve runs in the gfx950 kernels (rs_qr.hip,
// rs_factor.hip, rs_solve.hip, rs_apply.hip).  One host synchronisation per
// level reads back the ranks and pivot orders, which size the next level.
#include "rs.h"
#include "rs_internal.h"

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <exception>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#pragma clang fp contract(off)

using namespace rs;

namespace {

struct RsError {
  rs_status st;
  std::string msg;
};

#define HIP_CHECK(expr)                                                                   \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw RsError{e_ == hipErrorOutOfMemory ? RS_ERR_ALLOC : RS_ERR_DEVICE,             \
                    std::string(#expr) + ": " + hipGetErrorString(e_)};                   \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  // pinned host mirror used by upload(): the copy out of it is asynchronous,
  // `ev` marks its completion before the mirror is written again
  void* host = nullptr;
  size_t host_bytes = 0;
  hipEvent_t ev = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    release();
    if (ev) {
      (void)hipEventSynchronize(ev);
      (void)hipEventDestroy(ev);
    }
    if (host) (void)hipHostFree(host);
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void ensure(size_t nb) {
    if (nb <= bytes) return;
    release();
    if (nb == 0) return;
    HIP_CHECK(hipMalloc(&p, nb));
    bytes = nb;
  }
  // Copy nb bytes into the mirror once the previous copy out of it is done.
  void stage(const void* src, size_t nb) {
    if (ev) HIP_CHECK(hipEventSynchronize(ev));
    else HIP_CHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    if (nb > host_bytes) {
      if (host) HIP_CHECK(hipHostFree(host));
      host = nullptr;
      host_bytes = 0;
      const size_t cap = std::max<size_t>(nb + nb / 2, 4096);
      HIP_CHECK(hipHostMalloc(&host, cap, hipHostMallocDefault));
      host_bytes = cap;
    }
    std::memcpy(host, src, nb);
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// Host-to-device copy on the context stream through the buffer's pinned
// mirror; returns at once (the host vector may be reused immediately).
template <class T>
void upload(DevBuf& b, const std::vector<T>& v, hipStream_t s) {
  const size_t nb = v.size() * sizeof(T);
  b.ensure(std::max<size_t>(nb, 16));
  if (nb == 0) return;
  b.stage(v.data(), nb);
  HIP_CHECK(hipMemcpyAsync(b.p, b.host, nb, hipMemcpyHostToDevice, s));
  HIP_CHECK(hipEventRecord(b.ev, s));
}

// Pinned host buffer for device-to-host copies that stay asynchronous.
struct PinHost {
  void* p = nullptr;
  size_t bytes = 0;
  PinHost() = default;
  PinHost(const PinHost&) = delete;
  PinHost& operator=(const PinHost&) = delete;
  ~PinHost() {
    if (p) (void)hipHostFree(p);
  }
  template <class T>
  T* get(size_t n) {   // contents are not kept when the buffer grows
    const size_t nb = n * sizeof(T);
    if (nb > bytes) {
      if (p) HIP_CHECK(hipHostFree(p));
      p = nullptr;
      bytes = 0;
      const size_t cap = std::max<size_t>(nb + nb / 2, 4096);
      HIP_CHECK(hipHostMalloc(&p, cap, hipHostMallocDefault));
      bytes = cap;
    }
    return static_cast<T*>(p);
  }
};

struct Box {
  int level = 0;
  double cx = 0, cy = 0, side = 0;
  long long ix = 0, iy = 0;
  int parent = -1;
  int child[4] = {-1, -1, -1, -1};
  int nchild = 0;
  std::vector<int> nodes;
  std::vector<int> dofs;        // leaf: its unknowns, ascending
  // boxes whose square comes within the proxy radius of this box's centre:
  // same-level boxes and coarser leaves (the only holders of active unknowns
  // that can lie inside the proxy circle when this box is compressed)
  std::vector<int> near_same, near_leaf;
  bool leaf() const { return nchild == 0; }
};

struct BoxFac {
  int n = 0, k = 0, level = 0;
  bool active = false;        // compressed (n > 0, not the root)
  std::vector<int> I;         // active unknowns, ascending
  std::vector<int> perm;      // pivot order (positions into I)
  double* T = nullptr;
  double* E = nullptr;
  double* F = nullptr;
  double* Xinv = nullptr;
  double* Xss = nullptr;
  double* W = nullptr;
  float* Tf = nullptr;        // float copies (mixed precision)
  float* Ef = nullptr;
  float* Ff = nullptr;
  float* Xinvf = nullptr;
  int arena = -1;             // id of the device arena holding T, E, F, Xinv, Xss
  int rank0 = 0;
  double rcond = 1.0;         // rcond_1 of the accepted X_RR
  std::vector<int> fint;      // near field F_int used by the compression
};

using BoxKey = std::tuple<int, long long, long long>;   // (level, ix, iy)

// Factorization state before an update: boxes are matched by BoxKey.
struct OldState {
  std::vector<Box> boxes;
  std::vector<BoxFac> fac;
  std::map<BoxKey, int> by_key;
  std::vector<char> moved;    // per node of the new geometry
};

constexpr int kMaxDepth = 48;
constexpr int kGuardExtra = 8;

inline long long key2(long long ix, long long iy) { return (ix << 32) ^ (iy & 0xffffffffLL); }

}  // namespace

struct rs_ctx {
  rs_params prm{};
  // host clock at the end of the previous level's read-back (timing only)
  std::chrono::steady_clock::time_point level_done{};
  bool level_done_set = false;
  int N = 0, p = 0;
  std::vector<double> x, y, nx, ny, w, kap, hole;
  std::vector<int> curve;
  hipStream_t stream = nullptr;
  std::string err;
  int device = 0;

  // device geometry
  DevBuf d_x, d_y, d_nx, d_ny, d_w, d_kap, d_curve, d_hole;

  // tree
  std::vector<Box> boxes;
  int L = 0;
  double root_cx = 0, root_cy = 0, root_side = 0;

  // factorization
  bool factored = false;
  std::vector<BoxFac> fac;
  std::map<int, std::unique_ptr<DevBuf>> arenas;   // factor storage, one per level launch
  std::vector<std::unique_ptr<DevBuf>> arena_pool;  // released arenas kept for reuse
  int next_arena = 0;
  std::vector<char> recomputed;   // per box of the current tree
  std::vector<int> lvl_pos;       // host scratch of prepare_level
  PinHost h_rank, h_perm, h_small, h_rc;  // pinned read-back buffers
  const OldState* old = nullptr;  // set while an update runs
  // level workspaces (reused level to level)
  // a level launch's inputs (index lists, descriptors, QR tasks and work lists)
  // in one device buffer per level parity, filled by one copy
  DevBuf ws_in_a, ws_in_b;
  int desc_flip = 0;
  // ws_out: a level's per-box results read back by the host in one copy:
  // error flags (4 ints) | k (nb ints, padded to even) | status (same) | rcond (nb doubles)
  DevBuf ws_M, ws_R, ws_A, ws_scr, ws_src, ws_perm, ws_kx, ws_coop, ws_tq, ws_out;
  int n_cu = 0;                   // compute units of the device
  // root
  std::vector<int> I0;
  DevBuf d_I0, d_X0, d_Z, d_Zinv, d_gjwork, d_gjiwork, d_rcond, d_rstatus, d_root_box;
  DevBuf d_H, d_Hh, d_Ph, d_Gpart, d_G, d_W, d_Wf;
  int nz = 0;
  // solve metadata
  std::vector<std::vector<SolveBox>> sboxes;   // per level
  std::vector<int> lvl_maxn, lvl_maxr;
  DevBuf d_sboxes, d_sidx, d_ridx;
  std::vector<size_t> sbox_off;                 // offset of each level's boxes in d_sboxes
  int n_solve_boxes = 0;
  int n_ridx = 0;                 // length of the concatenated R lists
  int all_maxr = 0;
  // solve work
  DevBuf d_f, d_c, d_v, d_sol, d_parts, d_rhs2, d_xout, d_res, d_frows, d_xs, d_r, d_dx,
      d_ys, d_norms, d_apply;
  // evaluation at target points
  DevBuf d_evx, d_evy, d_evu, d_evpart;
  std::vector<double> last_res;   // relative residual per column of the last refined solve

  rs_stats stats{};

  // refinement iterations captured as a HIP graph (rebuilt after each factorization)
  long long factor_epoch = 0;
  bool root_pending = false;   // the root inverse was launched and not yet joined
  bool capturing = false;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t refine_exec = nullptr;   // one refinement iteration
  int refine_nrhs = 0;
  long long refine_epoch = -1;
  // device addresses of every buffer the captured iteration reads or writes;
  // a buffer that grew since the capture (rs_apply with more columns, a solve
  // without refinement) has moved, and the graph is captured again
  std::vector<const void*> refine_sig;
  double refine_prev = 1.0;       // largest relative residual before the last launch
  int refine_last = 0;            // iterations in the last launch
  DevBuf d_flag;                  // [converged, corrections applied, next residual updated, pair dropped]
  DevBuf d_corr;                  // scratch of the float32 correction images
  DevBuf d_fflag;                 // flags of rs_apply_f32
  int refine_which = 0;           // eager refinement: residual of the next iteration (0 exact, 1 updated)
  hipEvent_t ev_qr = nullptr;     // a level's QR ranks and pivot orders have reached the host
  // second stream of a level's pivoted QR: the cooperative and memory-route
  // launches run beside the row-reduced boxes (fork after assembly, join before
  // A_BB)
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_pre = nullptr;    // the next level's assembly and row reduction are done (second stream)
  hipEvent_t ev_tune[4] = {};     // launch-shape trials: memory-route QR, elimination (start, end)
  PinHost h_flag;

  // kernel timing (HIP events around launches)
  int timing = 0;                 // 0 off, 1 per kernel family, 2 per family and level,
                                  // 3 the pivoted-QR family only (no host phases)
  int cur_level = -1;
  struct Pending { int fam; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  std::vector<std::string> fam_name;
  std::vector<int> fam_launches;
  std::vector<double> fam_ms;

  ~rs_ctx() {
    if (refine_exec) (void)hipGraphExecDestroy(refine_exec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (ev_qr) (void)hipEventDestroy(ev_qr);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (ev_pre) (void)hipEventDestroy(ev_pre);
    for (hipEvent_t e : ev_tune)
      if (e) (void)hipEventDestroy(e);
    if (side_stream) (void)hipStreamDestroy(side_stream);
    for (auto& p : pending) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (auto e : event_pool) (void)hipEventDestroy(e);
  }
};

namespace {

thread_local std::string g_build_error;

void geo_of(const rs_ctx* c, Geo& g) {
  g.x = c->d_x.as<double>();
  g.y = c->d_y.as<double>();
  g.nx = c->d_nx.as<double>();
  g.ny = c->d_ny.as<double>();
  g.w = c->d_w.as<double>();
  g.kap = c->d_kap.as<double>();
  g.N = c->N;
  g.kernel = c->prm.kernel;
}

// ---- kernel timing --------------------------------------------------------
hipEvent_t take_event(rs_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIP_CHECK(hipEventCreate(&e));
  return e;
}

int family(rs_ctx* c, const char* name) {
  for (size_t i = 0; i < c->fam_name.size(); ++i)
    if (c->fam_name[i] == name) return (int)i;
  c->fam_name.push_back(name);
  c->fam_launches.push_back(0);
  c->fam_ms.push_back(0.0);
  return (int)c->fam_name.size() - 1;
}

// Brackets one launch (or a group of launches) with events when timing is on.
struct KTimer {
  rs_ctx* c;
  hipStream_t st;
  int fam = -1;
  hipEvent_t a{};
  // detail: a sub-phase, timed only in per-level mode; on: the stream the
  // phase is launched on (the context's stream when null)
  KTimer(rs_ctx* ctx, const char* name, bool detail = false, hipStream_t on = nullptr)
      : c(ctx), st(on ? on : ctx->stream) {
    if (!c->timing || c->capturing || (detail && c->timing != 2)) return;
    if (c->timing == 3 && std::strcmp(name, "cpqr") != 0) return;
    if (c->timing == 4 && std::strcmp(name, "apply_operator") != 0 && std::strcmp(name, "apply_correction") != 0)
      return;
    if (c->timing == 2 && c->cur_level >= 0) {
      const std::string full = std::string(name) + "@L" + std::to_string(c->cur_level);
      fam = family(c, full.c_str());
    } else {
      fam = family(c, name);
    }
    a = take_event(c);
    HIP_CHECK(hipEventRecord(a, st));
  }
  ~KTimer() {
    if (fam < 0) return;
    hipEvent_t b{};
    if (!c->event_pool.empty()) {
      b = c->event_pool.back();
      c->event_pool.pop_back();
    } else if (hipEventCreate(&b) != hipSuccess) {
      return;
    }
    if (hipEventRecord(b, st) == hipSuccess) c->pending.push_back({fam, a, b});
  }
};

// Wall time of a host phase (name "host:..."), accumulated when timing is on.
struct HTimer {
  rs_ctx* c;
  int fam = -1;
  std::chrono::steady_clock::time_point t0;
  HTimer(rs_ctx* ctx, const char* name) : c(ctx) {
    if (!c->timing || c->timing >= 3) return;
    fam = family(c, name);
    t0 = std::chrono::steady_clock::now();
  }
  ~HTimer() {
    if (fam < 0) return;
    c->fam_ms[fam] += 1e3 * std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    c->fam_launches[fam] += 1;
  }
};

// Resolve recorded event pairs; call after the stream has been synchronised.
// Pairs on the second stream that have not completed yet stay pending.
void resolve_timers(rs_ctx* c) {
  std::vector<decltype(c->pending)::value_type> keep;
  for (auto& p : c->pending) {
    if (hipEventQuery(p.b) == hipErrorNotReady) {
      keep.push_back(p);
      continue;
    }
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, p.a, p.b));
    c->fam_ms[p.fam] += ms;
    c->fam_launches[p.fam] += 1;
    c->event_pool.push_back(p.a);
    c->event_pool.push_back(p.b);
  }
  c->pending.swap(keep);
}

// Process-wide pool of host threads for the per-box host work of a level
// (near fields, unknown lists).  run(n, f) calls f(i) for every i < n, the
// caller taking part; small n runs on the caller alone.  Calls from several
// host threads are serialized.  A level's host work comes as a burst of two
// jobs, and the next level's preparation is on the critical path of the
// level pipeline, so workers poll for a new job for kSpinUs after finishing
// one before they block, and the caller polls for their completion.
class HostPool {
 public:
  static HostPool& instance() {
    static HostPool pool;
    return pool;
  }
  // f(0 .. n-1) over the pool.  Fine-grained items (n below kSerialBelow run
  // inline); a call made from inside pool work runs inline too, so a task of
  // run_tasks may itself call run.
  void run(int n, const std::function<void(int)>& f) { run_impl(n, f, kSerialBelow, false); }
  // Coarse tasks (one per context of a batch): every task may go to its own
  // thread.  An exception of a task is rethrown here once all have ended.
  void run_tasks(int n, const std::function<void(int)>& f) {
    std::vector<std::exception_ptr> errs(std::max(n, 0));
    const std::function<void(int)> g = [&](int i) {
      try {
        f(i);
      } catch (...) {
        errs[i] = std::current_exception();
      }
    };
    run_impl(n, g, 2, true);
    for (auto& e : errs)
      if (e) std::rethrow_exception(e);
  }
  void run_impl(int n, const std::function<void(int)>& f, int serial_below, bool unit_chunks) {
    if (n < serial_below || workers_.empty() || tl_in_pool) {
      for (int i = 0; i < n; ++i) f(i);
      return;
    }
    std::lock_guard<std::mutex> serial(run_mu_);
    {
      std::lock_guard<std::mutex> lk(mu_);
      fn_ = &f;
      n_ = n;
      chunk_ = unit_chunks ? 1 : std::max(1, n / (4 * (int)(workers_.size() + 1)));
      next_.store(0);
      active_.store((int)workers_.size());
      gen_.fetch_add(1, std::memory_order_release);
    }
    cv_.notify_all();
    tl_in_pool = true;
    work();
    tl_in_pool = false;
    while (active_.load(std::memory_order_acquire) != 0) std::this_thread::yield();
    fn_ = nullptr;
  }
  ~HostPool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_.store(true);
    }
    cv_.notify_all();
    for (auto& t : workers_) t.join();
  }

 private:
  static constexpr int kSerialBelow = 32;
  static constexpr int kSpinUs = 200;
  HostPool() {
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int nthreads = (int)std::min(16u, hw);
    for (int i = 0; i + 1 < nthreads; ++i)
      workers_.emplace_back([this] {
        tl_in_pool = true;
        loop();
      });
  }
  static thread_local bool tl_in_pool;
  void work() {
    for (;;) {
      const int b = next_.fetch_add(chunk_);
      if (b >= n_) return;
      const int e = std::min(n_, b + chunk_);
      for (int i = b; i < e; ++i) (*fn_)(i);
    }
  }
  void loop() {
    unsigned seen = 0;
    for (;;) {
      bool got = false;
      const auto t0 = std::chrono::steady_clock::now();
      while (!stop_.load(std::memory_order_relaxed) &&
             std::chrono::steady_clock::now() - t0 < std::chrono::microseconds(kSpinUs)) {
        if (gen_.load(std::memory_order_acquire) != seen) {
          got = true;
          break;
        }
      }
      if (!got) {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stop_.load() || gen_.load(std::memory_order_acquire) != seen; });
      }
      if (stop_.load()) return;
      seen = gen_.load(std::memory_order_acquire);
      work();
      active_.fetch_sub(1, std::memory_order_acq_rel);
    }
  }
  std::vector<std::thread> workers_;
  std::mutex run_mu_, mu_;
  std::condition_variable cv_;
  const std::function<void(int)>* fn_ = nullptr;
  int n_ = 0, chunk_ = 1;
  std::atomic<int> active_{0};
  std::atomic<unsigned> gen_{0};
  std::atomic<bool> stop_{false};
  std::atomic<int> next_{0};
};
thread_local bool HostPool::tl_in_pool = false;

// Leaf unknowns and the near-box lists of every box (static for a tree).  A
// box is listed when the distance from the compressed box's centre to its
// square is at most the proxy radius (with a relative margin of 1e-9, so that
// rounding in box centres never drops a box whose points may pass the strict
// inside test).
void build_neighbors(rs_ctx* c) {
  std::vector<std::unordered_map<long long, int>> cells(c->L + 1);
  for (size_t bi = 0; bi < c->boxes.size(); ++bi) {
    const Box& B = c->boxes[bi];
    cells[B.level][key2(B.ix, B.iy)] = (int)bi;
  }
  const double ratio = c->prm.proxy_ratio;
  auto near = [](const Box& B, const Box& Q, double rp) {
    const double h = 0.5 * Q.side;
    const double ex = std::max(0.0, std::fabs(B.cx - Q.cx) - h);
    const double ey = std::max(0.0, std::fabs(B.cy - Q.cy) - h);
    return ex * ex + ey * ey <= rp * rp * (1.0 + 1e-9);
  };
  // boxes are independent here (the cell maps are only read)
  HostPool::instance().run((int)c->boxes.size(), [&](int bi) {
    Box& B = c->boxes[bi];
    B.dofs.clear();
    B.near_same.clear();
    B.near_leaf.clear();
    if (B.leaf()) {
      // the Laplace Neumann kernel's second unknown per node is uncoupled
      // (row lambda x): it joins no box and the solve divides it by lambda
      const bool both = c->prm.kernel != 1;
      B.dofs.reserve(2 * B.nodes.size());
      for (int j : B.nodes) {
        B.dofs.push_back(2 * j);
        if (both) B.dofs.push_back(2 * j + 1);
      }
      std::sort(B.dofs.begin(), B.dofs.end());
    }
    if (B.level == 0) return;
    const int l = B.level;
    const double rp = ratio * B.side;
    const long long D = (long long)std::floor(ratio + 0.5) + 1;
    for (long long dx = -D; dx <= D; ++dx)
      for (long long dy = -D; dy <= D; ++dy) {
        if (dx == 0 && dy == 0) continue;
        auto it = cells[l].find(key2(B.ix + dx, B.iy + dy));
        if (it != cells[l].end() && near(B, c->boxes[it->second], rp)) B.near_same.push_back(it->second);
      }
    for (int lc = 0; lc < l; ++lc) {
      const long long ax = B.ix >> (l - lc), ay = B.iy >> (l - lc);
      const double sc = std::ldexp(B.side, l - lc);
      const long long Dc = (long long)std::ceil(rp / sc) + 1;
      for (long long dx = -Dc; dx <= Dc; ++dx)
        for (long long dy = -Dc; dy <= Dc; ++dy) {
          auto it = cells[lc].find(key2(ax + dx, ay + dy));
          if (it == cells[lc].end()) continue;
          const Box& Q = c->boxes[it->second];
          if (Q.leaf() && near(B, Q, rp)) B.near_leaf.push_back(it->second);
        }
    }
  });
}

void build_tree(rs_ctx* c) {
  c->boxes.clear();
  Box root;
  if (c->prm.has_root) {
    root.cx = c->prm.root[0];
    root.cy = c->prm.root[1];
    root.side = c->prm.root[2];
  } else {
    double xmin = c->x[0], xmax = c->x[0], ymin = c->y[0], ymax = c->y[0];
    for (int i = 1; i < c->N; ++i) {
      xmin = std::min(xmin, c->x[i]);
      xmax = std::max(xmax, c->x[i]);
      ymin = std::min(ymin, c->y[i]);
      ymax = std::max(ymax, c->y[i]);
    }
    root.cx = 0.5 * (xmin + xmax);
    root.cy = 0.5 * (ymin + ymax);
    root.side = (1.0 + std::ldexp(1.0, -20)) * std::max(xmax - xmin, ymax - ymin);
    if (root.side == 0.0) root.side = 1.0;
  }
  root.nodes.resize(c->N);
  for (int i = 0; i < c->N; ++i) root.nodes[i] = i;
  c->root_cx = root.cx;
  c->root_cy = root.cy;
  c->root_side = root.side;
  c->boxes.push_back(std::move(root));
  const int leaf = c->prm.leaf_size;
  // level by level: the boxes of a level split on host threads, and their
  // children are appended in box order (breadth-first numbering)
  size_t lo = 0, hi = 1;
  while (lo < hi) {
    const int nl = (int)(hi - lo);
    std::vector<std::array<std::vector<int>, 4>> parts(nl);
    bool too_deep = false;
    for (size_t bi = lo; bi < hi; ++bi)
      if ((int)c->boxes[bi].nodes.size() > leaf && c->boxes[bi].level >= kMaxDepth) too_deep = true;
    if (too_deep) throw RsError{RS_ERR_ARG, "quadtree deeper than 48 levels (coincident nodes?)"};
    HostPool::instance().run(nl, [&](int t) {
      const Box& B = c->boxes[lo + t];
      if ((int)B.nodes.size() <= leaf) return;
      for (int j : B.nodes) {
        const int q = (c->x[j] >= B.cx ? 1 : 0) + 2 * (c->y[j] >= B.cy ? 1 : 0);
        parts[t][q].push_back(j);
      }
    });
    for (size_t bi = lo; bi < hi; ++bi) {
      auto& part = parts[bi - lo];
      const double cx = c->boxes[bi].cx, cy = c->boxes[bi].cy, side = c->boxes[bi].side;
      const double h = side / 4.0;
      for (int q = 0; q < 4; ++q) {
        if (part[q].empty()) continue;
        Box ch;
        ch.level = c->boxes[bi].level + 1;
        ch.cx = (q % 2 == 0) ? cx - h : cx + h;
        ch.cy = (q < 2) ? cy - h : cy + h;
        ch.side = side / 2.0;
        ch.ix = 2 * c->boxes[bi].ix + (q & 1);
        ch.iy = 2 * c->boxes[bi].iy + (q >> 1);
        ch.parent = (int)bi;
        ch.nodes = std::move(part[q]);
        const int id = (int)c->boxes.size();
        c->boxes[bi].child[c->boxes[bi].nchild++] = id;
        c->boxes.push_back(std::move(ch));
      }
    }
    lo = hi;
    hi = c->boxes.size();
  }
  c->L = 0;
  for (const Box& b : c->boxes) c->L = std::max(c->L, b.level);
  HTimer ht_(c, "host:tree.neighbors");
  build_neighbors(c);
}

std::vector<int> skeleton_of(const BoxFac& f) {
  std::vector<int> s(f.k);
  for (int i = 0; i < f.k; ++i) s[i] = f.I[f.perm[i]];
  return s;
}

std::vector<int> redundant_of(const BoxFac& f) {
  std::vector<int> r(f.n - f.k);
  for (int i = f.k; i < f.n; ++i) r[i - f.k] = f.I[f.perm[i]];
  return r;
}

// Unknowns of box b and, for a parent, where each one sits in its child's X_SS.
void box_unknowns(const rs_ctx* c, int b, std::vector<int>& I, std::vector<ChildSrc>* src) {
  const Box& B = c->boxes[b];
  I.clear();
  if (src) src->clear();
  if (B.leaf()) {
    I = B.dofs;
    return;
  }
  struct E { int dof; int child; int idx; };
  std::vector<E> ents;
  for (int q = 0; q < B.nchild; ++q) {
    const int ch = B.child[q];
    const BoxFac& f = c->fac[ch];
    for (int i = 0; i < f.k; ++i) ents.push_back({f.I[f.perm[i]], ch, i});
  }
  std::sort(ents.begin(), ents.end(), [](const E& a, const E& b2) { return a.dof < b2.dof; });
  I.resize(ents.size());
  if (src) src->resize(ents.size());
  for (size_t i = 0; i < ents.size(); ++i) {
    I[i] = ents[i].dof;
    if (src) {
      const BoxFac& f = c->fac[ents[i].child];
      (*src)[i] = ChildSrc{f.Xss, ents[i].idx, f.k, ents[i].child, 0};
    }
  }
}

double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Updating rule (Section 2.8): a box is recompressed when an input of its
// compression changed.  Leaf: new box, different node set, or a moved node.
// Parent: new box, different children, or a recompressed child.  Any box: a
// different near field F_int or a moved node in it.  Otherwise the stored
// factors are exactly those a fresh factorization would compute.
bool compress_needed(const rs_ctx* c, int b, const std::vector<int>& F) {
  const OldState& O = *c->old;
  const Box& B = c->boxes[b];
  auto it = O.by_key.find(BoxKey{B.level, B.ix, B.iy});
  if (it == O.by_key.end()) return true;
  const Box& OB = O.boxes[it->second];
  const BoxFac& OF = O.fac[it->second];
  if (!OF.active || OB.leaf() != B.leaf()) return true;
  if (B.leaf()) {
    if (OB.nodes != B.nodes) return true;
    for (int j : B.nodes)
      if (O.moved[j]) return true;
  } else {
    std::vector<BoxKey> ok, nk;
    for (int q = 0; q < OB.nchild; ++q) {
      const Box& C = O.boxes[OB.child[q]];
      ok.emplace_back(C.level, C.ix, C.iy);
    }
    for (int q = 0; q < B.nchild; ++q) {
      const Box& C = c->boxes[B.child[q]];
      nk.emplace_back(C.level, C.ix, C.iy);
      if (c->recomputed[B.child[q]]) return true;
    }
    std::sort(ok.begin(), ok.end());
    std::sort(nk.begin(), nk.end());
    if (ok != nk) return true;
  }
  if (F != OF.fint) return true;
  for (int d : F)
    if (O.moved[d >> 1]) return true;
  return false;
}


// Work of one context at one level: the boxes it compresses, prepared on the host.
struct LevelPrep {
  std::vector<int> ids;          // all boxes of the level
  std::vector<int> sel;          // positions in ids that are compressed now
  std::vector<LevelBox> lb;      // their descriptors (device pointers filled)
  std::vector<int> doff;         // offset of each compressed box's I_B in the context's list
  std::vector<int> perm;         // pivot orders read back
  std::vector<int> dofs, fint;   // I_B and F_int of the compressed boxes, concatenated
  std::vector<ChildSrc> src;     // where each parent unknown's child block is
  int max_m = 0, max_n = 0;
  int aid = -1;
  size_t first = 0;              // index of the first box in the batched launch
};

constexpr int kMaxCoop = 64;     // most workgroups per box in the cooperative kernels

// A factor arena of at least `bytes`: the smallest pooled one that fits, else
// the largest pooled one grown, else a new one.  Work that read a pooled arena
// has completed (every entry point returns after its device work).
std::unique_ptr<DevBuf> take_arena(rs_ctx* c, size_t bytes) {
  auto& pool = c->arena_pool;
  int best = -1, largest = -1;
  for (int i = 0; i < (int)pool.size(); ++i) {
    if (pool[i]->bytes >= bytes && (best < 0 || pool[i]->bytes < pool[best]->bytes)) best = i;
    if (largest < 0 || pool[i]->bytes > pool[largest]->bytes) largest = i;
  }
  const int pick = best >= 0 ? best : largest;
  std::unique_ptr<DevBuf> a;
  if (pick >= 0) {
    a = std::move(pool[pick]);
    pool.erase(pool.begin() + pick);
  } else {
    a = std::make_unique<DevBuf>();
  }
  a->ensure(bytes);
  return a;
}

// Host part of one level for one context: unknowns, near fields, reuse
// decisions, workspace and arena allocation, uploads of the index lists.
void prepare_level(rs_ctx* c, int l, const std::vector<int>& ids, const std::vector<char>& active,
                   LevelPrep& P) {
  HTimer ht_(c, "host:prepare");
  const rs_params& prm = c->prm;
  Geo g;
  geo_of(c, g);
  P = LevelPrep();
  P.ids = ids;
  const int nids = (int)ids.size();
  std::vector<std::vector<int>> Is(nids);
  std::vector<std::vector<ChildSrc>> srcs(nids);
  HostPool& pool = HostPool::instance();
  {
    HTimer ht2_(c, "host:prep.unknowns");
    pool.run(nids, [&](int t) { box_unknowns(c, ids[t], Is[t], &srcs[t]); });
  }
  // position of each box of this level in ids (-1: other levels)
  std::vector<int>& pos_of = c->lvl_pos;
  pos_of.assign(c->boxes.size(), -1);
  for (int t = 0; t < nids; ++t) pos_of[ids[t]] = t;
  // near field F_int of every box (active unknowns strictly inside the proxy
  // circle, not in I_B) and whether an update can keep its factors; boxes are
  // independent here
  std::vector<std::vector<int>> Fs(nids);
  std::vector<char> keep(nids, 0);
  {
  HTimer ht3_(c, "host:prep.near");
  pool.run(nids, [&](int t) {
    if (Is[t].empty()) return;
    const int b = ids[t];
    const Box& B = c->boxes[b];
    const double rp = prm.proxy_ratio * B.side;
    const double rp2 = rp * rp;
    std::vector<int>& F = Fs[t];
    auto take = [&](const std::vector<int>& cand) {
      for (int d : cand) {
        if (!active[d]) continue;
        const int j = d >> 1;
        const double ddx = c->x[j] - B.cx, ddy = c->y[j] - B.cy;
        if (ddx * ddx + ddy * ddy < rp2) F.push_back(d);
      }
    };
    for (int q : B.near_same)
      if (pos_of[q] >= 0) take(Is[pos_of[q]]);
    for (int q : B.near_leaf) take(c->boxes[q].dofs);
    std::sort(F.begin(), F.end());
    if (c->old && !compress_needed(c, b, F)) keep[t] = 1;
  });
  }
  std::vector<int> dofs, fint;
  std::vector<ChildSrc> src_all;
  std::vector<int> soff;
  size_t totM = 0, totN2 = 0, totArena = 0, totScr = 0;
  for (int t = 0; t < nids; ++t) {
    const int b = ids[t];
    const Box& B = c->boxes[b];
    BoxFac& f = c->fac[b];
    f.level = l;
    f.I = std::move(Is[t]);
    f.n = (int)f.I.size();
    f.active = f.n > 0;
    if (f.n == 0) {
      f.k = 0;
      f.perm.clear();
      continue;
    }
    const std::vector<int>& F = Fs[t];
    if (keep[t]) {
      // every input of this box's compression is unchanged: keep its factors
      const OldState& O = *c->old;
      const BoxFac& of = O.fac[O.by_key.at(BoxKey{B.level, B.ix, B.iy})];
      f = of;
      c->recomputed[b] = 0;
      continue;
    }
    c->recomputed[b] = 1;
    f.fint = F;
    LevelBox x{};
    x.cx = B.cx;
    x.cy = B.cy;
    x.side = B.side;
    x.wscale = 0.0;
    for (int d : f.I) x.wscale = std::max(x.wscale, c->w[d >> 1]);
    x.n = f.n;
    x.nF = (int)F.size();
    // near field both ways, 2 rows per proxy point in each proxy block (three
    // blocks for Stokes, two for the Laplace kernel), the two rank-one rows
    x.m = 2 * x.nF + (prm.kernel == 1 ? 4 : 6) * prm.n_proxy + 2;
    x.geo = g;
    P.doff.push_back((int)dofs.size());
    soff.push_back(B.leaf() ? -1 : (int)src_all.size());
    x.fint = reinterpret_cast<const int*>((uintptr_t)fint.size());   // offsets for now
    dofs.insert(dofs.end(), f.I.begin(), f.I.end());
    fint.insert(fint.end(), F.begin(), F.end());
    if (!B.leaf()) src_all.insert(src_all.end(), srcs[t].begin(), srcs[t].end());
    totM += (size_t)x.m * x.n;
    const size_t n2 = (size_t)x.n * x.n;
    totN2 += n2;
    totScr += 3 * n2 + 128 * (size_t)x.n + 2048;
    totArena += 3 * (n2 / 4 + x.n) + 2 * n2;
    if (prm.precision >= 1) totArena += (3 * (n2 / 4 + x.n) + n2 + 1) / 2 + 4;
    P.max_m = std::max(P.max_m, x.m);
    P.max_n = std::max(P.max_n, x.n);
    P.lb.push_back(x);
    P.sel.push_back((int)t);
  }
  const int nb = (int)P.lb.size();
  if (nb == 0) return;
  // workspaces and the factor arena of this level
  HTimer ht4_(c, "host:prep.alloc");
  c->ws_M.ensure(totM * sizeof(double));
  c->ws_R.ensure(totN2 * sizeof(double));
  c->ws_A.ensure(totN2 * sizeof(double));
  c->ws_scr.ensure(totScr * sizeof(double));
  size_t totCoop = 0;
  for (const LevelBox& x : P.lb) totCoop += 8 + 2 + 3 * (size_t)kMaxCoop + (size_t)x.m;
  c->ws_coop.ensure(totCoop * sizeof(double));
  P.aid = c->next_arena++;
  c->arenas[P.aid] = take_arena(c, totArena * sizeof(double));
  DevBuf* arena = c->arenas[P.aid].get();
  c->ws_perm.ensure(std::max<size_t>(dofs.size(), 4) * sizeof(int));
  double* pM = c->ws_M.as<double>();
  double* pR = c->ws_R.as<double>();
  double* pA = c->ws_A.as<double>();
  double* pS = c->ws_scr.as<double>();
  double* pa = arena->as<double>();
  double* pc = c->ws_coop.as<double>();
  for (int i = 0; i < nb; ++i) {
    LevelBox& x = P.lb[i];
    const size_t n2 = (size_t)x.n * x.n;
    const size_t kr = n2 / 4 + x.n;
    // dofs, fint and src hold offsets into P's lists (src: offset + 1, 0 for a
    // leaf) until the level plan places the lists in the launch's input buffer
    x.dofs = reinterpret_cast<const int*>((uintptr_t)P.doff[i]);
    x.src = reinterpret_cast<const ChildSrc*>((uintptr_t)(soff[i] + 1));
    x.perm = c->ws_perm.as<int>() + P.doff[i];
    x.M = pM;
    pM += (size_t)x.m * x.n;
    x.R = pR;
    pR += n2;
    x.Ap = pA;
    pA += n2;
    x.scr = pS;
    pS += 3 * n2 + 128 * (size_t)x.n + 2048;
    x.T = pa;
    pa += kr;
    x.E = pa;
    pa += kr;
    x.F = pa;
    pa += kr;
    x.Xinv = pa;
    pa += n2;
    x.Xss = pa;
    pa += n2;
    if (prm.precision >= 1) {
      float* pf = reinterpret_cast<float*>(pa);
      x.Tf = pf;
      pf += kr;
      x.Ef = pf;
      pf += kr;
      x.Ff = pf;
      pf += kr;
      x.Xinvf = pf;
      pa += (3 * kr + n2 + 1) / 2 + 4;
    }
    x.bar = reinterpret_cast<unsigned*>(pc);
    pc += 8;
    x.hh = pc;
    pc += 2;
    x.cval = pc;
    pc += 2 * (size_t)kMaxCoop;
    x.cphys = reinterpret_cast<int*>(pc);
    pc += kMaxCoop;
    x.vbuf = pc;
    pc += x.m;
    BoxFac& f = c->fac[ids[P.sel[i]]];
    f.T = x.T;
    f.E = x.E;
    f.F = x.F;
    f.Xinv = x.Xinv;
    f.Xss = x.Xss;
    f.Tf = x.Tf;
    f.Ef = x.Ef;
    f.Ff = x.Ff;
    f.Xinvf = x.Xinvf;
  }
  P.dofs = std::move(dofs);
  P.fint = std::move(fint);
  P.src = std::move(src_all);
}

// Ranks and pivot orders read back for one context: fill its box records.
void finish_level(rs_ctx* c, LevelPrep& P, const int* k0, const int* kk, const int* st, const double* rc,
                  std::vector<int>& boxes_done) {
  HTimer ht_(c, "host:finish");
  for (size_t i = 0; i < P.lb.size(); ++i) {
    const int b = P.ids[P.sel[i]];
    BoxFac& f = c->fac[b];
    const LevelBox& x = P.lb[i];
    f.perm.assign(P.perm.begin() + P.doff[i], P.perm.begin() + P.doff[i] + x.n);
    f.k = kk[i];
    f.rank0 = k0[i];
    f.rcond = rc[i];
    f.arena = P.aid;
    if (st[i] != 0)
      throw RsError{RS_ERR_SINGULAR, "X_RR stayed singular after the pivot guard (box " +
                                         std::to_string(b) + ")"};
    c->stats.guard_bumps += f.k - f.rank0;
    // algorithmic flop counts.  ID: the pivoted QR of the m x n matrix M_B
    // stopped after k steps plus T = R11^{-1} R12, 4mnk - 2(m+n)k^2 +
    // (4/3)k^3 + k^2 r, whatever route computed it (the row reduction and
    // the head-room steps for the guard are not counted)
    const double m = x.m, n = x.n, k = f.k, r = n - k;
    const double fid = 4.0 * m * n * k - 2.0 * (m + n) * k * k + (4.0 / 3.0) * k * k * k + k * k * r;
    c->stats.flops_id += std::max(fid, 0.0);
    c->stats.flops_elim += k * k * r + 4 * k * k * r + 4 * k * r * r + 2 * r * r * r +
                           4 * k * r * r + 2 * k * k * r;
    c->stats.max_box_unknowns = std::max(c->stats.max_box_unknowns, x.n);
    c->stats.max_rank = std::max(c->stats.max_rank, f.k);
    boxes_done.push_back(b);
  }
}

// Pivoted-QR route of an m x n ID matrix (depends on m and n only):
//   1  the 16-lane kernel on M_B itself (m <= 256, n <= 128);
//   2  row reduction by 256-row blocks, then the 16-lane kernel on the stack
//      of factors (n <= 128): h = rows per first-round block, P[r] = factors
//      left after round r;
//   0  otherwise (the 64-lane register kernel or the memory-resident one).
int qr_route(int m, int n, int& h, std::vector<int>& P) {
  auto fits16 = [](int rows, int cols) { return rows <= 16 * kR16MaxRU && cols <= kR16MaxN; };
  P.clear();
  if (n == 0 || n > kR16MaxN) return 0;
  if (fits16(m, n)) return 1;
  h = 16 * kR16MaxRU;
  const int s = h / n;
  P.push_back((m + h - 1) / h);
  while (!fits16(P.back() * n, n)) P.push_back((P.back() + s - 1) / s);
  return 2;
}

// One launch per kernel over the boxes of all contexts at this level (the
// lead context provides the stream, the descriptor array and the rank arrays).
// Host work run while the level's elimination is on the device: called with
// the pivoted QR's ranks (indexed by box slot) once they and the pivot orders
// (in each LevelPrep::perm) have arrived.
// Wait for an event by polling it.  Used where the host's own work is the
// critical path (the speculative preparation of the next level starts when
// the QR ranks arrive), so that a blocking wait's wake-up latency is not added.
void poll_event(hipEvent_t ev) {
  for (;;) {
    const hipError_t e = hipEventQuery(ev);
    if (e == hipSuccess) return;
    if (e != hipErrorNotReady) HIP_CHECK(e);
  }
}

using LevelOverlap = std::function<void(const int* qr_rank)>;


// The context's second stream, made to wait for everything enqueued so far on
// its main stream (ev_fork); join_side makes the main stream wait for it.
hipStream_t fork_side(rs_ctx* c) {
  if (!c->side_stream) HIP_CHECK(hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking));
  if (!c->ev_fork) HIP_CHECK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  if (!c->ev_join) HIP_CHECK(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
  HIP_CHECK(hipEventRecord(c->ev_fork, c->stream));
  HIP_CHECK(hipStreamWaitEvent(c->side_stream, c->ev_fork, 0));
  return c->side_stream;
}
void join_side(rs_ctx* c) {
  HIP_CHECK(hipEventRecord(c->ev_join, c->side_stream));
  HIP_CHECK(hipStreamWaitEvent(c->stream, c->ev_join, 0));
}

// Autotuner of the cooperative launch shapes (a11): the workgroups per box of
// the memory-resident pivoted QR (G) and of the elimination (Ge).  Neither
// changes any result (every reduction is done by one fixed workgroup in a fixed
// order), so the choice only affects speed.  For a launch signature (kernel,
// boxes, largest n and m rounded up) the candidates are the heuristic value,
// half and double it (within the co-resident capacity); successive
// factorizations in the process try them in turn, each timed with events
// around its launch, and every later launch of that signature takes the
// fastest.
struct ShapeTune {
  std::vector<int> cand;
  std::vector<double> ms;     // < 0: not tried yet
  int best = -1;
  int next() const {
    for (size_t i = 0; i < ms.size(); ++i)
      if (ms[i] < 0) return (int)i;
    return -1;
  }
};
struct ShapeTuneCache {
  std::mutex mu;
  std::map<std::tuple<int, int, int, int>, ShapeTune> t;
};
ShapeTuneCache& shape_tune_cache() {
  static ShapeTuneCache cache;
  return cache;
}

// The value to launch with for a signature (and, when it is a trial, the
// entry and candidate index to report the time to).
int tuned_shape(int kind, int nbox, int n, int m, int g0, int cap, ShapeTune** entry, int* idx) {
  *entry = nullptr;
  *idx = -1;
  if (g0 < 2) return g0;
  ShapeTuneCache& tc = shape_tune_cache();
  std::lock_guard<std::mutex> lk(tc.mu);
  ShapeTune& e = tc.t[std::make_tuple(kind, nbox, (n + 31) / 32, (m + 255) / 256)];
  if (e.cand.empty()) {
    for (int g : {g0, g0 / 2, 2 * g0}) {
      g = std::min(std::max(g, 2), cap);
      if (std::find(e.cand.begin(), e.cand.end(), g) == e.cand.end()) e.cand.push_back(g);
    }
    e.ms.assign(e.cand.size(), -1.0);
  }
  const int i = e.next();
  if (i < 0) return e.cand[e.best];
  *entry = &e;
  *idx = i;
  return e.cand[i];
}

void report_shape(ShapeTune* e, int idx, double ms) {
  if (!e || idx < 0) return;
  ShapeTuneCache& tc = shape_tune_cache();
  std::lock_guard<std::mutex> lk(tc.mu);
  e->ms[idx] = ms;
  if (e->best < 0 || ms < e->ms[e->best]) e->best = idx;
}

struct LevelPlan {
  std::vector<LevelBox> all;
  int nb = 0, max_m = 0, max_n = 0;
  std::vector<QRTask> tasks;
  std::vector<int> round_first;
  std::vector<int4> work16, work;
  std::vector<int> fb;
  std::vector<std::pair<int, int>> coop;   // (first work item, count) of each cooperative launch
  int fb_m = 0, fb_n = 0, G = 1, Ge = 1;
  // launch-shape autotuner: the cache entries (null: not tuned) whose
  // candidate this launch tries, and that candidate's index
  struct ShapeTune* tq = nullptr;
  struct ShapeTune* te = nullptr;
  int tq_i = -1, te_i = -1;
  size_t rq_lds = 0;
  DevBuf* in = nullptr;                    // the launch's input buffer (one per level parity)
  std::vector<char> image;                 // its host image
  const LevelBox* dboxes = nullptr;        // device addresses of the sections
  const QRTask* dtasks = nullptr;
  const int4* dwork = nullptr;
  const int4* dwork16 = nullptr;
  const int* dfb = nullptr;
};

// Host plan of a level launch: descriptors, QR routes and tasks, workgroups per box.
void plan_level(std::vector<rs_ctx*>& cs, std::vector<LevelPrep>& preps, LevelPlan& P) {
  rs_ctx* c = cs[0];
  const rs_params& prm = c->prm;
  std::vector<LevelBox> all;
  int max_m = 0, max_n = 0;
  for (size_t i = 0; i < cs.size(); ++i) {
    preps[i].first = all.size();
    all.insert(all.end(), preps[i].lb.begin(), preps[i].lb.end());
    max_m = std::max(max_m, preps[i].max_m);
    max_n = std::max(max_n, preps[i].max_n);
  }
  const int nb = (int)all.size();
  P.nb = nb;
  if (nb == 0) return;
  std::unique_ptr<HTimer> plan_timer(new HTimer(c, "host:plan"));
  for (int i = 0; i < nb; ++i) all[i].slot = i;
  // Pivoted-QR routes (depend on m and n only): most boxes are reduced by
  // blocks of rows to a stack of triangular factors (which has the same
  // pivots, ranks and R up to row signs) and factored by one workgroup.
  std::vector<QRTask> tasks;
  std::vector<int> round_first{0};
  std::vector<int4> work16;
  std::vector<int> route(nb, 0);
  {
    std::vector<std::vector<int>> plans(nb);
    std::vector<int> hrows(nb, 0);
    size_t tq = 0;
    int rounds = 0;
    for (int i = 0; i < nb; ++i) {
      all[i].Mq = all[i].M;
      all[i].mq = all[i].m;
      route[i] = qr_route(all[i].m, all[i].n, hrows[i], plans[i]);
      if (route[i] == 2) {
        const size_t n2 = (size_t)all[i].n * all[i].n;
        tq += n2 * (plans[i][0] + (plans[i].size() > 1 ? plans[i][1] : 0));
        rounds = std::max(rounds, (int)plans[i].size());
      }
    }
    c->ws_tq.ensure(std::max<size_t>(tq, 1) * sizeof(double));
    std::vector<std::vector<QRTask>> by_round(rounds);
    double* base = c->ws_tq.as<double>();
    for (int i = 0; i < nb; ++i) {
      LevelBox& x = all[i];
      if (route[i] == 2) {
        const std::vector<int>& P = plans[i];
        const int n = x.n, h = hrows[i], s_per = h / n;
        double* buf[2] = {base, base + (size_t)n * n * P[0]};
        base += (size_t)n * n * (P[0] + (P.size() > 1 ? P[1] : 0));
        for (int b = 0; b < P[0]; ++b) {
          const int rows = std::min(h, x.m - b * h);
          // the row class covers the n output rows too (a short last block)
          by_round[0].push_back(QRTask{x.M + (size_t)b * h, buf[0] + (size_t)b * n, x.m, P[0] * n, rows, n,
                                       r16_row_class(std::max(rows, n)), 0});
        }
        for (size_t r = 1; r < P.size(); ++r) {
          const double* in = buf[(r - 1) & 1];
          double* out = buf[r & 1];
          for (int t = 0; t < P[r]; ++t) {
            const int cnt = std::min(s_per, P[r - 1] - t * s_per);
            by_round[r].push_back(QRTask{in + (size_t)t * s_per * n, out + (size_t)t * n, P[r - 1] * n,
                                         P[r] * n, cnt * n, n, r16_row_class(std::max(cnt * n, n)), 0});
          }
        }
        x.Mq = buf[(P.size() - 1) & 1];
        x.mq = P.back() * n;
      }
      if (route[i]) work16.push_back(make_int4(i, 0, 1, r16_row_class(x.mq)));
    }
    for (auto& r : by_round) {
      tasks.insert(tasks.end(), r.begin(), r.end());
      round_first.push_back((int)tasks.size());
    }
    // the per-context records keep the reduced row count (flop accounting)
    for (size_t ci = 0; ci < cs.size(); ++ci)
      for (size_t t = 0; t < preps[ci].lb.size(); ++t) preps[ci].lb[t].mq = all[preps[ci].first + t].mq;
  }
  // Pivoted-QR plan.  Boxes whose (reduced) matrix has at most 2560 rows
  // take the register-resident kernel with the fewest workgroups that hold
  // their columns (G = 1: an ordinary launch; G > 1: cooperative launches of
  // at most the resident capacity); taller ones take the memory-resident
  // kernel.  Neither result depends on G; which kernel a box takes depends on
  // its m and n only.
  std::vector<int4> work;
  std::vector<int> fb;
  std::vector<std::pair<int, int>> coop;      // (first work item, count)
  int fb_m = 0, fb_n = 0, rq_ru = 2, rq_n = 1;
  {
    std::vector<int4> wide;
    for (int i = 0; i < nb; ++i) {
      const LevelBox& x = all[i];
      if (route[i]) continue;
      if (x.mq > 64 * kRQMaxRU) {
        fb.push_back(i);
        fb_m = std::max(fb_m, x.m);
        fb_n = std::max(fb_n, x.n);
        continue;
      }
      const int ru = rq_row_class(x.mq);
      const int per = kRQWaves * rq_cols_per_wave(ru);
      const int G = std::max(1, (x.n + per - 1) / per);
      if (G > kMaxCoop) {
        fb.push_back(i);
        fb_m = std::max(fb_m, x.m);
        fb_n = std::max(fb_n, x.n);
        continue;
      }
      rq_ru = std::max(rq_ru, ru);
      rq_n = std::max(rq_n, x.n);
      if (G == 1) work.push_back(make_int4(i, 0, 1, ru));
      else wide.push_back(make_int4(i, 0, G, ru));
    }
    const size_t lds = cpqr_reg_lds_bytes(rq_ru, rq_n);
    const int cap = cpqr_reg_blocks_per_cu(lds) * c->n_cu;
    int first = (int)work.size(), used = 0;
    for (const int4& w : wide) {
      if (w.z > cap)
        throw RsError{RS_ERR_ARG, "box too large for the pivoted-QR kernel (m=" + std::to_string(all[w.x].m) +
                                      ", n=" + std::to_string(all[w.x].n) + ")"};
      if (used + w.z > cap) {
        coop.push_back({first, used});
        first = (int)work.size();
        used = 0;
      }
      for (int g = 0; g < w.z; ++g) work.push_back(make_int4(w.x, g, w.z, w.w));
      used += w.z;
    }
    if (used) coop.push_back({first, used});
  }
  const size_t rq_lds = cpqr_reg_lds_bytes(rq_ru, rq_n);
  const size_t qr_lds = cpqr_lds_bytes(fb_m, fb_n);
  if (!fb.empty() && qr_lds > 160 * 1024)
    throw RsError{RS_ERR_ARG, "box too large for the pivoted-QR kernel (m=" + std::to_string(fb_m) +
                                  ", n=" + std::to_string(fb_n) + ")"};
  // workgroups per box for the memory-resident QR and the elimination: spread
  // the few large boxes near the root over the device (cooperative launch: all
  // of them co-resident).  Results do not depend on G: every reduction is done
  // by one fixed workgroup.
  int G = 1, Ge = 1;
  const int nfb = (int)fb.size();
  if (nfb && nfb <= c->n_cu / 4) {
    const int capq = cpqr_blocks_per_cu(qr_lds) * c->n_cu;
    if (capq > 0) G = std::min({capq / nfb, std::max(1, fb_n / 16), kMaxCoop});
    if (G < 2) G = 1;
    else G = tuned_shape(0, nfb, fb_n, fb_m, G, std::min(capq / nfb, kMaxCoop), &P.tq, &P.tq_i);
  }
  if (nb <= c->n_cu / 4) {
    const int cape = eliminate_blocks_per_cu(max_n) * c->n_cu;
    if (cape > 0) Ge = std::min({cape / nb, std::max(1, max_n / 8), kMaxCoop});
    if (Ge < 2) Ge = 1;
    else Ge = tuned_shape(1, nb, max_n, max_m, Ge, std::min(cape / nb, kMaxCoop), &P.te, &P.te_i);
  }
  plan_timer.reset();
  P.all = std::move(all);
  P.max_m = max_m;
  P.max_n = max_n;
  P.tasks = std::move(tasks);
  P.round_first = std::move(round_first);
  P.work16 = std::move(work16);
  P.work = std::move(work);
  P.fb = std::move(fb);
  P.coop = std::move(coop);
  P.fb_m = fb_m;
  P.fb_n = fb_n;
  P.rq_lds = rq_lds;
  P.G = G;
  P.Ge = Ge;
  c->desc_flip ^= 1;
  P.in = c->desc_flip ? &c->ws_in_b : &c->ws_in_a;
  // input buffer layout: per context its I_B, F_int and child-source lists,
  // then descriptors, QR tasks, work lists (each section 256-byte aligned)
  size_t off = 0;
  auto place = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) & ~(size_t)255;
    return o;
  };
  std::vector<size_t> o_dofs(cs.size()), o_fint(cs.size()), o_src(cs.size());
  for (size_t i = 0; i < cs.size(); ++i) {
    o_dofs[i] = place(preps[i].dofs.size() * sizeof(int));
    o_fint[i] = place(preps[i].fint.size() * sizeof(int));
    o_src[i] = place(preps[i].src.size() * sizeof(ChildSrc));
  }
  const size_t o_boxes = place(P.all.size() * sizeof(LevelBox));
  const size_t o_tasks = place(P.tasks.size() * sizeof(QRTask));
  const size_t o_work = place(P.work.size() * sizeof(int4));
  const size_t o_work16 = place(P.work16.size() * sizeof(int4));
  const size_t o_fb = place(P.fb.size() * sizeof(int));
  P.in->ensure(std::max<size_t>(off, 256));
  char* base = static_cast<char*>(P.in->p);
  for (size_t i = 0; i < cs.size(); ++i)
    for (size_t t = 0; t < preps[i].lb.size(); ++t) {
      LevelBox& x = P.all[preps[i].first + t];
      x.dofs = reinterpret_cast<const int*>(base + o_dofs[i]) + reinterpret_cast<uintptr_t>(x.dofs);
      x.fint = reinterpret_cast<const int*>(base + o_fint[i]) + reinterpret_cast<uintptr_t>(x.fint);
      const uintptr_t so = reinterpret_cast<uintptr_t>(x.src);
      x.src = so == 0 ? nullptr : reinterpret_cast<const ChildSrc*>(base + o_src[i]) + (so - 1);
    }
  P.image.assign(off, 0);
  auto put = [&](size_t o, const void* src, size_t bytes) {
    if (bytes) std::memcpy(P.image.data() + o, src, bytes);
  };
  for (size_t i = 0; i < cs.size(); ++i) {
    put(o_dofs[i], preps[i].dofs.data(), preps[i].dofs.size() * sizeof(int));
    put(o_fint[i], preps[i].fint.data(), preps[i].fint.size() * sizeof(int));
    put(o_src[i], preps[i].src.data(), preps[i].src.size() * sizeof(ChildSrc));
  }
  put(o_boxes, P.all.data(), P.all.size() * sizeof(LevelBox));
  put(o_tasks, P.tasks.data(), P.tasks.size() * sizeof(QRTask));
  put(o_work, P.work.data(), P.work.size() * sizeof(int4));
  put(o_work16, P.work16.data(), P.work16.size() * sizeof(int4));
  put(o_fb, P.fb.data(), P.fb.size() * sizeof(int));
  P.dboxes = reinterpret_cast<const LevelBox*>(base + o_boxes);
  P.dtasks = reinterpret_cast<const QRTask*>(base + o_tasks);
  P.dwork = reinterpret_cast<const int4*>(base + o_work);
  P.dwork16 = reinterpret_cast<const int4*>(base + o_work16);
  P.dfb = reinterpret_cast<const int*>(base + o_fb);
}

// Matrix assembly and row reduction of a planned level on stream st: they read
// the geometry, the level's index lists and M_B only, so while level l is
// eliminated they can already run for level l - 1 (on the second stream).
void pre_launch(std::vector<rs_ctx*>& cs, LevelPlan& P, hipStream_t st) {
  rs_ctx* c = cs[0];
  const rs_params& prm = c->prm;
  upload(*P.in, P.image, st);
  const LevelBox* dlb = P.dboxes;
  {
    KTimer kt_(c, "assemble_M", false, st);
    launch_assemble_M(dlb, P.nb, P.max_m, prm.n_proxy, prm.proxy_ratio, prm.precision == 2, st);
  }
  if (P.round_first.size() > 1) {
    KTimer kt_(c, "cpqr", false, st);
    for (size_t r = 0; r + 1 < P.round_first.size(); ++r) {
      KTimer kt2_(c, "cpqr.rows", true, st);
      launch_tsqr(P.dtasks + P.round_first[r], P.round_first[r + 1] - P.round_first[r], st);
    }
  }
}

// The rest of a level: pivoted QR, A_BB, elimination and the read-backs.  With
// pre == null the level is planned and pre-launched here first; otherwise the
// main stream waits for the pre-launch on the second stream (ev_pre).
void launch_level(std::vector<rs_ctx*>& cs, std::vector<LevelPrep>& preps, LevelPlan* pre,
                  const LevelOverlap& overlap) {
  rs_ctx* c = cs[0];
  const rs_params& prm = c->prm;
  hipStream_t s = c->stream;
  if (!c->ev_tune[0])
    for (hipEvent_t& e : c->ev_tune) HIP_CHECK(hipEventCreate(&e));
  LevelPlan own;
  if (!pre) {
    plan_level(cs, preps, own);
    if (own.nb == 0) return;
    pre_launch(cs, own, s);
    pre = &own;
  } else {
    HIP_CHECK(hipStreamWaitEvent(s, c->ev_pre, 0));
    if (pre->nb == 0) return;
  }
  LevelPlan& P = *pre;
  const int nb = P.nb, max_n = P.max_n, fb_m = P.fb_m, fb_n = P.fb_n, G = P.G, Ge = P.Ge;
  const size_t rq_lds = P.rq_lds;
  const std::vector<int4>& work = P.work;
  const std::vector<int>& fb = P.fb;
  const std::vector<std::pair<int, int>>& coop = P.coop;
  const int nfb = (int)fb.size();
  c->ws_kx.ensure(nb * sizeof(int));
  const size_t nbp = ((size_t)nb + 1) & ~(size_t)1;   // keeps the rcond block 8-byte aligned
  const size_t out_bytes = (4 + 2 * nbp) * sizeof(int) + (size_t)nb * sizeof(double);
  c->ws_out.ensure(out_bytes);
  int* d_err = c->ws_out.as<int>();
  int* d_k = d_err + 4;
  int* d_status = d_k + nbp;
  double* d_rc = reinterpret_cast<double*>(d_status + nbp);
  const LevelBox* dlb = P.dboxes;
  if ((c->timing == 1 || c->timing == 2) && c->level_done_set) {
    const int fam = family(c, "host:between_levels");
    c->fam_ms[fam] += 1e3 * std::chrono::duration<double>(std::chrono::steady_clock::now() - c->level_done).count();
    c->fam_launches[fam] += 1;
    c->level_done_set = false;
  }
  {
    KTimer kt_(c, "cpqr");
    launch_zero_bars(dlb, nb, d_err, s);
    const int4* dw = P.dwork;
    const int nA = coop.empty() ? (int)work.size() : coop.front().first;
    auto check = [&](hipError_t e, const char* what, int blocks) {
      if (e != hipSuccess)
        throw RsError{RS_ERR_DEVICE, std::string("pivoted-QR launch failed (") + what + ", " +
                                         hipGetErrorString(e) + ", blocks " + std::to_string(blocks) + ")"};
    };
    // The few boxes of the cooperative and memory routes (wide or tall M_B)
    // are factored on a second stream while the row-reduced boxes are: their
    // boxes, rank slots and barrier words are disjoint, so the results do not
    // depend on the overlap.
    const bool side = !coop.empty() || nfb > 0;
    if (side) {
      hipStream_t s2 = fork_side(c);
      for (const auto& ch : coop) {
        KTimer kt2_(c, "cpqr.coop", true, s2);
        check(launch_cpqr_reg(dlb, dw + ch.first, ch.second, true, prm.tol, kGuardExtra, d_k,
                              c->ws_kx.as<int>(), d_err, rq_lds, s2), "register, cooperative",
              ch.second);
      }
      {
        KTimer kt2_(c, "cpqr.mem", true, s2);
        if (P.tq) HIP_CHECK(hipEventRecord(c->ev_tune[0], s2));
        check(launch_cpqr(dlb, P.dfb, nfb, G, prm.tol, kGuardExtra, d_k,
                          c->ws_kx.as<int>(), d_err, fb_m, fb_n, s2), "memory", nfb * G);
        if (P.tq) HIP_CHECK(hipEventRecord(c->ev_tune[1], s2));
      }
    }
    {
      KTimer kt2_(c, "cpqr.r16", true);
      check(launch_cpqr16(dlb, P.dwork16, (int)P.work16.size(), prm.tol, kGuardExtra,
                          d_k, c->ws_kx.as<int>(), d_err, s),
            "16-lane", (int)P.work16.size());
    }
    {
      KTimer kt2_(c, "cpqr.reg", true);
      check(launch_cpqr_reg(dlb, dw, nA, false, prm.tol, kGuardExtra, d_k, c->ws_kx.as<int>(),
                            d_err, rq_lds, s), "register", nA);
    }
    if (side) join_side(c);
  }
  {
    KTimer kt_(c, "assemble_abb");
    launch_assemble_abb(dlb, nb, max_n, prm.lambda, true, prm.precision == 2, s);
  }
  // read-backs into pinned memory stay asynchronous: one wait per level
  int* k0 = c->h_rank.get<int>(nb);
  HIP_CHECK(hipMemcpyAsync(k0, d_k, nb * sizeof(int), hipMemcpyDeviceToHost, s));
  // pivot orders are final after the QR (the elimination's guard only moves k)
  std::vector<int*> hperm(cs.size(), nullptr);
  for (size_t i = 0; i < cs.size(); ++i) {
    LevelPrep& P = preps[i];
    if (P.lb.empty()) continue;
    const size_t np = P.doff.back() + P.lb.back().n;
    hperm[i] = cs[i]->h_perm.get<int>(np);
    HIP_CHECK(hipMemcpyAsync(hperm[i], cs[i]->ws_perm.p, np * sizeof(int), hipMemcpyDeviceToHost, s));
  }
  if (!c->ev_qr) HIP_CHECK(hipEventCreateWithFlags(&c->ev_qr, hipEventDisableTiming));
  HIP_CHECK(hipEventRecord(c->ev_qr, s));
  {
    KTimer kt_(c, "eliminate");
    if (P.te) HIP_CHECK(hipEventRecord(c->ev_tune[2], s));
    HIP_CHECK(launch_eliminate(dlb, nb, Ge, d_k, c->ws_kx.as<int>(), prm.rcond_min,
                               d_status, d_rc, d_err + 1,
                               max_n, prm.precision == 2, prm.mixed_rcond_min, s));
    if (P.te) HIP_CHECK(hipEventRecord(c->ev_tune[3], s));
    if (prm.precision >= 1) launch_factor_to_float(dlb, nb, d_k, s);
  }
  HIP_CHECK(hipGetLastError());
  int* qr_err = reinterpret_cast<int*>(c->h_rc.get<double>(out_bytes / sizeof(double)));
  HIP_CHECK(hipMemcpyAsync(qr_err, c->ws_out.p, out_bytes, hipMemcpyDeviceToHost, s));
  int* kk = qr_err + 4;
  int* st = kk + nbp;
  double* hrc = reinterpret_cast<double*>(st + nbp);
  if (overlap) {
    {
      HTimer ht_(c, "host:level_wait");
      HTimer ht2_(c, "host:qr_wait");
      poll_event(c->ev_qr);
    }
    for (size_t i = 0; i < cs.size(); ++i)
      if (hperm[i]) preps[i].perm.assign(hperm[i], hperm[i] + preps[i].doff.back() + preps[i].lb.back().n);
    HTimer ht_(c, "host:speculate");
    overlap(k0);
  }
  {
    HTimer ht_(c, "host:level_wait");
    HTimer ht2_(c, overlap ? "host:elim_wait" : "host:last_wait");
    HIP_CHECK(hipStreamSynchronize(s));
  }
  for (size_t i = 0; i < cs.size(); ++i)
    if (hperm[i]) preps[i].perm.assign(hperm[i], hperm[i] + preps[i].doff.back() + preps[i].lb.back().n);
  resolve_timers(c);
  // launch-shape trials (both streams are complete here)
  for (int t = 0; t < 2; ++t) {
    ShapeTune* e = t == 0 ? P.tq : P.te;
    if (!e) continue;
    ++c->stats.shape_trials;
    float ms = 0.f;
    HIP_CHECK(hipEventSynchronize(c->ev_tune[2 * t + 1]));
    HIP_CHECK(hipEventElapsedTime(&ms, c->ev_tune[2 * t], c->ev_tune[2 * t + 1]));
    report_shape(e, t == 0 ? P.tq_i : P.te_i, ms);
  }
  if (qr_err[2]) throw RsError{RS_ERR_ARG, "non-finite entries in an ID matrix (coincident nodes?)"};
  if (qr_err[0] || qr_err[1]) throw RsError{RS_ERR_DEVICE, "box barrier timed out"};
  for (size_t i = 0; i < cs.size(); ++i) {
    LevelPrep& P = preps[i];
    if (P.lb.empty()) continue;
    std::vector<int> done;
    finish_level(cs[i], P, k0 + P.first, kk + P.first, st + P.first, hrc + P.first, done);
  }
  if (c->timing) {
    c->level_done = std::chrono::steady_clock::now();
    c->level_done_set = true;
  }
}

void build_solve_meta(rs_ctx* c) {
  HTimer ht_(c, "host:solve_meta");
  const int L = c->L;
  c->sboxes.assign(L + 1, {});
  c->lvl_maxn.assign(L + 1, 0);
  c->lvl_maxr.assign(L + 1, 0);
  std::vector<int> sidx, ridx;
  int part = 0;
  c->all_maxr = 0;
  c->stats.factor_bytes = 0;
  for (size_t b = 1; b < c->boxes.size(); ++b) {
    const BoxFac& f = c->fac[b];
    if (!f.active) continue;
    SolveBox sb{};
    sb.k = f.k;
    sb.r = f.n - f.k;
    sb.s_off = (int)sidx.size();
    sb.r_off = (int)ridx.size();
    sb.part = part++;
    sb.T = f.T;
    sb.E = f.E;
    sb.F = f.F;
    sb.Xinv = f.Xinv;
    sb.W = nullptr;
    // mixed precision: the float copies serve the solve only where X_RR is
    // well conditioned; elsewhere the box's float64 factors are read
    const bool use_f = c->prm.precision >= 1 && f.rcond >= c->prm.mixed_rcond_min && f.Tf;
    sb.Tf = use_f ? f.Tf : nullptr;
    sb.Ef = use_f ? f.Ef : nullptr;
    sb.Ff = use_f ? f.Ff : nullptr;
    sb.Xinvf = use_f ? f.Xinvf : nullptr;
    sb.Wf = nullptr;
    for (int i = 0; i < f.k; ++i) sidx.push_back(f.I[f.perm[i]]);
    for (int i = f.k; i < f.n; ++i) ridx.push_back(f.I[f.perm[i]]);
    c->sboxes[f.level].push_back(sb);
    c->lvl_maxn[f.level] = std::max(c->lvl_maxn[f.level], f.n);
    c->lvl_maxr[f.level] = std::max(c->lvl_maxr[f.level], sb.r);
    c->all_maxr = std::max(c->all_maxr, sb.r);
    c->stats.factor_bytes += (long long)(3LL * sb.k * sb.r + 1LL * sb.r * sb.r) * 8;
  }
  c->n_solve_boxes = part;
  c->n_ridx = (int)ridx.size();
  // border W slots
  const int p3 = 3 * c->p;
  if (p3) {
    size_t totW = 0;
    for (auto& lv : c->sboxes)
      for (auto& sb : lv) totW += (size_t)sb.r * p3;
    c->d_W.ensure(std::max<size_t>(totW, 1) * sizeof(double));
    double* pw = c->d_W.as<double>();
    float* pwf = nullptr;
    if (c->prm.precision >= 1) {
      c->d_Wf.ensure(std::max<size_t>(totW, 1) * sizeof(float));
      pwf = c->d_Wf.as<float>();
    }
    for (auto& lv : c->sboxes)
      for (auto& sb : lv) {
        // the W blocks follow the order of the concatenated R lists (the
        // gathered product for G relies on it)
        if (pw != c->d_W.as<double>() + (size_t)sb.r_off * p3)
          throw RsError{RS_ERR_DEVICE, "border W blocks out of the R-list order"};
        sb.W = pw;
        pw += (size_t)sb.r * p3;
        if (pwf) {
          if (sb.Tf) sb.Wf = pwf;
          pwf += (size_t)sb.r * p3;
        }
      }
  }
  // Every solve kernel reads a box's float factors together (T, E, F in the
  // sweeps; X_RR^-1 in the diagonal step; W in the border fix) once Tf is set,
  // and its float64 factors otherwise: the float pointers must be all set or
  // all null, and W's float copy must exist exactly for the float boxes.
  for (auto& lv : c->sboxes)
    for (auto& sb : lv) {
      const bool f = sb.Tf != nullptr;
      const bool wf_ok = !p3 || (sb.Wf != nullptr) == (f && c->prm.precision >= 1);
      if ((sb.Ef != nullptr) != f || (sb.Ff != nullptr) != f || (sb.Xinvf != nullptr) != f || !wf_ok ||
          (sb.r > 0 && !sb.Xinv) || (p3 && !sb.W))
        throw RsError{RS_ERR_DEVICE, "inconsistent factor pointers in the solve metadata"};
    }
  std::vector<SolveBox> flat;
  c->sbox_off.assign(L + 2, 0);
  for (int l = 0; l <= L; ++l) {
    c->sbox_off[l] = flat.size();
    flat.insert(flat.end(), c->sboxes[l].begin(), c->sboxes[l].end());
  }
  c->sbox_off[L + 1] = flat.size();
  upload(c->d_sboxes, flat, c->stream);
  upload(c->d_sidx, sidx, c->stream);
  upload(c->d_ridx, ridx, c->stream);
}

const SolveBox* level_sboxes(const rs_ctx* c, int l) {
  return c->d_sboxes.as<SolveBox>() + c->sbox_off[l];
}
int level_count(const rs_ctx* c, int l) { return (int)(c->sbox_off[l + 1] - c->sbox_off[l]); }

template <typename T>
void sweep_all(rs_ctx* c, T* buf, int ncols, int mode, hipStream_t on = nullptr) {
  const int L = c->L;
  hipStream_t st = on ? on : c->stream;
  KTimer kt_(c, mode == 0 ? "sweep_U" : (mode == 1 ? "sweep_PsiV" : "sweep_V"), false, st);
  if (mode == 2) {
    for (int l = 1; l <= L; ++l)
      launch_sweep(level_sboxes(c, l), level_count(c, l), c->d_sidx.as<int>(), c->d_ridx.as<int>(),
                   buf, ncols, mode, c->lvl_maxn[l], st);
  } else {
    for (int l = L; l >= 1; --l)
      launch_sweep(level_sboxes(c, l), level_count(c, l), c->d_sidx.as<int>(), c->d_ridx.as<int>(),
                   buf, ncols, mode, c->lvl_maxn[l], st);
  }
}

void ensure_solve_buffers(rs_ctx* c, int ncols);
void refine_graph_capture(rs_ctx* c, int nrhs);

// The root (Section 3.2's bordered system when there are holes) in two parts:
// factor_root_launch enqueues everything and leaves the inverse running on the
// context's side stream; factor_root_finish joins it and checks its status.
// A batch launches every context's root before it waits for any, so the
// root inverses (single-workgroup chains of pivot steps) run side by side.
void factor_root_launch(rs_ctx* c) {
  HTimer ht_(c, "host:root");
  hipStream_t s = c->stream;
  Geo g;
  geo_of(c, g);
  const int p3 = 3 * c->p;
  if (p3) {
    // the border columns H and rows Psi^T depend on the geometry only: they
    // are assembled first, while the host builds the root and solve metadata
    const size_t hn = (size_t)2 * c->N * p3;
    c->d_H.ensure(hn * sizeof(double));
    c->d_Hh.ensure(hn * sizeof(double));
    c->d_Ph.ensure(hn * sizeof(double));
    KTimer kt_(c, "border_H");
    launch_assemble_H(g, c->d_hole.as<double>(), c->p, c->d_curve.as<int>(), c->d_Hh.as<double>(),
                      c->d_Ph.as<double>(), s);
  }
  std::vector<ChildSrc> src;
  box_unknowns(c, 0, c->I0, &src);
  const int n0 = (int)c->I0.size();
  c->nz = n0 + p3;
  upload(c->d_I0, c->I0, s);
  c->d_X0.ensure(std::max<size_t>((size_t)n0 * n0, 1) * sizeof(double));
  if (n0 > 0) {
    LevelBox rb{};
    rb.n = n0;
    rb.geo = g;
    rb.dofs = c->d_I0.as<int>();
    rb.Ap = c->d_X0.as<double>();
    upload(c->ws_src, src, s);
    rb.src = c->boxes[0].leaf() ? nullptr : c->ws_src.as<ChildSrc>();
    std::vector<LevelBox> v{rb};
    upload(c->d_root_box, v, s);
    {
      KTimer kt_(c, "root_abb");
      launch_assemble_abb(c->d_root_box.as<LevelBox>(), 1, n0, c->prm.lambda, false, false, s);
    }
  }
  build_solve_meta(c);
  const int nz = c->nz;
  c->d_Zinv.ensure(std::max<size_t>((size_t)nz * nz, 1) * sizeof(double));
  c->d_gjwork.ensure(((size_t)3 * nz * 32 + 32 * 32) * sizeof(double));
  c->d_gjiwork.ensure(((size_t)nz + 32) * sizeof(int));
  c->d_rcond.ensure(sizeof(double));
  c->d_rstatus.ensure(sizeof(int));
  const double* Zsrc = c->d_X0.as<double>();
  if (p3) {
    // the Psi^T V rows are swept on the second stream beside the U sweep of
    // the border columns and the W blocks (which read only the latter)
    hipStream_t s2 = fork_side(c);
    sweep_all(c, c->d_Ph.as<double>(), p3, 1, s2);
    sweep_all(c, c->d_Hh.as<double>(), p3, 0);
    // W_B of every box, then G = sum_B (Psi^T V)_R W_B as one gathered product
    // W_B of each box is independent of the others: one launch per level,
    // its grid sized by the level's largest r
    {
      KTimer kt_(c, "border_box");
      for (int l = c->L; l >= 1; --l)
        launch_border_w(level_sboxes(c, l), level_count(c, l), c->d_ridx.as<int>(), c->d_Hh.as<double>(), p3,
                        c->lvl_maxr[l], s);
      join_side(c);   // Psi^T V rows
      const int nch = border_g_chunks(c->n_ridx, p3);
      const size_t gparts = (size_t)nch * p3 * p3;
      c->d_Gpart.ensure((gparts + sum_parts_scratch_doubles(nch, p3 * p3)) * sizeof(double));
      launch_border_g(c->d_ridx.as<int>(), c->n_ridx, c->d_Ph.as<double>(), c->d_W.as<double>(), p3, nch,
                      c->d_Gpart.as<double>(), s);
      c->d_G.ensure((size_t)p3 * p3 * sizeof(double));
      launch_sum_parts(c->d_Gpart.as<double>(), nch, (long long)p3 * p3, p3 * p3, 1.0, c->d_G.as<double>(),
                       c->d_Gpart.as<double>() + gparts, s);
    }
    if (c->prm.precision >= 1) {
      const int all_nb = c->L >= 1 ? (int)(c->sbox_off[c->L + 1] - c->sbox_off[1]) : 0;
      launch_w_to_float(level_sboxes(c, 1), all_nb, p3, s);
    }
    c->d_Z.ensure((size_t)nz * nz * sizeof(double));
    {
      KTimer kt_(c, "root_Z");
      launch_assemble_Z(c->d_X0.as<double>(), n0, c->d_Hh.as<double>(), c->d_Ph.as<double>(),
                        c->d_I0.as<int>(), p3, c->d_G.as<double>(), c->d_Z.as<double>(), s);
    }
    Zsrc = c->d_Z.as<double>();
  }
  c->root_pending = false;
  if (nz > 0) {
    hipStream_t s2 = fork_side(c);
    {
      KTimer kt_(c, "root_inverse", false, s2);
      launch_gj_blocked(const_cast<double*>(Zsrc), nz, c->d_Zinv.as<double>(), c->d_gjwork.as<double>(),
                        c->d_gjiwork.as<int>(), c->d_rstatus.as<int>(), s2);
    }
    HIP_CHECK(hipGetLastError());
    c->root_pending = true;
    // While the root inverse runs, the refinement graph for the last solve's
    // number of right-hand sides is captured anew (capture records launches
    // only; the factors' buffers and the solve metadata are final here).  A
    // solve with another count captures its own graph as before.
    if (c->refine_exec && c->refine_nrhs > 0) {
      ensure_solve_buffers(c, c->refine_nrhs);
      refine_graph_capture(c, c->refine_nrhs);
    }
  }
  c->stats.root_skeleton = n0;
}

void factor_root_finish(rs_ctx* c) {
  if (!c->root_pending) return;
  HTimer ht_(c, "host:root_wait");
  c->root_pending = false;
  join_side(c);
  int st = 0;
  HIP_CHECK(hipMemcpyAsync(&st, c->d_rstatus.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_CHECK(hipStreamSynchronize(c->stream));
  resolve_timers(c);
  if (st) throw RsError{RS_ERR_SINGULAR, "root system is singular"};
}

// Return factor arenas no box refers to any more to the pool.
void collect_arenas(rs_ctx* c) {
  std::vector<char> used(c->next_arena, 0);
  for (const BoxFac& f : c->fac)
    if (f.active && f.arena >= 0) used[f.arena] = 1;
  for (auto it = c->arenas.begin(); it != c->arenas.end();) {
    if (!used[it->first]) {
      c->arena_pool.push_back(std::move(it->second));
      it = c->arenas.erase(it);
    } else {
      ++it;
    }
  }
}

void release_all_arenas(rs_ctx* c) {
  for (auto& a : c->arenas) c->arena_pool.push_back(std::move(a.second));
  c->arenas.clear();
}

// The large level workspaces (ID matrices, R, A_BB, elimination scratch,
// cooperation records: about 17 KB per unknown at the leaf level) are needed
// only while a factorization runs.  They come from a per-device pool for the
// duration of one factorization call and go back to it afterwards, so
// factorizations that run one after another (single contexts, or batches
// factored in parts) share one set per context of the largest call instead of
// one per context.  The pool is never destroyed: its memory stays with the
// process (no device frees run at exit).
struct WorkSet {
  DevBuf M, R, A, scr, coop;
};
struct WorkPool {
  std::mutex mu;
  std::map<int, std::vector<std::unique_ptr<WorkSet>>> free;
};
WorkPool& work_pool() {
  static WorkPool* pool = new WorkPool;
  return *pool;
}
void swap_buf(DevBuf& a, DevBuf& b) {
  std::swap(a.p, b.p);
  std::swap(a.bytes, b.bytes);
}
void swap_work(rs_ctx* c, WorkSet& w) {
  swap_buf(c->ws_M, w.M);
  swap_buf(c->ws_R, w.R);
  swap_buf(c->ws_A, w.A);
  swap_buf(c->ws_scr, w.scr);
  swap_buf(c->ws_coop, w.coop);
}
struct WorkLease {
  std::vector<rs_ctx*> cs;
  std::vector<std::unique_ptr<WorkSet>> sets;
  explicit WorkLease(const std::vector<rs_ctx*>& v) : cs(v) {
    WorkPool& wp = work_pool();
    std::lock_guard<std::mutex> lk(wp.mu);
    for (rs_ctx* c : cs) {
      auto& fl = wp.free[c->device];
      std::unique_ptr<WorkSet> w;
      if (!fl.empty()) {
        w = std::move(fl.back());
        fl.pop_back();
      } else {
        w = std::make_unique<WorkSet>();
      }
      swap_work(c, *w);
      sets.push_back(std::move(w));
    }
  }
  ~WorkLease() {
    // the buffers go back only once the work that used them is done
    for (rs_ctx* c : cs) (void)hipStreamSynchronize(c->stream);
    for (rs_ctx* c : cs)
      if (c->side_stream) (void)hipStreamSynchronize(c->side_stream);
    WorkPool& wp = work_pool();
    std::lock_guard<std::mutex> lk(wp.mu);
    for (size_t i = 0; i < cs.size(); ++i) {
      swap_work(cs[i], *sets[i]);
      wp.free[cs[i]->device].push_back(std::move(sets[i]));
    }
  }
};

// Factor several contexts level-synchronously: every level is one launch per
// kernel over the boxes of all contexts (a single context is the plain case).
void do_factor_multi(std::vector<rs_ctx*>& cs) {
  WorkLease lease(cs);
  auto t0 = std::chrono::steady_clock::now();
  const size_t nc = cs.size();
  for (rs_ctx* c : cs) c->level_done_set = false;
  int L = 0;
  std::vector<std::vector<char>> active(nc);
  std::vector<std::vector<std::vector<int>>> by_level(nc);
  for (size_t i = 0; i < nc; ++i) {
    rs_ctx* c = cs[i];
    if (!c->old) release_all_arenas(c);
    c->fac.assign(c->boxes.size(), BoxFac());
    c->recomputed.assign(c->boxes.size(), 1);
    c->stats.guard_bumps = 0;
    c->stats.shape_trials = 0;
    c->stats.flops_id = 0;
    c->stats.flops_elim = 0;
    c->stats.max_box_unknowns = 0;
    c->stats.max_rank = 0;
    active[i].assign(2 * (size_t)c->N, 1);
    by_level[i].assign(c->L + 1, {});
    for (size_t b = 0; b < c->boxes.size(); ++b) by_level[i][c->boxes[b].level].push_back((int)b);
    L = std::max(L, c->L);
  }
  // the redundant unknowns of every box of level l (recompressed or kept) leave the active set
  auto drop_redundant = [&](int l, std::vector<std::vector<char>>& act) {
    for (size_t i = 0; i < nc; ++i) {
      if (cs[i]->L < l) continue;
      for (int b : by_level[i][l]) {
        const BoxFac& f = cs[i]->fac[b];
        if (!f.active) continue;
        for (int t = f.k; t < f.n; ++t) act[i][f.I[f.perm[t]]] = 0;
      }
    }
  };
  // While level l's elimination runs, level l - 1 is prepared on the host
  // with the ranks of level l's QR.  The elimination's guard can still raise a
  // rank (rarely); then that preparation is discarded and done again.
  // The speculative preparation also plans level l - 1 and enqueues its matrix
  // assembly and row reduction on the second stream (they read no output of
  // level l's elimination); a discarded pre-launch is waited for before its
  // buffers are written again.
  std::vector<LevelPrep> preps(nc), next(nc);
  LevelPlan next_plan;
  bool have_next = false, pre_pending = false;
  rs_ctx* c0 = cs[0];
  for (int l = L; l >= 1; --l) {
    c0->cur_level = l;
    LevelPlan cur_plan;
    LevelPlan* planned = nullptr;
    if (have_next) {
      preps.swap(next);
      std::swap(cur_plan, next_plan);
      planned = &cur_plan;
    } else {
      if (pre_pending) HIP_CHECK(hipStreamWaitEvent(c0->stream, c0->ev_pre, 0));
      preps.assign(nc, LevelPrep());
      // the contexts of a batch are independent here: one host thread each
      HostPool::instance().run_tasks((int)nc, [&](int i) {
        if (cs[i]->L >= l) prepare_level(cs[i], l, by_level[i][l], active[i], preps[i]);
      });
    }
    have_next = false;
    pre_pending = false;
    bool speculated = false;
    std::vector<std::vector<int>> spec_k(nc);
    LevelOverlap overlap;
    if (l > 1) {
      overlap = [&](const int* qr_rank) {
        for (size_t i = 0; i < nc; ++i) {
          const LevelPrep& P = preps[i];
          for (size_t t = 0; t < P.lb.size(); ++t) {
            BoxFac& f = cs[i]->fac[P.ids[P.sel[t]]];
            f.k = qr_rank[P.first + t];
            f.perm.assign(P.perm.begin() + P.doff[t], P.perm.begin() + P.doff[t] + P.lb[t].n);
            spec_k[i].push_back(f.k);
          }
        }
        std::vector<std::vector<char>> act(active);
        drop_redundant(l, act);
        // the second stream starts after level l's QR and A_BB (ev_qr): the
        // index lists of level l are no longer read
        if (!c0->side_stream) HIP_CHECK(hipStreamCreateWithFlags(&c0->side_stream, hipStreamNonBlocking));
        if (!c0->ev_pre) HIP_CHECK(hipEventCreateWithFlags(&c0->ev_pre, hipEventDisableTiming));
        hipStream_t s2 = c0->side_stream;
        HIP_CHECK(hipStreamWaitEvent(s2, c0->ev_qr, 0));
        next.assign(nc, LevelPrep());
        HostPool::instance().run_tasks((int)nc, [&](int i) {
          if (cs[i]->L >= l - 1) prepare_level(cs[i], l - 1, by_level[i][l - 1], act[i], next[i]);
        });
        next_plan = LevelPlan();
        c0->cur_level = l - 1;
        plan_level(cs, next, next_plan);
        if (next_plan.nb > 0) pre_launch(cs, next_plan, s2);
        c0->cur_level = l;
        HIP_CHECK(hipEventRecord(c0->ev_pre, s2));
        pre_pending = true;
        speculated = true;
      };
    }
    launch_level(cs, preps, planned, overlap);
    {
      HTimer ht_(cs[0], "host:drop");
      drop_redundant(l, active);
    }
    if (speculated) {
      bool same = true;
      for (size_t i = 0; i < nc && same; ++i) {
        const LevelPrep& P = preps[i];
        for (size_t t = 0; t < P.lb.size(); ++t)
          if (cs[i]->fac[P.ids[P.sel[t]]].k != spec_k[i][t]) {
            same = false;
            break;
          }
      }
      have_next = same;
    }
  }
  cs[0]->cur_level = -1;
  for (size_t i = 0; i < nc; ++i) {
    cs[i]->factor_epoch++;
    factor_root_launch(cs[i]);
  }
  for (size_t i = 0; i < nc; ++i) {
    rs_ctx* c = cs[i];
    factor_root_finish(c);
    collect_arenas(c);
    c->factored = true;
    c->stats.boxes_recomputed = 0;
    for (size_t b = 1; b < c->boxes.size(); ++b)
      if (c->fac[b].active && c->recomputed[b]) c->stats.boxes_recomputed++;
    c->stats.n_levels = c->L + 1;
    c->stats.n_boxes = (int)c->boxes.size();
  }
  const double ms = 1e3 * seconds_since(t0);
  for (rs_ctx* c : cs) c->stats.ms_factor = ms;
}

void do_factor(rs_ctx* c) {
  std::vector<rs_ctx*> cs{c};
  do_factor_multi(cs);
}

// Apply the factored inverse in place: cbuf (rows layout, ncols columns) holds
// the first 2N rows of the right-hand side on entry and [mu; lambda] (2N + 3p
// rows) on exit.  rbot (nullable, float64, 3p x ncols) is the right-hand side
// of the border rows (zero when null).
template <typename T>
void solve_rows(rs_ctx* c, T* cbuf, int ncols, const double* rbot) {
  hipStream_t s = c->stream;
  const int p3 = 3 * c->p;
  const int n0 = (int)c->I0.size();
  sweep_all<T>(c, cbuf, ncols, 0);
  // The diagonal blocks, the border right-hand side and the border fix touch
  // only each box's own R rows (disjoint over all levels) and its own partial
  // slot: one launch over the boxes of every level (stored level after level).
  const SolveBox* all_sb = level_sboxes(c, 1);
  const int all_nb = c->L >= 1 ? (int)(c->sbox_off[c->L + 1] - c->sbox_off[1]) : 0;
  {
    KTimer kt_(c, "diag");
    launch_diag<T>(all_sb, all_nb, c->d_ridx.as<int>(), cbuf, ncols, c->all_maxr, s);
  }
  const int nz = c->nz;
  c->d_v.ensure(std::max<size_t>((size_t)nz * ncols, 1) * sizeof(double));
  c->d_sol.ensure(std::max<size_t>((size_t)nz * ncols, 1) * sizeof(double));
  const double* rhs2 = nullptr;
  if (p3) {
    const int nsb = c->n_solve_boxes;
    const size_t nparts = (size_t)nsb * p3 * ncols;
    c->d_parts.ensure((nparts + sum_parts_scratch_doubles(nsb, p3 * ncols)) * sizeof(double));
    {
      KTimer kt_(c, "border_rhs");
      launch_border_rhs<T>(all_sb, all_nb, c->d_ridx.as<int>(), c->d_Ph.as<double>(), p3, cbuf, ncols,
                           c->d_parts.as<double>(), s);
    }
    c->d_rhs2.ensure((size_t)p3 * ncols * sizeof(double));
    launch_sum_parts(c->d_parts.as<double>(), nsb, (long long)p3 * ncols, p3 * ncols, -1.0,
                     c->d_rhs2.as<double>(), c->d_parts.as<double>() + nparts, s);
    if (rbot) launch_accumulate(rbot, (long long)p3 * ncols, c->d_rhs2.as<double>(), s);
    rhs2 = c->d_rhs2.as<double>();
  }
  if (nz > 0) {
    launch_root_gather<T>(cbuf, ncols, c->d_I0.as<int>(), n0, rhs2, p3, c->d_v.as<double>(), s);
    {
      KTimer kt_(c, "root_apply");
      launch_dense_apply(c->d_Zinv.as<double>(), nz, c->d_v.as<double>(), ncols,
                         c->d_sol.as<double>(), s);
    }
    if (n0) launch_root_scatter<T>(c->d_sol.as<double>(), ncols, c->d_I0.as<int>(), n0, cbuf, s);
  }
  if (p3) {
    const double* lam = c->d_sol.as<double>() + (size_t)n0 * ncols;
    {
      KTimer kt_(c, "border_fix");
      launch_border_fix<T>(all_sb, all_nb, c->d_ridx.as<int>(), p3, lam, cbuf, ncols, s);
    }
    // lambda rows follow the 2N density rows
    T* dst = cbuf + (size_t)2 * c->N * ncols;
    HIP_CHECK(hipMemcpyAsync(dst, lam, (size_t)p3 * ncols * sizeof(T), hipMemcpyDeviceToDevice, s));
  }
  sweep_all<T>(c, cbuf, ncols, 2);
  // Laplace Neumann: the uncoupled second unknown of each node is in no box;
  // its equation is lambda x = b
  if (c->prm.kernel == 1) launch_scale_odd_rows(cbuf, c->N, ncols, 1.0 / c->prm.lambda, s);
}

// out (float64 rows, 2N+3p) = factored inverse applied to rhs (float64 rows,
// 2N + 3p; the border rows are used as their right-hand side).
void apply_inverse(rs_ctx* c, const double* rhs, int ncols, double* out) {
  const size_t n2 = 2 * (size_t)c->N;
  const size_t ns = n2 + 3 * (size_t)c->p;
  const double* rbot = c->p ? rhs + n2 * ncols : nullptr;
  (void)ns;
  // vectors stay float64 in both precisions; mixed precision only changes
  // which factor copies the boxes read
  HIP_CHECK(hipMemcpyAsync(out, rhs, n2 * ncols * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  solve_rows<double>(c, out, ncols, rbot);
}

void apply_device_rows(rs_ctx* c, const double* xrows, int ncols, double* yrows, const int* skip);
int apply_config_for(rs_ctx* c, int ncols, const double* xrows, double* yrows);

// Every buffer one refinement iteration touches, allocated up front (a
// captured graph must not allocate).
void ensure_solve_buffers(rs_ctx* c, int ncols) {
  const size_t n2 = 2 * (size_t)c->N;
  const size_t ns = n2 + 3 * (size_t)c->p;
  const size_t rows = ns * ncols;
  const int p3 = 3 * c->p;
  c->d_r.ensure(rows * sizeof(double));
  c->d_dx.ensure(rows * sizeof(double));
  c->d_ys.ensure(rows * sizeof(double));
  // colsq, fsq, bsq, acc (ncols each), then the residual's partial sums
  c->d_norms.ensure((4 * (size_t)ncols + residual_scratch_doubles(ncols)) * sizeof(double));
  c->d_v.ensure(std::max<size_t>((size_t)c->nz * ncols, 1) * sizeof(double));
  c->d_sol.ensure(std::max<size_t>((size_t)c->nz * ncols, 1) * sizeof(double));
  if (p3) {
    c->d_parts.ensure(((size_t)c->n_solve_boxes * p3 * ncols +
                       sum_parts_scratch_doubles(c->n_solve_boxes, p3 * ncols)) *
                      sizeof(double));
    c->d_rhs2.ensure((size_t)p3 * ncols * sizeof(double));
  }
  c->d_apply.ensure(apply_scratch_doubles(c->N, ncols) * sizeof(double));
  if (c->prm.refine_update) c->d_corr.ensure(corr_scratch_bytes(c->N, ncols));
  c->d_flag.ensure(4 * sizeof(int));
}

// The apply of one refinement iteration (rows layout): the exact apply of x,
// or the float32 image of the correction dx, as the device flags say; which:
// -1 both launched (graph capture), 0 or 1 only that one (eager iterations).
void refine_apply(rs_ctx* c, int ncols, int which) {
  if (!c->prm.refine_update) which = 0;
  const int cfg = apply_config_for(c, ncols, c->d_xs.as<double>(), c->d_ys.as<double>());
  Geo g;
  geo_of(c, g);
  KTimer kt_(c, which == 1 ? "apply_correction" : "apply_operator");
  launch_apply_refine(g, c->d_curve.as<int>(), c->d_hole.as<double>(), c->p, c->prm.lambda, c->d_xs.as<double>(),
                      c->d_dx.as<double>(), ncols, c->d_ys.as<double>(), c->d_apply.as<double>(),
                      c->prm.refine_update ? c->d_corr.p : nullptr, c->d_flag.as<int>(), c->prm.refine_max, cfg,
                      which, c->stream);
  HIP_CHECK(hipGetLastError());
}

// One refinement iteration on the context's buffers: dx = inverse(r),
// x += dx (unless converged), then the new residual: r = [f; 0] - A x with
// the exact apply, or r = r - A dx with the float32 image of the correction
// (the device flags choose), and the flags.  which: as for refine_apply.
void refine_iteration(rs_ctx* c, int nrhs, int which) {
  const int n2 = 2 * c->N;
  const int ns = n2 + 3 * c->p;
  const size_t rows = (size_t)ns * nrhs;
  double* colsq = c->d_norms.as<double>();
  apply_inverse(c, c->d_r.as<double>(), nrhs, c->d_dx.as<double>());
  launch_accumulate_unless(c->d_dx.as<double>(), (long long)rows, c->d_xs.as<double>(), c->d_flag.as<int>(),
                           c->prm.refine_max, c->stream);
  refine_apply(c, nrhs, which);
  const double* bt = c->prm.refine_update ? corr_bound_rows(c->d_corr.p, c->N, nrhs) : nullptr;
  launch_residual(c->d_frows.as<double>(), n2, c->d_ys.as<double>(), ns, nrhs, c->d_r.as<double>(), colsq,
                  colsq + nrhs, colsq + 2 * nrhs, colsq + 4 * nrhs, c->d_flag.as<int>(), c->prm.refine_max, bt,
                  c->stream);
  launch_refine_flag(colsq, colsq + nrhs, colsq + 2 * nrhs, colsq + 3 * nrhs, nrhs, c->prm.refine_tol,
                     c->prm.refine_max, c->prm.refine_update, corr_bound_scale(), c->d_flag.as<int>(), c->stream);
}

// x = 0, r = [f; 0], flags cleared (f already in d_frows).
void refine_begin(rs_ctx* c, int nrhs) {
  const int n2 = 2 * c->N;
  const int ns = n2 + 3 * c->p;
  ensure_solve_buffers(c, nrhs);
  double* colsq = c->d_norms.as<double>();
  launch_fill(c->d_xs.as<double>(), (long long)ns * nrhs, 0.0, c->stream);
  launch_residual(c->d_frows.as<double>(), n2, c->d_xs.as<double>(), ns, nrhs, c->d_r.as<double>(), colsq,
                  colsq + nrhs, colsq + 2 * nrhs, colsq + 4 * nrhs, nullptr, 0, nullptr, c->stream);
  launch_set_ints(c->d_flag.as<int>(), 4, 0, c->stream);
  c->refine_which = 0;
  c->refine_prev = 1.0;
  c->refine_last = 0;
}

// Addresses of the buffers one refinement iteration touches (graph key).
std::vector<const void*> refine_graph_sig(const rs_ctx* c) {
  const DevBuf* bufs[] = {&c->d_r,     &c->d_dx,     &c->d_ys,   &c->d_xs,     &c->d_frows, &c->d_norms,
                          &c->d_v,     &c->d_sol,    &c->d_parts, &c->d_rhs2,  &c->d_apply, &c->d_flag,
                          &c->d_corr,
                          &c->d_sboxes, &c->d_sidx,  &c->d_ridx,  &c->d_I0,    &c->d_Zinv,  &c->d_Ph,
                          &c->d_W,     &c->d_Wf,     &c->d_x,     &c->d_y,     &c->d_nx,    &c->d_ny,
                          &c->d_w,     &c->d_kap,    &c->d_curve, &c->d_hole};
  std::vector<const void*> sig;
  sig.reserve(sizeof(bufs) / sizeof(bufs[0]));
  for (const DevBuf* b : bufs) sig.push_back(b->p);
  return sig;
}

// Capture one refinement iteration as a graph (once per factorization, nrhs
// and set of buffer addresses).
void refine_graph_capture(rs_ctx* c, int nrhs) {
  if (c->refine_exec && c->refine_nrhs == nrhs && c->refine_epoch == c->factor_epoch &&
      c->refine_sig == refine_graph_sig(c))
    return;
  HTimer ht_(c, "host:capture");
  if (c->refine_exec) {
    HIP_CHECK(hipGraphExecDestroy(c->refine_exec));
    c->refine_exec = nullptr;
  }
  if (!c->cap_stream) HIP_CHECK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  hipStream_t saved = c->stream;
  c->stream = c->cap_stream;
  c->capturing = true;
  hipGraph_t g = nullptr;
  HIP_CHECK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  try {
    refine_iteration(c, nrhs, -1);
  } catch (...) {
    (void)hipStreamEndCapture(c->cap_stream, &g);
    if (g) (void)hipGraphDestroy(g);
    c->stream = saved;
    c->capturing = false;
    throw;
  }
  const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
  c->stream = saved;
  c->capturing = false;
  if (e != hipSuccess) throw RsError{RS_ERR_DEVICE, std::string("graph capture failed: ") + hipGetErrorString(e)};
  const hipError_t e2 = hipGraphInstantiate(&c->refine_exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) {
    c->refine_exec = nullptr;
    throw RsError{RS_ERR_DEVICE, std::string("graph instantiation failed: ") + hipGetErrorString(e2)};
  }
  c->refine_nrhs = nrhs;
  c->refine_epoch = c->factor_epoch;
  c->refine_sig = refine_graph_sig(c);
}

// Iterations for the next round of graph replays (1 or 2) before the host
// looks at the residual again: the remaining count predicted from the
// contraction observed so far (per iteration, geometric mean over the last
// round); 2 before the first round.  Replays after convergence change nothing
// (the device flag skips them), so a prediction only trades a host poll
// against a skipped iteration.
int refine_next_iters(rs_ctx* c) {
  if (c->refine_last == 0 || c->last_res.empty()) return 2;
  double cur = 0.0;
  for (double r : c->last_res) cur = std::max(cur, r);
  const double prev = std::max(c->refine_prev, 1e-300);
  double rho = std::pow(std::max(cur, 1e-300) / prev, 1.0 / c->refine_last);
  rho = std::min(std::max(rho, 1e-12), 0.99);
  const double need = std::log(c->prm.refine_tol / std::max(cur, 1e-300)) / std::log(rho);
  return need > 1.5 ? 2 : 1;   // an extra poll costs far less than a skipped iteration
}

void refine_graph_launch(rs_ctx* c, int nrhs) {
  const int iters = refine_next_iters(c);
  if (!c->last_res.empty()) {
    double cur = 0.0;
    for (double r : c->last_res) cur = std::max(cur, r);
    c->refine_prev = cur;
  }
  refine_graph_capture(c, nrhs);
  c->refine_last = iters;
  KTimer kt_(c, "refine_graph");
  for (int it = 0; it < iters; ++it) HIP_CHECK(hipGraphLaunch(c->refine_exec, c->stream));
}

// Read the flags and norms after a graph launch; true when refinement is over
// (conv receives whether it converged).  Fills last_res and refine_iters.
bool refine_poll(rs_ctx* c, int nrhs, bool& conv) {
  int* hf = c->h_flag.get<int>(4 + 8 * (size_t)nrhs);
  double* hn = reinterpret_cast<double*>(hf + 4);
  HIP_CHECK(hipMemcpyAsync(hf, c->d_flag.p, 4 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_CHECK(hipMemcpyAsync(hn, c->d_norms.p, 4 * (size_t)nrhs * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  HIP_CHECK(hipStreamSynchronize(c->stream));
  resolve_timers(c);
  c->stats.refine_iters = hf[1];
  c->refine_which = hf[2] == 1 ? 1 : 0;
  // the certified relative residual: the computed norm plus the accumulated
  // rounding bound of updated residuals
  c->last_res.assign(nrhs, 0.0);
  for (int q = 0; q < nrhs; ++q) {
    const double fq = hn[nrhs + q] > 0 ? hn[nrhs + q] : 1.0;
    c->last_res[q] = (std::sqrt(hn[q]) + hn[3 * nrhs + q]) / std::sqrt(fq);
  }
  conv = hf[0] != 0;
  return conv || hf[1] >= c->prm.refine_max;
}

// The same iterations launched one by one, the host testing after each.
bool refine_eager(rs_ctx* c, int nrhs) {
  for (;;) {
    refine_iteration(c, nrhs, c->refine_which);
    bool conv;
    if (refine_poll(c, nrhs, conv)) return conv;
  }
}

// Solve with f_dev (2N x nrhs, column-major) into x_dev ((2N+3p) x nrhs,
// column-major).  With refine_max > 0: iterative refinement, the residual
// [f; 0] - A x evaluated exactly in float64 and the factored inverse (float64
// or float32) as the inner solver, until max_q ||r_q|| / ||f_q|| <= refine_tol.
// Returns false if refinement did not reach the tolerance.
bool solve_device(rs_ctx* c, int nrhs, const double* f_dev, double* x_dev) {
  const int n2 = 2 * c->N;
  const int ns = n2 + 3 * c->p;
  hipStream_t s = c->stream;
  const size_t rows = (size_t)ns * nrhs;
  c->d_frows.ensure((size_t)n2 * nrhs * sizeof(double));
  c->d_xs.ensure(rows * sizeof(double));
  launch_to_rows(f_dev, n2, n2, nrhs, c->d_frows.as<double>(), s);
  c->last_res.clear();
  c->stats.refine_iters = 0;
  if (c->prm.refine_max <= 0) {
    c->d_r.ensure(rows * sizeof(double));
    // right-hand side rows [f; 0]
    launch_fill(c->d_r.as<double>(), (long long)rows, 0.0, s);
    HIP_CHECK(hipMemcpyAsync(c->d_r.p, c->d_frows.p, (size_t)n2 * nrhs * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
    apply_inverse(c, c->d_r.as<double>(), nrhs, c->d_xs.as<double>());
    launch_from_rows(c->d_xs.as<double>(), ns, nrhs, x_dev, ns, s);
    HIP_CHECK(hipGetLastError());
    return true;
  }
  refine_begin(c, nrhs);
  apply_config_for(c, nrhs, c->d_xs.as<double>(), c->d_ys.as<double>());   // before any capture
  bool conv;
  // timing mode 4 times every launch of the exact apply: the iterations are
  // launched one by one (events are not recorded inside a captured graph)
  if (c->prm.solve_graph && c->timing != 4) {
    refine_graph_launch(c, nrhs);
    while (!refine_poll(c, nrhs, conv)) refine_graph_launch(c, nrhs);
  } else {
    conv = refine_eager(c, nrhs);
  }
  launch_from_rows(c->d_xs.as<double>(), ns, nrhs, x_dev, ns, s);
  HIP_CHECK(hipGetLastError());
  return conv;
}

// Autotuner of the operator apply: the kernel shape (columns per pass,
// targets per thread) for a problem shape (N, ncols) is chosen once per
// process by timing every valid shape on the context's stream (all shapes
// give bitwise the same result, so the choice only affects speed).
struct ApplyTuneCache {
  std::mutex mu;
  std::map<std::pair<int, int>, std::pair<int, double>> best;   // -> (config, ms per apply)
};
ApplyTuneCache& apply_tune_cache() {
  static ApplyTuneCache cache;
  return cache;
}

int apply_config_for(rs_ctx* c, int ncols, const double* xrows, double* yrows) {
  if (c->prm.kernel == 1) {   // the Laplace apply has one shape per column count
    c->stats.apply_config = apply_default_config(ncols);
    return c->stats.apply_config;
  }
  if (c->prm.apply_shape >= 0) {
    const int cfg = apply_config_valid(c->prm.apply_shape, ncols) ? c->prm.apply_shape
                                                                   : apply_default_config(ncols);
    c->stats.apply_config = cfg;
    return cfg;
  }
  const std::pair<int, int> key{c->N, ncols};
  ApplyTuneCache& tc = apply_tune_cache();
  {
    std::lock_guard<std::mutex> lk(tc.mu);
    auto it = tc.best.find(key);
    if (it != tc.best.end()) {
      c->stats.apply_config = it->second.first;
      c->stats.apply_ms = it->second.second;
      return it->second.first;
    }
  }
  if (c->capturing) return apply_default_config(ncols);
  Geo g;
  geo_of(c, g);
  c->d_apply.ensure(apply_scratch_doubles(c->N, ncols) * sizeof(double));
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  int best = apply_default_config(ncols);
  float best_ms = -1.0f;
  constexpr int kReps = 2;
  for (int cfg = 0; cfg < apply_config_count(); ++cfg) {
    if (!apply_config_valid(cfg, ncols)) continue;
    auto run = [&]() {
      launch_apply_operator(g, c->d_curve.as<int>(), c->d_hole.as<double>(), c->p, c->prm.lambda, xrows,
                            ncols, yrows, c->d_apply.as<double>(), nullptr, 0, cfg, c->stream);
    };
    run();   // warm-up
    HIP_CHECK(hipEventRecord(e0, c->stream));
    for (int r = 0; r < kReps; ++r) run();
    HIP_CHECK(hipEventRecord(e1, c->stream));
    HIP_CHECK(hipEventSynchronize(e1));
    float ms = 0.0f;
    HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    ms /= kReps;
    if (best_ms < 0.0f || ms < best_ms) {
      best_ms = ms;
      best = cfg;
    }
  }
  HIP_CHECK(hipEventDestroy(e0));
  HIP_CHECK(hipEventDestroy(e1));
  HIP_CHECK(hipGetLastError());
  {
    std::lock_guard<std::mutex> lk(tc.mu);
    tc.best[key] = {best, (double)best_ms};
  }
  c->stats.apply_config = best;
  c->stats.apply_ms = best_ms;
  return best;
}

// The apply shape without running the autotuner (no launches, no memory):
// the fixed shape, the tuned one if this problem shape was tuned before in
// the process, else the default.
int apply_config_cached(const rs_ctx* c, int ncols) {
  if (c->prm.kernel == 1) return apply_default_config(ncols);
  if (c->prm.apply_shape >= 0)
    return apply_config_valid(c->prm.apply_shape, ncols) ? c->prm.apply_shape : apply_default_config(ncols);
  ApplyTuneCache& tc = apply_tune_cache();
  std::lock_guard<std::mutex> lk(tc.mu);
  auto it = tc.best.find(std::pair<int, int>{c->N, ncols});
  return it != tc.best.end() ? it->second.first : apply_default_config(ncols);
}

// y = A x on the device (rows layout).  skip (nullable): refinement flags; the
// apply is skipped on the device once they say converged or exhausted.
void apply_device_rows(rs_ctx* c, const double* xrows, int ncols, double* yrows, const int* skip) {
  const int cfg = apply_config_for(c, ncols, xrows, yrows);
  Geo g;
  geo_of(c, g);
  {
    KTimer kt_(c, "apply_operator");
    c->d_apply.ensure(apply_scratch_doubles(c->N, ncols) * sizeof(double));
    launch_apply_operator(g, c->d_curve.as<int>(), c->d_hole.as<double>(), c->p, c->prm.lambda, xrows,
                          ncols, yrows, c->d_apply.as<double>(), skip, c->prm.refine_max, cfg, c->stream);
  }
  HIP_CHECK(hipGetLastError());
}

rs_status fail(rs_ctx* c, const RsError& e) {
  if (c) c->err = e.msg;
  else g_build_error = e.msg;
  return e.st;
}

bool finite_all(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

void validate_nodes(int n, const double* xy, const double* normal, const double* weight,
                    const double* curvature) {
  if (!xy || !normal || !weight || !curvature) throw RsError{RS_ERR_ARG, "NULL node array"};
  if (!finite_all(xy, 2 * (size_t)n) || !finite_all(normal, 2 * (size_t)n) ||
      !finite_all(weight, n) || !finite_all(curvature, n))
    throw RsError{RS_ERR_ARG, "non-finite node data"};
  for (int i = 0; i < n; ++i) {
    const double nn = std::sqrt(normal[2 * i] * normal[2 * i] + normal[2 * i + 1] * normal[2 * i + 1]);
    if (std::fabs(nn - 1.0) > 1e-12) throw RsError{RS_ERR_ARG, "normal " + std::to_string(i) + " is not unit length"};
    if (!(weight[i] > 0.0)) throw RsError{RS_ERR_ARG, "weight " + std::to_string(i) + " is not positive"};
  }
}

void upload_geometry(rs_ctx* c) {
  const size_t N = c->N;
  auto up = [&](DevBuf& b, const void* src, size_t bytes) {
    b.ensure(std::max<size_t>(bytes, 16));
    if (bytes) HIP_CHECK(hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
  };
  up(c->d_x, c->x.data(), N * sizeof(double));
  up(c->d_y, c->y.data(), N * sizeof(double));
  up(c->d_nx, c->nx.data(), N * sizeof(double));
  up(c->d_ny, c->ny.data(), N * sizeof(double));
  up(c->d_w, c->w.data(), N * sizeof(double));
  up(c->d_kap, c->kap.data(), N * sizeof(double));
  up(c->d_curve, c->curve.data(), N * sizeof(int));
  up(c->d_hole, c->hole.data(), c->hole.size() * sizeof(double));
}

bool inside_root(const rs_ctx* c, double x, double y) {
  const double h = 0.5 * c->root_side;
  return x >= c->root_cx - h && x < c->root_cx + h && y >= c->root_cy - h && y < c->root_cy + h;
}

}  // namespace

// ============================== C ABI ========================================

extern "C" {

void rs_default_params(rs_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->lambda = -0.5;
  p->tol = 1e-10;
  p->leaf_size = 64;
  p->n_proxy = 64;
  p->proxy_ratio = 1.5;
  p->rcond_min = 1e-12;
  p->precision = 0;
  p->refine_tol = 1e-8;
  p->refine_max = 0;
  p->has_root = 0;
  p->solve_graph = 1;
  p->mixed_rcond_min = 1e-4;
  p->apply_shape = -1;
  p->refine_update = 1;
}

rs_status rs_build_tree(const rs_params* prm, int n_nodes, const double* xy, const double* normal,
                        const double* weight, const double* curvature, const int* curve_id,
                        int n_holes, const double* hole_xy, rs_ctx** out) {
  rs_ctx* c = nullptr;
  try {
    if (!prm || !out) throw RsError{RS_ERR_ARG, "NULL params or output handle"};
    if (n_nodes <= 0) throw RsError{RS_ERR_ARG, "n_nodes must be positive"};
    if (n_holes < 0) throw RsError{RS_ERR_ARG, "n_holes must be >= 0"};
    if (!curve_id) throw RsError{RS_ERR_ARG, "NULL curve_id"};
    if (!(prm->tol > 0.0) || prm->leaf_size < 1 || prm->n_proxy < 4 || !(prm->proxy_ratio > 1.0))
      throw RsError{RS_ERR_ARG, "invalid tolerance, leaf size, proxy count or proxy ratio"};
    if (prm->precision < 0 || prm->precision > 2) throw RsError{RS_ERR_ARG, "precision must be 0, 1 or 2"};
    if (!(prm->mixed_rcond_min >= 0.0) || !std::isfinite(prm->mixed_rcond_min))
      throw RsError{RS_ERR_ARG, "mixed_rcond_min must be finite and >= 0"};
    if (prm->refine_update != 0 && prm->refine_update != 1)
      throw RsError{RS_ERR_ARG, "refine_update must be 0 or 1"};
    if (prm->kernel != 0 && prm->kernel != 1) throw RsError{RS_ERR_ARG, "kernel must be 0 or 1"};
    if (prm->kernel == 1 && n_holes != 0)
      throw RsError{RS_ERR_ARG, "the Laplace Neumann kernel has no augmentation: n_holes must be 0"};
    validate_nodes(n_nodes, xy, normal, weight, curvature);
    std::vector<int> count(n_holes + 1, 0);
    for (int i = 0; i < n_nodes; ++i) {
      if (curve_id[i] < 0 || curve_id[i] > n_holes) throw RsError{RS_ERR_ARG, "curve_id out of range"};
      count[curve_id[i]]++;
    }
    for (int h = 1; h <= n_holes; ++h)
      if (!count[h]) throw RsError{RS_ERR_ARG, "hole " + std::to_string(h) + " has no nodes"};
    if (hole_xy && !finite_all(hole_xy, 2 * (size_t)n_holes)) throw RsError{RS_ERR_ARG, "non-finite hole point"};
    c = new rs_ctx();
    c->prm = *prm;
    if (c->prm.kernel == 1) c->prm.refine_update = 0;   // no float32 image of the Laplace operator
    c->N = n_nodes;
    c->p = n_holes;
    c->x.resize(n_nodes);
    c->y.resize(n_nodes);
    c->nx.resize(n_nodes);
    c->ny.resize(n_nodes);
    for (int i = 0; i < n_nodes; ++i) {
      c->x[i] = xy[2 * i];
      c->y[i] = xy[2 * i + 1];
      c->nx[i] = normal[2 * i];
      c->ny[i] = normal[2 * i + 1];
    }
    c->w.assign(weight, weight + n_nodes);
    c->kap.assign(curvature, curvature + n_nodes);
    c->curve.assign(curve_id, curve_id + n_nodes);
    c->hole.assign(2 * (size_t)n_holes, 0.0);
    for (int h = 0; h < n_holes; ++h) {
      if (hole_xy) {
        c->hole[2 * h] = hole_xy[2 * h];
        c->hole[2 * h + 1] = hole_xy[2 * h + 1];
      } else {
        double sx = 0, sy = 0;
        for (int i = 0; i < n_nodes; ++i)
          if (curve_id[i] == h + 1) { sx += c->x[i]; sy += c->y[i]; }
        c->hole[2 * h] = sx / count[h + 1];
        c->hole[2 * h + 1] = sy / count[h + 1];
      }
    }
    if (prm->has_root) {
      if (!(prm->root[2] > 0.0) || !finite_all(prm->root, 3)) throw RsError{RS_ERR_ARG, "invalid fixed root"};
      c->root_cx = prm->root[0];
      c->root_cy = prm->root[1];
      c->root_side = prm->root[2];
      for (int i = 0; i < n_nodes; ++i)
        if (!inside_root(c, c->x[i], c->y[i]))
          throw RsError{RS_ERR_OUT_OF_ROOT, "node " + std::to_string(i) + " lies outside the fixed root"};
    }
    build_tree(c);
    HIP_CHECK(hipGetDevice(&c->device));
    HIP_CHECK(hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device));
    upload_geometry(c);
    c->stats.n_nodes = n_nodes;
    c->stats.n_holes = n_holes;
    c->stats.n_levels = c->L + 1;
    c->stats.n_boxes = (int)c->boxes.size();
    *out = c;
    return RS_OK;
  } catch (const RsError& e) {
    delete c;
    return fail(nullptr, e);
  } catch (const std::exception& e) {
    delete c;
    return fail(nullptr, RsError{RS_ERR_ALLOC, e.what()});
  }
}

rs_status rs_factor(rs_ctx* c) {
  if (!c) return RS_ERR_ARG;
  try {
    HIP_CHECK(hipSetDevice(c->device));
    c->factored = false;
    do_factor(c);
    return RS_OK;
  } catch (const RsError& e) {
    c->factored = false;
    return fail(c, e);
  } catch (const std::exception& e) {
    c->factored = false;
    return fail(c, RsError{RS_ERR_ALLOC, e.what()});
  }
}

rs_status rs_factor_batch(rs_ctx** ctxs, int n) {
  if (!ctxs || n <= 0) return RS_ERR_ARG;
  for (int i = 0; i < n; ++i)
    if (!ctxs[i]) return RS_ERR_ARG;
  rs_ctx* lead = ctxs[0];
  try {
    std::vector<rs_ctx*> cs(ctxs, ctxs + n);
    for (rs_ctx* c : cs) {
      const rs_params& a = lead->prm;
      const rs_params& b = c->prm;
      if (c->device != lead->device) throw RsError{RS_ERR_ARG, "contexts of a batch must share the device"};
      if (a.tol != b.tol || a.n_proxy != b.n_proxy || a.proxy_ratio != b.proxy_ratio ||
          a.lambda != b.lambda || a.rcond_min != b.rcond_min || a.precision != b.precision)
        throw RsError{RS_ERR_ARG, "contexts of a batch must share lambda, tol, proxy, rcond and precision"};
    }
    std::vector<rs_ctx*> sorted(cs);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
      throw RsError{RS_ERR_ARG, "a context appears twice in the batch"};
    HIP_CHECK(hipSetDevice(lead->device));
    for (rs_ctx* c : cs) c->factored = false;
    do_factor_multi(cs);
    return RS_OK;
  } catch (const RsError& e) {
    for (int i = 0; i < n; ++i) ctxs[i]->factored = false;
    for (int i = 0; i < n; ++i) ctxs[i]->err = e.msg;
    return e.st;
  } catch (const std::exception& e) {
    for (int i = 0; i < n; ++i) ctxs[i]->factored = false;
    return fail(lead, RsError{RS_ERR_ALLOC, e.what()});
  }
}

// Refined solves of n contexts interleaved: every context's first graph
// launch is queued before the first wait, and each later round relaunches
// only the contexts still iterating.  Contexts with refine_max = 0 or without
// the graph path are solved one after another.
rs_status rs_solve_batch(rs_ctx** ctxs, int n, int nrhs, const double* const* f_dev,
                         double* const* x_dev) {
  if (!ctxs || n <= 0 || !f_dev || !x_dev) return RS_ERR_ARG;
  for (int i = 0; i < n; ++i)
    if (!ctxs[i] || !f_dev[i] || !x_dev[i]) return RS_ERR_ARG;
  rs_status worst = RS_OK;
  std::vector<int> active;
  for (int i = 0; i < n; ++i) {
    rs_ctx* c = ctxs[i];
    if (!c->factored || nrhs <= 0 || c->prm.refine_max <= 0 || !c->prm.solve_graph || c->timing == 4) {
      const rs_status st = rs_solve_dev(c, nrhs, f_dev[i], x_dev[i]);
      if (st != RS_OK && worst == RS_OK) worst = st;
    } else {
      active.push_back(i);
    }
  }
  std::vector<std::chrono::steady_clock::time_point> t0(n);
  std::vector<char> conv(n, 0);
  std::vector<int> live;
  for (int i : active) {
    rs_ctx* c = ctxs[i];
    try {
      HIP_CHECK(hipSetDevice(c->device));
      t0[i] = std::chrono::steady_clock::now();
      const int n2 = 2 * c->N;
      const size_t rows = (size_t)(n2 + 3 * c->p) * nrhs;
      c->d_frows.ensure((size_t)n2 * nrhs * sizeof(double));
      c->d_xs.ensure(rows * sizeof(double));
      launch_to_rows(f_dev[i], n2, n2, nrhs, c->d_frows.as<double>(), c->stream);
      c->last_res.clear();
      c->stats.refine_iters = 0;
      refine_begin(c, nrhs);
      apply_config_for(c, nrhs, c->d_xs.as<double>(), c->d_ys.as<double>());
      refine_graph_launch(c, nrhs);
      live.push_back(i);
    } catch (const RsError& e) {
      const rs_status st = fail(c, e);
      if (worst == RS_OK) worst = st;
    }
  }
  while (!live.empty()) {
    std::vector<int> next;
    for (int i : live) {
      rs_ctx* c = ctxs[i];
      try {
        HIP_CHECK(hipSetDevice(c->device));
        bool cv = false;
        if (refine_poll(c, nrhs, cv)) {
          conv[i] = cv;
          const int ns = 2 * c->N + 3 * c->p;
          launch_from_rows(c->d_xs.as<double>(), ns, nrhs, x_dev[i], ns, c->stream);
          HIP_CHECK(hipStreamSynchronize(c->stream));
          c->stats.ms_solve = 1e3 * seconds_since(t0[i]);
          if (!cv) throw RsError{RS_ERR_NOCONV, "refinement did not reach refine_tol"};
        } else {
          refine_graph_launch(c, nrhs);
          next.push_back(i);
        }
      } catch (const RsError& e) {
        const rs_status st = fail(c, e);
        if (worst == RS_OK) worst = st;
      }
    }
    live.swap(next);
  }
  return worst;
}

rs_status rs_solve_dev(rs_ctx* c, int nrhs, const double* f_dev, double* x_dev) {
  if (!c) return RS_ERR_ARG;
  try {
    if (!c->factored) throw RsError{RS_ERR_STATE, "rs_solve before rs_factor"};
    if (nrhs <= 0 || !f_dev || !x_dev) throw RsError{RS_ERR_ARG, "bad nrhs or NULL pointer"};
    HIP_CHECK(hipSetDevice(c->device));
    auto t0 = std::chrono::steady_clock::now();
    const bool conv = solve_device(c, nrhs, f_dev, x_dev);
    HIP_CHECK(hipStreamSynchronize(c->stream));
    c->stats.ms_solve = 1e3 * seconds_since(t0);
    resolve_timers(c);
    if (!conv) throw RsError{RS_ERR_NOCONV, "refinement did not reach refine_tol"};
    return RS_OK;
  } catch (const RsError& e) {
    return fail(c, e);
  }
}

rs_status rs_solve(rs_ctx* c, int nrhs, const double* f, double* x, double* rel_residual) {
  if (!c) return RS_ERR_ARG;
  try {
    if (!c->factored) throw RsError{RS_ERR_STATE, "rs_solve before rs_factor"};
    if (nrhs <= 0 || !f || !x) throw RsError{RS_ERR_ARG, "bad nrhs or NULL pointer"};
    const size_t n2 = 2 * (size_t)c->N;
    const size_t ns = n2 + 3 * (size_t)c->p;
    if (!finite_all(f, n2 * nrhs)) throw RsError{RS_ERR_ARG, "non-finite right-hand side"};
    HIP_CHECK(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    auto t0 = std::chrono::steady_clock::now();
    c->d_f.ensure(n2 * nrhs * sizeof(double));
    c->d_xout.ensure(ns * nrhs * sizeof(double));
    HIP_CHECK(hipMemcpyAsync(c->d_f.p, f, n2 * nrhs * sizeof(double), hipMemcpyHostToDevice, s));
    const bool conv = solve_device(c, nrhs, c->d_f.as<double>(), c->d_xout.as<double>());
    std::vector<double> xo(ns * nrhs);
    HIP_CHECK(hipMemcpyAsync(xo.data(), c->d_xout.p, xo.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    c->stats.ms_solve = 1e3 * seconds_since(t0);
    resolve_timers(c);
    if (rel_residual) {
      if ((int)c->last_res.size() == nrhs) {
        std::copy(c->last_res.begin(), c->last_res.end(), rel_residual);
      } else {
        // residual of the direct solve: x rows are in d_xs
        c->d_ys.ensure(ns * nrhs * sizeof(double));
        c->d_r.ensure(ns * nrhs * sizeof(double));
        c->d_norms.ensure((4 * (size_t)nrhs + residual_scratch_doubles(nrhs)) * sizeof(double));
        apply_device_rows(c, c->d_xs.as<double>(), nrhs, c->d_ys.as<double>(), nullptr);
        double* colsq = c->d_norms.as<double>();
        launch_residual(c->d_frows.as<double>(), (int)n2, c->d_ys.as<double>(), (int)ns, nrhs,
                        c->d_r.as<double>(), colsq, colsq + nrhs, colsq + 2 * nrhs, colsq + 4 * nrhs, nullptr, 0,
                        nullptr, s);
        std::vector<double> nrm(2 * nrhs);
        HIP_CHECK(hipMemcpyAsync(nrm.data(), colsq, nrm.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        resolve_timers(c);
        for (int q = 0; q < nrhs; ++q)
          rel_residual[q] = std::sqrt(nrm[q] / (nrm[nrhs + q] > 0 ? nrm[nrhs + q] : 1.0));
      }
    }
    std::memcpy(x, xo.data(), xo.size() * sizeof(double));
    if (!conv) throw RsError{RS_ERR_NOCONV, "refinement did not reach refine_tol"};
    return RS_OK;
  } catch (const RsError& e) {
    return fail(c, e);
  }
}

rs_status rs_apply(rs_ctx* c, int ncols, const double* x, double* y) {
  if (!c) return RS_ERR_ARG;
  try {
    if (ncols <= 0 || !x || !y) throw RsError{RS_ERR_ARG, "bad ncols or NULL pointer"};
    HIP_CHECK(hipSetDevice(c->device));
    const size_t ns = 2 * (size_t)c->N + 3 * (size_t)c->p;
    c->d_f.ensure(ns * ncols * sizeof(double));
    c->d_c.ensure(ns * ncols * sizeof(double));
    c->d_res.ensure(ns * ncols * sizeof(double));
    HIP_CHECK(hipMemcpyAsync(c->d_f.p, x, ns * ncols * sizeof(double), hipMemcpyHostToDevice, c->stream));
    launch_to_rows(c->d_f.as<double>(), (int)ns, (int)ns, ncols, c->d_c.as<double>(), c->stream);
    apply_device_rows(c, c->d_c.as<double>(), ncols, c->d_res.as<double>(), nullptr);
    launch_from_rows(c->d_res.as<double>(), (int)ns, ncols, c->d_f.as<double>(), (int)ns, c->stream);
    HIP_CHECK(hipMemcpyAsync(y, c->d_f.p, ns * ncols * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_CHECK(hipStreamSynchronize(c->stream));
    resolve_timers(c);
    return RS_OK;
  } catch (const RsError& e) {
    return fail(c, e);
  }
}

rs_status rs_apply_f32(rs_ctx* c, int ncols, const double* x, double* y, double* bound) {
  if (!c) return RS_ERR_ARG;
  try {
    if (ncols <= 0 || !x || !y) throw RsError{RS_ERR_ARG, "bad ncols or NULL pointer"};
    if (c->prm.kernel == 1) throw RsError{RS_ERR_ARG, "no float32 image of the Laplace Neumann operator"};
    HIP_CHECK(hipSetDevice(c->device));
    const size_t ns = 2 * (size_t)c->N + 3 * (size_t)c->p;
    hipStream_t s = c->stream;
    c->d_f.ensure(ns * ncols * sizeof(double));
    c->d_c.ensure(ns * ncols * sizeof(double));
    c->d_res.ensure(ns * ncols * sizeof(double));
    c->d_apply.ensure(apply_scratch_doubles(c->N, ncols) * sizeof(double));
    c->d_corr.ensure(corr_scratch_bytes(c->N, ncols));
    // flags of a refinement iteration whose residual is updated: the image runs
    c->d_fflag.ensure(4 * sizeof(int));
    launch_set_ints(c->d_fflag.as<int>(), 4, 0, s);
    launch_set_ints(c->d_fflag.as<int>() + 2, 1, 1, s);
    HIP_CHECK(hipMemcpyAsync(c->d_f.p, x, ns * ncols * sizeof(double), hipMemcpyHostToDevice, s));
    launch_to_rows(c->d_f.as<double>(), (int)ns, (int)ns, ncols, c->d_c.as<double>(), s);
    Geo g;
    geo_of(c, g);
    {
      KTimer kt_(c, "apply_correction");
      launch_apply_refine(g, c->d_curve.as<int>(), c->d_hole.as<double>(), c->p, c->prm.lambda,
                          c->d_c.as<double>(), c->d_c.as<double>(), ncols, c->d_res.as<double>(),
                          c->d_apply.as<double>(), c->d_corr.p, c->d_fflag.as<int>(), 1, 0, 1, s);
    }
    launch_from_rows(c->d_res.as<double>(), (int)ns, ncols, c->d_f.as<double>(), (int)ns, s);
    HIP_CHECK(hipMemcpyAsync(y, c->d_f.p, ns * ncols * sizeof(double), hipMemcpyDeviceToHost, s));
    std::vector<double> bt((size_t)c->N * ncols);
    int hflag[4];
    HIP_CHECK(hipMemcpyAsync(bt.data(), corr_bound_rows(c->d_corr.p, c->N, ncols), bt.size() * sizeof(double),
                             hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipMemcpyAsync(hflag, c->d_fflag.p, sizeof(hflag), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    resolve_timers(c);
    if (hflag[3]) throw RsError{RS_ERR_ARG, "two distinct nodes are too close for the float32 image"};
    if (bound) {
      const double sc = corr_bound_scale();
      for (int q = 0; q < ncols; ++q)
        for (int i = 0; i < c->N; ++i) bound[(size_t)q * c->N + i] = sc * bt[(size_t)i * ncols + q];
    }
    return RS_OK;
  } catch (const RsError& e) {
    return fail(c, e);
  }
}

rs_status rs_apply_inverse(rs_ctx* c, int ncols, const double* b, double* x) {
  if (!c) return RS_ERR_ARG;
  try {
    if (!c->factored) throw RsError{RS_ERR_STATE, "rs_apply_inverse before rs_factor"};
    if (ncols <= 0 || !b || !x) throw RsError{RS_ERR_ARG, "bad ncols or NULL pointer"};
    const size_t ns = 2 * (size_t)c->N + 3 * (size_t)c->p;
    if (!finite_all(b, ns * ncols)) throw RsError{RS_ERR_ARG, "non-finite right-hand side"};
    HIP_CHECK(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    c->d_f.ensure(ns * ncols * sizeof(double));
    c->d_c.ensure(ns * ncols * sizeof(double));
    c->d_res.ensure(ns * ncols * sizeof(double));
    HIP_CHECK(hipMemcpyAsync(c->d_f.p, b, ns * ncols * sizeof(double), hipMemcpyHostToDevice, s));
    launch_to_rows(c->d_f.as<double>(), (int)ns, (int)ns, ncols, c->d_c.as<double>(), s);
    apply_inverse(c, c->d_c.as<double>(), ncols, c->d_res.as<double>());
    launch_from_rows(c->d_res.as<double>(), (int)ns, ncols, c->d_f.as<double>(), (int)ns, s);
    HIP_CHECK(hipMemcpyAsync(x, c->d_f.p, ns * ncols * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    resolve_timers(c);
    return RS_OK;
  } catch (const RsError& e) {
    return fail(c, e);
  }
}

rs_status rs_apply_dev_noalloc(rs_ctx* c, int ncols, const double* x_dev, double* y_dev) {
  if (!c) return RS_ERR_ARG;
  try {
    if (ncols <= 0 || !x_dev || !y_dev) throw RsError{RS_ERR_ARG, "bad ncols or NULL pointer"};
    HIP_CHECK(hipSetDevice(c->device));
    const size_t ns = 2 * (size_t)c->N + 3 * (size_t)c->p;
    const size_t rows = ns * (size_t)ncols;
    const size_t off = (2 * rows + 31) / 32 * 32;         // partial sums 256-byte aligned
    const size_t need = off + apply_scratch_doubles(c->N, ncols);
    if (need > noalloc_scratch_doubles())
      throw RsError{RS_ERR_ARG, "rs_apply_dev_noalloc: " + std::to_string(ncols) + " columns of " +
                                    std::to_string(ns) + " unknowns need " + std::to_string(need) +
                                    " doubles of scratch; the fixed per-device array holds " +
                                    std::to_string(noalloc_scratch_doubles())};
    double* scr = nullptr;
    HIP_CHECK(noalloc_scratch(c->device, &scr));
    hipStream_t s = c->stream;
    Geo g;
    geo_of(c, g);
    launch_to_rows(x_dev, (int)ns, (int)ns, ncols, scr, s);
    launch_apply_operator(g, c->d_curve.as<int>(), c->d_hole.as<double>(), c->p, c->prm.lambda, scr, ncols,
                          scr + rows, scr + off, nullptr, 0, apply_config_cached(c, ncols), s);
    launch_from_rows(scr + rows, (int)ns, ncols, y_dev, (int)ns, s);
    HIP_CHECK(hipGetLastError());
    return RS_OK;
  } catch (const RsError& e) {
    return fail(c, e);
  }
}

rs_status rs_evaluate(rs_ctx* c, int n_targets, const double* targets_xy, int ncols, const double* x,
                      double* u) {
  if (!c) return RS_ERR_ARG;
  try {
    if (n_targets <= 0 || ncols <= 0 || !targets_xy || !x || !u)
      throw RsError{RS_ERR_ARG, "bad n_targets or ncols, or NULL pointer"};
    if (!finite_all(targets_xy, 2 * (size_t)n_targets)) throw RsError{RS_ERR_ARG, "non-finite target"};
    HIP_CHECK(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    const int ns = 2 * c->N + 3 * c->p;
    const int nt = n_targets;
    std::vector<double> tx(nt), ty(nt);
    for (int t = 0; t < nt; ++t) {
      tx[t] = targets_xy[2 * t];
      ty[t] = targets_xy[2 * t + 1];
    }
    upload(c->d_evx, tx, s);
    upload(c->d_evy, ty, s);
    c->d_f.ensure((size_t)ns * ncols * sizeof(double));
    c->d_c.ensure((size_t)ns * ncols * sizeof(double));
    c->d_res.ensure((size_t)ns * ncols * sizeof(double));
    c->d_evu.ensure((size_t)2 * nt * ncols * sizeof(double));
    c->d_evpart.ensure(std::max<size_t>(eval_scratch_doubles(c->N, nt, ncols), 1) * sizeof(double));
    HIP_CHECK(hipMemcpyAsync(c->d_f.p, x, (size_t)ns * ncols * sizeof(double), hipMemcpyHostToDevice, s));
    launch_to_rows(c->d_f.as<double>(), ns, ns, ncols, c->d_c.as<double>(), s);
    const int cfg = apply_config_for(c, ncols, c->d_c.as<double>(), c->d_res.as<double>());
    Geo g;
    geo_of(c, g);
    {
      KTimer kt_(c, "evaluate");
      launch_evaluate(g, c->d_hole.as<double>(), c->p, c->d_evx.as<double>(), c->d_evy.as<double>(), nt,
                      c->d_c.as<double>(), ncols, c->d_evu.as<double>(), c->d_evpart.as<double>(), cfg, s);
    }
    c->d_res.ensure((size_t)2 * nt * ncols * sizeof(double));
    launch_from_rows(c->d_evu.as<double>(), 2 * nt, ncols, c->d_res.as<double>(), 2 * nt, s);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipMemcpyAsync(u, c->d_res.p, (size_t)2 * nt * ncols * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    resolve_timers(c);
    return RS_OK;
  } catch (const RsError& e) {
    return fail(c, e);
  }
}

rs_status rs_dense_inverse(rs_ctx* c, int n, const double* a, double* ainv) {
  if (!c) return RS_ERR_ARG;
  try {
    if (n <= 0 || !a || !ainv) throw RsError{RS_ERR_ARG, "bad size or NULL pointer"};
    const size_t nn = (size_t)n * n;
    if (!finite_all(a, nn)) throw RsError{RS_ERR_ARG, "non-finite matrix entry"};
    HIP_CHECK(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    DevBuf dA, dAi, dW, dI, dS;
    dA.ensure(nn * sizeof(double));
    dAi.ensure(nn * sizeof(double));
    dW.ensure(((size_t)3 * n * 32 + 32 * 32) * sizeof(double));
    dI.ensure(((size_t)n + 32) * sizeof(int));
    dS.ensure(sizeof(int));
    HIP_CHECK(hipMemcpyAsync(dA.p, a, nn * sizeof(double), hipMemcpyHostToDevice, s));
    launch_gj_blocked(dA.as<double>(), n, dAi.as<double>(), dW.as<double>(), dI.as<int>(),
                      dS.as<int>(), s);
    HIP_CHECK(hipGetLastError());
    int st = 0;
    HIP_CHECK(hipMemcpyAsync(&st, dS.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (st) throw RsError{RS_ERR_SINGULAR, "matrix is singular"};
    HIP_CHECK(hipMemcpyAsync(ainv, dAi.p, nn * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    return RS_OK;
  } catch (const RsError& e) {
    return fail(c, e);
  }
}

}  // extern "C"

namespace {

// Checks of one update's inputs (nothing is changed).
void validate_update(const rs_ctx* c, int n_moved, const int* idx, const double* xy, const double* normal,
                     const double* weight, const double* curvature, const double* hole_xy) {
  if (!c->factored) throw RsError{RS_ERR_STATE, "rs_update_moved_nodes before rs_factor"};
  if (n_moved < 0 || (n_moved > 0 && !idx)) throw RsError{RS_ERR_ARG, "bad moved-node list"};
  if (n_moved) validate_nodes(n_moved, xy, normal, weight, curvature);
  std::vector<char> seen(c->N, 0);
  for (int t = 0; t < n_moved; ++t) {
    if (idx[t] < 0 || idx[t] >= c->N) throw RsError{RS_ERR_ARG, "moved index out of range"};
    if (seen[idx[t]]) throw RsError{RS_ERR_ARG, "duplicate moved index"};
    seen[idx[t]] = 1;
    if (!inside_root(c, xy[2 * t], xy[2 * t + 1]))
      throw RsError{RS_ERR_OUT_OF_ROOT, "moved node leaves the root square"};
  }
  if (hole_xy && !finite_all(hole_xy, 2 * (size_t)c->p)) throw RsError{RS_ERR_ARG, "non-finite hole point"};
}

// Moves the nodes, keeps the previous factorization in O (boxes matched by
// position) and rebuilds the tree on the same root square; the factorization
// that follows reads O through c->old.
void begin_update(rs_ctx* c, int n_moved, const int* idx, const double* xy, const double* normal,
                  const double* weight, const double* curvature, const double* hole_xy, OldState& O) {
  for (int t = 0; t < n_moved; ++t) {
    const int i = idx[t];
    c->x[i] = xy[2 * t];
    c->y[i] = xy[2 * t + 1];
    c->nx[i] = normal[2 * t];
    c->ny[i] = normal[2 * t + 1];
    c->w[i] = weight[t];
    c->kap[i] = curvature[t];
  }
  if (hole_xy) c->hole.assign(hole_xy, hole_xy + 2 * (size_t)c->p);
  HIP_CHECK(hipSetDevice(c->device));
  O.boxes = std::move(c->boxes);
  O.fac = std::move(c->fac);
  for (size_t b = 0; b < O.boxes.size(); ++b)
    O.by_key[BoxKey{O.boxes[b].level, O.boxes[b].ix, O.boxes[b].iy}] = (int)b;
  O.moved.assign(c->N, 0);
  for (int t = 0; t < n_moved; ++t) O.moved[idx[t]] = 1;
  c->prm.has_root = 1;
  c->prm.root[0] = c->root_cx;
  c->prm.root[1] = c->root_cy;
  c->prm.root[2] = c->root_side;
  build_tree(c);
  upload_geometry(c);
  c->old = &O;
}

// Update after curves were inserted or deleted: validate the new boundary and
// the node correspondence, carry the old tree's index sets into the new
// numbering (deleted nodes map to values no new index takes, so any set that
// held one differs), and install the new geometry.
void begin_update_geometry(rs_ctx* c, int n_nodes, const double* xy, const double* normal,
                           const double* weight, const double* curvature, const int* curve_id, int n_holes,
                           const double* hole_xy, const int* old_of_new, OldState& O) {
  if (n_nodes <= 0 || n_holes < 0 || !curve_id || !old_of_new)
    throw RsError{RS_ERR_ARG, "bad n_nodes or n_holes, or NULL curve_id / old_of_new"};
  if (c->prm.kernel == 1 && n_holes != 0)
    throw RsError{RS_ERR_ARG, "the Laplace Neumann kernel has no augmentation: n_holes must be 0"};
  HTimer htv_(c, "host:upd.validate");
  validate_nodes(n_nodes, xy, normal, weight, curvature);
  std::vector<int> count(n_holes + 1, 0);
  for (int i = 0; i < n_nodes; ++i) {
    if (curve_id[i] < 0 || curve_id[i] > n_holes) throw RsError{RS_ERR_ARG, "curve_id out of range"};
    count[curve_id[i]]++;
  }
  for (int h = 1; h <= n_holes; ++h)
    if (!count[h]) throw RsError{RS_ERR_ARG, "hole " + std::to_string(h) + " has no nodes"};
  if (hole_xy && !finite_all(hole_xy, 2 * (size_t)n_holes)) throw RsError{RS_ERR_ARG, "non-finite hole point"};
  const int n_old = c->N;
  std::vector<int> new_of_old(n_old, -1);
  int last = -1;
  for (int j = 0; j < n_nodes; ++j) {
    const int o = old_of_new[j];
    if (o < -1 || o >= n_old) throw RsError{RS_ERR_ARG, "old_of_new entry out of range"};
    if (o < 0) continue;
    if (o <= last) throw RsError{RS_ERR_ARG, "kept nodes must keep their relative order"};
    last = o;
    if (xy[2 * j] != c->x[o] || xy[2 * j + 1] != c->y[o] || normal[2 * j] != c->nx[o] ||
        normal[2 * j + 1] != c->ny[o] || weight[j] != c->w[o] || curvature[j] != c->kap[o])
      throw RsError{RS_ERR_ARG, "kept node " + std::to_string(j) + " changed its data"};
    new_of_old[o] = j;
  }
  for (int i = 0; i < n_nodes; ++i)
    if (!inside_root(c, xy[2 * i], xy[2 * i + 1]))
      throw RsError{RS_ERR_OUT_OF_ROOT, "node " + std::to_string(i) + " lies outside the fixed root"};
  HIP_CHECK(hipSetDevice(c->device));
  HTimer htt_(c, "host:upd.translate");
  auto node_new = [&](int o) { return new_of_old[o] >= 0 ? new_of_old[o] : -2 - o; };
  auto dof_new = [&](int d) { return new_of_old[d >> 1] >= 0 ? 2 * new_of_old[d >> 1] + (d & 1) : -2 - d; };
  O.boxes = std::move(c->boxes);
  O.fac = std::move(c->fac);
  for (size_t b = 0; b < O.boxes.size(); ++b) {
    const Box& B = O.boxes[b];
    O.by_key[BoxKey{B.level, B.ix, B.iy}] = (int)b;
  }
  HostPool::instance().run((int)O.boxes.size(), [&](int b) {
    Box& B = O.boxes[b];
    for (int& j : B.nodes) j = node_new(j);
    BoxFac& F = O.fac[b];
    bool gone = false;
    for (int& d : F.I) {
      d = dof_new(d);
      gone |= d < 0;
    }
    for (int& d : F.fint) d = dof_new(d);
    if (gone) F.active = false;      // its unknowns changed: recompressed
  });
  O.moved.assign(n_nodes, 0);
  for (int j = 0; j < n_nodes; ++j) O.moved[j] = old_of_new[j] < 0;
  c->N = n_nodes;
  c->p = n_holes;
  c->x.resize(n_nodes);
  c->y.resize(n_nodes);
  c->nx.resize(n_nodes);
  c->ny.resize(n_nodes);
  for (int i = 0; i < n_nodes; ++i) {
    c->x[i] = xy[2 * i];
    c->y[i] = xy[2 * i + 1];
    c->nx[i] = normal[2 * i];
    c->ny[i] = normal[2 * i + 1];
  }
  c->w.assign(weight, weight + n_nodes);
  c->kap.assign(curvature, curvature + n_nodes);
  c->curve.assign(curve_id, curve_id + n_nodes);
  c->hole.assign(2 * (size_t)n_holes, 0.0);
  for (int h = 0; h < n_holes; ++h) {
    if (hole_xy) {
      c->hole[2 * h] = hole_xy[2 * h];
      c->hole[2 * h + 1] = hole_xy[2 * h + 1];
    } else {
      double sx = 0, sy = 0;
      for (int i = 0; i < n_nodes; ++i)
        if (curve_id[i] == h + 1) { sx += c->x[i]; sy += c->y[i]; }
      c->hole[2 * h] = sx / count[h + 1];
      c->hole[2 * h + 1] = sy / count[h + 1];
    }
  }
  c->prm.has_root = 1;
  c->prm.root[0] = c->root_cx;
  c->prm.root[1] = c->root_cy;
  c->prm.root[2] = c->root_side;
  {
    HTimer ht_(c, "host:upd.tree");
    build_tree(c);
  }
  {
    HTimer ht_(c, "host:upd.upload");
    upload_geometry(c);
  }
  c->stats.n_nodes = n_nodes;
  c->stats.n_holes = n_holes;
  c->old = &O;
}

}  // namespace

extern "C" {

rs_status rs_update_moved_nodes(rs_ctx* c, int n_moved, const int* idx, const double* xy,
                                const double* normal, const double* weight, const double* curvature,
                                const double* hole_xy) {
  if (!c) return RS_ERR_ARG;
  try {
    validate_update(c, n_moved, idx, xy, normal, weight, curvature, hole_xy);
    auto t0 = std::chrono::steady_clock::now();
    OldState O;
    begin_update(c, n_moved, idx, xy, normal, weight, curvature, hole_xy, O);
    try {
      do_factor(c);
    } catch (...) {
      c->old = nullptr;
      throw;
    }
    c->old = nullptr;
    c->stats.ms_update = 1e3 * seconds_since(t0);
    return RS_OK;
  } catch (const RsError& e) {
    c->factored = false;
    return fail(c, e);
  }
}

rs_status rs_update_geometry(rs_ctx* c, int n_nodes, const double* xy, const double* normal,
                             const double* weight, const double* curvature, const int* curve_id, int n_holes,
                             const double* hole_xy, const int* old_of_new) {
  if (!c) return RS_ERR_ARG;
  try {
    if (!c->factored) throw RsError{RS_ERR_STATE, "rs_update_geometry before rs_factor"};
    auto t0 = std::chrono::steady_clock::now();
    OldState O;
    begin_update_geometry(c, n_nodes, xy, normal, weight, curvature, curve_id, n_holes, hole_xy, old_of_new, O);
    try {
      do_factor(c);
    } catch (...) {
      c->old = nullptr;
      throw;
    }
    c->old = nullptr;
    c->stats.n_levels = c->L + 1;
    c->stats.n_boxes = (int)c->boxes.size();
    c->stats.ms_update = 1e3 * seconds_since(t0);
    return RS_OK;
  } catch (const RsError& e) {
    // argument errors leave the context untouched; a failure past them leaves
    // it unfactored (the old factorization has been taken apart)
    if (e.st != RS_ERR_ARG && e.st != RS_ERR_OUT_OF_ROOT) c->factored = false;
    return fail(c, e);
  }
}

rs_status rs_update_moved_nodes_batch(rs_ctx** ctxs, int n, const int* n_moved, const int* const* idx,
                                      const double* const* xy, const double* const* normal,
                                      const double* const* weight, const double* const* curvature,
                                      const double* const* hole_xy) {
  if (!ctxs || n <= 0 || !n_moved || !idx || !xy || !normal || !weight || !curvature) return RS_ERR_ARG;
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return RS_ERR_ARG;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return fail(ctxs[i], RsError{RS_ERR_ARG, "a context appears twice in the batch"});
    const rs_params& a = ctxs[0]->prm;
    const rs_params& b = ctxs[i]->prm;
    if (ctxs[i]->device != ctxs[0]->device)
      return fail(ctxs[i], RsError{RS_ERR_ARG, "contexts of a batch must share the device"});
    if (a.tol != b.tol || a.n_proxy != b.n_proxy || a.proxy_ratio != b.proxy_ratio || a.lambda != b.lambda ||
        a.rcond_min != b.rcond_min || a.precision != b.precision)
      return fail(ctxs[i], RsError{RS_ERR_ARG, "contexts of a batch must share lambda, tol, proxy, rcond and precision"});
  }
  for (int i = 0; i < n; ++i) {
    try {
      validate_update(ctxs[i], n_moved[i], idx[i], xy[i], normal[i], weight[i], curvature[i],
                      hole_xy ? hole_xy[i] : nullptr);
    } catch (const RsError& e) {
      return fail(ctxs[i], e);
    }
  }
  std::vector<rs_ctx*> cs(ctxs, ctxs + n);
  std::vector<OldState> Os(n);
  auto t0 = std::chrono::steady_clock::now();
  try {
    // the contexts' new trees and geometry uploads are independent: one host
    // thread each
    HostPool::instance().run_tasks(n, [&](int i) {
      begin_update(cs[i], n_moved[i], idx[i], xy[i], normal[i], weight[i], curvature[i],
                   hole_xy ? hole_xy[i] : nullptr, Os[i]);
    });
    do_factor_multi(cs);
  } catch (const RsError& e) {
    rs_status st = RS_OK;
    for (rs_ctx* c : cs) {
      c->old = nullptr;
      c->factored = false;
      st = fail(c, e);
    }
    return st;
  }
  const double ms = 1e3 * seconds_since(t0);
  for (rs_ctx* c : cs) {
    c->old = nullptr;
    c->stats.ms_update = ms;
  }
  return RS_OK;
}

rs_status rs_set_stream(rs_ctx* c, void* stream) {
  if (!c) return RS_ERR_ARG;
  if (c->stream != static_cast<hipStream_t>(stream) && hipStreamSynchronize(c->stream) != hipSuccess) {
    c->err = "rs_set_stream: synchronising the previous stream failed";
    return RS_ERR_DEVICE;
  }
  c->stream = static_cast<hipStream_t>(stream);
  return RS_OK;
}

rs_status rs_get_stats(const rs_ctx* c, rs_stats* out) {
  if (!c || !out) return RS_ERR_ARG;
  *out = c->stats;
  return RS_OK;
}

void rs_reset_tuning(void) {
  {
    ShapeTuneCache& tc = shape_tune_cache();
    std::lock_guard<std::mutex> lk(tc.mu);
    tc.t.clear();
  }
  ApplyTuneCache& ta = apply_tune_cache();
  std::lock_guard<std::mutex> lk(ta.mu);
  ta.best.clear();
}

rs_status rs_get_boxes(const rs_ctx* c, int cap, int* n_boxes, int* level, int* n_active, int* rank,
                       double* box_geom) {
  if (!c || !n_boxes) return RS_ERR_ARG;
  const int nb = (int)c->boxes.size();
  *n_boxes = nb;
  if (cap < nb) {
    const_cast<rs_ctx*>(c)->err = "capacity smaller than the number of boxes";
    return RS_ERR_ARG;
  }
  for (int b = 0; b < nb; ++b) {
    const Box& B = c->boxes[b];
    if (level) level[b] = B.level;
    int n = -1, k = -1;
    if (c->factored) {
      if (b == 0) {
        n = (int)c->I0.size();
        k = n;
      } else if (c->fac[b].n > 0) {
        n = c->fac[b].n;
        k = c->fac[b].k;
      }
    }
    if (n_active) n_active[b] = n;
    if (rank) rank[b] = k;
    if (box_geom) {
      box_geom[3 * b] = B.cx;
      box_geom[3 * b + 1] = B.cy;
      box_geom[3 * b + 2] = B.side;
    }
  }
  return RS_OK;
}

rs_status rs_get_skeleton(const rs_ctx* c, int box, int cap, int* out, int* len) {
  if (!c || !len) return RS_ERR_ARG;
  if (!c->factored) {
    const_cast<rs_ctx*>(c)->err = "no factorization";
    return RS_ERR_STATE;
  }
  if (box < 0 || box >= (int)c->boxes.size()) {
    const_cast<rs_ctx*>(c)->err = "box index out of range";
    return RS_ERR_ARG;
  }
  std::vector<int> s = box == 0 ? c->I0 : skeleton_of(c->fac[box]);
  *len = (int)s.size();
  if (cap < (int)s.size() || (!out && !s.empty())) {
    const_cast<rs_ctx*>(c)->err = "capacity smaller than the skeleton";
    return RS_ERR_ARG;
  }
  std::copy(s.begin(), s.end(), out);
  return RS_OK;
}

rs_status rs_set_kernel_timing(rs_ctx* c, int enable) {
  if (!c) return RS_ERR_ARG;
  c->timing = enable < 0 ? 0 : (enable > 4 ? 4 : enable);
  return RS_OK;
}

rs_status rs_get_kernel_times(rs_ctx* c, int cap, rs_kernel_time* out, int* n, int reset) {
  if (!c || !n) return RS_ERR_ARG;
  try {
    HIP_CHECK(hipStreamSynchronize(c->stream));
    resolve_timers(c);
  } catch (const RsError& e) {
    return fail(c, e);
  }
  const int nf = (int)c->fam_name.size();
  *n = nf;
  for (int i = 0; i < nf && i < cap && out; ++i) {
    std::memset(out[i].name, 0, sizeof(out[i].name));
    std::strncpy(out[i].name, c->fam_name[i].c_str(), sizeof(out[i].name) - 1);
    out[i].launches = c->fam_launches[i];
    out[i].total_ms = c->fam_ms[i];
  }
  if (reset) {
    std::fill(c->fam_launches.begin(), c->fam_launches.end(), 0);
    std::fill(c->fam_ms.begin(), c->fam_ms.end(), 0.0);
  }
  return RS_OK;
}

void rs_destroy(rs_ctx* c) { delete c; }

const char* rs_last_error(const rs_ctx* c) { return c ? c->err.c_str() : g_build_error.c_str(); }

}  // extern "C"

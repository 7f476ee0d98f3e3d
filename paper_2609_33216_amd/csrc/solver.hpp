// Host driver of the HSS solver: box tree, proxy/near-field planning, work
// lists and the per-level launch sequence of compress, factor and solve.
#pragma once

#include <algorithm>
#include <chrono>
#include <functional>
#include <string>
#include <unordered_map>
#include <vector>

#include "bessel.hpp"
#include "kernels.hpp"
#include "mlp.hpp"
#include "../../include/symhss.h"

namespace symhss {

// Device memory of one context: the bytes its work buffers hold, and an
// optional limit (0: none) beyond which an allocation fails as if the device
// were full.  A call into a context makes its budget the thread's current one.
struct DeviceBudget {
  size_t used = 0, limit = 0;
};
inline thread_local DeviceBudget* tl_budget = nullptr;
struct BudgetScope {
  DeviceBudget* prev;
  explicit BudgetScope(DeviceBudget* b) : prev(tl_budget) { tl_budget = b; }
  ~BudgetScope() { tl_budget = prev; }
};

// A refinement that ended at its iteration limit above its target (the
// iterate is still returned).
struct NotConverged : std::runtime_error {
  using std::runtime_error::runtime_error;
};

// Device allocation owned by the context (charged to the budget current when
// it was made).
template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DeviceBudget* charged = nullptr;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n), charged(o.charged) {
    o.p = nullptr;
    o.n = 0;
    o.charged = nullptr;
  }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      charged = o.charged;
      o.p = nullptr;
      o.n = 0;
      o.charged = nullptr;
    }
    return *this;
  }
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    if (charged) charged->used -= std::min(charged->used, n * sizeof(T));
    p = nullptr;
    n = 0;
    charged = nullptr;
  }
  void ensure(size_t m) {
    if (m <= n) return;
    release();
    if (m == 0) return;
    DeviceBudget* b = tl_budget;
    if (b && b->limit && b->used + m * sizeof(T) > b->limit) throw std::bad_alloc();
    if (hipMalloc(&p, m * sizeof(T)) != hipSuccess) {
      p = nullptr;
      throw std::bad_alloc();
    }
    n = m;
    charged = b;
    if (b) b->used += m * sizeof(T);
  }
  size_t bytes() const { return n * sizeof(T); }
};

// Staging of descriptor and index arrays: pinned host memory copied to
// device chunks on the context's stream.  Chunks live until reset(), which the
// driver calls only after the stream has drained.
class Uploader {
 public:
  Uploader() = default;
  Uploader(const Uploader&) = delete;
  Uploader& operator=(const Uploader&) = delete;
  ~Uploader();
  void set_stream(hipStream_t st) { st_ = st; }
  template <class T>
  T* put(const std::vector<T>& v) {
    return static_cast<T*>(put_bytes(v.data(), v.size() * sizeof(T)));
  }
  void* put_bytes(const void* src, size_t bytes);
  // Several arrays in one copy: stage() reserves staging space (h: host
  // address, hd: the same bytes as the device reads them, d: the device
  // copy), the caller fills h, and commit() queues the copy from h to d.  A
  // kernel of the caller's may instead read hd directly, without commit().
  struct Span {
    char* h;
    char* hd;
    char* d;
    size_t bytes;
  };
  Span stage(size_t bytes);
  void commit(const Span& s);
  void reset();
  size_t used() const;
  // one chunk with at least `bytes` free, so that later puts allocate nothing
  void reserve(size_t bytes);

 private:
  struct Chunk {
    char* d;
    char* h;   // pinned staging
    char* hd;  // the staging as the device addresses it
    size_t cap, used;
  };
  hipStream_t st_ = nullptr;
  std::vector<Chunk> chunks_;
  Chunk& new_chunk(size_t cap);
};

// Workspace of the multi-workgroup LU for one batched launch: F, the row
// positions and counters, the panel's triangular inverses.
template <class C>
struct CaluWs {
  DBuf<C> F, tw;
  DBuf<int> iw;
  // size the buffers for the descriptors and point each descriptor at its part
  template <class D>
  void attach(std::vector<D>& v) {
    size_t fe = 0, ie = 0, te = 0;
    for (const D& d : v) {
      fe += (size_t)d.n * d.ncol;
      ie += (size_t)calu_iw_ints(d.n);
      te += (size_t)calu_tw_elems(d.ncol);
    }
    F.ensure(std::max<size_t>(fe, 1));
    iw.ensure(std::max<size_t>(ie, 1));
    tw.ensure(std::max<size_t>(te, 1));
    fe = ie = te = 0;
    for (D& d : v) {
      d.F = F.p + fe;
      d.iw = iw.p + ie;
      d.tw = tw.p + te;
      fe += (size_t)d.n * d.ncol;
      ie += (size_t)calu_iw_ints(d.n);
      te += (size_t)calu_tw_elems(d.ncol);
    }
  }
};

// Geometry of one box of a boundary's full binary tree.
struct BoxGeom {
  int lo = 0, hi = 0;  // node range (global node ids)
  double cx = 0, cy = 0, rad = 0;
  double kmean = 0, kmax = 0;  // mean and largest |curvature| over its nodes
};

struct Box {
  int lo = 0, hi = 0;         // node range of the box
  double cx = 0, cy = 0, rad = 0;
  int tree = 0;               // boundary of a batch
  int li = 0;                 // index among its tree's boxes at this height
  double kmean = 0, kmax = 0; // |curvature| statistics of its nodes
  std::vector<int> rows[2];   // active row node ids: first / second equation
  std::vector<int> cols[2];   // active column node ids: q / u unknowns
  std::vector<int> rsk[2];    // row skeleton: local indices into rows[h]
  std::vector<int> csk[2];    // column skeleton: local indices into cols[h]
  std::vector<int> nearr[2];  // near-field rows (node ids) for M_R
  std::vector<int> nearc[2];  // near-field columns (node ids) for M_L
  double Rp = 0;
  int np = 0;
  int np_rule = 0;            // proxy count of the rule (without the predictor)
  int khat = 0;               // predicted rank (0: no prediction)
  int sr() const { return (int)(rows[0].size() + rows[1].size()); }
  int sc() const { return (int)(cols[0].size() + cols[1].size()); }
  int kc() const { return (int)(csk[0].size() + csk[1].size()); }
  int kr() const { return (int)(rsk[0].size() + rsk[1].size()); }
  // offsets (elements) into the level's buffers
  size_t off_R = 0, off_L = 0, off_aug1 = 0, off_aug2 = 0;
  size_t off_piv1 = 0, off_piv2 = 0;
  size_t off_s = 0, off_k = 0;  // prefix sums of s and k (solve buffers, maps)
  size_t off_gen = 0;           // mixed precision: s x s generator block
};

// All boxes at one height of the forest (height 0: leaves).  The boxes of a
// tree are contiguous and in curve order, so the children of box li of tree t
// at height h are boxes 2 li and 2 li + 1 of t at height h - 1.
struct Level {
  std::vector<Box> boxes;
  std::vector<int> tstart;  // per tree: index of its first box here, -1 if absent
  DBuf<cplx> interp;     // R and L of every box
  DBuf<cplx> aug1;       // [D | L] -> [LU(D) | X]
  DBuf<cplx> aug2;       // [R X | I] -> [LU | A~]
  DBuf<int> piv;         // pivots of both factorisations
  DBuf<int> info;        // 2 per box
  DBuf<int> childmap;    // per box (levels >= 1): positions of its k unknowns in the parent
  DBuf<int> leafmap;     // leaves: global indices of the 2n local unknowns
  DBuf<int> rootmap;     // boxes of trees whose dense top-level system is at this height:
                         // positions of their unknowns in that system
  // solve buffers
  DBuf<cplx> F, G, Ft, Z;
  // mixed precision: FP64 generator blocks (leaf D, parent sibling blocks,
  // s x s per box) for the FP64 HSS product, and the FP32 factorisation
  DBuf<cplx> gen;
  DBuf<f32::cplx> aug1f, aug2f, interpf;
  DBuf<f32::cplx> Ff, Gf, Ftf, Zf;
  // multi-workgroup LU workspaces of the two factorisations (FP64, FP32)
  CaluWs<cplx> cw1, cw2;
  CaluWs<f32::cplx> cw1f, cw2f;
  int netperm1 = 0;  // the LU of [D | L] left a net permutation (multi-workgroup LU)
  size_t s_total = 0, k_total = 0;
};

// One boundary of a batch (a single-boundary context holds one).
struct Tree {
  int64_t base = 0, n = 0;  // nodes [base, base + n); unknowns [2 base, 2 base + 2 n)
  int L = 0;                // box-tree levels (leaves at level L, height 0)
  symhss_medium med{};
  MediumDev md{};
  std::vector<std::vector<BoxGeom>> geom;  // per height, the full binary tree
  int root_h = -1;          // height of the dense top-level system
  int root_n = 0;           // its order
  size_t root_off = 0;      // offset of its matrix in the root buffer
  size_t root_inv_off = 0;  // offset of its diagonal-block inverses (blocked substitution)
  size_t rootvec_off = 0;   // offset of its unknowns in the root vectors
};

struct TimerPair {
  hipEvent_t a, b;
  int what;      // 0 kblock-compress, 1 kblock-factor, 2 id, 3 lu batched, 4 lu multi
  double work;   // algorithmic flops (or bytes for kblock) of the timed launch
};

class Solver {
 public:
  Solver(int device, hipStream_t stream);
  ~Solver();

  void assemble(int64_t n, const double* x, const double* dx, const double* ddx, const symhss_medium& med,
                const symhss_opts& opts);
  // count boundaries of n[t] nodes each, geometry arrays concatenated
  void assemble_batch(int count, const int64_t* n, const double* x, const double* dx, const double* ddx,
                      const symhss_medium* med, const symhss_opts& opts);
  void compress();
  void factor();
  void solve(const symhss_z* b, symhss_z* x, int nrhs, int flags);
  // factor, then solve, with the solve's sweep up the levels run beside the
  // top-level LU (pipelined FP64 factorisations; otherwise factor + solve)
  void factor_solve(const symhss_z* b, symhss_z* x, int nrhs, int flags);
  void solve_incident(const symhss_z* uin, const symhss_z* qin, symhss_z* q, symhss_z* u, int nrhs, int flags);
  void plane_wave_incident(const double* angles, symhss_z* uin, symhss_z* qin, int flags);
  void rhs_plane_wave(double angle, symhss_z* b, int flags);
  void rhs_plane_wave_batch(const double* angles, symhss_z* b, int flags);
  void eval_entries(int64_t nr, const int64_t* rows, int64_t nc, const int64_t* cols, symhss_z* out);
  void eval_bessel(int64_t n, const double* z, double* out);
  void matvec_direct(const symhss_z* x, symhss_z* y, int flags);
  void box_query(int level, int box, int what, int64_t* count, void* out);
  void configure(int what, int64_t value);
  void hss_matvec(const symhss_z* x, symhss_z* y, int flags);
  Mlp& predictor() { return mlp_; }
  float* infer_scratch() const { return infer_scratch_; }
  void box_table(int64_t* count, float* feat, int32_t* rank, int32_t* info) const;
  symhss_stats stats() const {
    symhss_stats s = stats_;
    s.tuned_buckets = (int32_t)tuned_.size();
    return s;
  }
  hipStream_t stream() const { return st_; }
  DeviceBudget* budget() { return &budget_; }

  int stage = 0;  // 0 none, 1 assembled, 2 compressed, 3 factored

 private:
  // declared before every device buffer it is charged with, so that it is
  // destroyed after them
  DeviceBudget budget_;
  // planning
  void build_tree();
  void set_active(int h);
  void plan_proxy_near(int h);
  void plan_proxy(int h);  // proxy circles (geometry and the predictor)
  void plan_near(int h);   // near fields (active sets of the neighbours)
  // Height h built ahead, while height h - 1's IDs run: boxes, proxy circles
  // and proxy points of the trees that may continue (those below their last
  // height).  Kept when exactly those trees continue, else rebuilt.
  void preplan(int h);
  int preplanned_h_ = -1;
  std::vector<int> preplanned_trees_;
  // proxy points of the current pass: offsets of each box's points
  void proxy_points(int h, const std::vector<int>& which);
  std::vector<int> prox_off_;
  void add_height(int h, const std::vector<int>& trees);
  int level_of(int h) const { return Lmax_ - h; }
  const Box& child(int h, const Box& B, int w) const {
    return hev_[h - 1].boxes[hev_[h - 1].tstart[B.tree] + 2 * B.li + w];
  }
  // compress pieces
  void compress_impl();
  void compress_level(int h);
  // one generation + ID pass over some boxes of a height
  struct IdPass {
    DBuf<cplx> scratch;     // the boxes' proxy matrices, factored in place
    DBuf<int> idint;        // pivots, then ranks
    DBuf<double> r00;
    std::vector<IdDesc> ds;
    std::vector<size_t> permoff;
    std::vector<int> hint;  // host copy of idint
    std::vector<int> boxes; // box indices of the pass
    size_t ptot = 0;
    int per = 2;
  };
  IdPass pass_[2];  // [0] all boxes, [1] predictor fallbacks
  // points_ready: proxy_points already ran for these boxes
  void proxy_ids(int h, const std::vector<int>& which, IdPass& P, bool points_ready = false);
  void box_features_of(int h, const Box& B, float* f) const;
  // factor pieces
  void factor_impl();
  void factor_layout();
  void factor_layout_level(int h);
  void factor_layout_root();
  // f's launches go to the factor stream, after `after` (null: after
  // everything queued on the compress stream so far)
  void enqueue_on_factor_stream(const std::function<void()>& f, hipEvent_t after = nullptr);
  void queue_pending_factor();
  void factor_level(int h);
  void factor_root();
  void factor_root_blocks();
  void factor_root_lu();
  void factor_enqueue();
  uint64_t plan_signature() const;
  // launches with a choice of variant (autotuned per size bucket when enabled)
  template <class S>
  void run_gemm(const std::vector<typename S::GemmDesc>& g, int count, int mmax, int nmax);
  void run_cpqr(const IdDesc* d, int count, int mmax, int nmax, int want_T, cplx* data, size_t data_elems, int* ints,
                size_t nints, double* dbl, size_t ndbl);
  // returns 1 if the pivots hold the net permutation (the multi-workgroup LU,
  // or k_lu_fused up to order kLuPermLds), 0 for row interchanges; multi_ok:
  // the descriptors carry the multi-workgroup LU's workspace
  int run_lu(const LuDesc* d, int count, int nmax, int ncolmax, int nrhsmax, cplx* data, size_t data_elems,
             double flops, bool multi_ok);
  void solve_enqueue(const cplx* db, cplx* dx, int nrhs);
  // the solve of device vectors (graph replay, mixed-precision refinement);
  // false if a refinement stopped at its iteration limit above its target
  bool solve_device(const cplx* db, cplx* dx, int nrhs, int flags);
  struct Sweep64;
  struct Sweep32;
  template <class S>
  void solve_sweep(const typename S::C* db, typename S::C* dx, int nrhs);
  void root_solve_widened(int nrhs);
  // mixed precision: FP32 factorisation, FP64 HSS product, refinement
  void factor_level_mixed(int h);
  void factor_root_mixed();
  void hss_matvec_enqueue(const cplx* x, cplx* y);
  bool solve_mixed(const cplx* db, cplx* dx, int nrhs);
  void ensure_sweep_buffers(int nrhs, bool fp32);
  // kernel-block launches
  struct KBatch {
    std::vector<KJob> jobs;
    std::vector<int> rpt, rm1, rm2, cpt, cm1, cm2;
    int64_t entries = 0;
    void add(cplx* out, int ld, int mode, int med, const std::vector<int>& rp, const std::vector<int>& r1,
             const std::vector<int>& r2, const std::vector<int>& cp, const std::vector<int>& c1,
             const std::vector<int>& c2);
  };
  void run_kblock(KBatch& kb, int timer_kind);
  // host staging reused from call to call (their lists keep their storage)
  struct JobPiece {
    std::vector<int> rp, r1, r2, cp, c1, c2;
  };
  std::vector<JobPiece> pieces_;  // per-box job lists of the proxy matrices
  KBatch kbw_;                    // the proxy matrices' kernel-block batch
  std::vector<KTile> tiles_;      // tiles of the current kernel-block batch
  void root_block_jobs(KBatch& kb, const Tree& T, int t, cplx* out, int ld, const std::vector<int>& offs);
  PointsDev tree_points(const Tree& T) const;
  PointsDev points() const;
  void upload_proxies(const std::vector<double>& px, const std::vector<double>& py,
                      const std::vector<double>& nx, const std::vector<double>& ny,
                      const std::vector<double>& w);
  void timer_begin(int what, double work = 0.0);
  void timer_end();
  void collect_timers();
  void collect_timers(std::vector<TimerPair>& list);
  void sync();

  int device_;  // HIP device the context was created on
  hipStream_t st_;
  bool own_stream_;
  Uploader up_;          // eager work: reset after every phase
  Uploader fgup_, sgup_;  // descriptors read by the captured factor / solve graphs
  Uploader* upl_ = &up_;
  // geometry
  int64_t n_ = 0;                // nodes of all boundaries
  std::vector<Tree> trees_;
  DBuf<MediumDev> media_;        // one per tree
  int Lmax_ = 0;                 // deepest tree
  std::vector<double> hx_, hy_;  // host copy of the nodes (planning)
  std::vector<double> hk_;       // curvature at the nodes (predictor features)
  Mlp mlp_;
  float* infer_scratch_ = nullptr;  // this device's allocation-free inference scratch
  int use_predictor_ = 0, proxy_margin_ = 16;
  int rank_leaf_ = 0;        // fixed-rank schedule: k_L per half (0: tolerance mode)
  double rank_scale_ = 1.0;  // and the growth a per level
  DBuf<double> geo_;             // px, py, nx, ny, w, kappa, each of capacity cap_
  size_t cap_ = 0;
  symhss_opts opts_{};
  bool two_sided_ = false;
  int Htop_ = 0;            // highest height holding boxes (max over trees of root_h)
  std::vector<Level> hev_;  // index = height (0 = leaves)
  DBuf<cplx> root_;         // dense top-level systems of all trees
  CaluWs<cplx> rootcw_;
  CaluWs<f32::cplx> rootcwf_;
  int root_netperm_ = 0;    // their LU left a net permutation (multi-workgroup LU)
  DBuf<int> rootpiv_, rootinfo_;
  // inverses of the 64 x 64 diagonal blocks of the top-level LU factors, for
  // the blocked substitution of systems of order kTrsvMinOrder and more
  DBuf<cplx> root_inv_;
  DBuf<f32::cplx> root_invf_;
  static constexpr int kTrsvMinOrder = 512;
  void root_invert();
  size_t rootvec_total_ = 0;  // sum of the trees' root orders
  DBuf<cplx> rootF_, rootG_;
  // mixed precision
  int precision_ = 0;               // 0 FP64, 1 FP32 factorisation + FP64 refinement
  // mixed precision: the dense top-level system stays FP64 (its LU and block
  // inverses; the sweeps widen their vector for it and round the result)
  static constexpr bool kMixedRoot64 = true;
  int refine_digits_ = 10, refine_maxit_ = 10;
  DBuf<cplx> root_gen_;             // off-diagonal blocks of the top-level systems (FP64)
  DBuf<f32::cplx> rootf_, rootFf_, rootGf_;
  DBuf<cplx> rwork_;                // residual, product, correction vectors
  DBuf<f32::cplx> rworkf_;
  DBuf<double> norms_;
  DBuf<cplx> vec_;  // staging of b / x for host-pointer solves
  DBuf<cplx> inc_;  // incident data, right-hand sides and solutions of solve_incident
  // execution options (symhss_configure)
  int use_graphs_ = 0, autotune_ = 0, persistent_ = -1;
  int eq_ = kEqMuller;  // which system the entry generator evaluates
  uint64_t unhashed_plans_ = 0;  // compresses run without the structure hash
  // cos / sin of 2 pi i / np, i < np, per proxy count np
  std::unordered_map<int, std::vector<double>> unit_circle_;
  bool capturing_ = false;
  uint64_t plan_sig_ = 0;     // structure produced by the last compress
  uint64_t assemble_gen_ = 0;
  uint64_t fsig_ = 0;         // structure the factor graph was captured for
  int fseen_ = 0;             // factors run with that structure
  hipGraphExec_t fgraph_ = nullptr;
  uint64_t ssig_ = 0;
  int sseen_ = 0;
  hipGraphExec_t sgraph_ = nullptr;
  size_t last_factor_upload_ = 0, last_solve_upload_ = 0;
  double sync_wait_ = 0.0;  // host seconds spent waiting for the stream
  int* pinned_ = nullptr;   // pinned host staging of the ID results
  size_t pinned_cap_ = 0;  // descriptor bytes of the last eager runs
  void drop_graphs();
  // autotuner: size bucket -> chosen variant
  std::vector<std::pair<uint64_t, int>> tuned_;
  int tuned_choice(uint64_t key) const;
  DBuf<cplx> tune_backup_;
  DBuf<int> tune_backup_int_;
  DBuf<double> tune_backup_dbl_;
  DBuf<cplx> tune_backup_lu_;  // LU trials run on the factor stream
  DBuf<int> queue_;
  std::vector<TimerPair> timers_;
  std::vector<TimerPair> ftimers_;           // launches on the factor stream
  std::vector<TimerPair>* tl_ = &timers_;    // where timer_begin records
  // pipelining: per-level factor work on a second stream during compress
  hipStream_t fst_ = nullptr;
  hipEvent_t cev_ = nullptr;
  hipEvent_t fev_ = nullptr;   // end of the compression of height pending_factor_
  // factor_solve: the levels' factorisations done (lev_) and the top-level
  // LU done (rev_), both on the factor stream; root_wait_ = rev_ while a
  // solve must wait for the top level before its top-level part
  hipEvent_t lev_ = nullptr, rev_ = nullptr;
  hipEvent_t root_wait_ = nullptr;
  void solve_impl(const symhss_z* b, symhss_z* x, int nrhs, int flags);
  void factor_finish();  // pivot checks and device-byte statistics
  int pending_factor_ = -1;    // compressed height whose pipelined factorisation is not queued yet
  Uploader fup2_;
  int pipeline_opt_ = 1;
  bool pipelined_ = false;
  int pipelined_precision_ = 0;  // precision the pipelined factorisation was queued in
  std::vector<hipEvent_t> event_pool_;
  symhss_stats stats_{};
};

}  // namespace symhss

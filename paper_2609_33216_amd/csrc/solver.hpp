// Host driver of the HSS solver: box tree, proxy/near-field planning, work
// lists and the per-level launch sequence of compress, factor and solve.
#pragma once

#include <chrono>
#include <string>
#include <vector>

#include "bessel.hpp"
#include "kernels.hpp"
#include "../../include/symhss.h"

namespace symhss {

// Device allocation owned by the context.
template <class T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void ensure(size_t m) {
    if (m <= n) return;
    release();
    if (m == 0) return;
    if (hipMalloc(&p, m * sizeof(T)) != hipSuccess) {
      p = nullptr;
      throw std::bad_alloc();
    }
    n = m;
  }
  size_t bytes() const { return n * sizeof(T); }
};

// Staging of descriptor and index arrays: pinned host memory copied to
// device chunks on the context's stream.  Chunks live until reset(), which the
// driver calls only after the stream has drained.
class Uploader {
 public:
  explicit Uploader(hipStream_t st) : st_(st) {}
  ~Uploader();
  template <class T>
  T* put(const std::vector<T>& v) {
    return static_cast<T*>(put_bytes(v.data(), v.size() * sizeof(T)));
  }
  void* put_bytes(const void* src, size_t bytes);
  void reset();

 private:
  struct Chunk {
    char* d;
    char* h;
    size_t cap, used;
  };
  hipStream_t st_;
  std::vector<Chunk> chunks_;
};

struct Box {
  int lo = 0, hi = 0;         // node range of the box
  double cx = 0, cy = 0, rad = 0;
  std::vector<int> rows[2];   // active row node ids: first / second equation
  std::vector<int> cols[2];   // active column node ids: q / u unknowns
  std::vector<int> rsk[2];    // row skeleton: local indices into rows[h]
  std::vector<int> csk[2];    // column skeleton: local indices into cols[h]
  std::vector<int> nearr[2];  // near-field rows (node ids) for M_R
  std::vector<int> nearc[2];  // near-field columns (node ids) for M_L
  double Rp = 0;
  int np = 0;
  int sr() const { return (int)(rows[0].size() + rows[1].size()); }
  int sc() const { return (int)(cols[0].size() + cols[1].size()); }
  int kc() const { return (int)(csk[0].size() + csk[1].size()); }
  int kr() const { return (int)(rsk[0].size() + rsk[1].size()); }
  // offsets (elements) into the level's buffers
  size_t off_R = 0, off_L = 0, off_aug1 = 0, off_aug2 = 0;
  size_t off_piv1 = 0, off_piv2 = 0;
  size_t off_s = 0, off_k = 0;  // prefix sums of s and k (solve buffers, maps)
};

struct Level {
  std::vector<Box> boxes;
  DBuf<cplx> interp;     // R and L of every box
  DBuf<cplx> aug1;       // [D | L] -> [LU(D) | X]
  DBuf<cplx> aug2;       // [R X | I] -> [LU | A~]
  DBuf<int> piv;         // pivots of both factorisations
  DBuf<int> info;        // 2 per box
  DBuf<int> childmap;    // per box (levels >= 1): positions of its k unknowns in the parent
  DBuf<int> leafmap;     // leaves: global indices of the 2n local unknowns
  // solve buffers
  DBuf<cplx> F, G, Ft, Z;
  size_t s_total = 0, k_total = 0;
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
  void compress();
  void factor();
  void solve(const symhss_z* b, symhss_z* x, int nrhs, int flags);
  void rhs_plane_wave(double angle, symhss_z* b, int flags);
  void eval_entries(int64_t nr, const int64_t* rows, int64_t nc, const int64_t* cols, symhss_z* out);
  void eval_bessel(int64_t n, const double* z, double* out);
  void matvec_direct(const symhss_z* x, symhss_z* y, int flags);
  void box_query(int level, int box, int what, int64_t* count, void* out);
  symhss_stats stats() const { return stats_; }
  hipStream_t stream() const { return st_; }

  int stage = 0;  // 0 none, 1 assembled, 2 compressed, 3 factored

 private:
  // planning
  void build_tree();
  void set_active(int l);
  void plan_proxy_near(int l);
  // compress pieces
  void compress_level(int l);
  // factor pieces
  void factor_level(int l);
  void factor_root();
  // kernel-block launches
  struct KBatch {
    std::vector<KJob> jobs;
    std::vector<int> rpt, rm1, rm2, cpt, cm1, cm2;
    int64_t entries = 0;
    void add(cplx* out, int ld, int mode, const std::vector<int>& rp, const std::vector<int>& r1,
             const std::vector<int>& r2, const std::vector<int>& cp, const std::vector<int>& c1,
             const std::vector<int>& c2);
  };
  void run_kblock(KBatch& kb, int timer_kind);
  void root_block_jobs(KBatch& kb, cplx* out, int ld, const std::vector<int>& offs);
  PointsDev points() const;
  void upload_proxies(const std::vector<double>& px, const std::vector<double>& py,
                      const std::vector<double>& nx, const std::vector<double>& ny,
                      const std::vector<double>& w);
  void timer_begin(int what, double work = 0.0);
  void timer_end();
  void collect_timers();
  void sync();

  int device_;  // HIP device the context was created on
  hipStream_t st_;
  bool own_stream_;
  Uploader up_;
  // geometry
  int64_t n_ = 0;
  std::vector<double> hx_, hy_;  // host copy of the nodes (planning)
  DBuf<double> geo_;             // px, py, nx, ny, w, kappa, each of capacity cap_
  size_t cap_ = 0;
  symhss_medium med_{};
  symhss_opts opts_{};
  MediumDev md_{};
  bool two_sided_ = false;
  int L_ = 0;
  int root_level_ = 1;      // level whose compressed system is factored densely
  std::vector<Level> lev_;  // index = level 0..L
  DBuf<int> rootmap_;       // per box of the root level: positions of its unknowns in the root system
  DBuf<cplx> scratch_;      // proxy matrices of one level
  DBuf<IdDesc> iddesc_;
  DBuf<int> idint_;
  DBuf<double> idr00_;
  DBuf<cplx> root_;
  DBuf<int> rootpiv_, rootinfo_;
  int root_n_ = 0;
  DBuf<cplx> vec_;  // staging of b / x for host-pointer solves
  std::vector<TimerPair> timers_;
  std::vector<hipEvent_t> event_pool_;
  symhss_stats stats_{};
};

}  // namespace symhss

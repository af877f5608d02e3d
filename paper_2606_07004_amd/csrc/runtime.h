// Host runtime of liblogdet: contexts, the device-resident matrix registry
// and the estimate pipeline.  Internal header (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/liblogdet.h"
#include "ld_kernels.h"

namespace ld {

// Thread-local error text behind ld_last_error().
ld_status set_error(ld_status st, const std::string& msg);

// Device memory with a byte ledger.
struct DeviceBuffer {
  void* ptr = nullptr;
  size_t bytes = 0;
  ~DeviceBuffer();
  hipError_t ensure(size_t want);  // grow-only
  void release();
};

class Server;

// Identity of a blocking estimate's launch sequence: the matrix (its serial
// number and autotune version), every parameter except the seed (the probe
// kernels read it from device memory), and the workspace the buffers live in.
struct GraphKey {
  uint64_t serial = 0, tune_ver = 0;
  int32_t method = 0, precision = 0, n_probes = 0, sketch_rank = 0, krylov_steps = 0;
  int32_t iop_window = 0, probe_dist = 0, subspace_rank = 0, adapt_every = 0, sketch_passes = 0;
  double tol = 0, adapt_tol = 0;
  const void* ws = nullptr;
  size_t ws_bytes = 0;
  bool operator==(const GraphKey& o) const;
};

// Captured estimates of a context, least recently used dropped beyond kMax.
struct GraphCache {
  static constexpr int kMax = 8;
  static constexpr int kSeen = 16;
  struct Entry {
    GraphKey key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t last = 0;
  };
  std::vector<Entry> entries;
  std::deque<GraphKey> seen;  // keys run once without a graph (capture on the next)
  int mode = 1;
  bool failed = false;  // a capture failed: graphs switched off for the context
  uint64_t tick = 0, captures = 0, replays = 0, eager = 0;
  ~GraphCache() { clear(); }
  Entry* find(const GraphKey& k);
  bool seen_before(const GraphKey& k);  // records k when not
  hipError_t insert(const GraphKey& k, hipGraph_t g, hipGraphExec_t x);
  void drop_matrix(uint64_t serial);
  void drop_workspace();
  void clear();
};

// Host -> device uploads through two pinned staging buffers: host threads
// fill one while the other is in flight (pageable sources reach only a part
// of the link rate).  Created on the first large upload of a context.
struct Stager {
  static constexpr size_t kChunk = (size_t)64 << 20;
  char* buf[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipStream_t st = nullptr;
  ~Stager();
  hipError_t init();
  hipError_t upload(void* dst, const void* src, size_t bytes);
  // bytes of device data produced on the host chunk by chunk: fill(buf, off,
  // len) writes bytes off .. off+len-1 into the pinned buffer buf
  hipError_t upload_fill(void* dst, size_t bytes,
                         const std::function<void(char*, size_t, size_t)>& fill);
};

// Event-bracketed launch timing per kernel family (see ld_profile_enable).
class Profiler {
 public:
  ~Profiler();
  void enable(uint32_t mask);
  bool on(uint32_t fam) const { return (mask_ & fam) != 0; }
  bool any() const { return mask_ != 0; }
  hipError_t begin(uint32_t fam, hipStream_t st, hipEvent_t* a);
  hipError_t end(uint32_t fam, hipStream_t st, hipEvent_t a, double bytes);
  hipError_t harvest();  // waits for pending events and accumulates
  void query(uint32_t fam, int64_t* n, double* ms, double* bytes);

 private:
  hipEvent_t get_event();
  struct Pending {
    int fam_bit;
    hipEvent_t a, b;
    double bytes;
  };
  std::mutex mu_;
  uint32_t mask_ = 0;
  std::vector<Pending> pending_;
  std::vector<hipEvent_t> pool_;
  int64_t count_[8] = {};
  double ms_[8] = {};
  double bytes_[8] = {};
};

}  // namespace ld

struct ld_ctx {
  ld_ctx();
  ~ld_ctx();  // defined where ld::Server is complete
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  ld_ctx_opts opts{};
  std::mutex est_mu;             // blocking estimates share the stream and workspace
  ld::DeviceBuffer workspace;
  std::atomic<int> n_matrices{0};
  std::unique_ptr<ld::Server> server;
  std::mutex server_mu;
  ld::Profiler prof;
  std::mutex stage_mu;
  std::unique_ptr<ld::Stager> stager;
  // the blocking estimates' timing events, adaptive-check event, pinned
  // count of active runs and pinned result buffer, created with the context
  // (the blocking estimates run one at a time under est_mu)
  hipEvent_t na_ev[3] = {nullptr, nullptr, nullptr};
  int* na_nact = nullptr;
  void* na_pack = nullptr;
  ld::GraphCache graphs;         // captured blocking estimates (under est_mu)
};

struct ld_matrix {
  ld_ctx* ctx = nullptr;
  int64_t n = 0, nnz = 0;
  int* rp = nullptr;
  int* ci = nullptr;
  double* v64 = nullptr;    // FP64 values (LD_PREC_FP64 runs)
  void* vlo = nullptr;      // FP32 or BF16 values (LD_PREC_MIXED runs)
  int vt_lo = 1;            // storage type of vlo (VT_F32 or VT_BF16)
  int vt = 0;               // requested ld_value_type
  double glo = 0, ghi = 0;  // Gershgorin bounds
  // Gershgorin block partials, kept with the matrix: freeing device memory
  // synchronises the device, which would make a matrix created while
  // requests run wait for them
  double* gpart = nullptr;
  // row groups (FP32 or FP64 storage, where they gather much less than the
  // rows): group pointers, union columns and kRowGroup values per union
  // column, FP64 and (FP32 storage) FP32
  int* rg_gp = nullptr;
  int* rg_col = nullptr;
  float* rg_val = nullptr;
  double* rg_val64 = nullptr;
  int64_t rg_nu = 0;
  int* rg_unused = nullptr;  // a count buffer whose groups were not kept
  double lo_hint = 0, hi_hint = 0;
  double lo = 0, hi = 0;    // interval used by the estimators
  size_t bytes = 0;
  std::atomic<int> inflight{0};
  uint64_t serial = 0;                 // unique per process
  std::atomic<uint64_t> tune_ver{0};   // bumped on every change of `tune`
  // autotuned product/update geometry per Krylov block shape:
  // key (ld, bytes per element, value type, kernel) -> (lanes per row |
  // log2(entry split) << 8, chunks per lane)
  mutable std::mutex tune_mu;
  std::map<uint64_t, std::pair<int, int>> tune;
};

namespace ld {

// One Krylov step of one request as four batchable launches.
struct StepPlan {
  bool valid = false;
  SpmmItem spmm{};
  ReduceItem red{};
  UpdateItem upd{};
  FinishItem fin{};
};
hipError_t launch_step_plans(hipStream_t st, std::vector<StepPlan>& plans);

// One estimate: the device state of one (matrix, params) request and the
// ordered list of device operations that compute it.  advance() enqueues
// work on a stream in slices (at most `budget` Krylov steps per call) so that
// the serving scheduler can interleave many requests; a blocking estimate
// simply calls it until it reports that everything is enqueued.
class Run {
 public:
  Run(ld_matrix* a, const ld_params& p);
  ~Run();
  ld_status validate();                 // parameter checks, derived sizes
  size_t device_bytes() const;          // bytes needed on the device
  ld_status bind(void* base, size_t bytes);  // carve the device buffers
  // Enqueue up to `budget` Krylov steps (non-Krylov phases count as one).
  // Returns LD_OK when more work remains, LD_PENDING... see .cpp.
  // With `plan`, a Krylov step that can join a batch is returned in *plan
  // (and *planned set) instead of being launched; the caller must launch it
  // (launch_step_plans) before advancing this request again.
  ld_status advance(hipStream_t st, int budget, bool* done, StepPlan* plan = nullptr,
                    bool* planned = nullptr);
  // Waits for `done` when given (a stream shared with other requests), else
  // for the whole stream.
  ld_status collect(hipStream_t st, ld_result* out, const ld_detail* detail,
                    hipEvent_t done = nullptr);
  ld_matrix* matrix() const { return a_; }
  const ld_params& params() const { return p_; }

 private:
  struct Phase;
  ld_status run_prologue(hipStream_t st);
  ld_status run_krylov_step(hipStream_t st, int t, StepPlan* plan = nullptr);
  ld_status run_epilogue(hipStream_t st);
  ld_status sketch_qr(hipStream_t st, double* Y, int cols);
  ld_status osa_sketch_prologue(hipStream_t st);
  ld_status osa_sketch_combine(hipStream_t st);
  ld_status start_block(hipStream_t st, const double* A, int s_cols, bool zero_h);
  ld_status sketch_runs_start(hipStream_t st);     // start block of the sketch-image runs
  ld_status sketch_combine_upto(hipStream_t st, int upto);  // two-pass: X_comb_next_..X_upto into Y
  ld_status begin_krylov(int phase);
  size_t layout(char* base);
  // product (which = 0) or update (which = 1) geometry of a Krylov block of
  // width ld: the matrix's tuned choice when it holds one, else the default
  Geom krylov_geom(int ld, int which) const;
  bool rg_ok() const;             // the product may read the matrix's row groups
  RowGroups row_groups() const;
  int upd_steady_nv(bool presub) const;  // update vectors of a steady-state step
  int upd_which(bool presub) const;      // tuning key of the update (window class)
  bool presub_choice(int ld) const;      // the stored step schedule of block width ld
  Geom v1_geom(int ld, const Geom& gu, bool presub) const;  // update geometry with v1
  // rows of partial sums a window-dots launch may write: kDotsWide when a
  // window can hold more than kDotsPerLaunch vectors older than the two
  // newest (FP32 and FP64 vectors), else kDotsPerLaunch
  int dots_rows() const { return (k_ - 2 > kDotsPerLaunch && !half_) ? kDotsWide : kDotsPerLaunch; }
  double spmm_bytes(int ld, int xbytes) const;

  ld_matrix* a_;
  ld_params p_;
  // derived
  int64_t n_ = 0;
  int s_ = 0, r_ = 0, B_ = 0, m_ = 0, k_ = 0;
  int kb_ = 0;                // basis columns of the estimate phase (So-SLQ: subspace rank)
  int adapt_every_ = 5;
  double tol_ = 1e-10;
  double lo_ = 0, hi_ = 0, scale_ = 1, c_ = 0, opscale_ = 1;
  bool mixed_ = false;        // Krylov vectors narrower than FP64 (FP32 or FP16)
  bool half_ = false;         // FP16 Krylov vectors
  double vscale_ = 1.0;       // power-of-two scale of the stored product output
  double oscale_ = 1.0;       // power-of-two scale of the stored start block
  int xb_ = 8;                // bytes per Krylov element
  int lds_ = 0, ldr_ = 0, ldB_ = 0, ld1_ = 0, ldx_ = 0;
  Geom gB_, gS_, g1_;
  Geom gBp_, gBu_, g1p_, g1u_;  // Krylov product / update geometries
  bool psB_ = true, ps1_ = true;  // the product subtracts the second-newest vector
  Geom gBuv_;                     // the estimate block's update with v1 (OSA-IOP)
  // state machine
  int stage_ = 0;             // 0 prologue, 1 krylov, 2 epilogue..., see .cpp
  int t_ = 0;
  int kphase_ = 0;            // OSA-IOP: 0 sketch-image runs, 1 estimate runs
  int kend_ = 0;              // steps of the current Krylov phase
  // two-pass sketch image (sketch_passes = 2): the sketch-image runs on a
  // ring of blocks, first for H only (opass_ 0), then again adding their
  // basis vectors into Y in batches of kCombBatch while still in the ring
  static constexpr int kCombBatch = 8;
  bool two_pass_ = false;
  int opass_ = 0;
  int comb_next_ = 0;         // next basis vector index to add to Y
  double* multall_ = nullptr; // two-pass: [m+1][ld1] multipliers of every sketch-run vector
  bool kmfull_ = false;       // multipliers indexed by vector, not by ring slot
  // Krylov phase parameters (current)
  int kB_ = 0, kld_ = 0, kns_ = 0;
  bool kpin_ = false, kfull_ = false;
  bool sym_ready_ = false;    // the next step's second-newest window product is in dwin_
  Geom kg_, kgu_;             // product / dots-and-update geometry of the phase
  bool kps_ = true;           // the phase's product subtracts the second-newest vector
  Geom kguv_;                 // the phase's update when it also reads v1
  void* kslots_ = nullptr;
  double* kmult_ = nullptr;
  // device buffers
  double* S_ = nullptr;       // [n][lds] sketch probes (aliases G_)
  double* Y_ = nullptr;       // [n][lds] sketch image -> basis A
  double* G_ = nullptr;       // [n][ldr] residual probes (Gaussian)
  uint64_t* gmask_ = nullptr; // [n][nwr] residual probe signs (Rademacher)
  int nwr_ = 0;
  uint64_t* smask_ = nullptr; // [n][nws] OSLQ sketch probe signs (Rademacher, lds <= 128)
  int nws_ = 0;
  void* slots_ = nullptr;     // Krylov storage
  double* mult_ = nullptr;    // [nslots][ld]
  double* part_ = nullptr;    // per-block partial sums
  double* dwin_ = nullptr;    // [nvmax][ld] reduced window dots
  double* nsr_ = nullptr;     // [2][ld] reduced norm / v1 dots
  double* norm2_ = nullptr;   // [ld]
  double* K_ = nullptr;       // [ld]
  double* H_ = nullptr;       // [ld][(m+1) m]
  double* gq_ = nullptr;      // [ld][m+1]
  double* work_ = nullptr;    // quadrature / log work
  double* gram_ = nullptr;    // [s][s]
  double* rfac_ = nullptr;    // [s][s]
  double* rinv_ = nullptr;    // [s][s]
  double* umat_ = nullptr;    // So-SLQ: [s][kb] kept eigenvectors / sqrt(eigenvalue)
  double* pmat_ = nullptr;    // [s][r]
  double* ell_ = nullptr;     // OSA-IOP: [ld][m] log(H) e1 of the sketch runs
  double* coefs_ = nullptr;   // OSA-IOP: [m][ld1] combination coefficients
  int* meff_ = nullptr;
  int* active_ = nullptr;
  int* flags_ = nullptr;
  int* dflag_ = nullptr;      // [2] CholQR flags
  int* need_ = nullptr;       // OSA-IOP: runs needing the general Hessenberg log
  int* meff0_ = nullptr;      // OSA-IOP: Krylov dimensions of the sketch-image runs
  void* pack_ = nullptr;      // packed per-run results (launch_pack_results)
  uint64_t* seed_dev_ = nullptr;  // the probe seed, read by the probe kernels
  bool capturing_ = false;    // enqueue into a graph capture: no event records, no seed write
  void* hpack_ = nullptr;     // pinned host copy of pack_
  bool own_hpack_ = false;
  // asymmetry of H accepted by the symmetric fast path of log(H) e1: rounding
  // level of the vectors' precision
  // relative asymmetry of H below which log(H) e1 takes the symmetric
  // tridiagonal path: rounding level of the Krylov vectors' storage (FP16
  // entries carry 2^-11 relative rounding, which reaches the two estimates of
  // each off-diagonal entry differently)
  double symtol() const { return half_ ? 1e-3 : (mixed_ ? 1e-5 : 1e-12); }
  // spectral interval of the Gauss-quadrature runs' operator (Q / scale)
  double quad_a() const { return lo_ / scale_; }
  double quad_b() const { return hi_ / scale_; }
  bool adaptive() const { return p_.adapt_tol > 0.0 && p_.method != LD_METHOD_OSA_IOP &&
                                 (p_.method == LD_METHOD_OSLQ || kphase_ == 1); }
  // adaptive Krylov dimension
  int* nact_ = nullptr;        // device: runs still active after a check
  int* nact_host_ = nullptr;   // pinned copy
  double* kprev_ = nullptr;    // [ld] quadrature value at the previous check
  hipEvent_t check_ev_ = nullptr;
  bool pending_check_ = false;
  bool blocking_ = false;
  size_t part_elems_ = 0;
  size_t slot_elems_ = 0;     // elements of one [n][ld] slot
  int nslots_ = 0;
  int wstride_ = 0;           // OSA-IOP: per-run workspace of the Hessenberg log
  hipEvent_t ev0_ = nullptr, ev1_ = nullptr;
  bool ext_ = false;          // events and pinned count belong to the caller
  double t_submit_ = 0;
  Profiler* prof_ = nullptr;
 public:
  void set_profiler(Profiler* p) { prof_ = p; }
  // Use caller-owned events (start, end, adaptive check) and a pinned int
  // instead of creating them; the run then creates and frees nothing.
  void use_external(hipEvent_t e0, hipEvent_t e1, hipEvent_t chk, int* nact_pinned) {
    ev0_ = e0;
    ev1_ = e1;
    check_ev_ = chk;
    nact_host_ = nact_pinned;
    ext_ = true;
  }
  void set_blocking(bool b) { blocking_ = b; }
  // Pinned host buffer of at least kHostPackBytes for the packed results
  // (owned by the caller); without one the run allocates its own.
  void set_host_pack(void* p) { hpack_ = p; }
  // Graph capture of the whole estimate: the seed write and the timing
  // events stay out of the captured sequence (the replay does them around the
  // graph launch: record ev0, write_seed, launch, record ev1).
  void set_capturing(bool c) { capturing_ = c; }
  ld_status write_seed(hipStream_t st);
  ld_status enqueue_results(hipStream_t st);  // pack + copy to the pinned buffer
  hipEvent_t start_event() const { return ev0_; }
  hipEvent_t end_event() const { return ev1_; }
  // whether the launch sequence depends on nothing but (matrix, params minus
  // the seed): no adaptive host check, no per-launch profiling events
  bool capturable() const;
  // Time the candidate geometries of the Krylov-block product and update on
  // this request's matrix and block shape; store the fastest in the matrix.
  ld_status tune(hipStream_t st, int reps, ld_tune_result* out);
  ld_status tune_set(int spmm_lanes, int spmm_chunks, int spmm_split, int update_lanes,
                     int update_chunks, int spmm_interleave = 0, int spmm_row_stride = 0,
                     int step_presub = 1, int spmm_row_groups = 0);
  std::vector<int> stride_candidates(hipStream_t st) const;
  double submit_time() const { return t_submit_; }
  void set_submit_time(double t) { t_submit_ = t; }
  int64_t n() const { return n_; }
};

double now_seconds();

}  // namespace ld

// Host runtime of liblogdet: the estimate pipeline as a resumable sequence of
// device phases, plus the C ABI entry points.
//
// Pipeline of one OSLQ estimate (Alg 3), all on one HIP stream:
//   Rademacher S -> Y = J S (CSR x block) -> CholQR2(Y) = A
//   -> Rademacher G -> P = A^T G -> X0 = [A | G - A P], column norms
//   -> m windowed Krylov steps over the whole block of s + r runs
//   -> Golub-Welsch per run -> per-run K values back to the host, trace sum.
// OSA-IOP (Alg 2 with Alg 1) adds a first Krylov phase over S whose basis is
// kept, log(H) e1 per run, Y = L_c S assembled from the stored basis, then
// the same QR / projection and a second Krylov phase with v1 kept for the
// quadratic forms.
#include "runtime.h"
#include "serve.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

namespace ld {

static thread_local std::string g_last_error;

ld_status set_error(ld_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

double now_seconds() {
  using clk = std::chrono::steady_clock;
  return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

#define LD_HIP(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return set_error(LD_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

DeviceBuffer::~DeviceBuffer() { release(); }

void DeviceBuffer::release() {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  bytes = 0;
}

hipError_t DeviceBuffer::ensure(size_t want) {
  if (want <= bytes && ptr) return hipSuccess;
  release();
  hipError_t e = hipMalloc(&ptr, want);
  if (e != hipSuccess) {
    ptr = nullptr;
    return e;
  }
  bytes = want;
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Profiler
// ---------------------------------------------------------------------------
static int fam_index(uint32_t fam) {
  int i = 0;
  while (fam > 1u) {
    fam >>= 1;
    ++i;
  }
  return i;
}

Profiler::~Profiler() {
  for (auto& p : pending_) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : pool_) (void)hipEventDestroy(e);
}

void Profiler::enable(uint32_t mask) {
  std::lock_guard<std::mutex> lk(mu_);
  mask_ = mask;
  for (int i = 0; i < 8; ++i) {
    count_[i] = 0;
    ms_[i] = 0.0;
    bytes_[i] = 0.0;
  }
}

hipEvent_t Profiler::get_event() {
  if (!pool_.empty()) {
    hipEvent_t e = pool_.back();
    pool_.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

hipError_t Profiler::begin(uint32_t fam, hipStream_t st, hipEvent_t* a) {
  *a = nullptr;
  std::lock_guard<std::mutex> lk(mu_);
  if (!(mask_ & fam)) return hipSuccess;
  *a = get_event();
  if (!*a) return hipErrorOutOfMemory;
  return hipEventRecord(*a, st);
}

hipError_t Profiler::end(uint32_t fam, hipStream_t st, hipEvent_t a, double bytes) {
  if (!a) return hipSuccess;
  std::lock_guard<std::mutex> lk(mu_);
  hipEvent_t b = get_event();
  if (!b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(b, st);
  pending_.push_back({fam_index(fam), a, b, bytes});
  return e;
}

hipError_t Profiler::harvest() {
  std::lock_guard<std::mutex> lk(mu_);
  hipError_t err = hipSuccess;
  for (auto& p : pending_) {
    hipError_t e = hipEventSynchronize(p.b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.a, p.b);
    if (e == hipSuccess) {
      count_[p.fam_bit] += 1;
      ms_[p.fam_bit] += ms;
      bytes_[p.fam_bit] += p.bytes;
    } else {
      err = e;
    }
    pool_.push_back(p.a);
    pool_.push_back(p.b);
  }
  pending_.clear();
  return err;
}

void Profiler::query(uint32_t fam, int64_t* n, double* ms, double* bytes) {
  std::lock_guard<std::mutex> lk(mu_);
  *n = 0;
  *ms = 0.0;
  *bytes = 0.0;
  for (int i = 0; i < 8; ++i)
    if (fam & (1u << i)) {
      *n += count_[i];
      *ms += ms_[i];
      *bytes += bytes_[i];
    }
}

// Launch with optional event bracketing; `bytes` is the algorithmic traffic.
#define LD_LAUNCH(fam, bytes, expr)                                      \
  do {                                                                   \
    hipEvent_t pa_ = nullptr;                                            \
    if (prof_) LD_HIP(prof_->begin((fam), st, &pa_));                    \
    LD_HIP(expr);                                                        \
    if (prof_) LD_HIP(prof_->end((fam), st, pa_, (double)(bytes)));      \
  } while (0)

// ---------------------------------------------------------------------------
// Graph cache of blocking estimates
// ---------------------------------------------------------------------------
bool GraphKey::operator==(const GraphKey& o) const {
  return serial == o.serial && tune_ver == o.tune_ver && method == o.method &&
         precision == o.precision && n_probes == o.n_probes && sketch_rank == o.sketch_rank &&
         krylov_steps == o.krylov_steps && iop_window == o.iop_window &&
         probe_dist == o.probe_dist && subspace_rank == o.subspace_rank &&
         adapt_every == o.adapt_every && sketch_passes == o.sketch_passes && tol == o.tol &&
         adapt_tol == o.adapt_tol && ws == o.ws && ws_bytes == o.ws_bytes;
}

static void destroy_entry(GraphCache::Entry& e) {
  if (e.exec) (void)hipGraphExecDestroy(e.exec);
  if (e.graph) (void)hipGraphDestroy(e.graph);
  e.exec = nullptr;
  e.graph = nullptr;
}

GraphCache::Entry* GraphCache::find(const GraphKey& k) {
  for (Entry& e : entries)
    if (e.key == k) {
      e.last = ++tick;
      return &e;
    }
  return nullptr;
}

bool GraphCache::seen_before(const GraphKey& k) {
  for (const GraphKey& s : seen)
    if (s == k) return true;
  seen.push_back(k);
  if ((int)seen.size() > kSeen) seen.pop_front();
  return false;
}

hipError_t GraphCache::insert(const GraphKey& k, hipGraph_t g, hipGraphExec_t x) {
  if ((int)entries.size() >= kMax) {
    size_t lru = 0;
    for (size_t i = 1; i < entries.size(); ++i)
      if (entries[i].last < entries[lru].last) lru = i;
    destroy_entry(entries[lru]);
    entries.erase(entries.begin() + (long)lru);
  }
  Entry e;
  e.key = k;
  e.graph = g;
  e.exec = x;
  e.last = ++tick;
  entries.push_back(e);
  ++captures;
  return hipSuccess;
}

void GraphCache::drop_matrix(uint64_t serial) {
  for (size_t i = entries.size(); i-- > 0;)
    if (entries[i].key.serial == serial) {
      destroy_entry(entries[i]);
      entries.erase(entries.begin() + (long)i);
    }
  for (size_t i = seen.size(); i-- > 0;)
    if (seen[i].serial == serial) seen.erase(seen.begin() + (long)i);
}

void GraphCache::drop_workspace() {
  for (Entry& e : entries) destroy_entry(e);
  entries.clear();
  seen.clear();
}

void GraphCache::clear() { drop_workspace(); }

static inline int round4(int x) { return (x + 3) & ~3; }
static inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// FP16 Krylov vectors are accepted when lambda_hi / lambda_lo is at most
// this (LD_PREC_HALF refuses wider intervals).  Measured on the serving mix
// of Laplacians and Wendland covariances: FP16 stays within 1e-4 of FP64 up
// to a ratio of ~500 on every kind; beyond it Wendland covariances, whose
// spectra crowd near the nugget, exceed 1e-4.
constexpr double kHalfMaxRatio = 512.0;
// LD_PREC_AUTO takes FP32 vectors up to this ratio and FP64 beyond.  FP32
// held 1e-4 against FP64 on every request of the serving mix with a ratio
// below ~8700 (Wendland covariances with small nuggets were the first to
// fail); the cut keeps a factor of two below that.  AUTO never takes FP16:
// its relative error is bounded against sum |log lambda|, so a logdet whose
// terms nearly cancel can miss a 1e-4 relative gate inside the FP16 range.
constexpr double kAutoMixedRatio = 4096.0;

// ---------------------------------------------------------------------------
// Run
// ---------------------------------------------------------------------------
enum Stage : int {
  ST_PROLOGUE = 0,
  ST_KRYLOV = 1,
  ST_COMBINE = 2,   // OSA-IOP: between the two Krylov phases
  ST_EPILOGUE = 3,
  ST_DONE = 4,
};

Run::Run(ld_matrix* a, const ld_params& p) : a_(a), p_(p) {}

Run::~Run() {
  if (check_ev_ && pending_check_) (void)hipEventSynchronize(check_ev_);
  if (own_hpack_ && hpack_) (void)hipHostFree(hpack_);  // waits for a copy in flight
  if (ext_) return;
  if (ev0_) (void)hipEventDestroy(ev0_);
  if (ev1_) (void)hipEventDestroy(ev1_);
  if (check_ev_) {
    (void)hipEventSynchronize(check_ev_);
    (void)hipEventDestroy(check_ev_);
  }
  if (nact_host_) (void)hipHostFree(nact_host_);
}

ld_status Run::validate() {
  if (!a_) return set_error(LD_E_INVALID_ARG, "null matrix");
  n_ = a_->n;
  s_ = p_.sketch_rank;
  r_ = p_.n_probes - p_.sketch_rank;
  m_ = p_.krylov_steps;
  k_ = p_.iop_window;
  tol_ = p_.tol > 0 ? p_.tol : 1e-10;
  if (p_.method != LD_METHOD_OSLQ && p_.method != LD_METHOD_OSA_IOP &&
      p_.method != LD_METHOD_SO_SLQ)
    return set_error(LD_E_INVALID_ARG, "unknown method");
  if (p_.precision != LD_PREC_FP64 && p_.precision != LD_PREC_MIXED &&
      p_.precision != LD_PREC_HALF && p_.precision != LD_PREC_AUTO)
    return set_error(LD_E_INVALID_ARG, "unknown precision");
  if (p_.probe_dist != LD_PROBE_RADEMACHER && p_.probe_dist != LD_PROBE_GAUSSIAN)
    return set_error(LD_E_INVALID_ARG, "unknown probe distribution");
  if (p_.sketch_passes < 0 || p_.sketch_passes > 2 ||
      (p_.sketch_passes == 2 && p_.method == LD_METHOD_OSLQ))
    return set_error(LD_E_INVALID_ARG, "sketch_passes must be 0, 1 or 2 (2: OSA-IOP and "
                                       "So-SLQ, whose sketch image comes from Krylov runs)");
  two_pass_ = p_.sketch_passes == 2;
  if (!(p_.adapt_tol >= 0.0) || !std::isfinite(p_.adapt_tol) || p_.adapt_every < 0)
    return set_error(LD_E_INVALID_ARG, "adapt_tol must be finite and >= 0, adapt_every >= 0");
  if (p_.adapt_tol > 0.0 && p_.method == LD_METHOD_OSA_IOP)
    return set_error(LD_E_INVALID_ARG, "the adaptive Krylov dimension applies to the Gauss "
                                       "quadrature methods (OSLQ, SLQ, So-SLQ)");
  if (p_.method == LD_METHOD_SO_SLQ) {
    if (s_ < 1 || s_ > kSoSlqMaxSketch || (int64_t)s_ > n_)
      return set_error(LD_E_INVALID_ARG, "So-SLQ: sketch_rank q must satisfy 1 <= q <= min(n, 48)");
    kb_ = p_.subspace_rank > 0 ? p_.subspace_rank : std::min(10, s_);
    if (kb_ > s_) return set_error(LD_E_INVALID_ARG, "So-SLQ: subspace_rank must be <= sketch_rank");
  } else {
    if (p_.subspace_rank != 0)
      return set_error(LD_E_INVALID_ARG, "subspace_rank applies to So-SLQ only");
    if (s_ < 0 || s_ > 256 || (int64_t)s_ > n_)
      return set_error(LD_E_INVALID_ARG, "sketch_rank must satisfy 0 <= s <= min(n, 256)");
    kb_ = s_;
  }
  if (r_ < 1) return set_error(LD_E_INVALID_ARG, "n_probes - sketch_rank must be >= 1");
  B_ = kb_ + r_;
  if (m_ < 1 || m_ > 512 || (int64_t)m_ > n_)
    return set_error(LD_E_INVALID_ARG, "krylov_steps must satisfy 1 <= m <= min(n, 512)");
  if (k_ < 1) return set_error(LD_E_INVALID_ARG, "iop_window must be >= 1");
  adapt_every_ = p_.adapt_every > 0 ? p_.adapt_every : 5;
  mixed_ = p_.precision != LD_PREC_FP64;
  half_ = p_.precision == LD_PREC_HALF;
  if (p_.precision == LD_PREC_AUTO) mixed_ = a_->hi <= kAutoMixedRatio * a_->lo;
  xb_ = half_ ? 2 : (mixed_ ? 4 : 8);
  if (std::max(B_, s_) > (mixed_ ? 256 : 128))
    return set_error(LD_E_INVALID_ARG, mixed_ ? "n_probes must be <= 256 in mixed precision"
                                              : "n_probes must be <= 128 in FP64");
  if (half_ && k_ > 4)
    return set_error(LD_E_INVALID_ARG,
                     "FP16 Krylov vectors take iop_window <= 4: with more window vectors the "
                     "classical Gram-Schmidt step on FP16-rounded vectors loses stability");
  if (half_ && !(a_->hi <= kHalfMaxRatio * a_->lo))
    return set_error(LD_E_INVALID_ARG,
                     "FP16 Krylov vectors take matrices with lambda_hi <= 512 lambda_lo: on "
                     "wider spectral intervals the 2^-11 storage rounding can move the estimate "
                     "by more than 1e-4 (use LD_PREC_MIXED or LD_PREC_AUTO)");
  // Krylov blocks hold whole 16-byte chunks per row (8 FP16 values)
  auto roundv = [&](int x) { return half_ ? (x + 7) / 8 * 8 : round4(x); };
  lds_ = roundv(std::max(s_, 1));
  ldr_ = round4(r_);
  ldB_ = roundv(B_);
  ld1_ = lds_;
  ldx_ = std::max(ldB_, ld1_);
  lo_ = a_->lo;
  hi_ = a_->hi;
  if (p_.method != LD_METHOD_OSA_IOP) {
    // OSLQ and its comparators: J = Q / lambda_hi and c = log(lambda_hi) when
    // lambda_lo < 1, else J = Q, c = 0
    if (lo_ < 1.0) {
      scale_ = hi_;
      c_ = std::log(hi_);
    } else {
      scale_ = 1.0;
      c_ = 0.0;
    }
  } else {
    // Krylov on Q / gamma; traced operator log Q - c I
    scale_ = std::sqrt(lo_ * hi_);
    c_ = lo_ < 1.0 ? std::log(lo_) : std::log(scale_);
  }
  opscale_ = 1.0 / scale_;
  vscale_ = 1.0;
  oscale_ = 1.0;
  if (half_) {
    // FP16 Krylov vectors: the product output (and every vector derived from
    // it) is stored at a power-of-two scale that puts the entries of a unit
    // vector near 1 while |entries| <= vscale * ||operator|| stays far below
    // the FP16 maximum; the start block likewise (its entries are at most a
    // few units before scaling)
    const double opnorm = hi_ * opscale_;
    const double target = std::min(std::sqrt((double)n_), 4096.0 / opnorm);
    vscale_ = std::ldexp(1.0, std::max(-20, std::min(14, (int)std::floor(std::log2(target)))));
    oscale_ = std::ldexp(1.0, std::max(0, std::min(10, (int)std::floor(std::log2(std::sqrt((double)n_))))));
  }
  gB_ = make_geom(n_, ldB_, xb_);
  gS_ = make_geom(n_, lds_, 8);
  g1_ = make_geom(n_, ld1_, xb_);
  psB_ = presub_choice(ldB_);
  ps1_ = presub_choice(ld1_);
  gBp_ = krylov_geom(ldB_, 0);
  gBu_ = krylov_geom(ldB_, upd_which(psB_));
  gBuv_ = v1_geom(ldB_, gBu_, psB_);
  g1p_ = krylov_geom(ld1_, 0);
  g1u_ = krylov_geom(ld1_, upd_which(ps1_));
  return LD_OK;
}

// Key of a tuned geometry: block width, element bytes, matrix value type of
// the product, kernel (0 product; 1 | class << 4 the update of a window class;
// 3 | class << 4 the same update when it also reads v1 (OSA-IOP); 2 the step
// schedule: {1, 0} when the update, not the product, subtracts the
// second-newest window vector).
static uint64_t tune_key(int ld, int xbytes, int vt, int which) {
  return (uint64_t)ld | ((uint64_t)xbytes << 16) | ((uint64_t)vt << 24) | ((uint64_t)which << 32);
}

// The update's register footprint grows with the vectors it subtracts, so its
// tuned geometry is kept per class of the steady-state window: the window
// (up to 8 vectors per launch, 4 with FP16 vectors), less the second-newest
// vector when the product subtracts it (windows of two or more).
int Run::upd_steady_nv(bool presub) const {
  const int kw = std::max(1, std::min(k_, half_ ? 4 : kMaxNv));
  return (k_ >= 2 && presub) ? kw - 1 : kw;
}
int Run::upd_which(bool presub) const {
  const int nv = upd_steady_nv(presub);
  const int cls = nv <= 1 ? 1 : (nv == 2 ? 2 : (nv <= 4 ? 4 : 8));
  return 1 | (cls << 4);
}
// The OSA-IOP update that also reads v1 holds two more sets of FP64 column
// sums per lane, so a geometry with many chunks per lane costs it occupancy:
// it takes its own tuned geometry (key 3 | class << 4), else the plain
// update's when that has at most 8 elements per lane, else the power-of-two
// lanes with the fewest chunks up to 8 elements per lane.
Geom Run::v1_geom(int ld, const Geom& gu, bool presub) const {
  const int vt = mixed_ ? a_->vt_lo : VT_F64;
  {
    std::lock_guard<std::mutex> lk(a_->tune_mu);
    auto it = a_->tune.find(tune_key(ld, xb_, vt, upd_which(presub) + 2));
    if (it != a_->tune.end()) {
      const Geom g = make_geom_lc(n_, ld, xb_, it->second.first, it->second.second);
      if (geom_usable(g)) return g;
    }
  }
  const int vec = 16 / xb_;
  if (gu.C * vec <= 8) return gu;
  const int ncolv = ld / vec;
  const int cmax = std::max(1, 8 / vec);
  int L = 1;
  while (L * cmax < ncolv && L < 64) L <<= 1;
  const Geom g = make_geom_lc(n_, ld, xb_, L, std::min(cmax, (ncolv + L - 1) / L));
  return geom_usable(g) ? g : gu;
}

// The matrix's row groups serve the products over the values that the
// estimate reads: FP32 (or FP64, on FP64 storage) values with FP32 Krylov
// vectors, FP64 values with FP64 vectors.
bool Run::rg_ok() const {
  if (!a_->rg_gp) return false;
  if (!mixed_) return xb_ == 8 && a_->rg_val64;
  // mixed: the values in their storage type, FP32 or FP64, on FP32 vectors
  return xb_ == 4 && (a_->vt_lo == VT_F32 ? a_->rg_val != nullptr : a_->rg_val64 != nullptr);
}
RowGroups Run::row_groups() const {
  RowGroups r;
  r.gp = a_->rg_gp;
  r.col = a_->rg_col;
  r.val = a_->rg_val;
  r.val64 = a_->rg_val64;
  return r;
}

bool Run::presub_choice(int ld) const {
  const int vt = mixed_ ? a_->vt_lo : VT_F64;
  std::lock_guard<std::mutex> lk(a_->tune_mu);
  auto it = a_->tune.find(tune_key(ld, xb_, vt, 2));
  return it == a_->tune.end() || it->second.first == 0;
}

Geom Run::krylov_geom(int ld, int which) const {
  const int vt = mixed_ ? a_->vt_lo : VT_F64;
  {
    std::lock_guard<std::mutex> lk(a_->tune_mu);
    auto it = a_->tune.find(tune_key(ld, xb_, vt, which));
    if (it != a_->tune.end()) {
      Geom g = make_geom_lc(n_, ld, xb_, it->second.first & 0xff, it->second.second);
      g.lges = (it->second.first >> 8) & 0xf;  // entry split of the product
      g.xil = (it->second.first >> 12) & 1;    // chunk mapping of the product
      g.ts = (it->second.first >> 16) & 0x7fff;  // row tiles of the product
      g.rg = (it->second.first >> 13) & 1;       // row groups of the product
      if (geom_usable(g) && (g.rg == 0 || rg_ok())) return g;
    }
  }
  if (which == 0 && rg_ok() && ld >= 16 && !(mixed_ && a_->vt_lo == VT_F64)) {
    // row groups (blocks of 16 columns or more: on narrower ones the groups'
    // extra multiply-adds and shuffles weigh more than the gathers they
    // save): one chunk per lane with FP32 vectors, two with FP64 ones (the
    // 64-probe covariance: 16 x 2 0.55 ms, 32 x 1 0.67 ms per product).
    // FP64 values on FP32 vectors keep the CSR product by default (their
    // FP64 sums of 4 rows cost occupancy: on that covariance 22.3 against
    // 21.3 ms per estimate); the autotuner and ld_tune_set can still take
    // the groups there
    const int ncolv = ld / (16 / xb_);
    const int C = (xb_ == 8 && ncolv >= 4) ? 2 : 1;
    Geom g = make_geom_lc(n_, ld, xb_, (ncolv + C - 1) / C, C);
    g.rg = 1;
    if ((ncolv + C - 1) / C <= 64 && geom_usable(g)) return g;
  }
  if (which == 0 && a_->nnz >= 64 * a_->n) {
    // long rows: one chunk per lane and the row's entries over two lane
    // groups, which halves each lane's chain of dependent gathers
    const int ncolv = ld / (16 / xb_);
    int Lc = 1;
    while (Lc < ncolv) Lc <<= 1;
    if (Lc <= 32) {
      Geom g = make_geom_lc(n_, ld, xb_, 2 * Lc, 1);
      g.lges = 1;
      if (geom_usable(g)) return g;
    }
  }
  const Geom d = make_geom(n_, ld, xb_);
  if (which == 0 && xb_ == 2 && d.C == 1 && d.ncolv <= 64 &&
      (64 / d.ncolv) > (64 / d.L)) {
    // FP16 product: L = the row's chunks when that keeps more lanes of a
    // wave busy than the power of two above it (96 probes: 5 rows of 12
    // lanes per wave instead of 4 of 16 with 4 idle)
    Geom g = make_geom_lc(n_, ld, xb_, d.ncolv, 1);
    if (geom_usable(g)) return g;
  }
  return d;
}

// One layout for measuring and for carving: with base == nullptr only the
// size is computed.
size_t Run::layout(char* base) {
  size_t off = 0;
  auto take = [&](size_t sz) -> void* {
    void* q = base ? base + off : nullptr;
    off += align_up(sz);
    return q;
  };
  const size_t n = (size_t)n_;
  const int nvmax = std::min(k_, m_) + 1;
  size_t slot_bytes;
  // Krylov storage: OSLQ ring of min(k,m)+1 slots; OSA-IOP max(phase-1 full
  // basis, phase-2 ring with v1 kept).
  if (p_.method == LD_METHOD_OSLQ) {
    nslots_ = std::min(k_, m_) + 1;
    slot_bytes = (size_t)nslots_ * n * ldB_ * xb_;
  } else {
    // phase 0 keeps the sketch runs' whole basis (two passes: a ring of the
    // window plus one combine batch); phase 1 is a ring (OSA-IOP also keeps
    // v1)
    const int ring = std::min(k_, m_) + (p_.method == LD_METHOD_OSA_IOP ? 2 : 1);
    const int ring0 = two_pass_ ? std::min(m_ + 1, std::min(k_, m_) + 1 + kCombBatch) : m_ + 1;
    nslots_ = std::max(ring0, ring);
    slot_bytes = std::max((size_t)ring0 * n * ld1_ * xb_, (size_t)ring * n * ldB_ * xb_);
  }
  slots_ = take(slot_bytes);
  mult_ = static_cast<double*>(take((size_t)nslots_ * ldx_ * 8));
  // Rademacher residual probes as packed signs (64 per word); Gaussian ones
  // as FP64 columns in the sketch-probe buffer once the sketch is formed
  const bool gsigns = p_.probe_dist == LD_PROBE_RADEMACHER;
  nwr_ = (r_ + 63) / 64;
  // the OSLQ sketch product gathers sign words too (up to 128 columns), so
  // no FP64 sketch-probe block is needed
  const bool ssigns = gsigns && p_.method == LD_METHOD_OSLQ && s_ > 0 && lds_ <= 128;
  nws_ = (s_ + 63) / 64;
  S_ = static_cast<double*>(
      take(n * (gsigns ? (ssigns ? 0 : lds_) : std::max(lds_, ldr_)) * 8));
  G_ = gsigns ? nullptr : S_;
  gmask_ = gsigns ? static_cast<uint64_t*>(take(n * (size_t)nwr_ * 8)) : nullptr;
  smask_ = ssigns ? static_cast<uint64_t*>(take(n * (size_t)nws_ * 8)) : nullptr;
  Y_ = s_ > 0 ? static_cast<double*>(take(n * lds_ * 8)) : nullptr;
  // streaming kernels: fused product dots (2 rows of ld) and further dots
  // launches (up to 4 rows of ld, 8 for windows that have more than 4 older
  // vectors) in separate regions, kMaxBlocks each
  size_t pe = (size_t)kMaxBlocks * (2 + dots_rows()) * ldx_;
  if (s_ > 0) pe = std::max(pe, (size_t)gS_.nblk * s_ * std::max(s_, r_));
  part_elems_ = pe;
  part_ = static_cast<double*>(take(pe * 8));
  dwin_ = static_cast<double*>(take((size_t)nvmax * ldx_ * 8));
  nsr_ = static_cast<double*>(take((size_t)2 * ldx_ * 8));
  norm2_ = static_cast<double*>(take((size_t)ldx_ * 8));
  K_ = static_cast<double*>(take((size_t)ldx_ * 8));
  H_ = static_cast<double*>(take((size_t)ldx_ * (m_ + 1) * m_ * 8));
  gq_ = static_cast<double*>(take((size_t)ldx_ * (m_ + 1) * 8));
  wstride_ = hess_log_wstride(m_);
  work_ = (p_.method != LD_METHOD_OSLQ)
              ? static_cast<double*>(take((size_t)ldx_ * (size_t)wstride_ * 8))
              : nullptr;
  if (s_ > 0) {
    gram_ = static_cast<double*>(take((size_t)s_ * s_ * 8));
    rfac_ = static_cast<double*>(take((size_t)s_ * s_ * 8));
    rinv_ = static_cast<double*>(take((size_t)s_ * s_ * 8));
    pmat_ = static_cast<double*>(take((size_t)s_ * r_ * 8));
  }
  if (p_.method == LD_METHOD_SO_SLQ) umat_ = static_cast<double*>(take((size_t)s_ * kb_ * 8));
  ell_ = static_cast<double*>(take((size_t)ld1_ * m_ * 8));
  coefs_ = static_cast<double*>(take((size_t)(m_ + 1) * ld1_ * 8));
  multall_ = two_pass_ ? static_cast<double*>(take((size_t)(m_ + 1) * ld1_ * 8)) : nullptr;
  meff_ = static_cast<int*>(take((size_t)ldx_ * 4));
  active_ = static_cast<int*>(take((size_t)ldx_ * 4));
  flags_ = static_cast<int*>(take((size_t)ldx_ * 4));
  dflag_ = static_cast<int*>(take(16));
  nact_ = static_cast<int*>(take(16));
  kprev_ = static_cast<double*>(take((size_t)ldx_ * 8));
  need_ = static_cast<int*>(take((size_t)ldx_ * 4));
  meff0_ = static_cast<int*>(take((size_t)ldx_ * 4));
  pack_ = take(pack_results_bytes(ldx_));
  seed_dev_ = static_cast<uint64_t*>(take(8));
  return off;
}

size_t Run::device_bytes() const { return const_cast<Run*>(this)->layout(nullptr); }

ld_status Run::bind(void* base, size_t bytes) {
  const size_t need = layout(nullptr);
  if (need > bytes) return set_error(LD_E_NO_MEMORY, "workspace smaller than the request needs");
  layout(static_cast<char*>(base));
  stage_ = ST_PROLOGUE;
  t_ = 0;
  kphase_ = 0;
  return LD_OK;
}

// Algorithmic bytes of one CSR x block product: the matrix once (values,
// column indices, row pointers), the input block once, the output block once.
double Run::spmm_bytes(int ld, int xbytes) const {
  const int vb = mixed_ ? (a_->vt_lo == VT_BF16 ? 2 : (a_->vt_lo == VT_F32 ? 4 : 8)) : 8;
  return (double)a_->nnz * (vb + 4) + 4.0 * (n_ + 1) + 2.0 * (double)n_ * ld * xbytes;
}

// CholQR2: Y <- Y R1^{-1}, then again, so that Y = A R with A orthonormal and
// R = R2 R1 upper triangular with a positive diagonal (the QR convention of
// the oracle).  A column whose part orthogonal to the columns kept before it
// is at most 1e-6 of its norm is dropped (a zero column of A, whose run then
// contributes nothing): A spans range(Y) in column order also when the sketch
// image is rank-deficient.  dflag_[pass] is set on a non-finite pivot.
ld_status Run::sketch_qr(hipStream_t st, double* Y, int cols) {
  for (int pass = 0; pass < 2; ++pass) {
    LD_LAUNCH(LD_PROF_SKETCH, (double)n_ * cols * 8,
              launch_gemm_tn(st, gS_, Y, lds_, cols, Y, lds_, cols, part_));
    LD_LAUNCH(LD_PROF_REDUCE, (double)gS_.nblk * cols * cols * 8,
              launch_reduce(st, part_, gS_.nblk, cols * cols, gram_));
    LD_LAUNCH(LD_PROF_SKETCH, 0, launch_chol_inv(st, cols, gram_, rfac_, rinv_, dflag_ + pass));
    LD_LAUNCH(LD_PROF_SKETCH, (double)n_ * cols * 16,
              launch_trsm_rows(st, n_, Y, lds_, cols, rinv_));
  }
  return LD_OK;
}

// X0 = [A | G - A (A^T G)] in Krylov precision, its column norms, and the
// per-run start state.
ld_status Run::start_block(hipStream_t st, const double* A, int s_cols, bool zero_h) {
  // no previous quadrature value yet (all-ones bytes: NaN) for the adaptive
  // test; a fresh Hessenberg block for a phase that starts here
  FillItem fi[2] = {{kprev_, (size_t)ldx_ * 2, 0xFFFFFFFFu},
                    {H_, (size_t)ldx_ * (m_ + 1) * m_ * 2, 0u}};
  LD_HIP(launch_fill(st, fi, zero_h ? 2 : 1));
  GSrc gs{G_, ldr_, gmask_, nwr_};
  if (gmask_) {
    gs.dense = nullptr;
    LD_LAUNCH(LD_PROF_PROBES, (double)n_ * nwr_ * 8,
              launch_rademacher_mask(st, p_.seed, n_, s_, r_, gmask_, nwr_, seed_dev_));
  } else {
    gs.mask = nullptr;
    LD_LAUNCH(LD_PROF_PROBES, (double)n_ * ldr_ * 8,
              launch_probes(st, p_.probe_dist, p_.seed, n_, s_, ldr_, r_, G_, 8, ldr_, 0,
                            seed_dev_));
  }
  const double gbytes = gmask_ ? (double)n_ * nwr_ * 8 : (double)n_ * r_ * 8;
  if (s_cols > 0) {
    LD_LAUNCH(LD_PROF_SKETCH, (double)n_ * s_cols * 8 + gbytes,
              launch_gemm_tn_g(st, gS_, A, lds_, s_cols, gs, r_, part_));
    LD_LAUNCH(LD_PROF_REDUCE, (double)gS_.nblk * s_cols * r_ * 8,
              launch_reduce(st, part_, gS_.nblk, s_cols * r_, pmat_));
  }
  LD_LAUNCH(LD_PROF_SKETCH, (double)n_ * s_cols * 8 + gbytes + (double)n_ * ldB_ * xb_,
            launch_project(st, gB_, A, lds_, s_cols, gs, r_, pmat_, slots_, part_, oscale_));
  LD_LAUNCH(LD_PROF_SMALL, (double)gB_.nblk * ldB_ * 8,
            launch_start_finish(st, B_, ldB_, part_, gB_.nblk, norm2_, mult_, active_, meff_, gq_,
                                m_ + 1, 1.0 / oscale_));
  return LD_OK;
}

ld_status Run::begin_krylov(int phase) {
  kphase_ = phase;
  t_ = 0;
  sym_ready_ = false;
  if (p_.method == LD_METHOD_OSLQ || (p_.method == LD_METHOD_SO_SLQ && phase == 1)) {
    kB_ = B_;
    kld_ = ldB_;
    kg_ = gBp_;
    kgu_ = gBu_;
    kguv_ = gBuv_;
    kps_ = psB_;
    kpin_ = false;
    kfull_ = false;
    kns_ = std::min(k_, m_) + 1;
  } else if (phase == 0) {
    kB_ = s_;
    kld_ = ld1_;
    kg_ = g1p_;
    kgu_ = g1u_;
    kguv_ = g1u_;
    kps_ = ps1_;
    kpin_ = false;
    kfull_ = !two_pass_;
    kns_ = two_pass_ ? std::min(m_ + 1, std::min(k_, m_) + 1 + kCombBatch) : m_ + 1;
  } else {
    kB_ = B_;
    kld_ = ldB_;
    kg_ = gBp_;
    kgu_ = gBu_;
    kguv_ = gBuv_;
    kps_ = psB_;
    kpin_ = true;
    kfull_ = false;
    kns_ = std::min(k_, m_) + 2;
  }
  kslots_ = slots_;
  // the sketch-image runs of a two-pass sketch keep every vector's
  // multiplier (the combination coefficients need all of them)
  kmfull_ = kfull_ || (phase == 0 && two_pass_);
  kmult_ = (phase == 0 && two_pass_) ? multall_ : mult_;
  slot_elems_ = (size_t)n_ * kld_;
  pending_check_ = false;
  // the second pass of a two-pass sketch needs the basis vectors v_1 .. v_m
  // only: its last step (which forms v_m+1) is skipped
  kend_ = (phase == 0 && two_pass_ && opass_ == 1) ? m_ - 1 : m_;
  return LD_OK;
}

// Start block of the sketch-image runs: the sketch columns S themselves in
// Krylov precision, their norms and per-run start state.
ld_status Run::sketch_runs_start(hipStream_t st) {
  LD_LAUNCH(LD_PROF_PROBES, (double)n_ * ld1_ * xb_,
            launch_probes(st, p_.probe_dist, p_.seed, n_, 0, ld1_, s_, slots_, xb_, ld1_, 0,
                          seed_dev_));
  VecSet vs{};
  vs.x[0] = slots_;
  int nb = 0;
  LD_LAUNCH(LD_PROF_DOTS, (double)n_ * ld1_ * xb_,
            launch_dots(st, g1_, slots_, vs, 1, 0, part_, &nb));
  LD_LAUNCH(LD_PROF_SMALL, (double)nb * ld1_ * 8,
            launch_start_finish(st, s_, ld1_, part_, nb, norm2_, two_pass_ ? multall_ : mult_,
                                active_, meff_, nullptr, 0, 1.0));
  return LD_OK;
}

// Two-pass sketch image: Y (+)= sum_{j = comb_next_ .. upto} coef_j X_j,
// X_j the ring slot of basis vector j (at most two launches when the range
// wraps the ring); the FMA chain per entry runs over j in order, as in the
// one-pass combine over the kept basis.
ld_status Run::sketch_combine_upto(hipStream_t st, int upto) {
  while (comb_next_ <= upto) {
    const int slot = comb_next_ % kns_;
    const int cnt = std::min(upto - comb_next_ + 1, kns_ - slot);
    const void* base = static_cast<const char*>(slots_) + (size_t)slot * slot_elems_ * xb_;
    LD_LAUNCH(LD_PROF_SKETCH, (double)cnt * n_ * ld1_ * xb_ + (double)n_ * lds_ * 16,
              launch_combine(st, n_, ld1_, cnt, base, xb_, slot_elems_,
                             coefs_ + (size_t)comb_next_ * ld1_, Y_, lds_, comb_next_ > 0));
    comb_next_ += cnt;
  }
  return LD_OK;
}

// The probe kernels read the seed from a device word, so that the launch
// sequence of an estimate does not depend on it.
ld_status Run::write_seed(hipStream_t st) {
  const FillItem fi[2] = {{seed_dev_, 1, (uint32_t)(p_.seed & 0xFFFFFFFFu)},
                          {reinterpret_cast<uint32_t*>(seed_dev_) + 1, 1,
                           (uint32_t)(p_.seed >> 32)}};
  LD_HIP(launch_fill(st, fi, 2));
  return LD_OK;
}

ld_status Run::run_prologue(hipStream_t st) {
  if (!ev0_) LD_HIP(hipEventCreate(&ev0_));
  if (!ev1_) LD_HIP(hipEventCreate(&ev1_));
  if (!capturing_) {
    LD_HIP(hipEventRecord(ev0_, st));
    ld_status rc = write_seed(st);
    if (rc != LD_OK) return rc;
  }
  {
    // run flags, QR flags and (Arnoldi methods) the Hessenberg blocks start
    // at zero
    FillItem fi[3] = {{flags_, (size_t)ldB_, 0u},
                      {dflag_, 4, 0u},
                      {H_, (size_t)ldx_ * (m_ + 1) * m_ * 2, 0u}};
    LD_HIP(launch_fill(st, fi, p_.method == LD_METHOD_OSLQ ? 2 : 3));
  }
  const void* vals_sketch = (mixed_ && a_->vlo) ? a_->vlo : a_->v64;
  const int vt_sketch = mixed_ ? a_->vt_lo : VT_F64;
  if (p_.method == LD_METHOD_OSLQ) {
    if (s_ > 0) {
      // Y = J S, J = Q / alpha (Alg 3: sketch from J S, not from f(J) S)
      if (smask_) {
        const int vb = vt_sketch == VT_BF16 ? 2 : (vt_sketch == VT_F32 ? 4 : 8);
        LD_LAUNCH(LD_PROF_PROBES, (double)n_ * nws_ * 8,
                  launch_rademacher_mask(st, p_.seed, n_, 0, s_, smask_, nws_, seed_dev_));
        LD_LAUNCH(LD_PROF_SKETCH,
                  (double)a_->nnz * (vb + 4) + 4.0 * (n_ + 1) + (double)n_ * nws_ * 8 +
                      (double)n_ * lds_ * 8,
                  launch_spmm_signs(st, n_, a_->rp, a_->ci, vals_sketch, vt_sketch, smask_, nws_,
                                    s_, Y_, lds_, opscale_));
      } else {
        LD_LAUNCH(LD_PROF_PROBES, (double)n_ * lds_ * 8,
                  launch_probes(st, p_.probe_dist, p_.seed, n_, 0, lds_, s_, S_, 8, lds_, 0,
                                seed_dev_));
        LD_LAUNCH(LD_PROF_SPMM, spmm_bytes(lds_, 8),
                  launch_spmm(st, gS_, a_->rp, a_->ci, vals_sketch, vt_sketch, S_, Y_, nullptr,
                              opscale_, nullptr, 0, 0, nullptr, nullptr));
      }
      ld_status rc = sketch_qr(st, Y_, s_);
      if (rc != LD_OK) return rc;
    }
    ld_status rc = start_block(st, Y_, s_, false);
    if (rc != LD_OK) return rc;
    begin_krylov(0);
    return LD_OK;
  }
  // OSA-IOP: the sketch-image runs start from S itself (phase 0, basis kept
  // or, in two passes, a ring)
  if (s_ > 0) {
    ld_status rc = sketch_runs_start(st);
    if (rc != LD_OK) return rc;
    opass_ = 0;
    begin_krylov(0);
    return LD_OK;
  }
  ld_status rc = start_block(st, nullptr, 0, false);
  if (rc != LD_OK) return rc;
  begin_krylov(1);
  return LD_OK;
}

// OSA-IOP between the two Krylov phases: y_i = ||s_i|| V log(H) e1 +
// (log gamma - c) s_i for every sketch column (Alg 1 on each column of S),
// then A = orth(Y) and the start block [A | (I - A A^T) G] of the estimate
// runs (Alg 2).
ld_status Run::osa_sketch_combine(hipStream_t st) {
  const double shift = std::log(scale_) - c_;
  if (!two_pass_ || opass_ == 0) {
    // keep the sketch-image runs' Krylov dimensions for the step count
    LD_HIP(launch_copy_words(st, meff0_, meff_, (size_t)std::max(s_, 1)));
    LD_LAUNCH(LD_PROF_SMALL, 0,
              launch_hess_log(st, s_, m_, H_, meff_, quad_a(), quad_b(), work_, wstride_, 0, ell_,
                              nullptr, 0.0, nullptr, flags_, symtol(), need_));
    // the coefficient of v_t in each run's y (its multipliers folded in)
    LD_LAUNCH(LD_PROF_SMALL, 0,
              launch_osa_coef(st, s_, ld1_, m_, ell_, two_pass_ ? multall_ : mult_, norm2_, meff_,
                              shift, coefs_));
  }
  if (two_pass_ && opass_ == 0) {
    // second pass: the same runs again from S (the same kernels in the same
    // order give the same vectors), adding v_1 .. v_m into Y as they pass
    // through the ring; H is not needed again (the rewrite is identical)
    ld_status rc = sketch_runs_start(st);
    if (rc != LD_OK) return rc;
    opass_ = 1;
    comb_next_ = 0;
    begin_krylov(0);
    if (kend_ == 0) return sketch_combine_upto(st, m_ - 1);  // m = 1: v_1 only
    return LD_OK;
  }
  if (!two_pass_)
    LD_LAUNCH(LD_PROF_SKETCH, (double)m_ * n_ * ld1_ * xb_ + (double)n_ * lds_ * 8,
              launch_combine(st, n_, ld1_, m_, slots_, xb_, (size_t)n_ * ld1_, coefs_, Y_, lds_));
  if (p_.method == LD_METHOD_SO_SLQ) {
    // So-SLQ keeps the kb dominant left singular vectors of Y: Y V_k
    // Lambda_k^{-1/2} from the eigenpairs of Y^T Y (rank-deficient sketches
    // allowed), then CholQR2 of those kb columns
    LD_LAUNCH(LD_PROF_SKETCH, (double)n_ * s_ * 8,
              launch_gemm_tn(st, gS_, Y_, lds_, s_, Y_, lds_, s_, part_));
    LD_LAUNCH(LD_PROF_REDUCE, (double)gS_.nblk * s_ * s_ * 8,
              launch_reduce(st, part_, gS_.nblk, s_ * s_, gram_));
    LD_LAUNCH(LD_PROF_SKETCH, 0, launch_subspace_eig(st, s_, kb_, gram_, umat_, dflag_ + 2));
    LD_LAUNCH(LD_PROF_SKETCH, (double)n_ * (s_ + kb_) * 8,
              launch_rows_mat(st, n_, Y_, lds_, s_, umat_, kb_));
  }
  ld_status rc = sketch_qr(st, Y_, kb_);
  if (rc != LD_OK) return rc;
  rc = start_block(st, Y_, kb_, true);
  if (rc != LD_OK) return rc;
  begin_krylov(1);
  return LD_OK;
}

ld_status Run::run_krylov_step(hipStream_t st, int t, StepPlan* plan) {
  auto slot_of = [&](int j) -> int {
    if (kfull_) return j;
    if (kpin_) return j == 0 ? 0 : 1 + (j - 1) % (kns_ - 1);
    return j % kns_;
  };
  const size_t eb = (size_t)xb_;
  auto slot_ptr = [&](int j) -> void* {
    return static_cast<char*>(kslots_) + (size_t)slot_of(j) * slot_elems_ * eb;
  };
  auto mult_ptr = [&](int j) -> double* {
    return kmult_ + (size_t)(kmfull_ ? j : slot_of(j)) * kld_;
  };
  const void* vals = (mixed_ && a_->vlo) ? a_->vlo : a_->v64;
  const int vt = mixed_ ? a_->vt_lo : VT_F64;
  const double vec_bytes = (double)n_ * kld_ * xb_;
  void* W = slot_ptr(t + 1);
  const int j0 = std::max(0, t - k_ + 1);
  const int nv = t - j0 + 1;
  // Window inner products h_jt = v_j^T (J v_t), row v = j - j0 of dwin_.
  // The newest (j = t) is fused into the product's epilogue.  The second
  // newest, v_t-1^T J v_t = v_t^T (J v_t-1) since J is symmetric, was formed
  // by the previous step's update pass when that pass was a single launch
  // (sym_in); otherwise the product's epilogue reads v_t-1 for it.  Older
  // ones take separate passes.  Each launch writes its partial sums to its own
  // region of part_ with its own grid size and is reduced into its rows.
  // With sym_in the product also subtracts h_t-1,t v_t-1 from J v_t before
  // its epilogue (the coefficient is known), so the newest coefficient and
  // the older ones are taken from the reduced vector, and the update no
  // longer reads v_t-1: one vector pass less per step.
  const bool sym_in = sym_ready_ && nv >= 2;
  const int nf = sym_in ? 1 : std::min(2, nv);
  const int nold = nv - nf - (sym_in ? 1 : 0);  // rows [0, nold) need a dots pass
  // the update's vectors: the window without v_t-1 when the product took it
  // out (coefficient row nv - 2 skipped)
  const int upd_max = half_ ? 4 : kMaxNv;
  const bool presub = kps_ && sym_in && nv - 1 <= upd_max;
  const int nu = presub ? nv - 1 : nv;
  const int dhole = presub ? nv - 1 : 0;
  auto upd_vec = [&](int v) { return j0 + v + ((presub && v >= nv - 2) ? 1 : 0); };
  const void* sx = presub ? slot_ptr(t - 1) : nullptr;
  const double* smult = presub ? mult_ptr(t - 1) : nullptr;
  const double* sd = presub ? dwin_ + (size_t)(nv - 2) * kld_ : nullptr;
  VecSet vf{};
  for (int v = 0; v < nf; ++v) {
    vf.x[v] = slot_ptr(j0 + nv - nf + v);
    vf.mult[v] = mult_ptr(j0 + nv - nf + v);
  }
  // the update pass hands the next step its second-newest inner product when
  // it runs as one launch and the window holds two vectors or more
  const bool sym_out = k_ >= 2 && nv <= (half_ ? 4 : kMaxNv) && t + 1 < m_;
  // OSA-IOP estimate runs keep g_t = v1^T v_t.  v1 is read on odd steps only,
  // which form v1^T v_{t+1} (the new vector) and v1^T v_t (the step's input):
  // after any step t every g_0 .. g_t is known (g_0 = 1), which is all a run
  // that stops at that step (breakdown, adaptive test) uses.
  const bool v1step = kpin_ && (t & 1);
  const int nv_next = (t + 1) - std::max(0, t + 2 - k_) + 1;
  const bool check = adaptive() && (t + 1) % adapt_every_ == 0 && t + 1 < m_;
  // second pass of a two-pass sketch: after this step forms v_t+2 (index
  // t + 1), the vectors that fill a batch, or the last one needed, go into Y
  const bool pass_b = two_pass_ && kphase_ == 0 && opass_ == 1;
  const int produced = std::min(t + 1, m_ - 1);
  const bool comb = pass_b && (produced - comb_next_ + 1 >= kCombBatch || produced == m_ - 1);
  if (plan) {
    // a step of four launches (product, reduction, one update, bookkeeping)
    // can join a batch of other requests' steps; the caller launches it
    plan->valid = nold == 0 && nv <= 4 && !check && !prof_ && !pass_b;
    if (plan->valid) {
      SpmmItem& sp = plan->spmm;
      sp = SpmmItem{};
      sp.g = kg_;
      sp.rp = a_->rp;
      sp.ci = a_->ci;
      sp.va = vals;
      sp.vt = vt;
      sp.X = slot_ptr(t);
      sp.W = W;
      sp.xmult = mult_ptr(t);
      sp.opscale = opscale_ * vscale_;
      sp.fused = vf;
      sp.nf = nf;
      sp.voff = 0;
      sp.part = part_;
      sp.sx = sx;
      sp.smult = smult;
      sp.sd = sd;
      if (kg_.rg) sp.rg = row_groups();
      plan->red = ReduceItem{part_, 0, nf * kld_, dwin_ + (size_t)(nv - nf) * kld_};
      UpdateItem& up = plan->upd;
      up = UpdateItem{};
      up.g = v1step ? kguv_ : kgu_;
      up.W = W;
      for (int v = 0; v < nu; ++v) {
        up.vs.x[v] = slot_ptr(upd_vec(v));
        up.vs.mult[v] = mult_ptr(upd_vec(v));
      }
      up.nv = nu;
      up.d = dwin_;
      up.voff = 0;
      up.dhole = dhole;
      up.want_norm = 1;
      up.v1 = v1step ? slot_ptr(0) : nullptr;
      up.v1mult = v1step ? mult_ptr(0) : nullptr;
      up.sym = sym_out;
      up.part = part_;
      plan->fin = FinishItem{kB_, kld_, t, m_, dwin_, j0, nv, part_, 0, tol_, H_, meff_, active_,
                             mult_ptr(t + 1), v1step ? gq_ : nullptr, flags_,
                             sym_out ? nv_next - 2 : -1, 1.0 / vscale_,
                             v1step ? mult_ptr(t) : nullptr};
      sym_ready_ = sym_out;
      return LD_OK;
    }
  }
  int nb = 0;
  const RowGroups rgs = row_groups();
  LD_LAUNCH(LD_PROF_SPMM, spmm_bytes(kld_, xb_) + (nf - 1 + (presub ? 1 : 0)) * vec_bytes,
            launch_spmm(st, kg_, a_->rp, a_->ci, vals, vt, slot_ptr(t), W, mult_ptr(t),
                        opscale_ * vscale_, &vf, nf, 0, part_, &nb, sx, smult, sd,
                        kg_.rg ? &rgs : nullptr));
  LD_LAUNCH(LD_PROF_REDUCE, (double)nb * nf * kld_ * 8,
            launch_reduce(st, part_, nb, nf * kld_, dwin_ + (size_t)(nv - nf) * kld_));
  // more than 4 older vectors: one wide launch (up to 8) with one 16-byte
  // chunk per lane, when a row has at most 64 chunks
  Geom gd = kgu_;
  int dmax = kDotsPerLaunch;
  if (nold > kDotsPerLaunch && dots_rows() > kDotsPerLaunch) {
    const int ncolv = kld_ / (16 / xb_);
    const Geom g = make_geom_lc(n_, kld_, xb_, ncolv, 1);
    if (ncolv <= 64 && geom_usable(g)) {
      gd = g;
      dmax = kDotsWide;
    }
  }
  for (int c0 = 0; c0 < nold; c0 += dmax) {
    VecSet vs{};
    const int nc = std::min(dmax, nold - c0);
    for (int v = 0; v < nc; ++v) {
      vs.x[v] = slot_ptr(j0 + c0 + v);
      vs.mult[v] = mult_ptr(j0 + c0 + v);
    }
    double* pp = part_ + (size_t)2 * kld_ * kMaxBlocks;
    LD_LAUNCH(LD_PROF_DOTS, (double)(nc + 1) * vec_bytes,
              launch_dots(st, gd, W, vs, nc, 0, pp, &nb));
    LD_LAUNCH(LD_PROF_REDUCE, (double)nb * nc * kld_ * 8,
              launch_reduce(st, pp, nb, nc * kld_, dwin_ + (size_t)c0 * kld_));
  }
  // the update in one launch for windows up to 8 vectors (4 with FP16 vectors)
  for (int c0 = 0; c0 < nu; c0 += upd_max) {
    VecSet vs{};
    const int nc = std::min(upd_max, nu - c0);
    for (int v = 0; v < nc; ++v) {
      vs.x[v] = slot_ptr(upd_vec(c0 + v));
      vs.mult[v] = mult_ptr(upd_vec(c0 + v));
    }
    const bool last = c0 + nc >= nu;
    LD_LAUNCH(LD_PROF_UPDATE, (double)(nc + 2 + ((last && v1step) ? 1 : 0)) * vec_bytes,
              launch_update(st, (last && v1step) ? kguv_ : kgu_, W, vs, nc, dwin_, c0,
                            last ? 1 : 0,
                            (last && v1step) ? slot_ptr(0) : nullptr,
                            (last && v1step) ? mult_ptr(0) : nullptr, last && sym_out, part_, &nb,
                            dhole));
  }
  sym_ready_ = sym_out;
  LD_LAUNCH(LD_PROF_SMALL, (double)nb * 2 * kld_ * 8,
            launch_step_finish(st, kB_, kld_, t, m_, dwin_, j0, nv, part_, nb, tol_, H_,
                               meff_, active_, mult_ptr(t + 1), v1step ? gq_ : nullptr, flags_,
                               sym_out ? nv_next - 2 : -1, 1.0 / vscale_,
                               v1step ? mult_ptr(t) : nullptr));
  if (comb) {
    ld_status rc = sketch_combine_upto(st, produced);
    if (rc != LD_OK) return rc;
  }
  if (check) {
    // adaptive Krylov dimension: runs whose quadrature value settled stop;
    // the count of runs still going comes back to the host for the early exit
    if (!nact_host_) LD_HIP(hipHostMalloc((void**)&nact_host_, sizeof(int), hipHostMallocDefault));
    if (!check_ev_) LD_HIP(hipEventCreateWithFlags(&check_ev_, hipEventDisableTiming));
    const FillItem fi{nact_, 1, 0u};
    LD_HIP(launch_fill(st, &fi, 1));
    LD_LAUNCH(LD_PROF_SMALL, 0,
              launch_quad_check(st, kB_, m_, H_, meff_, quad_a(), quad_b(), t + 1, active_, kprev_,
                                p_.adapt_tol, mult_ptr(t + 1), flags_, nact_));
    LD_HIP(hipMemcpyAsync(nact_host_, nact_, sizeof(int), hipMemcpyDeviceToHost, st));
    LD_HIP(hipEventRecord(check_ev_, st));
    pending_check_ = true;
  }
  return LD_OK;
}

// Launch the planned steps of several requests: one launch per kernel for
// all of them (grouped by kernel instantiation), in the order of a step.
hipError_t launch_step_plans(hipStream_t st, std::vector<StepPlan>& plans) {
  const int n = (int)plans.size();
  if (n == 0) return hipSuccess;
  std::vector<SpmmItem> sp(n);
  std::vector<ReduceItem> rd(n);
  std::vector<UpdateItem> up(n);
  std::vector<FinishItem> fi(n);
  for (int i = 0; i < n; ++i) sp[i] = plans[i].spmm;
  hipError_t e = launch_spmm_batch(st, sp.data(), n);
  if (e != hipSuccess) return e;
  for (int i = 0; i < n; ++i) {
    rd[i] = plans[i].red;
    rd[i].nblk = sp[i].nblk;
    up[i] = plans[i].upd;
  }
  e = launch_reduce_batch(st, rd.data(), n);
  if (e != hipSuccess) return e;
  e = launch_update_batch(st, up.data(), n);
  if (e != hipSuccess) return e;
  for (int i = 0; i < n; ++i) {
    fi[i] = plans[i].fin;
    fi[i].nblk = up[i].nblk;
  }
  return launch_step_finish_batch(st, fi.data(), n);
}

ld_status Run::run_epilogue(hipStream_t st) {
  if (p_.method != LD_METHOD_OSA_IOP) {
    // K = e1^T log(T) e1 per run by the trapezoidal Stieltjes rule; runs whose
    // Ritz values leave the operator's spectral interval go to Golub-Welsch
    LD_LAUNCH(LD_PROF_SMALL, 0,
              launch_quad_log(st, B_, m_, H_, meff_, quad_a(), quad_b(), K_, need_, flags_));
    LD_LAUNCH(LD_PROF_SMALL, 0, launch_gauss_log(st, B_, m_, H_, meff_, K_, flags_, need_));
  } else {
    // x^T L_c x / ||x||^2 = sum_t g_t (log H e1)_t + log(gamma) - c
    LD_LAUNCH(LD_PROF_SMALL, 0,
              launch_hess_log(st, B_, m_, H_, meff_, quad_a(), quad_b(), work_, wstride_, 1,
                              nullptr, gq_, std::log(scale_) - c_, K_, flags_, symtol(), need_));
  }
  if (capturing_) return LD_OK;  // the replay enqueues the results after the graph
  LD_HIP(hipEventRecord(ev1_, st));
  return enqueue_results(st);
}

// The per-run results, packed on the device and copied to pinned host memory
// in stream order: collect() reads them once the stream (or the request's
// done event) has passed this point.
ld_status Run::enqueue_results(hipStream_t st) {
  if (!hpack_) {
    LD_HIP(hipHostMalloc(&hpack_, kHostPackBytes, hipHostMallocDefault));
    own_hpack_ = true;
  }
  const int ld = std::max(B_, s_);
  LD_HIP(launch_pack_results(st, ld, K_, norm2_, meff_, flags_, dflag_,
                             (p_.method != LD_METHOD_OSLQ && s_ > 0) ? meff0_ : nullptr, pack_));
  LD_HIP(hipMemcpyAsync(hpack_, pack_, pack_results_bytes(ld), hipMemcpyDeviceToHost, st));
  return LD_OK;
}

bool Run::capturable() const {
  return lo_ != hi_ && !(p_.adapt_tol > 0.0) && !(prof_ && prof_->any());
}

ld_status Run::advance(hipStream_t st, int budget, bool* done, StepPlan* plan, bool* planned) {
  *done = false;
  if (planned) *planned = false;
  while (budget > 0) {
    switch (stage_) {
      case ST_PROLOGUE: {
        if (lo_ == hi_) {
          // a zero-width Gershgorin interval means Q = q I exactly: every
          // traced operator L_c is a multiple of I and the estimate is
          // exactly n log q (collect forms it); no kernel runs
          if (!ev0_) LD_HIP(hipEventCreate(&ev0_));
          if (!ev1_) LD_HIP(hipEventCreate(&ev1_));
          LD_HIP(hipEventRecord(ev0_, st));
          LD_HIP(hipEventRecord(ev1_, st));
          stage_ = ST_DONE;
          --budget;
          break;
        }
        ld_status rc = run_prologue(st);
        if (rc != LD_OK) return rc;
        stage_ = ST_KRYLOV;
        --budget;
        break;
      }
      case ST_KRYLOV: {
        if (pending_check_) {
          // all runs stopped by the adaptive test: skip the remaining steps
          if (blocking_) LD_HIP(hipEventSynchronize(check_ev_));
          const hipError_t q = hipEventQuery(check_ev_);
          if (q == hipSuccess) {
            pending_check_ = false;
            if (*nact_host_ == 0) {
              t_ = m_;
              stage_ = ST_EPILOGUE;
              break;
            }
          } else if (q != hipErrorNotReady) {
            LD_HIP(q);
          }
        }
        if (t_ >= kend_) {
          // a phase without steps (the second sketch pass at m = 1)
          stage_ = (p_.method != LD_METHOD_OSLQ && kphase_ == 0) ? ST_COMBINE : ST_EPILOGUE;
          break;
        }
        ld_status rc = run_krylov_step(st, t_, plan);
        if (rc != LD_OK) return rc;
        ++t_;
        --budget;
        if (t_ >= kend_)
          stage_ = (p_.method != LD_METHOD_OSLQ && kphase_ == 0) ? ST_COMBINE : ST_EPILOGUE;
        if (plan && plan->valid) {
          // the caller launches this step (with other requests' steps) first
          *planned = true;
          return LD_OK;
        }
        break;
      }
      case ST_COMBINE: {
        ld_status rc = osa_sketch_combine(st);
        if (rc != LD_OK) return rc;
        stage_ = ST_KRYLOV;
        --budget;
        break;
      }
      case ST_EPILOGUE: {
        ld_status rc = run_epilogue(st);
        if (rc != LD_OK) return rc;
        stage_ = ST_DONE;
        --budget;
        break;
      }
      default:
        *done = true;
        return LD_OK;
    }
  }
  *done = stage_ == ST_DONE;
  return LD_OK;
}

ld_status Run::collect(hipStream_t st, ld_result* out, const ld_detail* detail, hipEvent_t done) {
  if (done)
    LD_HIP(hipEventSynchronize(done));  // a shared stream may hold later work of other requests
  else
    LD_HIP(hipStreamSynchronize(st));
  if (prof_) LD_HIP(prof_->harvest());
  if (lo_ == hi_) {
    // Q = q I (see advance): x^T L_c x / ||x||^2 = log q - c for every run
    float ms = 0.f;
    LD_HIP(hipEventElapsedTime(&ms, ev0_, ev1_));
    ld_result res{};
    res.logdet = (double)n_ * std::log(lo_);
    res.shift_c = c_;
    res.tr_sketch = 0.0;
    res.tr_resid = res.logdet - (double)n_ * c_;
    res.lambda_lo = lo_;
    res.lambda_hi = hi_;
    res.scale = scale_;
    res.device_ms = ms;
    res.latency_ms = (now_seconds() - t_submit_) * 1e3;
    if (detail) {
      for (int p = 0; p < B_; ++p) {
        if (detail->probe_K) detail->probe_K[p] = std::log(lo_) - c_;
        if (detail->probe_norm2) detail->probe_norm2[p] = 0.0;
        if (detail->probe_steps) detail->probe_steps[p] = 0;
      }
      if (detail->tri_alpha) std::memset(detail->tri_alpha, 0, (size_t)B_ * m_ * 8);
      if (detail->tri_beta) std::memset(detail->tri_beta, 0, (size_t)B_ * m_ * 8);
      if (detail->sketch_basis) std::memset(detail->sketch_basis, 0, (size_t)n_ * kb_ * 8);
    }
    *out = res;
    return LD_OK;
  }
  // the packed results the epilogue copied to pinned memory (layout of
  // launch_pack_results)
  const int ldp = std::max(B_, s_);
  const double* pK = static_cast<const double*>(hpack_);
  const double* pN = pK + ldp;
  const int* pM = reinterpret_cast<const int*>(pN + ldp);
  const int* pF = pM + ldp;
  const int* pD = pF + ldp;
  const int* pM0 = pD + 4;
  std::vector<double> K(pK, pK + B_), nrm(pN, pN + B_);
  std::vector<int> meff(pM, pM + B_), flags(pF, pF + B_);
  const int dflag[3] = {pD[0], pD[1], pD[2]};
  float ms = 0.f;
  LD_HIP(hipEventElapsedTime(&ms, ev0_, ev1_));
  if (dflag[0] || dflag[1])
    return set_error(LD_E_NUMERIC, "NaN/Inf in the Gram matrix of the sketch image");
  if (dflag[2])
    return set_error(LD_E_NUMERIC, "So-SLQ: the sketch has rank below subspace_rank, or the Jacobi "
                                   "eigen-decomposition of its Gram matrix did not converge");
  int nbreak = 0;
  for (int p = 0; p < B_; ++p) {
    if (flags[p] & 1) return set_error(LD_E_NUMERIC, "NaN/Inf in Krylov run " + std::to_string(p));
    if (flags[p] & 2)
      return set_error(LD_E_NOT_SPD, "non-positive Ritz value in Krylov run " + std::to_string(p));
    if (flags[p] & 8)
      return set_error(LD_E_NUMERIC, "tridiagonal eigenvalues did not converge, run " +
                                         std::to_string(p));
    if (flags[p] & 4) ++nbreak;
  }
  // trace assembly in a fixed order: basis runs, then residual runs (the
  // Gauss quadrature methods start from unit basis vectors; OSA-IOP's K is
  // per unit norm of its start vector)
  double tr_sketch = 0.0;
  int basis_rank = 0;  // basis columns kept by the QR (dropped ones are zero, K = 0)
  for (int i = 0; i < kb_; ++i) {
    tr_sketch += (p_.method != LD_METHOD_OSA_IOP) ? K[i] : nrm[i] * K[i];
    basis_rank += nrm[i] > 0.0 ? 1 : 0;
  }
  double acc = 0.0;
  for (int j = kb_; j < B_; ++j) acc += nrm[j] * K[j];
  const double tr_resid = acc / r_;
  ld_result res{};
  res.logdet = (double)n_ * c_ + (tr_sketch + tr_resid);
  res.tr_sketch = tr_sketch;
  res.tr_resid = tr_resid;
  res.shift_c = c_;
  res.lambda_lo = lo_;
  res.lambda_hi = hi_;
  res.scale = scale_;
  int64_t steps = 0;
  int minst = m_;
  for (int p = 0; p < B_; ++p) {
    steps += meff[p];
    if (nrm[p] > 0) minst = std::min(minst, meff[p]);
  }
  if (p_.method != LD_METHOD_OSLQ && s_ > 0) {
    // OSA-IOP and So-SLQ also ran s Krylov runs for the sketch image
    for (int p = 0; p < s_; ++p) steps += pM0[p];
  }
  res.probe_steps = steps;
  const int64_t sketch_mv = (p_.method == LD_METHOD_OSLQ) ? s_ : (int64_t)s_ * m_;  // S or L S
  res.matvecs = sketch_mv + (int64_t)B_ * m_;
  res.min_steps = minst;
  res.n_breakdowns = nbreak;
  res.basis_rank = basis_rank;
  res.device_ms = ms;
  res.latency_ms = (now_seconds() - t_submit_) * 1e3;
  if (detail) {
    if (detail->probe_K) std::memcpy(detail->probe_K, K.data(), (size_t)B_ * 8);
    if (detail->probe_norm2) std::memcpy(detail->probe_norm2, nrm.data(), (size_t)B_ * 8);
    if (detail->probe_steps) std::memcpy(detail->probe_steps, meff.data(), (size_t)B_ * 4);
    if (detail->tri_alpha || detail->tri_beta) {
      std::vector<double> H((size_t)B_ * (m_ + 1) * m_);
      LD_HIP(hipMemcpy(H.data(), H_, H.size() * 8, hipMemcpyDeviceToHost));
      for (int p = 0; p < B_; ++p)
        for (int t = 0; t < m_; ++t) {
          const double* Hp = H.data() + (size_t)p * (m_ + 1) * m_;
          const bool live = t < meff[p];
          if (detail->tri_alpha)
            detail->tri_alpha[(size_t)p * m_ + t] = live ? Hp[(size_t)t * m_ + t] : 0.0;
          if (detail->tri_beta)
            detail->tri_beta[(size_t)p * m_ + t] = live ? Hp[(size_t)(t + 1) * m_ + t] : 0.0;
        }
    }
    if (detail->sketch_basis && kb_ > 0) {
      std::vector<double> Y((size_t)n_ * lds_);
      LD_HIP(hipMemcpy(Y.data(), Y_, Y.size() * 8, hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < n_; ++i)
        for (int j = 0; j < kb_; ++j) detail->sketch_basis[i * kb_ + j] = Y[(size_t)i * lds_ + j];
    }
  }
  *out = res;
  return LD_OK;
}

// ---------------------------------------------------------------------------
// Autotuner of the Krylov-step geometry (lanes per row L, chunks per lane C).
// ---------------------------------------------------------------------------

// (L, C) pairs for a block of ld columns: L a power of two <= 64, C <= kMaxC,
// L * C chunks covering the row with at most half a row idle; the default
// geometry first.  With split > 0 (the product) also every entry split
// 2^e <= 8 of each pair with L 2^e <= 64 lanes per row, encoded as
// (L 2^e) | (e << 8).  Then the pairs L = ceil(chunks / C) where that is
// not a power of two (floor(64 / L) rows per wave).  With interleave, every
// candidate again with the product's chunks interleaved over the XCDs
// (bit 12), and every power-of-two one with its rows in tiles of each given
// stride that is a multiple of its rows per wave (bits 16..30), both timed
// for the product only.
static std::vector<std::pair<int, int>> tune_candidates(int64_t n, int ld, int xbytes,
                                                        bool split, bool interleave,
                                                        const std::vector<int>& strides) {
  const Geom d = make_geom(n, ld, xbytes);
  std::vector<std::pair<int, int>> out{{d.L, d.C}};
  for (int L = 1; L <= 64; L <<= 1)
    for (int C = 1; C <= kMaxC; ++C) {
      const int idle = L * C - d.ncolv;
      if (idle < 0 || 2 * idle > d.ncolv) continue;
      for (int e = 0; e <= (split ? 3 : 0); ++e) {
        if ((L << e) > 64 || (L == d.L && C == d.C && e == 0)) continue;
        Geom g = make_geom_lc(n, ld, xbytes, L << e, C);
        g.lges = e;
        if (geom_usable(g)) out.push_back({(L << e) | (e << 8), C});
      }
    }
  for (int C = 1; C <= kMaxC; ++C) {
    const int L = (d.ncolv + C - 1) / C;
    if (L > 64 || (L & (L - 1)) == 0) continue;
    if (geom_usable(make_geom_lc(n, ld, xbytes, L, C))) out.push_back({L, C});
  }
  if (interleave) {
    const size_t base = out.size();
    for (size_t i = 0; i < base; ++i) out.push_back({out[i].first | (1 << 12), out[i].second});
  }
  const size_t base = out.size();
  for (size_t i = 0; i < base; ++i) {
    const int L = out[i].first & 0xff;
    if (L & (L - 1)) continue;
    for (int S : strides) {
      Geom g = make_geom_lc(n, ld, xbytes, L, out[i].second);
      g.lges = (out[i].first >> 8) & 0xf;
      g.ts = S;
      if (S % (64 / L) == 0 && geom_usable(g)) out.push_back({out[i].first | (S << 16), out[i].second});
    }
  }
  return out;
}

static Geom candidate_geom(int64_t n, int ld, int xbytes, const std::pair<int, int>& c) {
  Geom g = make_geom_lc(n, ld, xbytes, c.first & 0xff, c.second);
  g.lges = (c.first >> 8) & 0xf;
  g.xil = (c.first >> 12) & 1;
  g.ts = (c.first >> 16) & 0x7fff;
  g.rg = (c.first >> 13) & 1;
  return g;
}

// Row strides worth a row-tile trial for the product: the positive column
// offsets (col - row) that occur in at least a quarter of the rows of two
// sampled windows (the start and the middle of the matrix), most frequent
// first, at most two.  A stencil on a grid gives its line and plane strides.
std::vector<int> Run::stride_candidates(hipStream_t st) const {
  constexpr int64_t kWin = 4096;
  std::map<int64_t, int64_t> count;
  int64_t rows = 0;
  for (int64_t r0 : {int64_t(0), n_ / 2}) {
    const int64_t r1 = std::min(n_, r0 + kWin);
    if (r1 <= r0 || (r0 > 0 && r0 < kWin)) continue;
    std::vector<int> rp((size_t)(r1 - r0 + 1));
    if (hipMemcpyAsync(rp.data(), a_->rp + r0, rp.size() * sizeof(int), hipMemcpyDeviceToHost,
                       st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
      return {};
    // at most kMaxEntries sampled entries per window (long rows)
    constexpr int kMaxEntries = 1 << 20;
    size_t nr = rp.size() - 1;
    while (nr > 1 && rp[nr] - rp.front() > kMaxEntries) nr /= 2;
    rp.resize(nr + 1);
    if (rp.back() - rp.front() > kMaxEntries) continue;
    const int64_t r1s = r0 + (int64_t)nr;
    std::vector<int> ci((size_t)(rp.back() - rp.front()));
    if (!ci.empty() &&
        (hipMemcpyAsync(ci.data(), a_->ci + rp.front(), ci.size() * sizeof(int),
                        hipMemcpyDeviceToHost, st) != hipSuccess ||
         hipStreamSynchronize(st) != hipSuccess))
      return {};
    for (int64_t i = r0; i < r1s; ++i) {
      for (int k = rp[i - r0] - rp.front(); k < rp[i - r0 + 1] - rp.front(); ++k) {
        const int64_t d = (int64_t)ci[k] - i;
        if (d >= 2 && d <= kMaxRowStride) ++count[d];
      }
      ++rows;
    }
  }
  std::vector<std::pair<int64_t, int>> byc;
  for (const auto& kv : count)
    if (4 * kv.second >= rows) byc.push_back({-kv.second, (int)kv.first});
  std::sort(byc.begin(), byc.end());
  std::vector<int> out;
  for (size_t i = 0; i < byc.size() && i < 2; ++i) out.push_back(byc[i].second);
  return out;
}

namespace {
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};
}  // namespace

ld_status Run::tune(hipStream_t st, int reps, ld_tune_result* out) {
  const int vt = mixed_ ? a_->vt_lo : VT_F64;
  std::vector<int> widths{ldB_};
  if (p_.method != LD_METHOD_OSLQ && s_ > 0 && ld1_ != ldB_) widths.push_back(ld1_);
  if (reps == 0) {
    std::lock_guard<std::mutex> lk(a_->tune_mu);
    for (int ld : widths) {
      a_->tune.erase(tune_key(ld, xb_, vt, 0));
      for (bool ps : {true, false}) {
        a_->tune.erase(tune_key(ld, xb_, vt, upd_which(ps)));
        a_->tune.erase(tune_key(ld, xb_, vt, upd_which(ps) + 2));
      }
      a_->tune.erase(tune_key(ld, xb_, vt, 2));
    }
    a_->tune_ver.fetch_add(1);
    if (out) *out = ld_tune_result{};
    return LD_OK;
  }
  const int ldmax = std::max(ldB_, ld1_);
  const size_t n = (size_t)n_;
  const size_t vec = align_up(n * ldmax * xb_);
  // X (the product's input and newest window vector), V (an older window
  // vector), W (product / update in place), column multipliers, zero
  // coefficients and the partial sums
  const size_t small = align_up((size_t)ldmax * 8) + align_up((size_t)kMaxNv * ldmax * 8);
  const size_t partb = align_up((size_t)kMaxBlocks * 4 * ldmax * 8);
  DeviceBuffer buf;
  LD_HIP(buf.ensure(3 * vec + small + partb));
  char* base = static_cast<char*>(buf.ptr);
  void* X = base;
  void* V = base + vec;
  void* W = base + 2 * vec;
  double* mult = reinterpret_cast<double*>(base + 3 * vec);
  double* dcoef = reinterpret_cast<double*>(base + 3 * vec + align_up((size_t)ldmax * 8));
  double* part = reinterpret_cast<double*>(base + 3 * vec + small);
  const std::vector<double> ones((size_t)ldmax, 1.0);
  LD_HIP(hipMemcpyAsync(mult, ones.data(), ones.size() * 8, hipMemcpyHostToDevice, st));
  LD_HIP(hipMemsetAsync(dcoef, 0, (size_t)kMaxNv * ldmax * 8, st));
  const void* vals = (mixed_ && a_->vlo) ? a_->vlo : a_->v64;
  // the launches of a steady-state step: with k >= 2 the product subtracts
  // the second-newest vector (V here) and the update takes the rest of the
  // window and forms the next second-newest inner product
  const bool sym = k_ >= 2;
  const int nv = upd_steady_nv(true);
  EventPair ev;
  LD_HIP(hipEventCreate(&ev.a));
  LD_HIP(hipEventCreate(&ev.b));
  for (size_t wi = 0; wi < widths.size(); ++wi) {
    const int ld = widths[wi];
    LD_HIP(launch_probes(st, PROBE_RADEMACHER, 0x7475u, n_, 0, ld, ld, X, xb_, ld, 0));
    LD_HIP(launch_probes(st, PROBE_RADEMACHER, 0x7476u, n_, 0, ld, ld, V, xb_, ld, 0));
    // entry splits only pay on rows of many entries
    auto cand = tune_candidates(n_, ld, xb_, a_->nnz >= 16 * a_->n, true,
                                stride_candidates(st));
    if (rg_ok()) {
      // the row-group product in every plain geometry of at most two chunks
      // per lane (both chunk mappings), and its default first among them
      const size_t base = cand.size();
      const int ncolv = ld / (16 / xb_);
      if (ncolv <= 64) cand.push_back({ncolv | (1 << 13), 1});
      for (size_t i = 0; i < base; ++i) {
        const Geom g = candidate_geom(n_, ld, xb_, cand[i]);
        if (g.lges == 0 && g.ts == 0 && g.C <= 2 && !(g.L == ncolv && g.C == 1 && g.xil == 0))
          cand.push_back({cand[i].first | (1 << 13), cand[i].second});
      }
    }
    const RowGroups rgs = row_groups();
    const int nc = (int)cand.size();
    std::vector<double> tp(nc, 1e300), tu(nc, 1e300);
    VecSet vf{};
    vf.x[0] = X;
    vf.mult[0] = mult;
    VecSet vu{};
    for (int v = 0; v < nv; ++v) {
      vu.x[v] = v + 1 == nv ? X : V;
      vu.mult[v] = mult;
    }
    for (int round = 0; round < 3; ++round)
      for (int c = 0; c < nc; ++c) {
        const Geom g = candidate_geom(n_, ld, xb_, cand[c]);
        int nb = 0;
        float ms = 0.f;
        auto product = [&]() {
          return launch_spmm(st, g, a_->rp, a_->ci, vals, vt, X, W, mult, opscale_ * vscale_, &vf, 1, 0,
                             part, &nb, sym ? V : nullptr, sym ? mult : nullptr,
                             sym ? dcoef : nullptr, g.rg ? &rgs : nullptr);
        };
        auto update = [&]() {
          return launch_update(st, g, W, vu, nv, dcoef, 0, 1, nullptr, nullptr, sym, part, &nb,
                               sym ? nv : 0);
        };
        LD_HIP(product());  // warm-up
        LD_HIP(hipEventRecord(ev.a, st));
        for (int i = 0; i < reps; ++i) LD_HIP(product());
        LD_HIP(hipEventRecord(ev.b, st));
        LD_HIP(hipEventSynchronize(ev.b));
        LD_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
        tp[c] = std::min(tp[c], (double)ms / reps);
        // the update has no sparse entries to split and keeps its own mapping
        if (g.lges != 0 || g.xil != 0 || g.ts != 0 || g.rg != 0) continue;
        LD_HIP(update());
        LD_HIP(hipEventRecord(ev.a, st));
        for (int i = 0; i < reps; ++i) LD_HIP(update());
        LD_HIP(hipEventRecord(ev.b, st));
        LD_HIP(hipEventSynchronize(ev.b));
        LD_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
        tu[c] = std::min(tu[c], (double)ms / reps);
      }
    // a candidate replaces the best so far only when more than 1% faster
    // (timing noise would otherwise pick geometries at random, and the
    // update's geometry also serves the wider OSA-IOP v1 pass, which the
    // tuner does not time)
    int bp = 0, bu = 0;
    for (int c = 1; c < nc; ++c) {
      if (tp[c] < 0.99 * tp[bp]) bp = c;
      if (tu[c] < 0.99 * tu[bu]) bu = c;
    }
    // the step schedule: the product subtracting the second-newest vector
    // (as swept above) or the update taking the whole window (the product
    // then streams one vector less and the update one more), both timed
    // again in the same rounds; the latter is kept only when its product
    // and update are more than 1% faster per step
    bool presub = true;
    int bun = 0;
    double ps_ms = tp[bp] + tu[bu], plain_ms = 0.0;
    if (sym) {
      const int nvn = upd_steady_nv(false);
      VecSet vun{};
      for (int v = 0; v < nvn; ++v) {
        vun.x[v] = v + 1 == nvn ? X : V;
        vun.mult[v] = mult;
      }
      const Geom gp = candidate_geom(n_, ld, xb_, cand[bp]);
      const Geom gu = candidate_geom(n_, ld, xb_, cand[bu]);
      std::vector<int> ucand;
      for (int c = 0; c < nc; ++c) {
        const Geom g = candidate_geom(n_, ld, xb_, cand[c]);
        if (g.lges == 0 && g.xil == 0 && g.ts == 0 && g.rg == 0) ucand.push_back(c);
      }
      double t_psp = 1e300, t_psu = 1e300, t_pp = 1e300;
      std::vector<double> t_pu(nc, 1e300);
      auto timed = [&](auto&& fn, double& best) -> hipError_t {
        hipError_t e = fn();  // warm-up
        if (e == hipSuccess) e = hipEventRecord(ev.a, st);
        for (int i = 0; i < reps && e == hipSuccess; ++i) e = fn();
        if (e == hipSuccess) e = hipEventRecord(ev.b, st);
        if (e == hipSuccess) e = hipEventSynchronize(ev.b);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.a, ev.b);
        if (e == hipSuccess) best = std::min(best, (double)ms / reps);
        return e;
      };
      int nb = 0;
      for (int round = 0; round < 3; ++round) {
        LD_HIP(timed([&]() {
          return launch_spmm(st, gp, a_->rp, a_->ci, vals, vt, X, W, mult, opscale_ * vscale_,
                             &vf, 1, 0, part, &nb, V, mult, dcoef, gp.rg ? &rgs : nullptr);
        }, t_psp));
        LD_HIP(timed([&]() {
          return launch_spmm(st, gp, a_->rp, a_->ci, vals, vt, X, W, mult, opscale_ * vscale_,
                             &vf, 1, 0, part, &nb, nullptr, nullptr, nullptr,
                             gp.rg ? &rgs : nullptr);
        }, t_pp));
        LD_HIP(timed([&]() {
          return launch_update(st, gu, W, vu, nv, dcoef, 0, 1, nullptr, nullptr, true, part,
                               &nb, nv);
        }, t_psu));
        for (int c : ucand) {
          const Geom g = candidate_geom(n_, ld, xb_, cand[c]);
          LD_HIP(timed([&]() {
            return launch_update(st, g, W, vun, nvn, dcoef, 0, 1, nullptr, nullptr, true, part,
                                 &nb);
          }, t_pu[c]));
        }
      }
      bun = ucand.front();
      for (int c : ucand)
        if (t_pu[c] < 0.99 * t_pu[bun]) bun = c;
      ps_ms = t_psp + t_psu;
      plain_ms = t_pp + t_pu[bun];
      presub = !(plain_ms < 0.99 * ps_ms);
    }
    // OSA-IOP estimate runs: the update that also reads v1 (every other
    // step), in the chosen schedule, over the update candidates
    int bv = -1;
    if (p_.method == LD_METHOD_OSA_IOP && wi == 0) {
      const int nvs = upd_steady_nv(presub);
      VecSet vv{};
      for (int v = 0; v < nvs; ++v) {
        vv.x[v] = v + 1 == nvs ? X : V;
        vv.mult[v] = mult;
      }
      std::vector<double> tv(nc, 1e300);
      for (int round = 0; round < 3; ++round)
        for (int c = 0; c < nc; ++c) {
          const Geom g = candidate_geom(n_, ld, xb_, cand[c]);
          if (g.lges != 0 || g.xil != 0 || g.ts != 0 || g.rg != 0) continue;
          int nb = 0;
          auto upd = [&]() {
            return launch_update(st, g, W, vv, nvs, dcoef, 0, 1, V, mult, sym, part, &nb,
                                 (sym && presub) ? nvs : 0);
          };
          LD_HIP(upd());
          LD_HIP(hipEventRecord(ev.a, st));
          for (int i = 0; i < reps; ++i) LD_HIP(upd());
          LD_HIP(hipEventRecord(ev.b, st));
          LD_HIP(hipEventSynchronize(ev.b));
          float ms = 0.f;
          LD_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
          tv[c] = std::min(tv[c], (double)ms / reps);
        }
      bv = 0;
      for (int c = 1; c < nc; ++c)
        if (tv[c] < 0.99 * tv[bv]) bv = c;
    }
    {
      std::lock_guard<std::mutex> lk(a_->tune_mu);
      a_->tune[tune_key(ld, xb_, vt, 0)] = cand[bp];
      if (bv >= 0) a_->tune[tune_key(ld, xb_, vt, upd_which(presub) + 2)] = cand[bv];
      if (presub) {
        a_->tune[tune_key(ld, xb_, vt, upd_which(true))] = cand[bu];
        a_->tune.erase(tune_key(ld, xb_, vt, 2));
      } else {
        a_->tune[tune_key(ld, xb_, vt, upd_which(false))] = cand[bun];
        a_->tune[tune_key(ld, xb_, vt, 2)] = {1, 0};
      }
      a_->tune_ver.fetch_add(1);
    }
    if (wi == 0 && out) {
      *out = ld_tune_result{};
      out->spmm_lanes = cand[bp].first & 0xff;
      out->spmm_chunks = cand[bp].second;
      out->spmm_entry_split = 1 << ((cand[bp].first >> 8) & 0xf);
      out->spmm_interleave = (cand[bp].first >> 12) & 1;
      out->spmm_row_stride = (cand[bp].first >> 16) & 0x7fff;
      out->spmm_row_groups = (cand[bp].first >> 13) & 1;
      out->update_lanes = cand[presub ? bu : bun].first;
      out->update_chunks = cand[presub ? bu : bun].second;
      out->spmm_ms = tp[bp];
      out->spmm_default_ms = tp[0];
      out->update_ms = tu[bu];
      out->update_default_ms = tu[0];
      out->candidates = nc;
      out->step_presub = presub ? 1 : 0;
      out->step_presub_ms = ps_ms;
      out->step_plain_ms = plain_ms;
    }
  }
  return LD_OK;
}

ld_status Run::tune_set(int spmm_lanes, int spmm_chunks, int spmm_split, int update_lanes,
                         int update_chunks, int spmm_interleave, int spmm_row_stride,
                         int step_presub, int spmm_row_groups) {
  int e = 0;
  while (e < 4 && (1 << e) < spmm_split) ++e;
  Geom gp = make_geom_lc(n_, ldB_, xb_, spmm_lanes, spmm_chunks);
  gp.lges = e;
  gp.ts = spmm_row_stride;
  gp.rg = spmm_row_groups == 1 ? 1 : 0;
  if ((1 << e) != spmm_split || !geom_usable(gp) || (spmm_interleave != 0 && spmm_interleave != 1) ||
      !geom_usable(make_geom_lc(n_, ldB_, xb_, update_lanes, update_chunks)) ||
      (step_presub != 0 && step_presub != 1) || (spmm_row_groups != 0 && spmm_row_groups != 1) ||
      (gp.rg && !rg_ok()))
    return set_error(LD_E_INVALID_ARG,
                     "lanes must be <= 64 (a power of two with an entry split), chunks in "
                     "[1, 4] and the entry split 1, 2, 4 or 8 (at most the lanes), the lanes "
                     "per split group and the chunks covering the probe block, interleave 0 "
                     "or 1, the row stride 0 or a multiple of the rows per wave (64 / lanes, "
                     "lanes a power of two) up to 32767, the step schedule 0 or 1, row "
                     "groups 0 or 1 (1: FP32 or FP64 Krylov vectors on a matrix that keeps "
                     "row groups, at most 2 chunks, no entry split, no row stride)");
  const int vt = mixed_ ? a_->vt_lo : VT_F64;
  std::lock_guard<std::mutex> lk(a_->tune_mu);
  a_->tune[tune_key(ldB_, xb_, vt, 0)] = {spmm_lanes | (e << 8) | (spmm_interleave << 12) |
                                             (gp.rg << 13) | (spmm_row_stride << 16),
                                         spmm_chunks};
  a_->tune[tune_key(ldB_, xb_, vt, upd_which(step_presub != 0))] = {update_lanes, update_chunks};
  if (step_presub)
    a_->tune.erase(tune_key(ldB_, xb_, vt, 2));
  else
    a_->tune[tune_key(ldB_, xb_, vt, 2)] = {1, 0};
  a_->tune_ver.fetch_add(1);
  return LD_OK;
}

// Host threads for a pass over `work` items: one per ~4M items, at most 16.
static int host_threads(int64_t work) {
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  const int64_t want = std::max<int64_t>(1, work / (int64_t(1) << 22));
  return (int)std::min<int64_t>(std::min(hw, 16), want);
}

// f(t, begin, end) on nt contiguous ranges of [0, count), in threads.
template <typename F>
static void parallel_ranges(int64_t count, int nt, F f) {
  if (nt <= 1) {
    f(0, 0, count);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t) {
    const int64_t b = count * t / nt, e = count * (t + 1) / nt;
    th.emplace_back([=, &f]() { f(t, b, e); });
  }
  for (auto& x : th) x.join();
}

Stager::~Stager() {
  if (st) (void)hipStreamSynchronize(st);
  for (int i = 0; i < 2; ++i) {
    if (buf[i]) (void)hipHostFree(buf[i]);
    if (ev[i]) (void)hipEventDestroy(ev[i]);
  }
  if (st) (void)hipStreamDestroy(st);
}

hipError_t Stager::init() {
  hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  for (int i = 0; i < 2 && e == hipSuccess; ++i) {
    e = hipHostMalloc((void**)&buf[i], kChunk, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
  }
  return e;
}

hipError_t Stager::upload_fill(void* dst, size_t bytes,
                               const std::function<void(char*, size_t, size_t)>& fill) {
  char* d = static_cast<char*>(dst);
  size_t i = 0;
  for (size_t off = 0; off < bytes; off += kChunk, ++i) {
    const size_t len = std::min(kChunk, bytes - off);
    char* b = buf[i & 1];
    if (i >= 2) {
      // the buffer's previous copy must have left it
      const hipError_t e = hipEventSynchronize(ev[i & 1]);
      if (e != hipSuccess) return e;
    }
    fill(b, off, len);
    hipError_t e = hipMemcpyAsync(d + off, b, len, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(ev[i & 1], st);
    if (e != hipSuccess) return e;
  }
  return hipStreamSynchronize(st);
}

hipError_t Stager::upload(void* dst, const void* src, size_t bytes) {
  const char* s = static_cast<const char*>(src);
  return upload_fill(dst, bytes, [&](char* b, size_t off, size_t len) {
    parallel_ranges((int64_t)len, host_threads((int64_t)len / 4), [&](int, int64_t b0, int64_t b1) {
      std::memcpy(b + b0, s + off + b0, (size_t)(b1 - b0));
    });
  });
}

}  // namespace ld

// ---------------------------------------------------------------------------
// Device-resident scratch of the no-allocation estimate.  A file-scope device
// array: every GPU the library runs on holds its own copy from module load
// until the process ends.  Host code never uses the array's name as an
// address: the device address of each GPU's copy is looked up once per device
// (with that device current) by hipGetSymbolAddress and kept here.
// ---------------------------------------------------------------------------
namespace ld {

constexpr size_t kScratchBytes = (size_t)256 << 20;  // 256 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
// calls of the no-allocation estimate on one device share its scratch: they
// run one at a time
std::mutex g_scratch_use_mu[kMaxDevices];
}  // namespace

// Device address of `device`'s scratch (looked up on the first call for the
// device; the device must be current).
static hipError_t scratch_ptr(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace ld

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace ld;

#define LD_HIP_API(expr)                                                                \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return set_error(LD_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Capture the launch sequence of a blocking estimate (everything between the
// seed write and the result pack) from the context's stream into a graph
// kept under `key`.  Nothing runs during the capture.
static ld_status capture_estimate(ld_ctx* ctx, Run& run, const GraphKey& key) {
  LD_HIP_API(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  run.set_capturing(true);
  bool done = false;
  ld_status rc = LD_OK;
  while (!done && rc == LD_OK) rc = run.advance(ctx->stream, 1 << 30, &done);
  run.set_capturing(false);
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(ctx->stream, &g);
  if (rc != LD_OK || ee != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    if (rc != LD_OK) return rc;
    return set_error(LD_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(ee));
  }
  hipGraphExec_t x = nullptr;
  const hipError_t ie = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (ie != hipSuccess) {
    (void)hipGraphDestroy(g);
    return set_error(LD_E_DEVICE, std::string("graph instantiation: ") + hipGetErrorString(ie));
  }
  LD_HIP_API(ctx->graphs.insert(key, g, x));
  return LD_OK;
}

extern "C" {

const char* ld_last_error(void) { return g_last_error.c_str(); }

ld_status ld_ctx_create(const ld_ctx_opts* opts, ld_ctx** out) {
  if (!out) return set_error(LD_E_INVALID_ARG, "null out pointer");
  ld_ctx_opts o{};
  if (opts) o = *opts;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return set_error(LD_E_DEVICE, "no HIP device available");
  if (o.device < 0 || o.device >= ndev) return set_error(LD_E_INVALID_ARG, "bad device ordinal");
  if (o.default_method != LD_METHOD_OSLQ && o.default_method != LD_METHOD_OSA_IOP &&
      o.default_method != LD_METHOD_SO_SLQ)
    return set_error(LD_E_INVALID_ARG, "bad default_method");
  if (o.default_precision != LD_PREC_FP64 && o.default_precision != LD_PREC_MIXED &&
      o.default_precision != LD_PREC_HALF && o.default_precision != LD_PREC_AUTO)
    return set_error(LD_E_INVALID_ARG, "bad default_precision");
  LD_HIP_API(hipSetDevice(o.device));
  std::unique_ptr<ld_ctx> c(new ld_ctx());
  c->device = o.device;
  c->opts = o;
  if (c->opts.max_slots <= 0) c->opts.max_slots = 16;
  if (o.hip_stream) {
    c->stream = static_cast<hipStream_t>(o.hip_stream);
    c->own_stream = false;
  } else {
    LD_HIP_API(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    c->own_stream = true;
  }
  if (c->opts.hbm_budget_bytes == 0) {
    size_t fr = 0, tot = 0;
    LD_HIP_API(hipMemGetInfo(&fr, &tot));
    c->opts.hbm_budget_bytes = (uint64_t)(0.8 * (double)fr);
  }
  // set-up of the no-allocation estimate: the device's scratch address, and
  // the events and pinned counter its runs use in place of creating their own
  void* sp = nullptr;
  LD_HIP_API(scratch_ptr(o.device, &sp));
  for (int i = 0; i < 3; ++i)
    LD_HIP_API(hipEventCreateWithFlags(&c->na_ev[i], i == 2 ? hipEventDisableTiming
                                                               : hipEventDefault));
  LD_HIP_API(hipHostMalloc((void**)&c->na_nact, sizeof(int), hipHostMallocDefault));
  LD_HIP_API(hipHostMalloc(&c->na_pack, kHostPackBytes, hipHostMallocDefault));
  *out = c.release();
  return LD_OK;
}

ld_status ld_ctx_destroy(ld_ctx* ctx) {
  if (!ctx) return set_error(LD_E_INVALID_ARG, "null context");
  if (ctx->n_matrices.load() > 0)
    return set_error(LD_E_BUSY, "destroy every matrix of the context first");
  (void)hipSetDevice(ctx->device);
  ctx->server.reset();
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  ctx->graphs.clear();
  ctx->workspace.release();
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  for (hipEvent_t& e : ctx->na_ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->na_nact) (void)hipHostFree(ctx->na_nact);
  if (ctx->na_pack) (void)hipHostFree(ctx->na_pack);
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return LD_OK;
}

// FP64 -> BF16 with a single round-to-nearest-even: truncate toward zero to
// FP32 (keeping whether anything was dropped), then round the low 16 bits.
static uint16_t double_to_bf16_rne(double d) {
  const double ad = std::fabs(d);
  float fa = (float)ad;
  if ((double)fa > ad) fa = std::nextafter(fa, 0.0f);
  const bool inexact = (double)fa != ad;
  uint32_t u;
  std::memcpy(&u, &fa, 4);
  const uint32_t lower = u & 0xFFFFu;
  uint32_t upper = u >> 16;
  if (lower > 0x8000u || (lower == 0x8000u && (inexact || (upper & 1u)))) ++upper;
  return (uint16_t)(upper | (std::signbit(d) ? 0x8000u : 0u));
}

// Row groups of kRowGroup consecutive rows (the sorted union of their
// columns, kRowGroup values per union column, zero where a row has no
// entry), kept where they gather much less than the rows: at least
// kRowGroupMinRatio entries per union column (covariance-like matrices; a
// 3D Laplacian has 1.3, a random graph 1.0), estimated first on a sample of
// groups on the host, then counted and built on the device.
static constexpr double kRowGroupMinRatio = 2.0;

// Union columns of group g (rows sorted, as the structure checks ensure).
static int64_t group_union_size(const int32_t* rp, const int32_t* ci, int64_t n, int64_t g) {
  const int64_t r0 = g * kRowGroup;
  const int nr = (int)std::min<int64_t>(kRowGroup, n - r0);
  int32_t k[kRowGroup], e[kRowGroup];
  for (int r = 0; r < nr; ++r) {
    k[r] = rp[r0 + r];
    e[r] = rp[r0 + r + 1];
  }
  int64_t cnt = 0;
  for (;;) {
    int32_t c = INT32_MAX;  // columns are below n <= INT32_MAX
    for (int r = 0; r < nr; ++r)
      if (k[r] < e[r]) c = std::min(c, ci[k[r]]);
    if (c == INT32_MAX) break;
    for (int r = 0; r < nr; ++r)
      if (k[r] < e[r] && ci[k[r]] == c) ++k[r];
    ++cnt;
  }
  return cnt;
}

ld_status ld_create_csr(ld_ctx* ctx, int64_t n, int64_t nnz, const int32_t* row_ptr,
                        const int32_t* col_idx, const double* values, int32_t vt,
                        double lambda_lo_hint, double lambda_hi_hint, ld_matrix** out) {
  if (!ctx || !out || !row_ptr || !col_idx || !values)
    return set_error(LD_E_INVALID_ARG, "null argument");
  if (n < 1 || nnz < n || n > INT32_MAX || nnz > INT32_MAX)
    return set_error(LD_E_INVALID_ARG, "need 1 <= n <= nnz <= 2^31-1");
  if (vt != LD_VT_FP64 && vt != LD_VT_FP32 && vt != LD_VT_BF16)
    return set_error(LD_E_INVALID_ARG, "bad value type");
  if (!(lambda_lo_hint >= 0.0) || !(lambda_hi_hint >= 0.0) ||
      (lambda_lo_hint > 0 && lambda_hi_hint > 0 && lambda_lo_hint > lambda_hi_hint))
    return set_error(LD_E_INVALID_ARG, "bad spectral hints");
  // structure checks on the host copy, rows split over host threads; the
  // error reported is the one the first failing row (in row order) gives
  if (row_ptr[0] != 0 || row_ptr[n] != nnz) return set_error(LD_E_BAD_CSR, "row_ptr[0] != 0 or row_ptr[n] != nnz");
  {
    struct Fail {
      int64_t row = INT64_MAX;
      ld_status st = LD_OK;
      const char* what = nullptr;
    };
    auto check_rows = [&](int64_t r0, int64_t r1, Fail* f) {
      for (int64_t i = r0; i < r1; ++i) {
        const int32_t a = row_ptr[i], b = row_ptr[i + 1];
        auto fail = [&](ld_status st, const char* what) {
          f->row = i;
          f->st = st;
          f->what = what;
        };
        if (b < a) return fail(LD_E_BAD_CSR, "row_ptr not monotone at row ");
        bool diag = false;
        for (int32_t k = a; k < b; ++k) {
          const int32_t c = col_idx[k];
          if (c < 0 || c >= n) return fail(LD_E_BAD_CSR, "column index out of range in row ");
          if (k > a && c <= col_idx[k - 1])
            return fail(LD_E_BAD_CSR, "columns not sorted/unique in row ");
          if (!std::isfinite(values[k])) return fail(LD_E_BAD_CSR, "non-finite value in row ");
          if (c == i) {
            diag = true;
            if (!(values[k] > 0.0)) return fail(LD_E_NOT_SPD, "non-positive diagonal entry in row ");
          }
        }
        if (!diag) return fail(LD_E_NOT_SPD, "missing diagonal entry in row ");
      }
    };
    const int nt = host_threads(nnz);
    std::vector<Fail> fails((size_t)nt);
    parallel_ranges(n, nt, [&](int t, int64_t r0, int64_t r1) { check_rows(r0, r1, &fails[t]); });
    const Fail* first = nullptr;
    for (const Fail& f : fails)
      if (f.st != LD_OK && (!first || f.row < first->row)) first = &f;
    if (first) return set_error(first->st, std::string(first->what) + std::to_string(first->row));
  }
  LD_HIP_API(hipSetDevice(ctx->device));
  static std::atomic<uint64_t> next_serial{1};
  std::unique_ptr<ld_matrix> m(new ld_matrix());
  m->serial = next_serial.fetch_add(1);
  m->ctx = ctx;
  m->n = n;
  m->nnz = nnz;
  m->vt = vt;
  m->lo_hint = lambda_lo_hint;
  m->hi_hint = lambda_hi_hint;
  auto cleanup = [&]() {
    if (m->rp) (void)hipFree(m->rp);
    if (m->ci) (void)hipFree(m->ci);
    if (m->v64) (void)hipFree(m->v64);
    if (m->vlo) (void)hipFree(m->vlo);
    if (m->gpart) (void)hipFree(m->gpart);
    if (m->rg_gp) (void)hipFree(m->rg_gp);
    if (m->rg_col) (void)hipFree(m->rg_col);
    if (m->rg_val) (void)hipFree(m->rg_val);
    if (m->rg_val64) (void)hipFree(m->rg_val64);
    if (m->rg_unused) (void)hipFree(m->rg_unused);
  };
  hipError_t e = hipMalloc(&m->rp, (size_t)(n + 1) * 4);
  if (e == hipSuccess) e = hipMalloc(&m->ci, (size_t)nnz * 4);
  if (e == hipSuccess) e = hipMalloc(&m->v64, (size_t)nnz * 8);
  // mixed-precision runs read the values in the storage type: FP32 or BF16
  // copies, or (FP64 storage) the FP64 values themselves
  m->vt_lo = (vt == LD_VT_BF16) ? VT_BF16 : (vt == LD_VT_FP32 ? VT_F32 : VT_F64);
  const size_t lo_bytes =
      m->vt_lo == VT_F64 ? 0 : (size_t)nnz * (m->vt_lo == VT_BF16 ? 2 : 4);
  if (e == hipSuccess && lo_bytes > 0) e = hipMalloc(&m->vlo, lo_bytes);
  if (e != hipSuccess) {
    cleanup();
    return set_error(e == hipErrorOutOfMemory ? LD_E_NO_MEMORY : LD_E_DEVICE,
                     std::string("matrix allocation: ") + hipGetErrorString(e));
  }
  m->bytes = (size_t)(n + 1) * 4 + (size_t)nnz * 12 + lo_bytes;
  // the FP32 or BF16 copy of values[k0 .. k1) into h (host threads)
  auto convert = [&](void* h, int64_t k0, int64_t k1) {
    const int nt = host_threads(k1 - k0);
    if (m->vt_lo == VT_BF16) {
      uint16_t* o = static_cast<uint16_t*>(h);
      parallel_ranges(k1 - k0, nt, [&](int, int64_t a, int64_t b) {
        for (int64_t k = a; k < b; ++k) o[k] = double_to_bf16_rne(values[k0 + k]);
      });
    } else {
      float* o = static_cast<float*>(h);
      parallel_ranges(k1 - k0, nt, [&](int, int64_t a, int64_t b) {
        for (int64_t k = a; k < b; ++k) o[k] = (float)values[k0 + k];
      });
    }
  };
  // large arrays go through the context's pinned staging buffers (the
  // narrowed values are converted straight into them)
  constexpr size_t kStageMin = (size_t)32 << 20;
  auto stager = [&]() -> hipError_t {
    if (!ctx->stager) {
      std::unique_ptr<Stager> sg(new Stager());
      const hipError_t ei = sg->init();
      if (ei != hipSuccess) return ei;
      ctx->stager = std::move(sg);
    }
    return hipSuccess;
  };
  auto upload = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    if (bytes < kStageMin) return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    std::lock_guard<std::mutex> lk(ctx->stage_mu);
    const hipError_t ei = stager();
    return ei != hipSuccess ? ei : ctx->stager->upload(dst, src, bytes);
  };
  e = upload(m->rp, row_ptr, (size_t)(n + 1) * 4);
  if (e == hipSuccess) e = upload(m->ci, col_idx, (size_t)nnz * 4);
  if (e == hipSuccess) e = upload(m->v64, values, (size_t)nnz * 8);
  if (e == hipSuccess && lo_bytes > 0) {
    const size_t vb = m->vt_lo == VT_BF16 ? 2 : 4;
    if (lo_bytes < kStageMin) {
      std::vector<char> lo_host(lo_bytes);
      convert(lo_host.data(), 0, nnz);
      e = hipMemcpy(m->vlo, lo_host.data(), lo_bytes, hipMemcpyHostToDevice);
    } else {
      std::lock_guard<std::mutex> lk(ctx->stage_mu);
      e = stager();
      if (e == hipSuccess)
        e = ctx->stager->upload_fill(m->vlo, lo_bytes, [&](char* b, size_t off, size_t len) {
          convert(b, (int64_t)(off / vb), (int64_t)((off + len) / vb));
        });
    }
  }
  // row groups (FP32 or FP64 storage; BF16 values keep the CSR product)
  if (e == hipSuccess && (m->vt_lo == VT_F32 || m->vt_lo == VT_F64)) {
    const int64_t ng = (n + kRowGroup - 1) / kRowGroup;
    const int64_t ns = std::min<int64_t>(ng, 256);
    int64_t se = 0, su = 0;
    for (int64_t i = 0; i < ns; ++i) {
      const int64_t g = i * ng / ns;
      se += row_ptr[std::min(n, (g + 1) * kRowGroup)] - row_ptr[g * kRowGroup];
      su += group_union_size(row_ptr, col_idx, n, g);
    }
    if ((double)se >= kRowGroupMinRatio * (double)su) {
      // counts into gp[1 ..], prefix sums on the host (a union column comes
      // from at least one entry: nu <= nnz < 2^31), then the fill
      std::vector<int32_t> gp((size_t)ng + 1, 0);
      e = hipMalloc(&m->rg_gp, ((size_t)ng + 1) * 4);
      if (e == hipSuccess) e = launch_rowgroup_count(ctx->stream, n, m->rp, m->ci, m->rg_gp + 1);
      if (e == hipSuccess)
        e = hipMemcpyAsync(gp.data() + 1, m->rg_gp + 1, (size_t)ng * 4, hipMemcpyDeviceToHost,
                           ctx->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
      int64_t nu = 0;
      for (int64_t g = 0; g < ng && e == hipSuccess; ++g) {
        nu += gp[g + 1];
        gp[g + 1] = (int32_t)nu;
      }
      if (e == hipSuccess && (double)nnz >= kRowGroupMinRatio * (double)nu) {
        e = hipMemcpyAsync(m->rg_gp, gp.data(), ((size_t)ng + 1) * 4, hipMemcpyHostToDevice,
                           ctx->stream);
        if (e == hipSuccess) e = hipMalloc(&m->rg_col, (size_t)nu * 4);
        // FP32 values only with FP32 storage (mixed runs read them); FP64
        // values always (FP64 runs, and mixed runs on FP64 storage)
        const bool f32 = m->vt_lo == VT_F32;
        if (e == hipSuccess && f32) e = hipMalloc(&m->rg_val, (size_t)nu * kRowGroup * 4);
        if (e == hipSuccess) e = hipMalloc(&m->rg_val64, (size_t)nu * kRowGroup * 8);
        if (e == hipSuccess)
          e = launch_rowgroup_fill(ctx->stream, n, m->rp, m->ci, m->v64, m->rg_gp, m->rg_col,
                                   m->rg_val, m->rg_val64);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e == hipSuccess) {
          m->rg_nu = nu;
          m->bytes += ((size_t)ng + 1) * 4 + (size_t)nu * (4 + (f32 ? 12 : 8) * kRowGroup);
        }
      } else if (e == hipSuccess) {
        // the full count missed the ratio the sample promised: no groups (the
        // count buffer stays with the matrix, since a free would synchronise
        // the device)
        m->rg_unused = m->rg_gp;
        m->rg_gp = nullptr;
      }
    }
  }
  // Gershgorin interval (Section 2.1), on the device
  const int nb = (int)((n + kThreads - 1) / kThreads);
  if (e == hipSuccess) e = hipMalloc(&m->gpart, (size_t)nb * 2 * 8);
  int nparts = 0;
  if (e == hipSuccess)
    e = launch_gershgorin(ctx->stream, n, m->rp, m->ci, m->v64, m->gpart, &nparts);
  std::vector<double> hp((size_t)nb * 2);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hp.data(), m->gpart, hp.size() * 8, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    cleanup();
    return set_error(LD_E_DEVICE, std::string("matrix upload: ") + hipGetErrorString(e));
  }
  double glo = INFINITY, ghi = -INFINITY;
  for (int b = 0; b < nparts; ++b) {
    glo = std::min(glo, hp[2 * b]);
    ghi = std::max(ghi, hp[2 * b + 1]);
  }
  m->glo = glo;
  m->ghi = ghi;
  double hi = lambda_hi_hint > 0 ? lambda_hi_hint : ghi;
  double lo = lambda_lo_hint > 0 ? lambda_lo_hint : glo;
  if (lo <= 0.0) lo = 1e-6 * hi;  // Gershgorin lower bound not positive: small positive floor
  if (!(lo > 0.0) || !(hi >= lo) || !std::isfinite(hi)) {
    cleanup();
    return set_error(LD_E_INVALID_ARG, "spectral interval is empty or not finite");
  }
  m->lo = lo;
  m->hi = hi;
  ctx->n_matrices.fetch_add(1);
  *out = m.release();
  return LD_OK;
}

ld_status ld_destroy(ld_matrix* a) {
  if (!a) return set_error(LD_E_INVALID_ARG, "null matrix");
  if (a->inflight.load() > 0) return set_error(LD_E_BUSY, "requests still use the matrix");
  (void)hipSetDevice(a->ctx->device);
  {
    std::lock_guard<std::mutex> lk(a->ctx->est_mu);
    a->ctx->graphs.drop_matrix(a->serial);
  }
  (void)hipStreamSynchronize(a->ctx->stream);
  if (a->rp) (void)hipFree(a->rp);
  if (a->ci) (void)hipFree(a->ci);
  if (a->v64) (void)hipFree(a->v64);
  if (a->vlo) (void)hipFree(a->vlo);
  if (a->gpart) (void)hipFree(a->gpart);
  if (a->rg_gp) (void)hipFree(a->rg_gp);
  if (a->rg_col) (void)hipFree(a->rg_col);
  if (a->rg_val) (void)hipFree(a->rg_val);
  if (a->rg_val64) (void)hipFree(a->rg_val64);
  if (a->rg_unused) (void)hipFree(a->rg_unused);
  a->ctx->n_matrices.fetch_sub(1);
  delete a;
  return LD_OK;
}

ld_status ld_matrix_bounds(const ld_matrix* a, double* lo, double* hi) {
  if (!a || !lo || !hi) return set_error(LD_E_INVALID_ARG, "null argument");
  *lo = a->lo;
  *hi = a->hi;
  return LD_OK;
}

ld_status ld_autotune(ld_matrix* a, const ld_params* p, int32_t reps, ld_tune_result* out) {
  if (!a || !p) return set_error(LD_E_INVALID_ARG, "null argument");
  if (reps < 0 || reps > 10000) return set_error(LD_E_INVALID_ARG, "reps must be in [0, 10000]");
  ld_ctx* ctx = a->ctx;
  std::lock_guard<std::mutex> lk(ctx->est_mu);
  LD_HIP_API(hipSetDevice(ctx->device));
  Run run(a, *p);
  ld_status rc = run.validate();
  if (rc != LD_OK) return rc;
  return run.tune(ctx->stream, reps, out);
}

ld_status ld_tune_set(ld_matrix* a, const ld_params* p, int32_t spmm_lanes, int32_t spmm_chunks,
                      int32_t spmm_entry_split, int32_t update_lanes, int32_t update_chunks,
                      int32_t spmm_interleave, int32_t spmm_row_stride,
                      int32_t step_presub, int32_t spmm_row_groups) {
  if (!a || !p) return set_error(LD_E_INVALID_ARG, "null argument");
  Run run(a, *p);
  ld_status rc = run.validate();
  if (rc != LD_OK) return rc;
  return run.tune_set(spmm_lanes, spmm_chunks, spmm_entry_split, update_lanes, update_chunks,
                      spmm_interleave, spmm_row_stride, step_presub, spmm_row_groups);
}

ld_status ld_quad_form(ld_matrix* a, const double* x, double* out) {
  if (!a || !x || !out) return set_error(LD_E_INVALID_ARG, "null argument");
  ld_ctx* ctx = a->ctx;
  std::lock_guard<std::mutex> lk(ctx->est_mu);
  LD_HIP_API(hipSetDevice(ctx->device));
  const int64_t n = a->n;
  // x as column 0 of an [n][4] FP64 block (the product kernels' minimum
  // width); W = Q X with the inner product x^T (Q x) fused in the epilogue
  const int ld = 4;
  const Geom g = make_geom(n, ld, 8);
  std::vector<double> hx((size_t)n * ld, 0.0);
  for (int64_t i = 0; i < n; ++i) hx[(size_t)i * ld] = x[i];
  DeviceBuffer buf;
  const size_t vec = (size_t)n * ld * 8;
  const size_t part = (size_t)kMaxBlocks * ld * 8;
  LD_HIP_API(buf.ensure(2 * vec + part + 64));
  char* base = static_cast<char*>(buf.ptr);
  double* X = reinterpret_cast<double*>(base);
  double* W = reinterpret_cast<double*>(base + vec);
  double* pt = reinterpret_cast<double*>(base + 2 * vec);
  double* res = reinterpret_cast<double*>(base + 2 * vec + part);
  LD_HIP_API(hipMemcpyAsync(X, hx.data(), vec, hipMemcpyHostToDevice, ctx->stream));
  VecSet vs{};
  vs.x[0] = X;
  int nb = 0;
  LD_HIP_API(launch_spmm(ctx->stream, g, a->rp, a->ci, a->v64, VT_F64, X, W, nullptr, 1.0, &vs, 1,
                         0, pt, &nb));
  LD_HIP_API(launch_reduce(ctx->stream, pt, nb, ld, res));
  double r[4];
  LD_HIP_API(hipMemcpyAsync(r, res, sizeof(r), hipMemcpyDeviceToHost, ctx->stream));
  LD_HIP_API(hipStreamSynchronize(ctx->stream));
  *out = r[0];
  return LD_OK;
}

ld_status ld_estimate_detail(ld_matrix* a, const ld_params* p, ld_result* out,
                             const ld_detail* detail) {
  if (!a || !p || !out) return set_error(LD_E_INVALID_ARG, "null argument");
  const double t0 = now_seconds();
  ld_ctx* ctx = a->ctx;
  std::lock_guard<std::mutex> lk(ctx->est_mu);
  LD_HIP_API(hipSetDevice(ctx->device));
  if (!ctx->na_ev[0] || !ctx->na_nact || !ctx->na_pack)
    return set_error(LD_E_INVALID_ARG, "context without its blocking-estimate set-up");
  // a run with the context's events and pinned buffers (a second one only
  // when a graph capture fails and the estimate runs kernel by kernel)
  auto make_run = [&](std::unique_ptr<Run>& r) -> ld_status {
    r.reset(new Run(a, *p));
    r->set_submit_time(t0);
    r->set_profiler(&ctx->prof);
    r->set_blocking(true);
    r->use_external(ctx->na_ev[0], ctx->na_ev[1], ctx->na_ev[2], ctx->na_nact);
    r->set_host_pack(ctx->na_pack);
    return r->validate();
  };
  std::unique_ptr<Run> runp;
  ld_status rc = make_run(runp);
  if (rc != LD_OK) return rc;
  const size_t need = runp->device_bytes();
  const void* ws0 = ctx->workspace.ptr;
  const size_t wb0 = ctx->workspace.bytes;
  hipError_t e = ctx->workspace.ensure(need);
  if (e != hipSuccess)
    return set_error(e == hipErrorOutOfMemory ? LD_E_NO_MEMORY : LD_E_DEVICE,
                     std::string("workspace allocation: ") + hipGetErrorString(e));
  // graphs captured on the old workspace point into freed memory
  if (ctx->workspace.ptr != ws0 || ctx->workspace.bytes != wb0) ctx->graphs.drop_workspace();
  rc = runp->bind(ctx->workspace.ptr, ctx->workspace.bytes);
  if (rc != LD_OK) return rc;
  GraphCache& gc = ctx->graphs;
  if (gc.mode == 1 && runp->capturable()) {
    Run& run = *runp;
    GraphKey key;
    key.serial = a->serial;
    key.tune_ver = a->tune_ver.load();
    key.method = p->method;
    key.precision = p->precision;
    key.n_probes = p->n_probes;
    key.sketch_rank = p->sketch_rank;
    key.krylov_steps = p->krylov_steps;
    key.iop_window = p->iop_window;
    key.probe_dist = p->probe_dist;
    key.subspace_rank = p->subspace_rank;
    key.adapt_every = p->adapt_every;
    key.sketch_passes = p->sketch_passes;
    key.tol = p->tol;
    key.adapt_tol = p->adapt_tol;
    key.ws = ctx->workspace.ptr;
    key.ws_bytes = ctx->workspace.bytes;
    GraphCache::Entry* ent = gc.find(key);
    if (!ent && gc.seen_before(key)) {
      // second estimate of this shape: capture its launches (nothing runs
      // during the capture), then replay below
      rc = capture_estimate(ctx, run, key);
      if (rc != LD_OK) {
        // the runtime would not capture or instantiate it: this context
        // launches kernel by kernel from now on, starting with a fresh run
        gc.mode = 0;
        gc.failed = true;
        gc.clear();
        rc = make_run(runp);
        if (rc == LD_OK) rc = runp->bind(ctx->workspace.ptr, ctx->workspace.bytes);
        if (rc != LD_OK) return rc;
      } else {
        ent = gc.find(key);
      }
    }
    if (ent) {
      // record start, seed, the graph, record end, results: the launches of
      // an eager estimate in the same order
      LD_HIP_API(hipEventRecord(run.start_event(), ctx->stream));
      rc = run.write_seed(ctx->stream);
      if (rc != LD_OK) return rc;
      LD_HIP_API(hipGraphLaunch(ent->exec, ctx->stream));
      LD_HIP_API(hipEventRecord(run.end_event(), ctx->stream));
      rc = run.enqueue_results(ctx->stream);
      if (rc != LD_OK) {
        (void)hipStreamSynchronize(ctx->stream);
        return rc;
      }
      ++gc.replays;
      return run.collect(ctx->stream, out, detail);
    }
  }
  ++gc.eager;
  Run& run = *runp;
  bool done = false;
  while (!done) {
    rc = run.advance(ctx->stream, 1 << 30, &done);
    if (rc != LD_OK) {
      (void)hipStreamSynchronize(ctx->stream);
      return rc;
    }
  }
  return run.collect(ctx->stream, out, detail);
}

ld_status ld_request_bytes(ld_matrix* a, const ld_params* p, uint64_t* bytes) {
  if (!a || !p || !bytes) return set_error(LD_E_INVALID_ARG, "null argument");
  Run run(a, *p);
  ld_status rc = run.validate();
  if (rc != LD_OK) return rc;
  *bytes = (uint64_t)run.device_bytes();
  return LD_OK;
}

ld_status ld_estimate_ex(ld_matrix* a, const ld_params* p, ld_result* out) {
  return ld_estimate_detail(a, p, out, nullptr);
}

ld_status ld_estimate_noalloc(ld_matrix* a, const ld_params* p, ld_result* out) {
  if (!a || !p || !out) return set_error(LD_E_INVALID_ARG, "null argument");
  const double t0 = now_seconds();
  ld_ctx* ctx = a->ctx;
  if (ctx->device < 0 || ctx->device >= kMaxDevices || !ctx->na_ev[0] || !ctx->na_nact ||
      !ctx->na_pack)
    return set_error(LD_E_INVALID_ARG, "context without the no-allocation set-up");
  std::lock_guard<std::mutex> lk(ctx->est_mu);
  std::lock_guard<std::mutex> lk_dev(g_scratch_use_mu[ctx->device]);
  LD_HIP_API(hipSetDevice(ctx->device));
  void* base = nullptr;
  LD_HIP_API(scratch_ptr(ctx->device, &base));
  Run run(a, *p);
  run.set_submit_time(t0);
  run.set_blocking(true);
  run.use_external(ctx->na_ev[0], ctx->na_ev[1], ctx->na_ev[2], ctx->na_nact);
  run.set_host_pack(ctx->na_pack);
  ld_status rc = run.validate();
  if (rc != LD_OK) return rc;
  const size_t need = run.device_bytes();
  if (need > kScratchBytes)
    return set_error(LD_E_INVALID_ARG,
                     "the request needs " + std::to_string(need) +
                         " device bytes; ld_estimate_noalloc holds at most " +
                         std::to_string(kScratchBytes) + " (use ld_estimate_ex)");
  rc = run.bind(base, kScratchBytes);
  if (rc != LD_OK) return rc;
  bool done = false;
  while (!done) {
    rc = run.advance(ctx->stream, 1 << 30, &done);
    if (rc != LD_OK) {
      (void)hipStreamSynchronize(ctx->stream);
      return rc;
    }
  }
  return run.collect(ctx->stream, out, nullptr);
}

ld_status ld_estimate(ld_matrix* a, int32_t n_probes, int32_t sketch_rank, int32_t krylov_steps,
                      int32_t iop_window, uint64_t seed, ld_result* out) {
  if (!a) return set_error(LD_E_INVALID_ARG, "null matrix");
  ld_params p{};
  p.method = a->ctx->opts.default_method;
  p.precision = a->ctx->opts.default_precision;
  p.n_probes = n_probes;
  p.sketch_rank = sketch_rank;
  p.krylov_steps = krylov_steps;
  p.iop_window = iop_window;
  p.seed = seed;
  p.tol = 0.0;
  return ld_estimate_detail(a, &p, out, nullptr);
}

ld_status ld_profile_enable(ld_ctx* ctx, uint32_t family_mask) {
  if (!ctx) return set_error(LD_E_INVALID_ARG, "null context");
  std::lock_guard<std::mutex> lk(ctx->est_mu);
  LD_HIP_API(hipSetDevice(ctx->device));
  LD_HIP_API(ctx->prof.harvest());
  ctx->prof.enable(family_mask & LD_PROF_ALL);
  return LD_OK;
}

ld_status ld_profile_query(ld_ctx* ctx, uint32_t family, int64_t* launches, double* total_ms,
                           double* total_bytes) {
  if (!ctx || !launches || !total_ms || !total_bytes)
    return set_error(LD_E_INVALID_ARG, "null argument");
  ctx->prof.query(family, launches, total_ms, total_bytes);
  return LD_OK;
}

ld_status ld_debug_copy(ld_ctx* ctx, uint64_t bytes, int32_t reps, double* ms) {
  if (!ctx || !ms || bytes < 16 || reps < 1) return set_error(LD_E_INVALID_ARG, "bad argument");
  std::lock_guard<std::mutex> lk(ctx->est_mu);
  LD_HIP_API(hipSetDevice(ctx->device));
  DeviceBuffer a, b;
  LD_HIP_API(a.ensure(bytes));
  LD_HIP_API(b.ensure(bytes));
  LD_HIP_API(hipMemsetAsync(a.ptr, 0, bytes, ctx->stream));
  hipEvent_t e0, e1;
  LD_HIP_API(hipEventCreate(&e0));
  LD_HIP_API(hipEventCreate(&e1));
  LD_HIP_API(launch_copy16(ctx->stream, a.ptr, b.ptr, bytes));  // warm-up
  LD_HIP_API(hipEventRecord(e0, ctx->stream));
  for (int i = 0; i < reps; ++i) LD_HIP_API(launch_copy16(ctx->stream, a.ptr, b.ptr, bytes));
  LD_HIP_API(hipEventRecord(e1, ctx->stream));
  LD_HIP_API(hipEventSynchronize(e1));
  float t = 0.f;
  LD_HIP_API(hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = t / reps;
  return LD_OK;
}

ld_status ld_debug_row_groups(ld_matrix* a, int64_t* n_union, int32_t* gp, int32_t* col,
                              double* val) {
  if (!a || !n_union) return set_error(LD_E_INVALID_ARG, "null argument");
  *n_union = a->rg_gp ? a->rg_nu : 0;
  if (!gp || !col || !val || !a->rg_gp) return LD_OK;
  ld_ctx* ctx = a->ctx;
  std::lock_guard<std::mutex> lk(ctx->est_mu);
  LD_HIP_API(hipSetDevice(ctx->device));
  const int64_t ng = (a->n + kRowGroup - 1) / kRowGroup;
  LD_HIP_API(hipMemcpy(gp, a->rg_gp, ((size_t)ng + 1) * 4, hipMemcpyDeviceToHost));
  LD_HIP_API(hipMemcpy(col, a->rg_col, (size_t)a->rg_nu * 4, hipMemcpyDeviceToHost));
  LD_HIP_API(hipMemcpy(val, a->rg_val64, (size_t)a->rg_nu * kRowGroup * 8, hipMemcpyDeviceToHost));
  return LD_OK;
}

ld_status ld_debug_stream(ld_ctx* ctx, uint64_t bytes, int32_t reads, int32_t writes,
                          int32_t reps, double* ms) {
  if (!ctx || !ms || bytes < 16 || reps < 1 || reads < 1 || reads > 3 || writes < 0 || writes > 1)
    return set_error(LD_E_INVALID_ARG, "bad argument");
  std::lock_guard<std::mutex> lk(ctx->est_mu);
  LD_HIP_API(hipSetDevice(ctx->device));
  DeviceBuffer in[3], out, sink;
  const void* src[3] = {nullptr, nullptr, nullptr};
  for (int r = 0; r < reads; ++r) {
    LD_HIP_API(in[r].ensure(bytes));
    LD_HIP_API(hipMemsetAsync(in[r].ptr, 0, bytes, ctx->stream));
    src[r] = in[r].ptr;
  }
  if (writes) LD_HIP_API(out.ensure(bytes));
  LD_HIP_API(sink.ensure((size_t)kMaxBlocks * kThreads * sizeof(float)));
  hipEvent_t e0, e1;
  LD_HIP_API(hipEventCreate(&e0));
  LD_HIP_API(hipEventCreate(&e1));
  auto go = [&]() {
    return launch_stream_rw(ctx->stream, reads, writes, src, out.ptr, static_cast<float*>(sink.ptr),
                            bytes);
  };
  hipError_t e = go();  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
  for (int i = 0; i < reps && e == hipSuccess; ++i) e = go();
  if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  LD_HIP_API(e);
  *ms = t / reps;
  return LD_OK;
}

ld_status ld_debug_rademacher(ld_ctx* ctx, uint64_t seed, int64_t n, int32_t col_begin,
                              int32_t col_end, double* out) {
  if (!ctx || !out || n < 1 || col_begin < 0 || col_end <= col_begin || n > INT32_MAX)
    return set_error(LD_E_INVALID_ARG, "bad argument");
  std::lock_guard<std::mutex> lk(ctx->est_mu);
  LD_HIP_API(hipSetDevice(ctx->device));
  const int nc = col_end - col_begin;
  const int ld = (nc + 3) & ~3;
  DeviceBuffer buf;
  LD_HIP_API(buf.ensure((size_t)n * ld * 8));
  LD_HIP_API(launch_rademacher(ctx->stream, seed, n, col_begin, ld, nc, buf.ptr, 8, ld, 0));
  LD_HIP_API(hipStreamSynchronize(ctx->stream));
  std::vector<double> h((size_t)n * ld);
  LD_HIP_API(hipMemcpy(h.data(), buf.ptr, h.size() * 8, hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < n; ++i)
    for (int j = 0; j < nc; ++j) out[i * nc + j] = h[(size_t)i * ld + j];
  return LD_OK;
}

ld_status ld_debug_quad_log(ld_ctx* ctx, int32_t runs, int32_t m, const double* alpha,
                           const double* beta, const int32_t* dims, double a, double b,
                           double* K, int32_t* need) {
  if (!ctx || !alpha || !beta || !dims || !K || !need || runs < 1 || m < 1 || m > 512 ||
      !(a > 0.0) || !(b >= a))
    return set_error(LD_E_INVALID_ARG, "bad argument");
  for (int p = 0; p < runs; ++p)
    if (dims[p] < 0 || dims[p] > m) return set_error(LD_E_INVALID_ARG, "dims[p] must be in [0, m]");
  std::lock_guard<std::mutex> lk(ctx->est_mu);
  LD_HIP_API(hipSetDevice(ctx->device));
  // the Hessenberg layout of the estimates: run p's (m+1) x m block, diagonal
  // h_tt and both off-diagonals h_t+1,t = h_t,t+1 = beta_t
  const size_t hb = (size_t)(m + 1) * m;
  std::vector<double> H((size_t)runs * hb, 0.0);
  for (int p = 0; p < runs; ++p)
    for (int t = 0; t < m; ++t) {
      double* Hp = H.data() + (size_t)p * hb;
      Hp[(size_t)t * m + t] = alpha[(size_t)p * m + t];
      Hp[(size_t)(t + 1) * m + t] = beta[(size_t)p * m + t];
      if (t + 1 < m) Hp[(size_t)t * m + t + 1] = beta[(size_t)p * m + t];
    }
  DeviceBuffer dH, dm, dK, dn, df;
  LD_HIP_API(dH.ensure(H.size() * 8));
  LD_HIP_API(dm.ensure((size_t)runs * 4));
  LD_HIP_API(dK.ensure((size_t)runs * 8));
  LD_HIP_API(dn.ensure((size_t)runs * 4));
  LD_HIP_API(df.ensure((size_t)runs * 4));
  LD_HIP_API(hipMemcpy(dH.ptr, H.data(), H.size() * 8, hipMemcpyHostToDevice));
  LD_HIP_API(hipMemcpy(dm.ptr, dims, (size_t)runs * 4, hipMemcpyHostToDevice));
  const FillItem fi{df.ptr, (size_t)runs, 0u};
  LD_HIP_API(launch_fill(ctx->stream, &fi, 1));
  double* hK = static_cast<double*>(dK.ptr);
  int* hn = static_cast<int*>(dn.ptr);
  int* hf = static_cast<int*>(df.ptr);
  const double* hH = static_cast<const double*>(dH.ptr);
  const int* hm = static_cast<const int*>(dm.ptr);
  LD_HIP_API(launch_quad_log(ctx->stream, runs, m, hH, hm, a, b, hK, hn, hf));
  LD_HIP_API(launch_gauss_log(ctx->stream, runs, m, hH, hm, hK, hf, hn));
  LD_HIP_API(hipStreamSynchronize(ctx->stream));
  std::vector<int> flags(runs);
  LD_HIP_API(hipMemcpy(K, dK.ptr, (size_t)runs * 8, hipMemcpyDeviceToHost));
  LD_HIP_API(hipMemcpy(need, dn.ptr, (size_t)runs * 4, hipMemcpyDeviceToHost));
  LD_HIP_API(hipMemcpy(flags.data(), df.ptr, (size_t)runs * 4, hipMemcpyDeviceToHost));
  for (int p = 0; p < runs; ++p)
    if (flags[p] & 11)
      return set_error(LD_E_NUMERIC, "run " + std::to_string(p) + ": flags " +
                                         std::to_string(flags[p]));
  return LD_OK;
}

ld_status ld_debug_probes(ld_ctx* ctx, uint64_t seed, int64_t n, int32_t col_begin,
                          int32_t col_end, int32_t dist, double* out) {
  if (!ctx || !out || n < 1 || col_begin < 0 || col_end <= col_begin || n > INT32_MAX ||
      (dist != LD_PROBE_RADEMACHER && dist != LD_PROBE_GAUSSIAN))
    return set_error(LD_E_INVALID_ARG, "bad argument");
  std::lock_guard<std::mutex> lk(ctx->est_mu);
  LD_HIP_API(hipSetDevice(ctx->device));
  const int nc = col_end - col_begin;
  const int ld = (nc + 3) & ~3;
  DeviceBuffer buf;
  LD_HIP_API(buf.ensure((size_t)n * ld * 8));
  LD_HIP_API(launch_probes(ctx->stream, dist, seed, n, col_begin, ld, nc, buf.ptr, 8, ld, 0));
  LD_HIP_API(hipStreamSynchronize(ctx->stream));
  std::vector<double> h((size_t)n * ld);
  LD_HIP_API(hipMemcpy(h.data(), buf.ptr, h.size() * 8, hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < n; ++i)
    for (int j = 0; j < nc; ++j) out[i * nc + j] = h[(size_t)i * ld + j];
  return LD_OK;
}

static ld::Server* server_of(ld_ctx* ctx) {
  std::lock_guard<std::mutex> lk(ctx->server_mu);
  if (!ctx->server) ctx->server.reset(new ld::Server(ctx));
  return ctx->server.get();
}

ld_status ld_graph_mode(ld_ctx* ctx, int32_t mode) {
  if (!ctx) return set_error(LD_E_INVALID_ARG, "null context");
  if (mode != 0 && mode != 1) return set_error(LD_E_INVALID_ARG, "graph mode must be 0 or 1");
  std::lock_guard<std::mutex> lk(ctx->est_mu);
  (void)hipSetDevice(ctx->device);
  if (mode == 0) {
    if (ctx->stream) LD_HIP_API(hipStreamSynchronize(ctx->stream));
    ctx->graphs.clear();
  }
  ctx->graphs.mode = mode;
  return LD_OK;
}

ld_status ld_graph_stats_get(ld_ctx* ctx, ld_graph_stats* out) {
  if (!ctx || !out) return set_error(LD_E_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(ctx->est_mu);
  ld_graph_stats o{};
  o.captures = ctx->graphs.captures;
  o.replays = ctx->graphs.replays;
  o.eager = ctx->graphs.eager;
  o.cached = (uint64_t)ctx->graphs.entries.size();
  o.mode = ctx->graphs.mode;
  o.capture_failed = ctx->graphs.failed ? 1 : 0;
  *out = o;
  return LD_OK;
}

ld_status ld_serving_stats_get(ld_ctx* ctx, ld_serving_stats* out) {
  if (!ctx || !out) return set_error(LD_E_INVALID_ARG, "null argument");
  ld_serving_stats o{};
  o.max_slots = ctx->opts.max_slots;
  o.budget_bytes = ctx->opts.hbm_budget_bytes;
  {
    std::lock_guard<std::mutex> lk(ctx->server_mu);
    if (ctx->server) {
      const ld::Server::Stats st = ctx->server->stats();
      o.submitted = st.submitted;
      o.completed = st.completed;
      o.ticks = st.ticks;
      o.batched_steps = st.batched_steps;
      o.batched_launches = st.batched_launches;
      o.held_bytes = st.held_bytes;
      o.peak_held_bytes = st.peak_bytes;
      o.buffer_allocs = st.buffer_allocs;
      o.buffer_frees = st.buffer_frees;
      o.peak_active = st.peak_active;
    }
  }
  *out = o;
  return LD_OK;
}

ld_status ld_submit(ld_matrix* a, const ld_params* p, uint64_t* ticket) {
  if (!a || !p || !ticket) return set_error(LD_E_INVALID_ARG, "null argument");
  return server_of(a->ctx)->submit(a, *p, ticket);
}

ld_status ld_poll(ld_ctx* ctx, uint64_t ticket, ld_result* out) {
  if (!ctx || !out) return set_error(LD_E_INVALID_ARG, "null argument");
  return server_of(ctx)->poll(ticket, out, false);
}

ld_status ld_wait(ld_ctx* ctx, uint64_t ticket, ld_result* out) {
  if (!ctx || !out) return set_error(LD_E_INVALID_ARG, "null argument");
  return server_of(ctx)->poll(ticket, out, true);
}

}  // extern "C"

// Host runtime of the C ABI declared in include/ctaux.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/ctaux.h"
#include "ctaux_internal.h"

using namespace ctaux;

namespace {

thread_local char g_create_error[512] = "";

struct TimedEvent {
  int name;
  hipEvent_t start, stop;
};

const char *kKernelNames[] = {"block_begin", "interp", "prep",     "propose",
                              "assemble",    "rankk",  "block_end", "measure", "refine"};
constexpr int kNumNames = sizeof(kKernelNames) / sizeof(kKernelNames[0]);

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Sequential carving of the workspace; with base == nullptr it only measures.
struct Carver {
  char *base;
  size_t off = 0;
  template <typename T>
  T *take(size_t count) {
    off = align_up(off, 256);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += align_up(count * sizeof(T), 256);
    return p;
  }
};

}  // namespace

struct ctaux_batch {
  Batch b;
  hipStream_t stream;
  // The measurement of a block runs on a stream of its own beside the next
  // block's proposals (it reads the block's N, configuration and state copy,
  // which the next block does not write before its k_block_end); the next
  // block's k_block_end waits for it.  For a few chains it is launched once the
  // next block's preparation is enqueued, so that it shares the GPU with the
  // one-workgroup-per-chain proposal kernel rather than with the preparation
  // products.
  hipStream_t mstream = nullptr;
  hipEvent_t ev_end = nullptr, ev_meas = nullptr;
  bool meas_owed = false;      // a block ended and its measurement is not launched yet
  bool meas_pending = false;   // ev_meas marks the end of the last launched measurement
  bool begun = false;          // the next block's start already ran (fused into the last block's end)
  std::vector<ChainDesc> desc;        // host copies
  std::vector<ChainState> state;      // host mirror (refreshed at sync points)
  std::vector<int32_t> obs_len;
  int64_t blocks_launched = 0;
  int32_t recompute_every = 0;
  int32_t recompute_mode = 0;       // 0: Newton step (from scratch when it cannot recover), 1: from scratch
  // Adaptive refinement schedule, per chain: chain c is refined after every
  // block whose count is a multiple of interval[c], a power of two in
  // [1, max_interval] (max_interval = the largest power of two <= recompute_every),
  // starting at 1.  Powers of two keep the refinements of
  // all chains aligned, so that a refinement (which synchronises the host with
  // the device) happens at most every min_c interval[c] blocks.  After each
  // refinement interval[c] is quartered when the drift of chain c exceeded the
  // drift target and doubled when it stayed below 1/16 of it.
  int32_t max_interval = 0;
  std::vector<int32_t> interval;
  double drift_target = 0.0;
  int64_t log_cap = 0;
  int32_t obs_len_max = 0;
  int32_t timing = 0;                 // bit i: time kernel i (kKernelNames)
  int32_t timing_every = 1;           // time one launch in timing_every of each selected kernel
  int64_t timing_seen[16] = {0};      // launches of each kernel since timing was set
  std::vector<TimedEvent> pool;       // created events
  size_t pool_used = 0;
  double ms[kNumNames] = {0};
  int64_t launches[kNumNames] = {0};
  // Block sequences replayed from a HIP graph (ctaux_set_graph): graph_blocks
  // blocks (each ending in k_block_turn) and the last one's measurement,
  // captured once and replayed where no refinement falls inside the window.
  int32_t graph_blocks = 0;
  bool capturing = false;
  hipStream_t cstream = nullptr;   // capture stream (the batch's stream may be the null stream)
  hipGraphExec_t gexec = nullptr;
  int64_t graph_launches = 0;
  std::string err;
};

namespace {

int set_err(ctaux_batch *b, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (b) b->err = buf;
  else snprintf(g_create_error, sizeof g_create_error, "%s", buf);
  return code;
}

#define HIPCHECK(b, call)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return set_err((b), CTAUX_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

}  // namespace

namespace ctaux {

int create_error(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_create_error, sizeof g_create_error, fmt, ap);
  va_end(ap);
  return code;
}

// Model of chain c (Sec. II A): parameters, sizes and finite tables.
int model_error(const ctaux_model &m, int c, ctaux_batch *eb) {
  if (!(m.beta > 0) || !(m.U >= 0) || !(m.K > 0) || !isfinite(m.beta) || !isfinite(m.U) || !isfinite(m.K))
    return set_err(eb, CTAUX_EINVAL, "chain %d: need beta > 0, U >= 0, K > 0", c);
  if (m.n_sites < 1 || m.n_sites > 128 || m.n_tau < 2 || m.n_disp < 1 || !m.site_disp || !m.g0_up || !m.g0_dn)
    return set_err(eb, CTAUX_EINVAL, "chain %d: invalid sizes or null tables (n_sites <= 128)", c);
  for (int i = 0; i < m.n_sites * m.n_sites; ++i)
    if (m.site_disp[i] < 0 || m.site_disp[i] >= m.n_disp)
      return set_err(eb, CTAUX_EINVAL, "chain %d: site_disp out of range", c);
  for (int64_t i = 0; i < static_cast<int64_t>(m.n_disp) * m.n_tau; ++i)
    if (!isfinite(m.g0_up[i]) || !isfinite(m.g0_dn[i]))
      return set_err(eb, CTAUX_EINVAL, "chain %d: non-finite G0 table entry %lld", c, (long long)i);
  return CTAUX_OK;
}

}  // namespace ctaux

namespace {

int validate(const ctaux_model *models, int32_t n_chains, const ctaux_opts *o, ctaux_batch *eb) {
  if (!models || !o || n_chains < 1 || n_chains > 8192)
    return set_err(eb, CTAUX_EINVAL, "null models/opts or n_chains not in 1..8192");
  if (o->k_max < 1 || o->k_max > kMaxKmax) return set_err(eb, CTAUX_EINVAL, "k_max must be in 1..%d", kMaxKmax);
  if (o->k_cap < 1 || o->k_cap > kMaxKcap || o->k_cap > o->k_max)
    return set_err(eb, CTAUX_EINVAL, "k_cap must be in 1..min(k_max, %d)", kMaxKcap);
  if (!(o->p_flip >= 0.0 && o->p_flip <= 1.0)) return set_err(eb, CTAUX_EINVAL, "p_flip must be in [0,1]");
  if (!(o->p_pair >= 0.0 && o->p_flip + o->p_pair <= 1.0))
    return set_err(eb, CTAUX_EINVAL, "p_pair must be in [0, 1 - p_flip]");
  // a pair needs two insertion candidates and two slots of Gamma in one block
  if (o->p_pair > 0.0 && (o->k_max < 2 || o->k_cap < 2))
    return set_err(eb, CTAUX_EINVAL, "pair updates need k_max >= 2 and k_cap >= 2");
  if (!isfinite(o->gamma_tol) || !isfinite(o->drift_tol))
    return set_err(eb, CTAUX_EINVAL, "gamma_tol and drift_tol must be finite");
  if (o->rankk_tile != 0 && o->rankk_tile != 32 && o->rankk_tile != 64)
    return set_err(eb, CTAUX_EINVAL, "rankk_tile must be 0, 32 or 64");
  if (o->precision != CTAUX_FP64 && o->precision != CTAUX_FP32 && o->precision != CTAUX_BF16X3)
    return set_err(eb, CTAUX_EINVAL, "precision must be CTAUX_FP64, CTAUX_FP32 or CTAUX_BF16X3");
  if (o->meas_every < 1 || o->n_tau_out < 0 || o->n_tau_out > 4096 || o->n_cap < 1 || o->n_cap > 65536 ||
      o->recompute_every < 0 || o->n_therm < 0 || o->log_cap < 0)
    return set_err(eb, CTAUX_EINVAL, "invalid meas_every/n_tau_out/n_cap/recompute_every/n_therm/log_cap");
  if (!isfinite(o->drift_target) || o->drift_target < 0.0 || o->recompute_mode < 0 || o->recompute_mode > 1)
    return set_err(eb, CTAUX_EINVAL, "drift_target must be finite and >= 0, recompute_mode 0 or 1");
  if (o->n_matsubara < 0 || o->n_matsubara > 32)
    return set_err(eb, CTAUX_EINVAL, "n_matsubara must be in 0..32");
  // the proposal kernel holds Gamma^{-1} of both sectors and the spins of the
  // augmented configuration in the LDS of one workgroup
  {
    const size_t lds = propose_lds_bytes(o->k_cap, o->k_max, o->n_cap) + kProposeStaticLds;
    if (lds > kLdsPerWorkgroup)
      return set_err(eb, CTAUX_EINVAL, "n_cap=%d with k_cap=%d needs %zu bytes of LDS in the proposal kernel "
                     "(limit %zu)", o->n_cap, o->k_cap, lds, kLdsPerWorkgroup);
  }
  for (int c = 0; c < n_chains; ++c) {
    const ctaux_model &m = models[c];
    int rc = model_error(m, c, eb);
    if (rc) return rc;
    if (o->n_matsubara > 0) {
      if (m.n_sites * o->n_matsubara > 2048)
        return set_err(eb, CTAUX_EINVAL, "chain %d: n_sites * n_matsubara must not exceed 2048", c);
      if (!m.site_pos || !m.kvecs || m.n_k < 1 || m.n_k > 512)
        return set_err(eb, CTAUX_EINVAL, "chain %d: the momentum measurement needs site_pos and 1..512 kvecs", c);
      for (int i = 0; i < 3 * m.n_sites; ++i)
        if (!isfinite(m.site_pos[i])) return set_err(eb, CTAUX_EINVAL, "chain %d: non-finite site_pos", c);
      for (int i = 0; i < 3 * m.n_k; ++i)
        if (!isfinite(m.kvecs[i])) return set_err(eb, CTAUX_EINVAL, "chain %d: non-finite kvecs", c);
    }
    // the table kernels index a chain's elements with 32-bit integers
    if (2ll * (o->n_tau_out + 1) * m.n_sites * o->n_cap >= (1ll << 31))
      return set_err(eb, CTAUX_EINVAL, "chain %d: 2 (n_tau_out + 1) n_sites n_cap must stay below 2^31", c);
  }
  return CTAUX_OK;
}

// Lays out (and, with a base, assigns) every buffer; returns total bytes.
size_t layout(const ctaux_model *models, int32_t n_chains, const ctaux_opts *o, char *base, Batch *bt,
              std::vector<ChainDesc> *descs) {
  Carver cv{base};
  const int n_cap = o->n_cap, kmax = o->k_max, kcap = o->k_cap;
  const int ld = static_cast<int>(align_up(n_cap, 64));
  const int lda = static_cast<int>(align_up(kcap, 8));
  const size_t es = o->precision == CTAUX_FP64 ? sizeof(double) : sizeof(float);
  ChainDesc *d_desc = cv.take<ChainDesc>(n_chains);
  ChainState *d_state = cv.take<ChainState>(n_chains);
  ChainState *d_mstate = cv.take<ChainState>(n_chains);
  // refinement pool: room for one chain at n_cap, and for all chains at n_cap
  // up to 4 GiB; chains are refined in groups that fit
  const size_t need_cap = refine_need_doubles(n_cap, o->precision);
  size_t pool = static_cast<size_t>(n_chains) * need_cap;
  const size_t pool_limit = (size_t{4} << 30) / sizeof(double);
  if (pool > pool_limit) pool = pool_limit > need_cap ? pool_limit : need_cap;
  double *r_pool = cv.take<double>(pool);
  RefineItem *r_items = cv.take<RefineItem>(n_chains);
  double *r_red = cv.take<double>(refine_red_doubles(n_chains));
  InvItem *r_inv = cv.take<InvItem>(2 * static_cast<size_t>(n_chains));
  if (bt) {
    bt->d_desc = d_desc; bt->d_state = d_state; bt->d_mstate = d_mstate;
    bt->r_pool = r_pool; bt->r_pool_doubles = pool; bt->r_items = r_items; bt->r_red = r_red;
    bt->r_inv = r_inv;
  }
  for (int c = 0; c < n_chains; ++c) {
    const ctaux_model &m = models[c];
    ChainDesc d;
    memset(&d, 0, sizeof d);
    const int nc = m.n_sites;
    for (int s = 0; s < 2; ++s) d.g0[s] = cv.take<double>(static_cast<size_t>(m.n_disp) * m.n_tau);
    d.site_disp = cv.take<int32_t>(static_cast<size_t>(nc) * nc);
    d.cls_off = cv.take<int32_t>(m.n_disp + 1);
    d.cls_pairs = cv.take<int32_t>(static_cast<size_t>(nc) * nc);
    for (int p = 0; p < 2; ++p)
      for (int s = 0; s < 2; ++s) d.N[p][s] = cv.take<char>(es * ld * ld);
    for (int p = 0; p < 2; ++p) {
      d.tau[p] = cv.take<double>(n_cap);
      d.site[p] = cv.take<int32_t>(n_cap);
      d.s0[p] = cv.take<int32_t>(n_cap);
      d.id[p] = cv.take<int64_t>(n_cap);
    }
    d.ptype = cv.take<int32_t>(kmax);
    d.pspin = cv.take<int32_t>(kmax);
    d.pspin2 = cv.take<int32_t>(kmax);
    d.pacc = cv.take<double>(kmax);
    d.ppick = cv.take<double>(kmax);
    d.ppick2 = cv.take<double>(kmax);
    d.ctau = cv.take<double>(kmax);
    d.csite = cv.take<int32_t>(kmax);
    d.cid = cv.take<int64_t>(kmax);
    for (int s = 0; s < 2; ++s) {
      d.X[s] = cv.take<double>(static_cast<size_t>(align_up(kmax, 16)) * ld);   // cand_offset order
      d.ZT[s] = cv.take<double>(static_cast<size_t>(align_up(kmax, 16)) * ld);
      d.YT[s] = cv.take<double>(static_cast<size_t>(kmax) * ld);
      d.Rt[s] = cv.take<double>(static_cast<size_t>(kmax) * ld);
      d.G0nn[s] = cv.take<double>(static_cast<size_t>(kmax) * kmax);
      d.Gnn[s] = cv.take<double>(static_cast<size_t>(kmax) * kmax);
      d.ghat[s] = cv.take<double>(kcap);
      d.Gam[s] = cv.take<double>(static_cast<size_t>(kcap) * kcap);
      d.Ginv[s] = cv.take<double>(static_cast<size_t>(kcap) * kcap);
      d.Rg[s] = cv.take<double>(static_cast<size_t>(kcap) * kcap);
      d.Ac[s] = cv.take<char>(es * ld * lda);
      d.Bc[s] = cv.take<char>(es * lda * ld);
      d.W[s] = cv.take<double>(static_cast<size_t>(n_cap) * nc);
      d.gR[s] = cv.take<double>(align_up(n_cap, 16) * align_up(nc, 16));   // cand_offset order
      d.Gxy[s] = cv.take<double>(static_cast<size_t>(o->n_tau_out + 1) * nc * nc);
      // gL as a table only where the measurement uses one (batches of fewer than 8 chains)
      d.gL[s] = n_chains < 8 ? cv.take<double>(static_cast<size_t>(o->n_tau_out + 1) * nc * ld) : nullptr;
    }
    {
      // time-ordered vertex records of the measurement (batches of 8 chains or more)
      const size_t nm = n_chains >= 8 ? static_cast<size_t>(n_cap) : 1;
      d.mpos = cv.take<int32_t>(nm);
      d.mtau = cv.take<double>(nm);
      d.msite = cv.take<int32_t>(nm);
      d.mfac = cv.take<double>(2 * nm);
    }
    d.P = cv.take<int32_t>(kcap);
    d.map = cv.take<int32_t>(n_cap + kmax);
    d.obs_len = 8 + 2 * m.n_disp * o->n_tau_out;
    d.obs = cv.take<double>(d.obs_len);
    d.log_cap = o->log_cap;
    d.log_acc = cv.take<uint8_t>(o->log_cap > 0 ? o->log_cap : 1);
    d.log_R = cv.take<double>(o->log_cap > 0 ? o->log_cap : 1);
    {
      const int nm = o->n_matsubara, nk = nm > 0 ? m.n_k : 0;
      d.n_mats = nm;
      d.n_k = nk;
      const size_t one = 1;
      d.kw_pos = cv.take<double>(nm > 0 ? 3 * static_cast<size_t>(nc) : one);
      d.kw_k = cv.take<double>(nm > 0 ? 3 * static_cast<size_t>(nk) : one);
      d.kw_g0 = cv.take<double>(nm > 0 ? 4 * static_cast<size_t>(nk) * nm : one);
      d.kw_off = cv.take<int32_t>(nm > 0 ? nc + 1 : 1);
      d.kw_list = cv.take<int32_t>(nm > 0 ? n_cap : 1);
      d.kw_ph = cv.take<double>(nm > 0 ? 2 * static_cast<size_t>(n_cap) * nm : one);
      // the C blocks also hold the transforms of the tables while G0(K, i w) is set up
      const size_t cblk = 4 * static_cast<size_t>(nc) * nc * nm, tblk = 4 * static_cast<size_t>(m.n_disp) * nm;
      d.kw_C = cv.take<double>(nm > 0 ? (cblk > tblk ? cblk : tblk) : one);
      d.obs_kw = cv.take<double>(nm > 0 ? 4 * static_cast<size_t>(nk) * nm : one);
    }
    if (descs) {
      d.beta = m.beta; d.K = m.K;
      d.gamma = acosh(1.0 + m.beta * m.U * nc / (2.0 * m.K));
      d.inv_h = static_cast<double>(m.n_tau - 1) / m.beta;
      d.p_flip = o->p_flip;
      d.p_pair = o->p_pair;
      d.gamma_tol = o->gamma_tol;
      d.drift_tol = o->drift_tol;
      for (int s = 0; s < 2; ++s) {
        const double sigma = s == 0 ? 1.0 : -1.0;
        for (int k = -2; k <= 2; ++k) d.evd[s][k + 2] = exp(d.gamma * sigma * k);
      }
      d.nc = nc; d.n_tau = m.n_tau; d.n_disp = m.n_disp; d.lda = lda;
      d.n_cap = n_cap; d.ld = ld; d.kmax = kmax; d.kcap = kcap;
      d.meas_every = o->meas_every; d.n_out = o->n_tau_out; d.n_therm = o->n_therm;
      d.seed_lo = static_cast<uint32_t>(o->seed);
      d.seed_hi = static_cast<uint32_t>(o->seed >> 32);
      d.chain_id = static_cast<uint32_t>(c);
      d.precision = o->precision;
      descs->push_back(d);
    }
  }
  return align_up(cv.off, 256);
}

int enqueue_block(ctaux_batch *h, bool next_follows);
int schedule_refinements(ctaux_batch *h);

struct Timer {
  ctaux_batch *h;
  int name;
  hipStream_t s;
  TimedEvent *ev = nullptr;
  Timer(ctaux_batch *h_, int name_, hipStream_t s_ = nullptr) : h(h_), name(name_), s(s_ ? s_ : h_->stream) {
    if (!(h->timing & (1 << name))) return;
    if (h->timing_seen[name]++ % h->timing_every != 0) return;
    if (h->pool_used == h->pool.size()) {
      TimedEvent e;
      e.name = name;
      (void)hipEventCreate(&e.start);
      (void)hipEventCreate(&e.stop);
      h->pool.push_back(e);
    }
    ev = &h->pool[h->pool_used++];
    ev->name = name;
    (void)hipEventRecord(ev->start, s);
  }
  ~Timer() {
    if (ev) (void)hipEventRecord(ev->stop, s);
  }
};

void flush_timing(ctaux_batch *h) {
  for (size_t i = 0; i < h->pool_used; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->pool[i].start, h->pool[i].stop) == hipSuccess) {
      h->ms[h->pool[i].name] += ms;
      h->launches[h->pool[i].name] += 1;
    }
  }
  h->pool_used = 0;
}

// Launches the measurement owed by the last block on the measurement stream,
// ordered after everything enqueued so far on the batch's stream.
int launch_owed_measure(ctaux_batch *h) {
  if (!h->meas_owed) return CTAUX_OK;
  HIPCHECK(h, hipEventRecord(h->ev_end, h->stream));
  HIPCHECK(h, hipStreamWaitEvent(h->mstream, h->ev_end, 0));
  { Timer t(h, 7, h->mstream); launch_measure(h->b, h->mstream); }
  HIPCHECK(h, hipEventRecord(h->ev_meas, h->mstream));
  h->meas_owed = false;
  h->meas_pending = true;
  return CTAUX_OK;
}

// Launches any owed measurement and waits for both streams of the batch.
int sync_all(ctaux_batch *h) {
  int rc = launch_owed_measure(h);
  if (rc) return rc;
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->mstream));
  return CTAUX_OK;
}

int sync_states(ctaux_batch *h) {
  int rc = sync_all(h);
  if (rc) return rc;
  if (h->timing) flush_timing(h);
  // device-to-host copies are ordered on the batch's stream and waited for
  HIPCHECK(h, hipMemcpyAsync(h->state.data(), h->b.d_state, sizeof(ChainState) * h->b.n_chains,
                             hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  return CTAUX_OK;
}

// N of a chain between the device (rows of ld entries) and a compact host
// array of n x n entries.  Whole padded rows move in one contiguous copy on the
// batch's stream; the (un)packing is done on the host.  (Two-dimensional copies
// between pageable host memory and the device have been seen to deliver zeros
// when the process runs under the ROCm kernel tracer.)
int n_to_host(ctaux_batch *h, void *dst, const void *src, int n, size_t es) {
  const size_t ld = static_cast<size_t>(h->b.ld);
  std::vector<char> rows(es * ld * n);
  HIPCHECK(h, hipMemcpyAsync(rows.data(), src, rows.size(), hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  for (int i = 0; i < n; ++i) memcpy(static_cast<char *>(dst) + es * n * i, rows.data() + es * ld * i, es * n);
  return CTAUX_OK;
}

int n_to_device(ctaux_batch *h, void *dst, const void *src, int n, size_t es) {
  const size_t ld = static_cast<size_t>(h->b.ld);
  std::vector<char> rows(es * ld * n, 0);
  for (int i = 0; i < n; ++i) memcpy(rows.data() + es * ld * i, static_cast<const char *>(src) + es * n * i, es * n);
  HIPCHECK(h, hipMemcpyAsync(dst, rows.data(), rows.size(), hipMemcpyHostToDevice, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));   // rows is freed on return
  return CTAUX_OK;
}

// Refinement of a set of chains.  A Newton step N <- N + N (I - M N) (k_refine.hip)
// squares the relative error of N; a chain whose drift after a step exceeds the
// storage's threshold `again` gets another step (up to kRefinePasses in all),
// each preceded by one synchronisation.  N is recomputed from scratch (M built
// from the tables and inverted by the pivoted elimination of k_invert.hip) when
// a step leaves a drift above kScratchDrift or a non-finite N (outside the
// region where the Newton iteration contracts), when a further step does not
// reduce the drift at least fourfold, or when the passes run out.  With
// scratch_only every chain is recomputed from scratch.  The first measured
// drift of each chain is its N error before the refinement; with adapt it sets
// the chain's next interval.
constexpr int kRefinePasses = 3;
constexpr double kScratchDrift = 1e-2;

// Packs the chains into groups whose scratch fits the pool, uploads the items
// (and, for a from-scratch recompute, the elimination items carved from the
// same scratch) and launches every group.
int launch_refinement(ctaux_batch *h, const std::vector<int> &chains, bool scratch, int pass) {
  const Batch &b = h->b;
  const size_t slots = static_cast<size_t>(refine_slots(b.precision));
  std::vector<RefineItem> items;
  std::vector<InvItem> inv;
  std::vector<int> starts;
  size_t used = 0;
  for (int c : chains) {
    const ChainState &st = h->state[c];
    if (scratch && st.n == 0) continue;
    const size_t need = refine_need_doubles(st.n, b.precision);
    if (starts.empty() || used + need > b.r_pool_doubles) {
      starts.push_back(static_cast<int>(items.size()));
      used = 0;
    }
    items.push_back(RefineItem{c, st.n, static_cast<int64_t>(used)});
    if (scratch) {
      const size_t nn = static_cast<size_t>(st.n) * st.n;
      for (int sec = 0; sec < 2; ++sec) {
        InvItem it;
        memset(&it, 0, sizeof it);
        double *W = b.r_pool + used + sec * slots * nn;   // the M slot of the sector
        double *scr = b.r_pool + used + 2 * slots * nn + sec * inv_scratch_doubles(st.n);
        inv_item_carve(it, W, st.n, st.n, scr);
        inv.push_back(it);
      }
    }
    used += need;
  }
  if (items.empty()) return CTAUX_OK;
  // host-to-device copies go on the batch's stream and are waited for: a
  // synchronous hipMemcpy from pageable memory may return before its DMA has
  // landed, and is not ordered with a stream other than the null stream
  HIPCHECK(h, hipMemcpyAsync(b.r_items, items.data(), sizeof(RefineItem) * items.size(), hipMemcpyHostToDevice,
                             h->stream));
  if (scratch)
    HIPCHECK(h, hipMemcpyAsync(b.r_inv, inv.data(), sizeof(InvItem) * inv.size(), hipMemcpyHostToDevice, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  starts.push_back(static_cast<int>(items.size()));
  Timer t(h, 8);
  for (size_t g = 0; g + 1 < starts.size(); ++g) {
    const int i0 = starts[g], cnt = starts[g + 1] - starts[g];
    if (scratch) {
      int n_max = 0;
      for (int i = i0; i < i0 + cnt; ++i) n_max = items[i].n > n_max ? items[i].n : n_max;
      launch_scratch_group(b, h->stream, b.r_items + i0, b.r_inv + 2 * i0, cnt, n_max, pass);
    } else {
      launch_refine_group(b, h->stream, b.r_items + i0, cnt, pass);
    }
  }
  return CTAUX_OK;
}

int refine_chains(ctaux_batch *h, const std::vector<int> &which, bool adapt, bool scratch_only) {
  const Batch &b = h->b;
  const double again = b.precision == kFP64 ? 1e-9 : 1e-4;
  int rc = sync_states(h);
  if (rc) return rc;
  std::vector<int> newton, scratch;
  for (int c : which)
    if (h->state[c].status == 0) (scratch_only ? scratch : newton).push_back(c);
  std::vector<double> prev(b.n_chains, INFINITY);
  int pass = 0;
  auto adapt_intervals = [&](const std::vector<int> &cs) {
    for (int c : cs) {
      const ChainState &st = h->state[c];
      if (st.status != 0) continue;
      const double d = st.last_drift;
      int32_t &iv = h->interval[c];
      if (!(d <= h->drift_target)) iv = iv > 4 ? iv / 4 : 1;
      else if (d < h->drift_target / 16.0) iv = 2 * iv < h->max_interval ? 2 * iv : h->max_interval;
    }
  };
  for (; pass < kRefinePasses && !newton.empty(); ++pass) {
    rc = launch_refinement(h, newton, false, pass);
    if (rc) return rc;
    rc = sync_states(h);
    if (rc) return rc;
    if (pass == 0 && adapt) adapt_intervals(newton);
    std::vector<int> next;
    for (int c : newton) {
      const ChainState &st = h->state[c];
      if (st.status != 0) continue;   // drift_tol stopped it
      const double d = st.pass_drift;
      if (!(d <= kScratchDrift)) scratch.push_back(c);
      else if (d > again) {
        if ((pass > 0 && d > 0.25 * prev[c]) || pass + 1 == kRefinePasses) scratch.push_back(c);
        else next.push_back(c);
      }
      prev[c] = d;
    }
    newton.swap(next);
  }
  if (!scratch.empty()) {
    // scratch_only: the recompute's drift is the chain's N error before it (pass 0)
    rc = launch_refinement(h, scratch, true, scratch_only ? 0 : pass);
    if (rc) return rc;
    rc = sync_states(h);
    if (rc) return rc;
    if (scratch_only && adapt) adapt_intervals(scratch);
  }
  return CTAUX_OK;
}

int refine_all(ctaux_batch *h, bool scratch_only) {
  std::vector<int> all(h->b.n_chains);
  for (int c = 0; c < h->b.n_chains; ++c) all[c] = c;
  return refine_chains(h, all, false, scratch_only);
}

// next_follows: another block is enqueued right after this one, so its start
// is fused into this block's end (k_block_turn).
int enqueue_block(ctaux_batch *h, bool next_follows) {
  const Batch &b = h->b;
  hipStream_t s = h->stream;
  if (!h->begun) {
    Timer t(h, 0);
    launch_block_begin(b, s);
  }
  h->begun = false;
  { Timer t(h, 1); launch_interp(b, s); }
  { Timer t(h, 2); launch_prep(b, s); }
  int rc = launch_owed_measure(h);   // the previous block's, beside this block's proposals
  if (rc) return rc;
  { Timer t(h, 3); launch_propose(b, s); }
  { Timer t(h, 4); launch_assemble(b, s); }
  { Timer t(h, 5); launch_rankk(b, s); }
  // k_block_end rewrites the state copy the previous measurement reads
  if (h->meas_pending) HIPCHECK(h, hipStreamWaitEvent(s, h->ev_meas, 0));
  if (next_follows) {
    Timer t(h, 6);
    launch_block_turn(b, s);
    h->begun = true;
  } else {
    Timer t(h, 6);
    launch_block_end(b, s);
  }
  h->meas_owed = true;
  // many chains: the measurement is the longest step of a block and the next
  // block's k_block_end waits for it, so it starts at once
  if (b.n_chains >= 8) {
    int rc2 = launch_owed_measure(h);
    if (rc2) return rc2;
  }
  if (h->capturing) return CTAUX_OK;   // counted and scheduled by the graph replay
  h->blocks_launched += 1;
  {
    int rc2 = schedule_refinements(h);
    if (rc2) return rc2;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(h, CTAUX_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  if (h->timing && h->pool_used > 16000) {
    int rc = sync_all(h);
    if (rc) return rc;
    flush_timing(h);
  }
  return CTAUX_OK;
}

// The refinements due after block blocks_launched (intervals are powers of two,
// so with every interval a multiple of a graph window they fall at its ends).
int schedule_refinements(ctaux_batch *h) {
  if (h->recompute_every <= 0) return CTAUX_OK;
  std::vector<int> due;
  for (int c = 0; c < h->b.n_chains; ++c)
    if (h->blocks_launched % h->interval[c] == 0) due.push_back(c);
  if (due.empty()) return CTAUX_OK;
  return refine_chains(h, due, true, h->recompute_mode == 1);
}

// Brings the streams to the state a graph window starts from: the next
// block's start launched, no measurement owed or in flight.
int graph_entry(ctaux_batch *h) {
  if (!h->begun) {
    Timer t(h, 0);
    launch_block_begin(h->b, h->stream);
    h->begun = true;
  }
  int rc = launch_owed_measure(h);
  if (rc) return rc;
  if (h->meas_pending) {
    HIPCHECK(h, hipStreamWaitEvent(h->stream, h->ev_meas, 0));
    h->meas_pending = false;
  }
  return CTAUX_OK;
}

// Captures graph_blocks blocks and the last one's measurement (joined back to
// the capture stream) and instantiates them; nothing runs during the capture.
// The capture runs on a stream of the library's own, since the batch's stream
// may be the null stream; the graph is then launched on the batch's stream.
int capture_window(ctaux_batch *h) {
  if (!h->cstream && hipStreamCreate(&h->cstream) != hipSuccess) {
    h->cstream = nullptr;
    return set_err(h, CTAUX_EDEVICE, "hipStreamCreate failed");
  }
  const hipStream_t orig = h->stream;
  const int32_t timing = h->timing;
  h->timing = 0;   // no event pairs inside the graph
  h->capturing = true;
  h->stream = h->cstream;
  int rc = CTAUX_OK;
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    rc = set_err(h, CTAUX_EDEVICE, "hipStreamBeginCapture failed");
  } else {
    for (int i = 0; i < h->graph_blocks && rc == CTAUX_OK; ++i) rc = enqueue_block(h, true);
    if (rc == CTAUX_OK) rc = launch_owed_measure(h);
    if (rc == CTAUX_OK && hipStreamWaitEvent(h->stream, h->ev_meas, 0) != hipSuccess)
      rc = set_err(h, CTAUX_EDEVICE, "graph capture: joining the measurement stream failed");
    const hipError_t e = hipStreamEndCapture(h->stream, &g);
    if (rc == CTAUX_OK && e != hipSuccess) rc = set_err(h, CTAUX_EDEVICE, "hipStreamEndCapture failed");
  }
  h->capturing = false;
  h->stream = orig;
  h->timing = timing;
  h->meas_owed = false;
  h->meas_pending = false;
  h->begun = true;
  if (rc == CTAUX_OK && hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
    h->gexec = nullptr;
    rc = set_err(h, CTAUX_EDEVICE, "hipGraphInstantiate failed");
  }
  if (g) (void)hipGraphDestroy(g);
  return rc;
}

// A graph window may start here: graph_blocks blocks remain before the last
// block of the run, the window is aligned to graph_blocks, and no chain's
// refinement interval is shorter than the window.
bool graph_window_ok(const ctaux_batch *h, int64_t blocks_left) {
  const int g = h->graph_blocks;
  if (g <= 0 || blocks_left <= g || h->blocks_launched % g != 0) return false;
  if (h->recompute_every > 0)
    for (int32_t iv : h->interval)
      if (iv < g) return false;
  return true;
}

int run_graph_window(ctaux_batch *h) {
  int rc = graph_entry(h);
  if (rc) return rc;
  if (!h->gexec) {
    rc = capture_window(h);
    if (rc) return rc;
  }
  HIPCHECK(h, hipGraphLaunch(h->gexec, h->stream));
  h->graph_launches += 1;
  h->blocks_launched += h->graph_blocks;
  return schedule_refinements(h);
}

int chain_error(ctaux_batch *h) {
  for (int c = 0; c < h->b.n_chains; ++c) {
    const ChainState &st = h->state[c];
    if (st.status == CTAUX_ECAPACITY)
      return set_err(h, CTAUX_ECAPACITY, "chain %d: an insertion at proposal %lld would exceed n_cap=%d", c,
                     (long long)st.err_index, h->b.n_cap);
    if (st.status != 0 && st.err_index == -6)
      return set_err(h, st.status, "chain %d: N^{-1} of the configuration is singular or not finite "
                     "(from-scratch recompute failed)", c);
    if (st.status != 0 && st.err_index == -5)
      return set_err(h, st.status, "chain %d: refinement drift %.3g exceeds drift_tol (N is no longer the "
                     "inverse of its definition: refine more often, or use FP64 storage)", c, st.last_drift);
    if (st.status != 0)
      return set_err(h, st.status, "chain %d: numerical failure (code %d) at proposal %lld, drift %.3g", c,
                     st.status, (long long)st.err_index, st.last_drift);
  }
  return CTAUX_OK;
}

}  // namespace

extern "C" {

size_t ctaux_workspace_bytes(const ctaux_model *models, int32_t n_chains, const ctaux_opts *opts) {
  if (validate(models, n_chains, opts, nullptr) != CTAUX_OK) return 0;
  return layout(models, n_chains, opts, nullptr, nullptr, nullptr);
}

int ctaux_create(const ctaux_model *models, int32_t n_chains, const ctaux_opts *opts, void *dev_workspace,
                 size_t ws_bytes, void *hip_stream, ctaux_batch **out) {
  if (!out) return set_err(nullptr, CTAUX_EINVAL, "out is null");
  *out = nullptr;
  int rc = validate(models, n_chains, opts, nullptr);
  if (rc) return rc;
  const size_t need = layout(models, n_chains, opts, nullptr, nullptr, nullptr);
  if (!dev_workspace || ws_bytes < need)
    return set_err(nullptr, CTAUX_ENOMEM, "workspace of %zu bytes needed, %zu given", need, ws_bytes);
  if (reinterpret_cast<uintptr_t>(dev_workspace) % 256 != 0)
    return set_err(nullptr, CTAUX_EINVAL, "workspace must be 256-byte aligned");
  ctaux_batch *h = new (std::nothrow) ctaux_batch();
  if (!h) return set_err(nullptr, CTAUX_ENOMEM, "host allocation failed");
  h->stream = static_cast<hipStream_t>(hip_stream);
  Batch &b = h->b;
  b.n_chains = n_chains;
  b.kmax = opts->k_max;
  b.kcap = opts->k_cap;
  b.n_cap = opts->n_cap;
  b.ld = static_cast<int>(align_up(opts->n_cap, 64));
  b.precision = opts->precision;
  b.nc_max = 1;
  b.n_out_max = opts->n_tau_out;
  b.n_tau_max = 2;
  b.n_mats = opts->n_matsubara;
  b.n_k_max = 0;
  for (int c = 0; c < n_chains; ++c) {
    b.nc_max = models[c].n_sites > b.nc_max ? models[c].n_sites : b.nc_max;
    b.n_tau_max = models[c].n_tau > b.n_tau_max ? models[c].n_tau : b.n_tau_max;
    if (opts->n_matsubara > 0 && models[c].n_k > b.n_k_max) b.n_k_max = models[c].n_k;
  }
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    delete h;
    return set_err(nullptr, CTAUX_EDEVICE, "no HIP device");
  }
  b.n_cu = prop.multiProcessorCount;
  b.rankk_tile = opts->rankk_tile == 32 ? 32 : 64;
  b.pairs = opts->p_pair > 0.0 ? 1 : 0;
  b.grid_per_chain = n_chains >= 2048 ? 1 : 2048 / n_chains;
  if (b.grid_per_chain > 1024) b.grid_per_chain = 1024;
  h->recompute_every = opts->recompute_every;
  h->recompute_mode = opts->recompute_mode;
  h->max_interval = 1;
  while (2 * h->max_interval <= opts->recompute_every) h->max_interval *= 2;
  h->interval.assign(n_chains, 1);
  h->drift_target = opts->drift_target > 0.0 ? opts->drift_target : (opts->precision == CTAUX_FP64 ? 1e-10 : 1e-4);
  h->log_cap = opts->log_cap;
  layout(models, n_chains, opts, static_cast<char *>(dev_workspace), &b, &h->desc);
  // upload tables, maps and descriptors
  std::vector<ChainState> st(n_chains);
  for (int c = 0; c < n_chains; ++c) {
    const ctaux_model &m = models[c];
    ChainDesc &d = h->desc[c];
    const size_t tb = sizeof(double) * m.n_disp * m.n_tau;
    const int nc = m.n_sites;
    std::vector<int32_t> off(m.n_disp + 1, 0), pairs;
    for (int dd = 0; dd < m.n_disp; ++dd) {
      for (int x = 0; x < nc; ++x)
        for (int y = 0; y < nc; ++y)
          if (m.site_disp[x * nc + y] == dd) pairs.push_back(x * nc + y);
      off[dd + 1] = static_cast<int32_t>(pairs.size());
    }
    if (hipMemcpyAsync(const_cast<double *>(d.g0[0]), m.g0_up, tb, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(const_cast<double *>(d.g0[1]), m.g0_dn, tb, hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(const_cast<int32_t *>(d.site_disp), m.site_disp, sizeof(int32_t) * nc * nc,
                       hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(const_cast<int32_t *>(d.cls_off), off.data(), sizeof(int32_t) * off.size(),
                       hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemcpyAsync(const_cast<int32_t *>(d.cls_pairs), pairs.data(), sizeof(int32_t) * pairs.size(),
                       hipMemcpyHostToDevice, h->stream) != hipSuccess ||
        hipMemsetAsync(d.obs, 0, sizeof(double) * d.obs_len, h->stream) != hipSuccess ||
        (d.n_mats > 0 &&
         (hipMemcpyAsync(d.kw_pos, m.site_pos, sizeof(double) * 3 * nc, hipMemcpyHostToDevice, h->stream) !=
              hipSuccess ||
          hipMemcpyAsync(d.kw_k, m.kvecs, sizeof(double) * 3 * d.n_k, hipMemcpyHostToDevice, h->stream) !=
              hipSuccess ||
          hipMemsetAsync(d.obs_kw, 0, sizeof(double) * 4 * d.n_k * d.n_mats, h->stream) != hipSuccess)) ||
        (opts->log_cap > 0 &&
         (hipMemsetAsync(d.log_acc, 0, opts->log_cap, h->stream) != hipSuccess ||
          hipMemsetAsync(d.log_R, 0, sizeof(double) * opts->log_cap, h->stream) != hipSuccess))) {
      delete h;
      return set_err(nullptr, CTAUX_EDEVICE, "upload of chain %d failed", c);
    }
    // hipMemcpyAsync of pageable host memory is staged before returning, so the
    // temporaries above may go out of scope; synchronize per chain to be safe.
    if (hipStreamSynchronize(h->stream) != hipSuccess) {
      delete h;
      return set_err(nullptr, CTAUX_EDEVICE, "stream synchronisation failed");
    }
    h->obs_len.push_back(d.obs_len);
    if (d.obs_len > h->obs_len_max) h->obs_len_max = d.obs_len;
    memset(&st[c], 0, sizeof(ChainState));
    st[c].sign = 1.0;
  }
  h->state = st;
  if (setup_propose(b) != 0 || setup_refine(b) != 0) {
    delete h;
    return set_err(nullptr, CTAUX_EDEVICE, "setting the dynamic LDS limits of the kernels failed (LDS of the "
                   "proposal kernel: %zu bytes)", propose_lds_bytes(b.kcap, b.kmax, b.n_cap));
  }
  if (hipMemcpyAsync(b.d_desc, h->desc.data(), sizeof(ChainDesc) * n_chains, hipMemcpyHostToDevice, h->stream) !=
          hipSuccess ||
      hipMemcpyAsync(b.d_state, st.data(), sizeof(ChainState) * n_chains, hipMemcpyHostToDevice, h->stream) !=
          hipSuccess ||
      hipMemcpyAsync(b.d_mstate, st.data(), sizeof(ChainState) * n_chains, hipMemcpyHostToDevice, h->stream) !=
          hipSuccess ||
      hipStreamSynchronize(h->stream) != hipSuccess) {
    delete h;
    return set_err(nullptr, CTAUX_EDEVICE, "descriptor upload failed");
  }
  if (b.n_mats > 0) {
    launch_kw_g0(b, h->stream);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess) {
      delete h;
      return set_err(nullptr, CTAUX_EDEVICE, "G0(K, i w_n) set-up failed");
    }
  }
  // measurement stream (default priority, no implicit synchronisation with the
  // null stream) and the two events that order it against the caller's stream.
  // The events only order kernels of this device (the host waits by
  // synchronising the streams), so they release at device scope, without the
  // system-scope fence.
  const unsigned ev_flags = hipEventDisableTiming | hipEventDisableSystemFence;
  if (hipStreamCreateWithFlags(&h->mstream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_end, ev_flags) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_meas, ev_flags) != hipSuccess) {
    ctaux_destroy(h);
    return set_err(nullptr, CTAUX_EDEVICE, "measurement stream creation failed");
  }
  *out = h;
  return CTAUX_OK;
}

int ctaux_run(ctaux_batch *h, int64_t n_proposals) {
  if (!h) return CTAUX_EINVAL;
  if (n_proposals < 0) return set_err(h, CTAUX_EINVAL, "n_proposals < 0");
  int rc = chain_error(h);
  if (rc) return rc;
  if (n_proposals == 0) return CTAUX_OK;
  launch_set_target(h->b, h->stream, n_proposals);
  int64_t iters = (n_proposals + h->b.kmax - 1) / h->b.kmax;
  int64_t prev_done = -1;
  while (true) {
    for (int64_t i = 0; i < iters;) {
      if (graph_window_ok(h, iters - i)) {
        rc = run_graph_window(h);
        i += h->graph_blocks;
      } else {
        rc = enqueue_block(h, i + 1 < iters);
        i += 1;
      }
      if (rc) return rc;
    }
    rc = sync_states(h);
    if (rc) return rc;
    rc = chain_error(h);
    if (rc) return rc;
    int64_t remaining = 0, done_sum = 0;
    for (const ChainState &st : h->state) {
      remaining = st.target - st.done > remaining ? st.target - st.done : remaining;
      done_sum += st.done;
    }
    if (remaining == 0) break;
    if (done_sum == prev_done) return set_err(h, CTAUX_EDEVICE, "no chain progressed");
    prev_done = done_sum;
    iters = (remaining + h->b.kmax - 1) / h->b.kmax;
  }
  return CTAUX_OK;
}

static int recompute_impl(ctaux_batch *h, double *max_drift_out, bool scratch_only) {
  if (!h) return CTAUX_EINVAL;
  int rc0 = refine_all(h, scratch_only);
  if (rc0) return rc0;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(h, CTAUX_EDEVICE, "refine launch failed: %s", hipGetErrorString(e));
  int rc = sync_states(h);
  if (rc) return rc;
  double m = 0.0;
  for (const ChainState &st : h->state) m = st.last_drift > m ? st.last_drift : m;
  if (max_drift_out) *max_drift_out = m;
  return chain_error(h);
}

int ctaux_recompute(ctaux_batch *h, double *max_drift_out) { return recompute_impl(h, max_drift_out, false); }

int ctaux_recompute_from_scratch(ctaux_batch *h, double *max_drift_out) {
  return recompute_impl(h, max_drift_out, true);
}

int32_t ctaux_obs_len(const ctaux_batch *h) { return h ? h->obs_len_max : 0; }

int ctaux_get_obs(ctaux_batch *h, int32_t chain, double *out, int32_t len) {
  if (!h || !out || chain < 0 || chain >= h->b.n_chains) return CTAUX_EINVAL;
  const int32_t L = h->obs_len[chain];
  if (len < L) return set_err(h, CTAUX_EINVAL, "obs buffer of %d doubles needed", L);
  {
    int rc_ = sync_all(h);
    if (rc_) return rc_;
  }
  HIPCHECK(h, hipMemcpyAsync(out, h->desc[chain].obs, sizeof(double) * L, hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  for (int32_t i = L; i < len; ++i) out[i] = 0.0;
  return CTAUX_OK;
}

int ctaux_get_obs_kw(ctaux_batch *h, int32_t chain, double *s_out, double *g0_out, int32_t len) {
  if (!h || !s_out || chain < 0 || chain >= h->b.n_chains) return CTAUX_EINVAL;
  const ChainDesc &d = h->desc[chain];
  if (d.n_mats == 0) return set_err(h, CTAUX_EINVAL, "the batch was created with n_matsubara = 0");
  const int32_t L = 4 * d.n_k * d.n_mats;
  if (len < L) return set_err(h, CTAUX_EINVAL, "kw buffer of %d doubles needed", L);
  {
    int rc_ = sync_all(h);
    if (rc_) return rc_;
  }
  HIPCHECK(h, hipMemcpyAsync(s_out, d.obs_kw, sizeof(double) * L, hipMemcpyDeviceToHost, h->stream));
  if (g0_out) HIPCHECK(h, hipMemcpyAsync(g0_out, d.kw_g0, sizeof(double) * L, hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  return CTAUX_OK;
}

int ctaux_reset_obs(ctaux_batch *h) {
  if (!h) return CTAUX_EINVAL;
  {
    int rc_ = sync_all(h);   // a measurement in flight writes obs
    if (rc_) return rc_;
  }
  for (int c = 0; c < h->b.n_chains; ++c) {
    HIPCHECK(h, hipMemsetAsync(h->desc[c].obs, 0, sizeof(double) * h->obs_len[c], h->stream));
    if (h->desc[c].n_mats > 0)
      HIPCHECK(h, hipMemsetAsync(h->desc[c].obs_kw, 0, sizeof(double) * 4 * h->desc[c].n_k * h->desc[c].n_mats,
                                 h->stream));
  }
  {
    int rc_ = sync_all(h);
    if (rc_) return rc_;
  }
  return CTAUX_OK;
}

int ctaux_get_stats(ctaux_batch *h, int32_t chain, ctaux_stats *out) {
  if (!h || !out || chain < 0 || chain >= h->b.n_chains) return CTAUX_EINVAL;
  int rc = sync_states(h);
  if (rc) return rc;
  const ChainState &st = h->state[chain];
  out->proposals = st.done;
  out->accepted = st.accepted;
  out->blocks = st.blocks;
  out->sum_ka = st.sum_ka;
  out->next_id = st.next_id;
  out->order = st.n;
  out->status = st.status;
  out->sign = st.sign;
  out->max_drift = st.max_drift;
  out->rankk_flops = st.rk_flops;
  out->rankk_bytes = st.rk_bytes;
  out->sum_order = st.sum_order;
  out->gj_fallbacks = st.gj_fallbacks;
  out->prep_flops = st.prep_flops;
  out->prep_bytes = st.prep_bytes;
  out->meas_flops = st.meas_flops;
  out->meas_bytes = st.meas_bytes;
  out->scratch_recomputes = st.scratch_recomputes;
  out->refine_interval = h->recompute_every > 0 ? h->interval[chain] : 0;
  return CTAUX_OK;
}

int ctaux_get_config(ctaux_batch *h, int32_t chain, int32_t cap, ctaux_vertex *out, int32_t *n_out) {
  if (!h || chain < 0 || chain >= h->b.n_chains || cap < 0 || (cap > 0 && !out)) return CTAUX_EINVAL;
  int rc = sync_states(h);
  if (rc) return rc;
  const ChainState &st = h->state[chain];
  const ChainDesc &d = h->desc[chain];
  const int n = st.n, par = st.parity;
  if (n_out) *n_out = n;
  const int m = n < cap ? n : cap;
  if (m == 0) return CTAUX_OK;
  std::vector<double> tau(m);
  std::vector<int32_t> site(m), s(m);
  std::vector<int64_t> id(m);
  HIPCHECK(h, hipMemcpyAsync(tau.data(), d.tau[par], sizeof(double) * m, hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(h, hipMemcpyAsync(site.data(), d.site[par], sizeof(int32_t) * m, hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(h, hipMemcpyAsync(s.data(), d.s0[par], sizeof(int32_t) * m, hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(h, hipMemcpyAsync(id.data(), d.id[par], sizeof(int64_t) * m, hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  for (int i = 0; i < m; ++i) out[i] = ctaux_vertex{id[i], tau[i], site[i], s[i]};
  return CTAUX_OK;
}

int ctaux_get_N(ctaux_batch *h, int32_t chain, int32_t sector, double *out, int32_t ld, int32_t *n_out) {
  if (!h || chain < 0 || chain >= h->b.n_chains || sector < 0 || sector > 1) return CTAUX_EINVAL;
  int rc = sync_states(h);
  if (rc) return rc;
  const ChainState &st = h->state[chain];
  const ChainDesc &d = h->desc[chain];
  const int n = st.n;
  if (n_out) *n_out = n;
  if (n == 0 || !out) return CTAUX_OK;   // out == NULL: query the order only
  if (ld < n) return set_err(h, CTAUX_EINVAL, "ld < order %d", n);
  const size_t es = h->b.precision == CTAUX_FP64 ? sizeof(double) : sizeof(float);
  std::vector<char> tmp(es * n * n);
  int rc2 = n_to_host(h, tmp.data(), d.N[st.parity][sector], n, es);
  if (rc2) return rc2;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      out[static_cast<size_t>(i) * ld + j] =
          es == sizeof(double) ? reinterpret_cast<double *>(tmp.data())[static_cast<size_t>(i) * n + j]
                               : reinterpret_cast<float *>(tmp.data())[static_cast<size_t>(i) * n + j];
  return CTAUX_OK;
}

int ctaux_get_decisions(ctaux_batch *h, int32_t chain, int64_t first, int64_t count, uint8_t *acc, double *R) {
  if (!h || chain < 0 || chain >= h->b.n_chains || first < 0 || count < 0 || first + count > h->log_cap ||
      (count > 0 && (!acc || !R)))
    return h ? set_err(h, CTAUX_EINVAL, "decision range outside the log") : CTAUX_EINVAL;
  if (count == 0) return CTAUX_OK;
  {
    int rc_ = sync_all(h);
    if (rc_) return rc_;
  }
  HIPCHECK(h, hipMemcpyAsync(acc, h->desc[chain].log_acc + first, count, hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(h, hipMemcpyAsync(R, h->desc[chain].log_R + first, sizeof(double) * count, hipMemcpyDeviceToHost,
                             h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  return CTAUX_OK;
}

int ctaux_set_timing(ctaux_batch *h, int32_t mask) {
  if (!h) return CTAUX_EINVAL;
  {
    int rc_ = sync_all(h);
    if (rc_) return rc_;
  }
  flush_timing(h);
  h->timing = mask;
  for (int i = 0; i < 16; ++i) h->timing_seen[i] = 0;
  for (int i = 0; i < kNumNames; ++i) {
    h->ms[i] = 0.0;
    h->launches[i] = 0;
  }
  return CTAUX_OK;
}

int32_t ctaux_get_timing(ctaux_batch *h, const char **names, double *ms, int64_t *launches, int32_t cap) {
  if (!h) return 0;
  if (sync_all(h) != CTAUX_OK) return 0;
  flush_timing(h);
  int32_t k = 0;
  for (int i = 0; i < kNumNames && k < cap; ++i, ++k) {
    if (names) names[k] = kKernelNames[i];
    if (ms) ms[k] = h->ms[i];
    if (launches) launches[k] = h->launches[i];
  }
  return k;
}

// Checkpoint blob: header, then id[n] (int64), tau[n] (double), site[n], s[n]
// (int32), N of both sectors (n x n each, storage type, row-major), obs.
struct CkptHeader {
  char magic[8];
  int32_t version, precision, nc, n_tau, n, obs_len;
  double beta, K, gamma;
  int64_t next_id, done, accepted, blocks, sum_ka;
  int64_t launches;   // blocks enqueued on the batch
  int64_t refine_interval, since_refine;   // the chain's refinement interval (since_refine unused)
  double sign, max_drift, last_drift, rk_flops, rk_bytes, sum_order;
  int64_t kw_len;   // doubles of the momentum / Matsubara accumulators
};
constexpr char kCkptMagic[8] = {'C', 'T', 'A', 'U', 'X', 'C', 'K', '1'};

size_t kw_len(const ctaux_batch *h, int chain) {
  return 4 * static_cast<size_t>(h->desc[chain].n_k) * h->desc[chain].n_mats;
}

size_t ckpt_bytes(const ctaux_batch *h, int chain, int n) {
  const size_t es = h->b.precision == CTAUX_FP64 ? sizeof(double) : sizeof(float);
  return sizeof(CkptHeader) + static_cast<size_t>(n) * (8 + 8 + 4 + 4) + 2 * es * n * n +
         sizeof(double) * (h->obs_len[chain] + kw_len(h, chain));
}

int ctaux_checkpoint(ctaux_batch *h, int32_t chain, void *buf, size_t *len) {
  if (!h || !len || chain < 0 || chain >= h->b.n_chains) return CTAUX_EINVAL;
  int rc = sync_states(h);
  if (rc) return rc;
  const ChainState &st = h->state[chain];
  const ChainDesc &d = h->desc[chain];
  const int n = st.n, par = st.parity;
  const size_t need = ckpt_bytes(h, chain, n);
  if (!buf) {
    *len = need;
    return CTAUX_OK;
  }
  if (*len < need) return set_err(h, CTAUX_EINVAL, "checkpoint buffer of %zu bytes needed", need);
  *len = need;
  CkptHeader hd;
  memset(&hd, 0, sizeof hd);
  memcpy(hd.magic, kCkptMagic, 8);
  hd.version = 2;
  hd.precision = h->b.precision;
  hd.nc = d.nc;
  hd.n_tau = d.n_tau;
  hd.n = n;
  hd.obs_len = h->obs_len[chain];
  hd.beta = d.beta;
  hd.K = d.K;
  hd.gamma = d.gamma;
  hd.next_id = st.next_id;
  hd.done = st.done;
  hd.accepted = st.accepted;
  hd.blocks = st.blocks;
  hd.sum_ka = st.sum_ka;
  hd.launches = h->blocks_launched;
  hd.refine_interval = h->recompute_every > 0 ? h->interval[chain] : 0;
  hd.since_refine = 0;
  hd.sign = st.sign;
  hd.max_drift = st.max_drift;
  hd.last_drift = st.last_drift;
  hd.rk_flops = st.rk_flops;
  hd.rk_bytes = st.rk_bytes;
  hd.sum_order = st.sum_order;
  hd.kw_len = static_cast<int64_t>(kw_len(h, chain));
  char *p = static_cast<char *>(buf);
  memcpy(p, &hd, sizeof hd);
  p += sizeof hd;
  const size_t es = h->b.precision == CTAUX_FP64 ? sizeof(double) : sizeof(float);
  if (n > 0) {
    HIPCHECK(h, hipMemcpyAsync(p, d.id[par], 8 * n, hipMemcpyDeviceToHost, h->stream));
    p += 8 * n;
    HIPCHECK(h, hipMemcpyAsync(p, d.tau[par], 8 * n, hipMemcpyDeviceToHost, h->stream));
    p += 8 * n;
    HIPCHECK(h, hipMemcpyAsync(p, d.site[par], 4 * n, hipMemcpyDeviceToHost, h->stream));
    p += 4 * n;
    HIPCHECK(h, hipMemcpyAsync(p, d.s0[par], 4 * n, hipMemcpyDeviceToHost, h->stream));
    p += 4 * n;
    for (int sec = 0; sec < 2; ++sec) {
      rc = n_to_host(h, p, d.N[par][sec], n, es);
      if (rc) return rc;
      p += es * n * n;
    }
  }
  HIPCHECK(h, hipMemcpyAsync(p, d.obs, sizeof(double) * h->obs_len[chain], hipMemcpyDeviceToHost, h->stream));
  p += sizeof(double) * h->obs_len[chain];
  if (kw_len(h, chain) > 0)
    HIPCHECK(h, hipMemcpyAsync(p, d.obs_kw, sizeof(double) * kw_len(h, chain), hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  return CTAUX_OK;
}

int ctaux_restore(ctaux_batch *h, int32_t chain, const void *buf, size_t len) {
  if (!h || !buf || chain < 0 || chain >= h->b.n_chains) return CTAUX_EINVAL;
  CkptHeader hd;
  if (len < sizeof hd) return set_err(h, CTAUX_EINVAL, "checkpoint truncated");
  memcpy(&hd, buf, sizeof hd);
  const ChainDesc &d = h->desc[chain];
  if (memcmp(hd.magic, kCkptMagic, 8) != 0 || hd.version != 2)
    return set_err(h, CTAUX_EINVAL, "not a version-2 checkpoint");
  if (hd.precision != h->b.precision || hd.nc != d.nc || hd.n_tau != d.n_tau || hd.beta != d.beta ||
      hd.K != d.K || hd.gamma != d.gamma || hd.obs_len != h->obs_len[chain] ||
      hd.kw_len != static_cast<int64_t>(kw_len(h, chain)))
    return set_err(h, CTAUX_EINVAL, "checkpoint of another model or precision");
  if (hd.n < 0 || hd.n > h->b.n_cap) return set_err(h, CTAUX_EINVAL, "checkpoint order %d exceeds n_cap", hd.n);
  if (len < ckpt_bytes(h, chain, hd.n)) return set_err(h, CTAUX_EINVAL, "checkpoint truncated");
  int rc = sync_states(h);
  if (rc) return rc;
  const int n = hd.n;
  const size_t es = h->b.precision == CTAUX_FP64 ? sizeof(double) : sizeof(float);
  const char *p = static_cast<const char *>(buf) + sizeof hd;
  if (n > 0) {
    HIPCHECK(h, hipMemcpyAsync(d.id[0], p, 8 * n, hipMemcpyHostToDevice, h->stream));
    p += 8 * n;
    HIPCHECK(h, hipMemcpyAsync(d.tau[0], p, 8 * n, hipMemcpyHostToDevice, h->stream));
    p += 8 * n;
    HIPCHECK(h, hipMemcpyAsync(d.site[0], p, 4 * n, hipMemcpyHostToDevice, h->stream));
    p += 4 * n;
    HIPCHECK(h, hipMemcpyAsync(d.s0[0], p, 4 * n, hipMemcpyHostToDevice, h->stream));
    p += 4 * n;
    for (int sec = 0; sec < 2; ++sec) {
      rc = n_to_device(h, d.N[0][sec], p, n, es);
      if (rc) return rc;
      p += es * n * n;
    }
  }
  HIPCHECK(h, hipMemcpyAsync(d.obs, p, sizeof(double) * hd.obs_len, hipMemcpyHostToDevice, h->stream));
  p += sizeof(double) * hd.obs_len;
  if (kw_len(h, chain) > 0)
    HIPCHECK(h, hipMemcpyAsync(d.obs_kw, p, sizeof(double) * kw_len(h, chain), hipMemcpyHostToDevice, h->stream));
  ChainState st;
  memset(&st, 0, sizeof st);
  st.n = n;
  st.n_new = n;
  st.parity = 0;
  st.done = hd.done;
  st.target = hd.done;
  st.next_id = hd.next_id;
  st.accepted = hd.accepted;
  st.blocks = hd.blocks;
  st.sum_ka = hd.sum_ka;
  st.sign = hd.sign;
  st.max_drift = hd.max_drift;
  st.last_drift = hd.last_drift;
  st.rk_flops = hd.rk_flops;
  st.rk_bytes = hd.rk_bytes;
  st.sum_order = hd.sum_order;
  HIPCHECK(h, hipMemcpyAsync(h->b.d_state + chain, &st, sizeof st, hipMemcpyHostToDevice, h->stream));
  // the copies above read the caller's buffer and st: wait for them on the
  // batch's stream (see refine_all on synchronous copies from pageable memory)
  HIPCHECK(h, hipStreamSynchronize(h->stream));
  h->state[chain] = st;
  // The refinement schedule belongs to the batch; a one-chain batch takes over
  // the schedule of the checkpointed one (when both use the same recompute_every).
  if (h->b.n_chains == 1) h->blocks_launched = hd.launches;
  if (h->recompute_every > 0 && hd.refine_interval >= 1 && hd.refine_interval <= h->max_interval &&
      (hd.refine_interval & (hd.refine_interval - 1)) == 0)
    h->interval[chain] = static_cast<int32_t>(hd.refine_interval);
  return CTAUX_OK;
}

int ctaux_set_graph(ctaux_batch *h, int32_t blocks) {
  if (!h) return CTAUX_EINVAL;
  if (blocks < 0 || blocks > 64 || (blocks & (blocks - 1)) != 0)
    return set_err(h, CTAUX_EINVAL, "graph window must be 0 or a power of two up to 64 blocks");
  int rc = sync_all(h);
  if (rc) return rc;
  if (h->gexec) {
    (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
  }
  h->graph_blocks = blocks;
  return CTAUX_OK;
}

int64_t ctaux_graph_launches(const ctaux_batch *h) { return h ? h->graph_launches : -1; }

int ctaux_set_timing_every(ctaux_batch *h, int32_t every) {
  if (!h || every < 1) return CTAUX_EINVAL;
  h->timing_every = every;
  return CTAUX_OK;
}

const char *ctaux_last_error(const ctaux_batch *h) { return h ? h->err.c_str() : g_create_error; }

void ctaux_destroy(ctaux_batch *h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  if (h->mstream) {
    (void)hipStreamSynchronize(h->mstream);
    (void)hipStreamDestroy(h->mstream);
  }
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->cstream) (void)hipStreamDestroy(h->cstream);
  if (h->ev_end) (void)hipEventDestroy(h->ev_end);
  if (h->ev_meas) (void)hipEventDestroy(h->ev_meas);
  for (TimedEvent &e : h->pool) {
    (void)hipEventDestroy(e.start);
    (void)hipEventDestroy(e.stop);
  }
  delete h;
}

}  // extern "C"

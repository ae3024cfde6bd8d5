// C ABI: validation, parameter derivation (Sec. 2.5), workspace layout, step
// loop and host orchestration. Every entry point returns an LBM_E* code and
// records a message retrievable with lbm_last_error().
#include <hip/hip_runtime.h>
#include <math.h>
#include <stddef.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <utility>

#include "lattice.h"
#include "runtime.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

#define HIPCHECK(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(LBM_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));           \
  } while (0)

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// a checkpoint slot: this many header bytes, then one population buffer
constexpr size_t kCkptHeaderBytes = 256;

size_t storage_bytes(int storage) {
  switch (storage) {
    case LBM_F64: return 8;
    case LBM_F32: return 4;
    case LBM_F16: return 2;
    case LBM_BF16: return 2;
    case LBM_BF16_F16S: return 2;  // flow and scalar elements have one size
  }
  return 0;
}

// bytes of one population buffer: x-blocked rows of ceil(nx / 64) blocks of
// qt populations x 64 values
size_t state_bytes_of(const lbm_config* c, int qt) {
  return (size_t)c->ny * c->nz * lbm::xblocks(c->nx) * qt * lbm::kXB * storage_bytes(c->storage);
}

struct Layout {
  size_t buf, chibar, partials, dres, d0, scratch, total;
  int diag_blocks;
};

int block_x(int nx) { return nx >= lbm::kBlock ? lbm::kBlock : ((nx + 63) / 64) * 64; }

Layout layout_of(const lbm_config* c, const lbm_params* p) {
  Layout L;
  const int64_t n = (int64_t)c->nx * c->ny * c->nz;
  const int qt = p->q_flow + p->q_scalar;
  const int nbx = (c->nx + block_x(c->nx) - 1) / block_x(c->nx);
  L.diag_blocks = nbx * c->nz;
  size_t off = 0;
  L.buf = align256(state_bytes_of(c, qt) + lbm::kBufferGuardBytes);
  L.chibar = 2 * L.buf;
  off = L.chibar + align256((size_t)c->nx * c->nz * sizeof(double));
  L.partials = off;
  off += align256((size_t)L.diag_blocks * lbm::kDiagSlots * sizeof(double));
  L.dres = off;
  off += 256;
  L.d0 = off;
  off += 256;
  L.scratch = off;
  off += align256((size_t)n * sizeof(double));
  L.total = off;
  return L;
}

// Third-order rates and fourth-order equilibrium coefficients of the
// parametrised cumulant (Geier, Pasquali and Schoenherr 2017, the method the
// paper's VirtualFluids runs apply, Sec. 2.3) for shear rate w1 and bulk rate
// w2. false if a denominator vanishes or a value is not finite.
bool parametrized_rates(double w1, double w2, lbm_params* p) {
  const double w1s = w1 * w1, w2s = w2 * w2;
  const double dp = 8.0 * (5.0 - 2.0 * w1) * w1 + w2 * (8.0 + w1 * (9.0 * w1 - 26.0));
  const double dm = w2 * (56.0 - 42.0 * w1 + 9.0 * w1s) - 8.0 * w1;
  const double dd = 16.0 * w1s * (w1 - 6.0) - 2.0 * w1 * w2 * (216.0 + 5.0 * w1 * (9.0 * w1 - 46.0)) +
                    w2s * (w1 * (3.0 * w1 - 10.0) * (15.0 * w1 - 28.0) - 48.0);
  const double dab = (w1 - w2) * (w2 * (2.0 + 3.0 * w1) - 8.0 * w1);
  const double tiny = 1e-12;
  if (fabs(dp) < tiny || fabs(dm) < tiny || fabs(dd) < tiny || fabs(dab) < tiny) return false;
  p->w_plus = 8.0 * (w1 - 2.0) * (w2 * (3.0 * w1 - 1.0) - 5.0 * w1) / dp;
  p->w_minus = 8.0 * (w1 - 2.0) * (w1 + w2 * (3.0 * w1 - 7.0)) / dm;
  p->w_111 = 24.0 * (w1 - 2.0) *
             (4.0 * w1s + w1 * w2 * (18.0 - 13.0 * w1) + w2s * (2.0 + w1 * (6.0 * w1 - 11.0))) / dd;
  p->coef_a = (4.0 * w1s + 2.0 * w1 * w2 * (w1 - 6.0) + w2s * (w1 * (10.0 - 3.0 * w1) - 4.0)) / dab;
  p->coef_b = (4.0 * w1 * w2 * (9.0 * w1 - 16.0) - 4.0 * w1s - 2.0 * w2s * (2.0 + 9.0 * w1 * (w1 - 2.0))) /
              (3.0 * dab);
  return std::isfinite(p->w_plus) && std::isfinite(p->w_minus) && std::isfinite(p->w_111) &&
         std::isfinite(p->coef_a) && std::isfinite(p->coef_b);
}

int validate(const lbm_config* c, lbm_params* out) {
  if (!c) return fail(LBM_EINVAL, "config is NULL");
  if (c->struct_size != sizeof(lbm_config))
    return fail(LBM_EINVAL, "config struct_size %u != %zu", c->struct_size, sizeof(lbm_config));
  if (c->nx < 1 || c->ny < 1 || c->nz < 1)
    return fail(LBM_EINVAL, "grid %d x %d x %d: every size must be >= 1", c->nx, c->ny, c->nz);
  const int64_t n = (int64_t)c->nx * c->ny * c->nz;
  if (n >= ((int64_t)1 << 31)) return fail(LBM_EINVAL, "grid has %lld nodes (limit 2^31 - 1)", (long long)n);
  if (c->model != LBM_CUMULANT27_Q7 && c->model != LBM_BGK19_SMAG_Q6 &&
      c->model != LBM_CUMULANT27_FCM27)
    return fail(LBM_EINVAL, "unknown model %d", c->model);
  if (storage_bytes(c->storage) == 0) return fail(LBM_EINVAL, "unknown storage %d", c->storage);
  if (!(c->re_b > 0) || !(c->sc > 0) || !(c->sc_t > 0))
    return fail(LBM_EINVAL, "Re_b, Sc and Sc_T must be > 0");
  if (!(c->g_prime >= 0) || !(c->ub_lu >= 0) || !(c->cs_smag >= 0))
    return fail(LBM_EINVAL, "g', ub_lu and C_s must be >= 0");
  const double rates[5] = {c->omega_bulk, c->omega3, c->omega4, c->omega5, c->omega6};
  for (double r : rates)
    if (!(r > 0 && r < 2)) return fail(LBM_EINVAL, "relaxation rates must lie in (0, 2)");
  lbm_params p;
  const double H = (double)c->nz;
  p.g_prime = c->ub_lu > 0 ? c->ub_lu * c->ub_lu / H : c->g_prime;
  p.u_b = sqrt(p.g_prime * H);
  p.nu0 = p.u_b * H / c->re_b;
  p.tau0 = 3.0 * p.nu0 + 0.5;
  p.d0 = p.nu0 / c->sc;
  p.cs2_phi = c->model == LBM_CUMULANT27_Q7 ? 0.25 : 1.0 / 3.0;
  p.tau_phi0 = 0.5 + p.d0 / p.cs2_phi;
  p.q_flow = c->model == LBM_BGK19_SMAG_Q6 ? 19 : 27;
  p.q_scalar = c->model == LBM_CUMULANT27_Q7 ? 7 : (c->model == LBM_BGK19_SMAG_Q6 ? 6 : 27);
  if (!(p.tau0 > 0.5))
    return fail(LBM_EINVAL, "tau0 = %.17g must be > 1/2 (g' = 0 or Re_b too large)", p.tau0);
  p.w_plus = p.w_minus = p.w_111 = p.coef_a = p.coef_b = 0.0;
  if (c->parametrized != 0 && c->parametrized != 1)
    return fail(LBM_EINVAL, "parametrized must be 0 or 1");
  if (c->smag_paper_form != 0 && c->smag_paper_form != 1)
    return fail(LBM_EINVAL, "smag_paper_form must be 0 or 1");
  if (!(c->limiter >= 0) || std::isinf(c->limiter))
    return fail(LBM_EINVAL, "limiter must be finite and >= 0");
  if (c->parametrized) {
    if (c->model == LBM_BGK19_SMAG_Q6)
      return fail(LBM_EINVAL, "the parametrised rates need a cumulant model");
    if (c->cs_smag != 0.0)
      return fail(LBM_EINVAL, "the parametrised cumulant runs without the Smagorinsky model (cs_smag = 0)");
    if (c->omega3 != 1.0 || c->omega4 != 1.0 || c->omega5 != 1.0 || c->omega6 != 1.0)
      return fail(LBM_EINVAL, "parametrised mode replaces omega3..omega6: leave them at 1");
    if (!parametrized_rates(1.0 / p.tau0, c->omega_bulk, &p))
      return fail(LBM_EINVAL, "parametrised rates are singular or not finite at omega1 = %.17g, "
                  "omega_bulk = %.17g", 1.0 / p.tau0, c->omega_bulk);
  }
  if (out) *out = p;
  return LBM_OK;
}

int require_ready(lbm_handle* h) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (!h->initialised) return fail(LBM_ESTATE, "state not initialised (call lbm_init_*)");
  return LBM_OK;
}

int set_device(lbm_handle* h) {
  HIPCHECK(hipSetDevice(h->device));
  return LBM_OK;
}

int run_diag(lbm_handle* h, double* dst) {
  HIPCHECK(lbm::launch_diag(h, dst));
  return LBM_OK;
}

}  // namespace

extern "C" {

const char* lbm_last_error(void) { return g_err; }

// ------------------------------------------------------------ adjoint
namespace {
struct AdjLayout {
  size_t buf, ckpt, traj, lam, gpart, fwpart, small, total;
  int64_t nseg, ktraj;
  bool overlap;  // two trajectory sets: segment s - 1 is recomputed while s is reversed
};

// A state of at most this size stays in the 256 MB last-level cache with the
// adjoint buffers, and its kernels are bound by latency, not bandwidth: the
// adjoint run then recomputes the next segment on a second stream while the
// reverse sweep runs, so that the two sets of kernels fill each other's
// stalls. Larger states are bandwidth bound and run both on one stream.
constexpr size_t kOverlapStateBytes = 64ull << 20;

AdjLayout adj_layout(const lbm_config* c, const lbm_params* p, int64_t n_steps, int64_t k) {
  AdjLayout L;
  const int qt = p->q_flow + p->q_scalar;
  // population states (checkpoints, trajectory) and the two adjoint buffers
  // share the population buffers' x-blocked layout and slot size
  L.buf = align256(state_bytes_of(c, qt) + lbm::kBufferGuardBytes);
  L.nseg = (n_steps + k - 1) / k;
  // a segment's first state is its checkpoint; the trajectory slots hold
  // the other k - 1 (fewer when the run is shorter)
  L.ktraj = (k < n_steps ? k : n_steps) - 1;
  L.overlap = L.nseg >= 2 && L.buf <= kOverlapStateBytes;
  const int bx = block_x(c->nx);
  const int64_t ablocks = (int64_t)((c->nx + bx - 1) / bx) * c->ny * c->nz;
  const int64_t fblocks = (int64_t)lbm::xblocks(c->nx) * c->ny * std::min(c->nz, 2);
  size_t off = 0;
  L.ckpt = off;
  off += (size_t)L.nseg * L.buf;
  L.traj = off;
  off += (size_t)(L.overlap ? 2 : 1) * L.ktraj * L.buf;
  L.lam = off;
  off += 2 * L.buf;
  L.gpart = off;
  off += align256((size_t)ablocks * 2 * sizeof(double));
  L.fwpart = off;
  // one slot set per step, plus one that takes the unused sums of step 0 and
  // of the recomputed steps
  off += align256((size_t)(n_steps + 1) * fblocks * 2 * sizeof(double));
  L.small = off;
  off += 256;
  L.total = off;
  return L;
}

int adjoint_supported(const lbm_config* c) {
  if (c->storage != LBM_F32 && c->storage != LBM_F64)
    return fail(LBM_EINVAL, "the adjoint needs LBM_F32 or LBM_F64 storage");
  if (c->model != LBM_BGK19_SMAG_Q6 &&
      (c->omega3 != 1.0 || c->omega4 != 1.0 || c->omega5 != 1.0 || c->omega6 != 1.0))
    return fail(LBM_EINVAL, "the cumulant adjoint needs omega3..omega6 = 1");
  return LBM_OK;
}
}  // namespace

size_t lbm_adjoint_workspace_bytes(const lbm_config* cfg, int64_t n_steps, int64_t k_ckpt) {
  lbm_params p;
  if (validate(cfg, &p) != LBM_OK || n_steps < 1 || k_ckpt < 1) return 0;
  if (adjoint_supported(cfg) != LBM_OK) return 0;
  return adj_layout(cfg, &p, n_steps, k_ckpt).total;
}

// The adjoint run's second stream (non-blocking, default priority) and the
// events that order it against the handle's stream, made once per handle.
static int ensure_side_stream(lbm_handle* h) {
  if (h->side) return LBM_OK;
  hipStream_t st = nullptr;
  hipEvent_t ev[5] = {};
  bool ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; ok && i < 5; ++i)
    ok = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    for (int i = 0; i < 5; ++i)
      if (ev[i]) (void)hipEventDestroy(ev[i]);
    if (st) (void)hipStreamDestroy(st);
    return fail(LBM_EDEVICE, "could not create the adjoint run's second stream");
  }
  h->side = st;
  h->ev_fork = ev[0];
  h->ev_rec[0] = ev[1];
  h->ev_rec[1] = ev[2];
  h->ev_rev[0] = ev[3];
  h->ev_rev[1] = ev[4];
  return LBM_OK;
}

int lbm_adjoint_run(lbm_handle* h, int64_t n_steps, int64_t k_ckpt, double w_front, double w_fw,
                    void* adj_ws, size_t adj_bytes, double* J_out, double* dJ_dcs,
                    double* dJ_dsct, double* dJ_dchi0_dev) {
  int rc = require_ready(h);
  if (rc) return rc;
  if (h->step != 0) return fail(LBM_ESTATE, "the adjoint run must start from step 0 (step is %lld)",
                                (long long)h->step);
  if (n_steps < 1 || k_ckpt < 1) return fail(LBM_EINVAL, "n_steps and k_ckpt must be >= 1");
  if (!adj_ws || !J_out || !dJ_dcs || !dJ_dsct || !dJ_dchi0_dev) return fail(LBM_EINVAL, "NULL argument");
  if (((uintptr_t)adj_ws & 255) != 0) return fail(LBM_EINVAL, "adjoint workspace not 256-byte aligned");
  rc = adjoint_supported(&h->cfg);
  if (rc) return rc;
  const AdjLayout L = adj_layout(&h->cfg, &h->prm, n_steps, k_ckpt);
  if (adj_bytes < L.total)
    return fail(LBM_ENOMEM, "adjoint workspace of %zu bytes, %zu needed", adj_bytes, L.total);
  rc = set_device(h);
  if (rc) return rc;
  char* ws = (char*)adj_ws;
  double* gpart = (double*)(ws + L.gpart);
  double* fwpart = (double*)(ws + L.fwpart);
  double* small = (double*)(ws + L.small);  // [0] F_w sum, [8..12] front seed, [16..17] params
  const int nblk = lbm::adjoint_blocks(h);
  const size_t sbytes = h->state_bytes;
  auto ckpt = [&](int64_t s) { return (void*)(ws + L.ckpt + (size_t)s * L.buf); };
  HIPCHECK(lbm::launch_zero(h, gpart, 2 * (int64_t)nblk));
  HIPCHECK(lbm::launch_zero(h, small, 32));
  // Storage of the forward states. State m of segment s (m0 = s k_ckpt <= m <
  // e) is checkpoint s when m = m0, else slot m - m0 (1 .. k - 1) of the
  // segment's trajectory set (set s mod 2 when two sets overlap the
  // recomputation with the reverse sweep, else the one set). The forward
  // pass writes every checkpoint state straight into its slot and the states
  // of the last segment straight into their trajectory set, so the reverse
  // pass recomputes every segment but the last and copies nothing; the other
  // states go through the handle's two buffers, and the final state n ends in
  // the handle's current buffer.
  auto traj_slot = [&](int64_t s, int64_t i) {
    const size_t set = L.overlap ? (size_t)(s % 2) : 0;
    return (void*)(ws + L.traj + (set * L.ktraj + (size_t)(i - 1)) * L.buf);
  };
  auto state_of = [&](int64_t m) {
    const int64_t s = m / k_ckpt, m0 = s * k_ckpt;
    return m == m0 ? ckpt(s) : traj_slot(s, m - m0);
  };
  if (L.overlap) {
    rc = ensure_side_stream(h);
    if (rc) return rc;
  }
  const int64_t last = L.nseg - 1;
  // forward; the wall-layer sums of F_w(m), m = 1..n, go to one slot set per
  // step (slot m - 1) and are reduced once, in fixed order, at the end. Step
  // m -> m + 1 gathers state m and writes F_w(m) itself; the final state's
  // F_w(n) takes the separate wall-layer kernel. Every forward and recomputed
  // step runs the same kernel (step 0 and the recomputation write into the
  // spare slot set), so the recomputed states are bitwise the forward pass's
  // whatever the checkpoint interval.
  const int fwb = lbm::fw_blocks(h);
  double* fw_spare = fwpart + 2 * (size_t)fwb * n_steps;
  HIPCHECK(hipMemcpyAsync(ckpt(0), h->buf[h->cur], sbytes, hipMemcpyDeviceToDevice, h->stream));
  const void* cur = ckpt(0);
  for (int64_t m = 0; m < n_steps; ++m) {
    const int64_t mn = m + 1;
    void* dst;
    if (mn == n_steps) {
      h->cur = (cur == h->buf[0]) ? 1 : 0;
      dst = h->buf[h->cur];
    } else if (mn % k_ckpt == 0 || mn / k_ckpt == last) {
      dst = state_of(mn);
    } else {
      dst = (cur == h->buf[0]) ? h->buf[1] : h->buf[0];
    }
    double* fw = m >= 1 ? fwpart + 2 * (size_t)fwb * (m - 1) : fw_spare;
    HIPCHECK(lbm::launch_step(h, cur, dst, fw));
    cur = dst;
    h->step += 1;
  }
  auto recompute = [&](int64_t s, hipStream_t st) -> hipError_t {
    const int64_t m0 = s * k_ckpt;
    const int64_t e = std::min<int64_t>(m0 + k_ckpt, n_steps);
    for (int64_t m = m0; m + 1 < e; ++m) {
      const hipError_t err = lbm::launch_step(h, state_of(m), state_of(m + 1), fw_spare, st);
      if (err != hipSuccess) return err;
    }
    return hipSuccess;
  };
  if (L.overlap) {
    // the second stream starts on segment last - 1 once the forward pass is done
    HIPCHECK(hipEventRecord(h->ev_fork, h->stream));
    HIPCHECK(hipStreamWaitEvent(h->side, h->ev_fork, 0));
    HIPCHECK(recompute(last - 1, h->side));
    HIPCHECK(hipEventRecord(h->ev_rec[(last - 1) % 2], h->side));
  }
  HIPCHECK(lbm::launch_fw_layers(h, h->buf[h->cur], fwpart + 2 * (size_t)fwb * (n_steps - 1)));
  HIPCHECK(lbm::launch_fw_reduce(h, fwpart, n_steps * fwb, small));
  // final state: front and its seed, lambda(n)
  HIPCHECK(lbm::launch_diag(h, h->dres));
  HIPCHECK(lbm::launch_front_seed(h, w_front, small + 8));
  const double a0 = h->cfg.nz >= 2 ? w_fw / (double)n_steps * h->prm.nu0 * 3.0 : 0.0;
  const double a1 = h->cfg.nz >= 2 ? -w_fw / (double)n_steps * h->prm.nu0 / 3.0 : 0.0;
  void* lam_next = ws + L.lam;
  void* lam_out = ws + L.lam + L.buf;
  HIPCHECK(lbm::launch_adjoint_seed(h, h->buf[h->cur], lam_next, a0, a1, small + 8));
  // reverse sweep over the segments, recomputing each from its checkpoint
  // (the last segment's states are still in the trajectory). With two
  // trajectory sets the second stream recomputes segment s - 1 (event
  // ev_rec[(s - 1) % 2]) while this stream reverses segment s, and it starts
  // on segment s - 2, whose set is s's, only once s is reversed (ev_rev[s % 2]).
  for (int64_t s = last; s >= 0; --s) {
    const int64_t m0 = s * k_ckpt;
    const int64_t e = std::min<int64_t>(m0 + k_ckpt, n_steps);
    if (s != last) {
      if (L.overlap)
        HIPCHECK(hipStreamWaitEvent(h->stream, h->ev_rec[s % 2], 0));
      else
        HIPCHECK(recompute(s, h->stream));
    }
    for (int64_t m = e - 1; m >= m0; --m) {
      const bool seed = m >= 1;
      HIPCHECK(lbm::launch_adjoint_step(h, state_of(m), lam_next, lam_out, seed ? a0 : 0.0,
                                        seed ? a1 : 0.0, gpart, m == 0 ? dJ_dchi0_dev : nullptr));
      std::swap(lam_next, lam_out);
    }
    if (L.overlap && s >= 2) {
      HIPCHECK(hipEventRecord(h->ev_rev[s % 2], h->stream));
      HIPCHECK(hipStreamWaitEvent(h->side, h->ev_rev[s % 2], 0));
      HIPCHECK(recompute(s - 2, h->side));
      HIPCHECK(hipEventRecord(h->ev_rec[s % 2], h->side));
    }
  }
  // every recomputation on the second stream ended before a reverse step of
  // this stream that waited for it, the last one (segment 0) before step 0
  HIPCHECK(lbm::launch_sum_pairs(h, gpart, nblk, small + 16));
  double hs[32], r[8];
  HIPCHECK(hipMemcpyAsync(hs, small, sizeof(hs), hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipMemcpyAsync(r, h->dres, sizeof(r), hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  *J_out = w_front * (r[3] - h->x0) + w_fw * hs[0] / (double)n_steps;
  *dJ_dcs = hs[16];
  *dJ_dsct = hs[17];
  return LBM_OK;
}

int lbm_stream_copy(void* dst_dev, const void* src_dev, size_t bytes, void* hip_stream) {
  if (!dst_dev || !src_dev) return fail(LBM_EINVAL, "NULL pointer");
  if (bytes % 16 != 0) return fail(LBM_EINVAL, "bytes must be a multiple of 16");
  HIPCHECK(lbm::launch_stream_copy(dst_dev, src_dev, bytes, (hipStream_t)hip_stream));
  return LBM_OK;
}

int lbm_derive_params(const lbm_config* cfg, lbm_params* out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  return validate(cfg, out);
}

size_t lbm_workspace_bytes(const lbm_config* cfg) {
  lbm_params p;
  if (validate(cfg, &p) != LBM_OK) return 0;
  return layout_of(cfg, &p).total;
}

size_t lbm_state_bytes(const lbm_config* cfg) {
  lbm_params p;
  if (validate(cfg, &p) != LBM_OK) return 0;
  return kCkptHeaderBytes + layout_of(cfg, &p).buf;
}

int lbm_create(const lbm_config* cfg, void* dev_workspace, size_t bytes, void* hip_stream,
               lbm_handle** out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  lbm_params p;
  int rc = validate(cfg, &p);
  if (rc) return rc;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return fail(LBM_ENODEV, "no GPU visible to the HIP runtime");
  if (!dev_workspace) return fail(LBM_EINVAL, "workspace is NULL");
  if (((uintptr_t)dev_workspace & 255) != 0) return fail(LBM_EINVAL, "workspace not 256-byte aligned");
  const Layout L = layout_of(cfg, &p);
  if (bytes < L.total)
    return fail(LBM_ENOMEM, "workspace of %zu bytes, %zu needed", bytes, L.total);
  lbm_handle* h = new (std::nothrow) lbm_handle();
  if (!h) return fail(LBM_ENOMEM, "host allocation failed");
  h->cfg = *cfg;
  h->prm = p;
  h->qf = p.q_flow;
  h->qs = p.q_scalar;
  h->qt = p.q_flow + p.q_scalar;
  h->n = (int64_t)cfg->nx * cfg->ny * cfg->nz;
  h->esize = storage_bytes(cfg->storage);
  h->state_bytes = state_bytes_of(cfg, h->qt);
  if (hipGetDevice(&h->device) != hipSuccess ||
      hipDeviceGetAttribute(&h->cu_count, hipDeviceAttributeMultiprocessorCount, h->device) !=
          hipSuccess) {
    delete h;
    return fail(LBM_EDEVICE, "hipGetDevice or hipDeviceGetAttribute failed");
  }
  h->stream = (hipStream_t)hip_stream;
  h->ws = (char*)dev_workspace;
  h->ws_bytes = bytes;
  h->buf[0] = h->ws;
  h->buf[1] = h->ws + L.buf;
  h->cur = 0;
  h->chibar = (double*)(h->ws + L.chibar);
  h->partials = (double*)(h->ws + L.partials);
  h->dres = (double*)(h->ws + L.dres);
  h->d0 = (double*)(h->ws + L.d0);
  h->scratch = (double*)(h->ws + L.scratch);
  h->diag_blocks = L.diag_blocks;
  h->step = 0;
  h->initialised = false;
  h->x0 = (int)floor(0.125 * cfg->nx);
  *out = h;
  return LBM_OK;
}

int lbm_destroy(lbm_handle* h) {
  if (h && h->side) {
    // the adjoint run's second stream is idle: every run ends with a
    // synchronisation of the handle's stream, which waited for it
    int prev = -1;
    const bool had = hipGetDevice(&prev) == hipSuccess;
    if (hipSetDevice(h->device) == hipSuccess) {
      (void)hipEventDestroy(h->ev_fork);
      for (int i = 0; i < 2; ++i) {
        (void)hipEventDestroy(h->ev_rec[i]);
        (void)hipEventDestroy(h->ev_rev[i]);
      }
      (void)hipStreamDestroy(h->side);
      if (had && prev != h->device) (void)hipSetDevice(prev);
    }
  }
  delete h;
  return LBM_OK;
}

static int after_init(lbm_handle* h) {
  h->step = 0;
  h->initialised = true;
  return run_diag(h, h->d0);
}

int lbm_init_lock_exchange(lbm_handle* h, double lock_fraction, double noise_amp, uint64_t seed) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (!(lock_fraction > 0 && lock_fraction < 1)) return fail(LBM_EINVAL, "lock_fraction must be in (0, 1)");
  if (!(noise_amp >= 0 && noise_amp < 1)) return fail(LBM_EINVAL, "noise_amp must be in [0, 1)");
  int rc = set_device(h);
  if (rc) return rc;
  h->cur = 0;
  h->x0 = (int)floor(lock_fraction * h->cfg.nx);
  HIPCHECK(lbm::launch_init_lock(h, lock_fraction, noise_amp, seed));
  return after_init(h);
}

int lbm_init_from_field(lbm_handle* h, const double* chi0_dev, double lock_fraction) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (!chi0_dev) return fail(LBM_EINVAL, "chi0 is NULL");
  if (!(lock_fraction >= 0 && lock_fraction < 1)) return fail(LBM_EINVAL, "lock_fraction must be in [0, 1)");
  int rc = set_device(h);
  if (rc) return rc;
  h->cur = 0;
  h->x0 = (int)floor(lock_fraction * h->cfg.nx);
  HIPCHECK(lbm::launch_init_field(h, chi0_dev));
  return after_init(h);
}

int lbm_step(lbm_handle* h, int64_t n) {
  int rc = require_ready(h);
  if (rc) return rc;
  if (n < 0) return fail(LBM_EINVAL, "negative step count");
  if (n == 0) return LBM_OK;
  rc = set_device(h);
  if (rc) return rc;
  for (int64_t i = 0; i < n; ++i) {
    HIPCHECK(lbm::launch_step(h, h->buf[h->cur], h->buf[h->cur ^ 1]));
    h->cur ^= 1;
    h->step += 1;
  }
  return LBM_OK;
}

int lbm_moments(lbm_handle* h, int dtype, void* rho, void* ux, void* uy, void* uz, void* chi) {
  int rc = require_ready(h);
  if (rc) return rc;
  if (dtype != LBM_OUT_F32 && dtype != LBM_OUT_F64) return fail(LBM_EINVAL, "dtype must be LBM_OUT_F32 or LBM_OUT_F64");
  rc = set_device(h);
  if (rc) return rc;
  HIPCHECK(lbm::launch_moments(h, dtype, rho, ux, uy, uz, chi));
  return LBM_OK;
}

int lbm_wall_shear(lbm_handle* h, int dtype, void* tau, void* tau_bar) {
  int rc = require_ready(h);
  if (rc) return rc;
  if (dtype != LBM_OUT_F32 && dtype != LBM_OUT_F64) return fail(LBM_EINVAL, "dtype must be LBM_OUT_F32 or LBM_OUT_F64");
  if (h->cfg.nz < 2) return fail(LBM_EINVAL, "the wall shear stress needs nz >= 2");
  rc = set_device(h);
  if (rc) return rc;
  HIPCHECK(lbm::launch_wall_shear(h, dtype, tau, tau_bar));
  return LBM_OK;
}

int lbm_get_step(const lbm_handle* h, int64_t* step) {
  if (!h || !step) return fail(LBM_EINVAL, "NULL argument");
  *step = h->step;
  return LBM_OK;
}

// lbm_diag from the diagnostics kernels' result slot r and the initial
// diagnostics r0 of a run at `step` with gate index x0
static int fill_diag(lbm_diag* out, const double* r, const double* r0, int64_t step, int x0,
                     const lbm_config& cfg, const lbm_params& prm) {
  const double H = (double)cfg.nz, ub = prm.u_b;
  out->step = step;
  out->t_nd = (double)step * ub / H;
  out->mass = r[0];
  out->mass0 = r0[0];
  out->chi_mass = r[1];
  out->chi_mass0 = r0[1];
  out->fw = r[2];
  out->fw_nd = ub > 0 ? r[2] / (ub * ub * H * H) : 0.0;
  out->x_front = r[3];
  out->x_f = r[3] - x0;
  out->x_f_nd = out->x_f / H;
  out->umax = r[4];
  out->nonfinite = (int64_t)r[5];
  if (out->nonfinite > 0)
    return fail(LBM_EUNSTABLE, "%lld nodes hold non-finite moments at step %lld",
                (long long)out->nonfinite, (long long)step);
  return LBM_OK;
}

int lbm_diagnostics(lbm_handle* h, lbm_diag* out) {
  int rc = require_ready(h);
  if (rc) return rc;
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  rc = set_device(h);
  if (rc) return rc;
  rc = run_diag(h, h->dres);
  if (rc) return rc;
  double r[8], r0[8];
  HIPCHECK(hipMemcpyAsync(r, h->dres, sizeof(r), hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipMemcpyAsync(r0, h->d0, sizeof(r0), hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  return fill_diag(out, r, r0, h->step, h->x0, h->cfg, h->prm);
}

// Header of a checkpoint slot, in its first 256 bytes (the population buffer
// follows): the configuration it belongs to, the step counter, the gate index
// and the diagnostics at initialisation (so that a fresh handle restored from
// the slot reports mass drift and front position against the saved run's
// start). The header comes first so that reading it stays inside any slot,
// whichever configuration wrote it; the populations are copied only once it
// matches the handle's.
struct CkptHeader {
  uint64_t magic;
  int32_t nx, ny, nz, model, storage, x0;
  int64_t step;
  double d0[8];
};
constexpr uint64_t kCkptMagic = 0x31544B43504D424Cull;  // "LBMPCKT1"
static_assert(sizeof(CkptHeader) <= kCkptHeaderBytes, "checkpoint header must fit its 256 bytes");

int lbm_checkpoint_save(lbm_handle* h, void* dev_slot) {
  int rc = require_ready(h);
  if (rc) return rc;
  if (!dev_slot) return fail(LBM_EINVAL, "slot is NULL");
  rc = set_device(h);
  if (rc) return rc;
  char* hdr = (char*)dev_slot;
  HIPCHECK(lbm::launch_copy_state(h, h->buf[h->cur], hdr + kCkptHeaderBytes));
  static thread_local CkptHeader hh;
  hh.magic = kCkptMagic;
  hh.nx = h->cfg.nx;
  hh.ny = h->cfg.ny;
  hh.nz = h->cfg.nz;
  hh.model = h->cfg.model;
  hh.storage = h->cfg.storage;
  hh.x0 = h->x0;
  hh.step = h->step;
  HIPCHECK(hipMemcpyAsync(hdr, &hh, offsetof(CkptHeader, d0), hipMemcpyHostToDevice, h->stream));
  HIPCHECK(hipMemcpyAsync(hdr + offsetof(CkptHeader, d0), h->d0, sizeof(hh.d0), hipMemcpyDeviceToDevice,
                          h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

int lbm_checkpoint_load(lbm_handle* h, const void* dev_slot) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (!dev_slot) return fail(LBM_EINVAL, "slot is NULL");
  int rc = set_device(h);
  if (rc) return rc;
  const char* hdr = (const char*)dev_slot;
  CkptHeader hh;
  HIPCHECK(hipMemcpyAsync(&hh, hdr, offsetof(CkptHeader, d0), hipMemcpyDeviceToHost, h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  if (hh.magic != kCkptMagic)
    return fail(LBM_EINVAL, "slot does not hold a checkpoint (bad header)");
  const lbm_config& c = h->cfg;
  if (hh.nx != c.nx || hh.ny != c.ny || hh.nz != c.nz || hh.model != c.model || hh.storage != c.storage)
    return fail(LBM_EINVAL, "checkpoint of a %d x %d x %d grid, model %d, storage %d does not match "
                "the handle's %d x %d x %d, model %d, storage %d", hh.nx, hh.ny, hh.nz, hh.model,
                hh.storage, c.nx, c.ny, c.nz, c.model, c.storage);
  if (hh.step < 0 || hh.x0 < 0 || hh.x0 >= c.nx)
    return fail(LBM_EINVAL, "checkpoint header holds step %lld, gate %d", (long long)hh.step, hh.x0);
  HIPCHECK(lbm::launch_copy_state(h, hdr + kCkptHeaderBytes, h->buf[h->cur]));
  HIPCHECK(hipMemcpyAsync(h->d0, hdr + offsetof(CkptHeader, d0), sizeof(hh.d0), hipMemcpyDeviceToDevice,
                          h->stream));
  HIPCHECK(hipStreamSynchronize(h->stream));
  h->step = hh.step;
  h->x0 = hh.x0;
  h->initialised = true;
  return LBM_OK;
}

int lbm_checkpoint_diagnostics(const lbm_config* cfg, const void* dev_slot, void* hip_stream,
                               lbm_diag* out) {
  if (!dev_slot || !out) return fail(LBM_EINVAL, "NULL argument");
  lbm_params p;
  int rc = validate(cfg, &p);
  if (rc) return rc;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return fail(LBM_ENODEV, "no GPU visible to the HIP runtime");
  // scratch of the diagnostics kernels, as a handle's workspace holds it:
  // span sums of chi, per-block partials, one result slot
  const Layout L = layout_of(cfg, &p);
  const size_t n_chibar = align256((size_t)cfg->nx * cfg->nz * sizeof(double)) / sizeof(double);
  const size_t n_part = align256((size_t)L.diag_blocks * lbm::kDiagSlots * sizeof(double)) / sizeof(double);
  const size_t need = n_chibar + n_part + 32;
  if (need > lbm::kStaticScratchDoubles)
    return fail(LBM_ENOMEM, "the diagnostics of a %d x %d x %d grid need %zu bytes of scratch; the "
                "allocation-free entry point holds %zu (nx * nz up to about %zu)", cfg->nx, cfg->ny,
                cfg->nz, need * sizeof(double), lbm::kStaticScratchDoubles * sizeof(double),
                lbm::kStaticScratchDoubles - n_part - 32);
  double* sp = nullptr;
  HIPCHECK(lbm::static_scratch(&sp));
  hipStream_t stream = (hipStream_t)hip_stream;
  const char* hdr = (const char*)dev_slot;
  CkptHeader hh;
  HIPCHECK(hipMemcpyAsync(&hh, hdr, sizeof(hh), hipMemcpyDeviceToHost, stream));
  HIPCHECK(hipStreamSynchronize(stream));
  if (hh.magic != kCkptMagic)
    return fail(LBM_EINVAL, "slot does not hold a checkpoint (bad header)");
  if (hh.nx != cfg->nx || hh.ny != cfg->ny || hh.nz != cfg->nz || hh.model != cfg->model ||
      hh.storage != cfg->storage)
    return fail(LBM_EINVAL, "checkpoint of a %d x %d x %d grid, model %d, storage %d does not match "
                "the configuration's %d x %d x %d, model %d, storage %d", hh.nx, hh.ny, hh.nz, hh.model,
                hh.storage, cfg->nx, cfg->ny, cfg->nz, cfg->model, cfg->storage);
  // a handle on the host stack (no device memory of its own): the slot's
  // populations and the static scratch
  lbm_handle t{};
  t.cfg = *cfg;
  t.prm = p;
  t.qf = p.q_flow;
  t.qs = p.q_scalar;
  t.qt = p.q_flow + p.q_scalar;
  t.n = (int64_t)cfg->nx * cfg->ny * cfg->nz;
  t.esize = storage_bytes(cfg->storage);
  t.state_bytes = state_bytes_of(cfg, t.qt);
  HIPCHECK(hipGetDevice(&t.device));
  t.stream = stream;
  t.buf[0] = (void*)(hdr + kCkptHeaderBytes);
  t.buf[1] = nullptr;
  t.cur = 0;
  t.chibar = sp;
  t.partials = sp + n_chibar;
  t.dres = sp + n_chibar + n_part;
  t.diag_blocks = L.diag_blocks;
  t.step = hh.step;
  t.x0 = hh.x0;
  t.initialised = true;
  HIPCHECK(lbm::launch_diag(&t, t.dres));
  double r[8];
  HIPCHECK(hipMemcpyAsync(r, t.dres, sizeof(r), hipMemcpyDeviceToHost, stream));
  HIPCHECK(hipStreamSynchronize(stream));
  return fill_diag(out, r, hh.d0, hh.step, hh.x0, *cfg, p);
}

int lbm_get_populations(lbm_handle* h, double* host_f, double* host_phi) {
  int rc = require_ready(h);
  if (rc) return rc;
  if (!host_f || !host_phi) return fail(LBM_EINVAL, "NULL output");
  rc = set_device(h);
  if (rc) return rc;
  for (int a = 0; a < h->qt; ++a) {
    double* dst = a < h->qf ? host_f + (int64_t)a * h->n : host_phi + (int64_t)(a - h->qf) * h->n;
    HIPCHECK(lbm::launch_get_pop(h, a, h->scratch));
    HIPCHECK(hipMemcpyAsync(dst, h->scratch, h->n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
  }
  return LBM_OK;
}

int lbm_set_populations(lbm_handle* h, const double* host_f, const double* host_phi) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (!host_f || !host_phi) return fail(LBM_EINVAL, "NULL input");
  int rc = set_device(h);
  if (rc) return rc;
  for (int a = 0; a < h->qt; ++a) {
    const double* srcp = a < h->qf ? host_f + (int64_t)a * h->n : host_phi + (int64_t)(a - h->qf) * h->n;
    HIPCHECK(hipMemcpyAsync(h->scratch, srcp, h->n * sizeof(double), hipMemcpyHostToDevice, h->stream));
    HIPCHECK(lbm::launch_set_pop(h, a, h->scratch));
    HIPCHECK(hipStreamSynchronize(h->stream));
  }
  if (!h->initialised) {
    h->step = 0;
    h->initialised = true;
    return run_diag(h, h->d0);
  }
  return LBM_OK;
}

}  // extern "C"

// Handle and launcher interface shared by the C ABI (abi.cpp) and the kernel
// translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/lbm.h"

struct lbm_handle {
  lbm_config cfg;
  lbm_params prm;
  int qf, qs, qt;     // flow, scalar, total populations
  int64_t n;          // nodes
  size_t esize;       // bytes per stored population value
  size_t state_bytes; // bytes of one population buffer (x-blocked, padded rows)
  int device;
  int cu_count;       // compute units of the device
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  void* buf[2];       // population buffers (post-collision values, pull layout)
  int cur;            // index of the buffer holding the current state
  double* chibar;     // nx * nz span sums of chi (diagnostics)
  double* partials;   // per-block diagnostic partial sums
  double* dres;       // 8 doubles: current diagnostics
  double* d0;         // 8 doubles: diagnostics at initialisation
  double* scratch;    // n doubles (get/set hooks)
  int64_t step;
  bool initialised;
  int x0;             // gate index
  int diag_blocks;
  // the adjoint run's second stream (default priority) and its events, made
  // on first use for a grid whose recomputation overlaps the reverse sweep
  hipStream_t side;
  hipEvent_t ev_fork, ev_rec[2], ev_rev[2];
};

namespace lbm {

constexpr int kBlock = 256;  // threads per block along x (multiple of 64)
constexpr int kNodesPerThread = 2;  // step kernel: nodes per thread along x (FP32, FP64)
// The cumulant + D3Q27-scalar model holds 54 populations per node: one node
// per thread keeps its register count (and so its occupancy) near the others'.
// With 16-bit storage one node per thread also measured faster (FP16 +5 %,
// BF16 +13 % at 2048 x 128 x 256); FP32 is faster at two.
template <int MODEL, typename ST>
constexpr int nodes_per_thread() {
  return MODEL == 2 ? 1 : (sizeof(ST) == 2 ? 1 : kNodesPerThread);
}
constexpr int kDiagSlots = 8;  // partial sums per diagnostic block

// kernels.hip
// one step src -> dst; fw (the adjoint's forward pass, FP32 / FP64 storage):
// also the wall-layer sums of F_w of the gathered state into
// fw[2 fw_blocks], as launch_fw_layers writes them. st: the stream to launch
// on (null: the handle's)
hipError_t launch_step(lbm_handle* h, const void* src, void* dst, double* fw = nullptr,
                       hipStream_t st = nullptr);
hipError_t launch_init_lock(lbm_handle* h, double lock_fraction, double amp, uint64_t seed);
hipError_t launch_init_field(lbm_handle* h, const double* chi0);
hipError_t launch_moments(lbm_handle* h, int dtype, void* rho, void* ux, void* uy, void* uz,
                          void* chi);
hipError_t launch_wall_shear(lbm_handle* h, int dtype, void* tau, void* tau_bar);
hipError_t launch_diag(lbm_handle* h, double* out);
hipError_t launch_get_pop(lbm_handle* h, int q, double* dst);
hipError_t launch_set_pop(lbm_handle* h, int q, const double* src);
hipError_t launch_copy_state(lbm_handle* h, const void* src, void* dst);
hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t stream);
// device address, on the current device, of the static scratch array of the
// allocation-free diagnostics (kStaticScratchDoubles doubles)
constexpr size_t kStaticScratchDoubles = (size_t)1 << 22;
hipError_t static_scratch(double** ptr);

// adjoint.hip
int adjoint_blocks(const lbm_handle* h);
int fw_blocks(const lbm_handle* h);
hipError_t launch_adjoint_step(lbm_handle* h, const void* state, const void* lam_next,
                               void* lam_out, double a0, double a1, double* gpart, double* dchi0);
hipError_t launch_adjoint_seed(lbm_handle* h, const void* state, void* lam, double a0, double a1,
                               const double* fs);
hipError_t launch_front_seed(lbm_handle* h, double w_front, double* out);
// wall-layer sums of F_w of the current state into part[2 fw_blocks]
hipError_t launch_fw_layers(lbm_handle* h, const void* state, double* part);
// out[0] += nu0 (9 S0 - S1) / 3 over nparts partial pairs (fixed order)
hipError_t launch_fw_reduce(lbm_handle* h, const double* part, int64_t nparts, double* out);
hipError_t launch_sum_pairs(lbm_handle* h, const double* part, int nparts, double* out);
hipError_t launch_zero(lbm_handle* h, double* p, int64_t n);

}  // namespace lbm

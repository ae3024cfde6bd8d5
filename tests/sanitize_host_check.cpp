// Host-only build of the C ABI's host code (csrc/abi.cpp) under AddressSanitizer
// and UndefinedBehaviorSanitizer: every validation path that runs before any
// device work, on valid, invalid and extreme configurations. The kernel
// launchers are replaced by stubs that report "no device" (none of the paths
// below reaches them: the library checks for a GPU first). Exit status 0 and
// "sanitize ok" on success; a sanitizer report aborts the run.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "runtime.h"

namespace lbm {
hipError_t launch_step(lbm_handle*, const void*, void*, double*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_init_lock(lbm_handle*, double, double, uint64_t) { return hipErrorNoDevice; }
hipError_t launch_init_field(lbm_handle*, const double*) { return hipErrorNoDevice; }
hipError_t launch_moments(lbm_handle*, int, void*, void*, void*, void*, void*) { return hipErrorNoDevice; }
hipError_t launch_wall_shear(lbm_handle*, int, void*, void*) { return hipErrorNoDevice; }
hipError_t launch_diag(lbm_handle*, double*) { return hipErrorNoDevice; }
hipError_t launch_get_pop(lbm_handle*, int, double*) { return hipErrorNoDevice; }
hipError_t launch_set_pop(lbm_handle*, int, const double*) { return hipErrorNoDevice; }
hipError_t launch_copy_state(lbm_handle*, const void*, void*) { return hipErrorNoDevice; }
hipError_t launch_stream_copy(void*, const void*, size_t, hipStream_t) { return hipErrorNoDevice; }
int adjoint_blocks(const lbm_handle*) { return 1; }
int fw_blocks(const lbm_handle*) { return 1; }
hipError_t launch_adjoint_step(lbm_handle*, const void*, const void*, void*, double, double, double*,
                               double*) { return hipErrorNoDevice; }
hipError_t launch_adjoint_seed(lbm_handle*, const void*, void*, double, double, const double*) {
  return hipErrorNoDevice;
}
hipError_t launch_front_seed(lbm_handle*, double, double*) { return hipErrorNoDevice; }
hipError_t launch_fw_layers(lbm_handle*, const void*, double*) { return hipErrorNoDevice; }
hipError_t launch_fw_reduce(lbm_handle*, const double*, int64_t, double*) { return hipErrorNoDevice; }
hipError_t launch_sum_pairs(lbm_handle*, const double*, int, double*) { return hipErrorNoDevice; }
hipError_t launch_zero(lbm_handle*, double*, int64_t) { return hipErrorNoDevice; }
hipError_t static_scratch(double**) { return hipErrorNoDevice; }
}  // namespace lbm

static int fails = 0;
#define EXPECT(c)                                                   \
  do {                                                              \
    if (!(c)) {                                                     \
      ++fails;                                                      \
      printf("FAIL line %d: %s (%s)\n", __LINE__, #c, lbm_last_error()); \
    }                                                               \
  } while (0)

static lbm_config base(int nx, int ny, int nz, int model, int storage) {
  lbm_config c;
  memset(&c, 0, sizeof(c));
  c.struct_size = sizeof(lbm_config);
  c.nx = nx;
  c.ny = ny;
  c.nz = nz;
  c.model = model;
  c.storage = storage;
  c.re_b = 30000.0;
  c.sc = 1.0;
  c.g_prime = 1e-4;
  c.cs_smag = 0.1;
  c.sc_t = 1.0;
  c.omega_bulk = c.omega3 = c.omega4 = c.omega5 = c.omega6 = 1.0;
  return c;
}

int main() {
  // valid configurations, including the largest grid (64-bit sizes)
  const int grids[][3] = {{1, 1, 1}, {65, 3, 2}, {1024, 64, 128}, {4096, 256, 512}, {256, 16, 32}};
  for (auto& gr : grids)
    for (int model = 0; model < 3; ++model)
      for (int st = 0; st < 5; ++st) {
        lbm_config c = base(gr[0], gr[1], gr[2], model, st);
        lbm_params p;
        EXPECT(lbm_derive_params(&c, &p) == LBM_OK);
        EXPECT(lbm_workspace_bytes(&c) > 0);
        EXPECT(lbm_state_bytes(&c) > 0);
        if (st == LBM_F32 || st == LBM_F64) {
          EXPECT(lbm_adjoint_workspace_bytes(&c, 2000, 100) > 0);
          EXPECT(lbm_adjoint_workspace_bytes(&c, 0, 100) == 0);
        } else {
          EXPECT(lbm_adjoint_workspace_bytes(&c, 100, 10) == 0);
        }
        // lbm_create: no GPU behind the stubbed launchers or the runtime, or a null
        // workspace: never a handle
        lbm_handle* h = (lbm_handle*)0x1;
        const int rc = lbm_create(&c, nullptr, 0, nullptr, &h);
        EXPECT(rc == LBM_ENODEV || rc == LBM_EINVAL);
        EXPECT(h == nullptr);
      }
  // the parametrised rates
  {
    lbm_config c = base(64, 4, 8, 0, LBM_F32);
    c.cs_smag = 0.0;
    c.parametrized = 1;
    c.limiter = 1e-2;
    c.omega_bulk = 1.3;
    lbm_params p;
    EXPECT(lbm_derive_params(&c, &p) == LBM_OK);
    EXPECT(isfinite(p.w_plus) && isfinite(p.coef_a) && isfinite(p.coef_b));
  }
  // invalid configurations: every one rejected with a message
  {
    lbm_config bad[16];
    int n = 0;
    bad[n] = base(0, 1, 1, 0, 1); ++n;
    bad[n] = base(2048, 1024, 1024, 0, 1); ++n;
    bad[n] = base(8, 8, 8, 7, 1); ++n;
    bad[n] = base(8, 8, 8, 0, 9); ++n;
    bad[n] = base(8, 8, 8, 0, 1); bad[n].re_b = -1.0; ++n;
    bad[n] = base(8, 8, 8, 0, 1); bad[n].g_prime = 0.0; ++n;
    bad[n] = base(8, 8, 8, 0, 1); bad[n].omega4 = 2.0; ++n;
    bad[n] = base(8, 8, 8, 0, 1); bad[n].sc_t = NAN; ++n;
    bad[n] = base(8, 8, 8, 0, 1); bad[n].cs_smag = -0.1; ++n;
    bad[n] = base(8, 8, 8, 0, 1); bad[n].struct_size = 4; ++n;
    bad[n] = base(8, 8, 8, 1, 1); bad[n].parametrized = 1; ++n;
    bad[n] = base(8, 8, 8, 0, 1); bad[n].limiter = INFINITY; ++n;
    bad[n] = base(8, 8, 8, 0, 1); bad[n].smag_paper_form = 2; ++n;
    for (int i = 0; i < n; ++i) {
      lbm_params p;
      EXPECT(lbm_derive_params(&bad[i], &p) == LBM_EINVAL);
      EXPECT(strlen(lbm_last_error()) > 0);
      EXPECT(lbm_workspace_bytes(&bad[i]) == 0);
      lbm_handle* h = nullptr;
      EXPECT(lbm_create(&bad[i], (void*)256, 1 << 20, nullptr, &h) == LBM_EINVAL && h == nullptr);
    }
    EXPECT(lbm_derive_params(nullptr, nullptr) == LBM_EINVAL);
    EXPECT(lbm_workspace_bytes(nullptr) == 0);
  }
  // entry points on a null handle or null arguments
  lbm_diag d;
  int64_t s;
  EXPECT(lbm_step(nullptr, 1) == LBM_EINVAL);
  EXPECT(lbm_diagnostics(nullptr, &d) == LBM_EINVAL);
  EXPECT(lbm_moments(nullptr, LBM_OUT_F32, nullptr, nullptr, nullptr, nullptr, nullptr) == LBM_EINVAL);
  EXPECT(lbm_wall_shear(nullptr, LBM_OUT_F32, nullptr, nullptr) == LBM_EINVAL);
  EXPECT(lbm_get_step(nullptr, &s) == LBM_EINVAL);
  EXPECT(lbm_init_lock_exchange(nullptr, 0.125, 1e-3, 0) == LBM_EINVAL);
  EXPECT(lbm_init_from_field(nullptr, nullptr, 0.125) == LBM_EINVAL);
  EXPECT(lbm_checkpoint_save(nullptr, nullptr) == LBM_EINVAL);
  EXPECT(lbm_checkpoint_load(nullptr, nullptr) == LBM_EINVAL);
  EXPECT(lbm_get_populations(nullptr, nullptr, nullptr) == LBM_EINVAL);
  EXPECT(lbm_set_populations(nullptr, nullptr, nullptr) == LBM_EINVAL);
  EXPECT(lbm_stream_copy(nullptr, nullptr, 16, nullptr) == LBM_EINVAL);
  EXPECT(lbm_stream_copy((void*)256, (void*)512, 17, nullptr) == LBM_EINVAL);
  double J, a, b;
  EXPECT(lbm_adjoint_run(nullptr, 10, 5, 1.0, 1.0, nullptr, 0, &J, &a, &b, nullptr) == LBM_EINVAL);
  EXPECT(lbm_checkpoint_diagnostics(nullptr, nullptr, nullptr, &d) == LBM_EINVAL);
  {
    lbm_config c = base(64, 4, 8, 0, LBM_F32);
    const int rc = lbm_checkpoint_diagnostics(&c, (void*)256, nullptr, &d);
    EXPECT(rc == LBM_ENODEV || rc == LBM_EDEVICE);
  }
  EXPECT(lbm_destroy(nullptr) == LBM_OK);
  printf("fails %d\nsanitize ok\n", fails);
  return fails != 0;
}

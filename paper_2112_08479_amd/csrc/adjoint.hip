// Differentiation form: adjoint of an n-step run with checkpoint-recompute.
//
// Forward map per step: f(m+1) = G(C(f(m))), G the gather with half-way
// bounce-back (a permutation of the population slots), C the local collision.
// With lambda(m) = dJ/df(m):
//   lambda(m) = C'(f(m))^T G^T lambda(m+1) + dJ_m/df(m),
// where G^T lambda is again a gather with the velocities reversed:
//   (G^T lambda)_q(x) = lambda_q(x + c_q) if x + c_q is a fluid node, else
//   lambda_opp(q)(x). Parameter gradients sum the parameter part of each
// collision's adjoint; dJ/dchi0 = sum_p w_p lambda_phi,p(0) (phi(0) = w chi0).
//
// Objective J = w_front x_f(n) + w_fw (1/n) sum_{m=1..n} F_w(m); F_w depends
// on u_x = j_x / rho at z = 0, 1; x_f on the span-averaged concentration at
// the front's two columns (see the diagnostics).
#include <math.h>
#include <string.h>

#include <algorithm>

#include "adjoint.h"
#include "collide.h"
#include "lattice.h"
#include "runtime.h"

namespace lbm {

template <int MODEL>
struct AModel;
template <>
struct AModel<0> {
  using LF = Q27;
  using LS = Q7;
};
template <>
struct AModel<1> {
  using LF = Q19;
  using LS = Q6;
};
template <>
struct AModel<2> {
  using LF = Q27;
  using LS = Q27;
};

struct AdjStep {
  double a0, a1;        // F_w seed coefficients at z = 0 and z = 1 (0 when not seeded)
  double dcs_dc;        // d c_les / d C_s: 36 sqrt(2) C_s, or 18 sqrt(2) in the printed form
  double disct_dsct;    // d (1/Sc_T) / d Sc_T = -1 / Sc_T^2
  double* gpart;        // per-block accumulators (2 doubles per block)
  double* dchi0;        // non-null: write dJ/dchi0 (the step m = 0)
};

template <int MODEL, typename ST, typename CT, bool LES, bool PARAM = false>
__global__ __launch_bounds__(kBlock) void k_adjoint_step(const ST* __restrict__ state,
                                                         const CT* __restrict__ lam_next,
                                                         CT* __restrict__ lam_out, Grid g,
                                                         Phys<CT> p, AdjStep a, int nbx) {
  using LF = typename AModel<MODEL>::LF;
  using LS = typename AModel<MODEL>::LS;
  constexpr int QT = LF::Q + LS::Q;
  // a row's tiles on one XCD, as in the step kernel: the pulls across tile
  // edges then find the neighbouring tile's lines in the same L2
  const int b = xcd_row_order(blockIdx.x, gridDim.x, nbx);
  const int row = b / nbx;
  const int x0 = (b - row * nbx) * (int)blockDim.x;
  const int y = row % g.ny, z = row / g.ny;
  // The step kernel's addressing: block-uniform row segments (scalar
  // registers) plus the lane's own, x - 1 and x + 1 offsets. Lanes past the
  // row's end read its last node (their results are dropped), so that every
  // lane takes part in the loads and in the x-wall fix-up's wave ballot.
  const TileLanes<QT, 1> t = tile_lanes<QT, 1>(g, x0, (int)threadIdx.x, (int)blockDim.x);
  const int x = t.x[0];
  const bool active = x < g.nx;
  CT fg1[1][LF::Q], ph1[1][LS::Q], gb[LF::Q], pb[LS::Q];
  gather_rows<LF, LS, 1, ST, CT>(state, g, t, y, z, fg1, ph1);
  const CT* fg = fg1[0];
  const CT* ph = ph1[0];
  const bool wave_at_wall = __builtin_amdgcn_ballot_w64(x == 0 || x == g.nx - 1) != 0;
  // reverse pulls of lambda(m + 1) (the pull on the reversed velocities),
  // issued with the state's loads so that their latencies overlap (the
  // register allocation is the same either way)
  CT lg[1][LF::Q], lp[1][LS::Q];
  pull_lattice<Rev<LF>, 0, QT, 1, CT, CT>(lam_next, g, y, z, t, wave_at_wall, lg);
  pull_lattice<Rev<LS>, LF::Q, QT, 1, CT, CT>(lam_next, g, y, z, t, wave_at_wall, lp);
  // the F_w seed at this step needs rho and u_x of the gathered state: taken
  // before the collision's adjoint so that the gathered values need not
  // stay live through it (block-uniform branch: the block's row has one z)
  const double az = (z == 0) ? a.a0 : ((z == 1) ? a.a1 : 0.0);
  CT sd_ir = CT(0), sd_ux = CT(0);
  if (az != 0.0) {
    CT drho = CT(0), jx = CT(0);
    static_for<0, LF::Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      drho += fg[q];
      if (LF::cx[q]) jx += CT(LF::cx[q]) * fg[q];
    });
    sd_ir = CT(1) / (CT(1) + drho);
    sd_ux = jx * sd_ir;
  }
  CT bc = CT(0), bi = CT(0);
  if constexpr ((MODEL == 0 || MODEL == 2) && PARAM) {
    // the scalar populations and their adjoints wait in LDS, each thread in
    // its own column, while the flow's reverse sweep runs
    // (vjp_cumulant27_param takes the scalar part last): that keeps the FP32
    // model-3 kernel at two waves per SIMD
    __shared__ CT stash[2 * LS::Q][kBlock];
    const int tid = (int)threadIdx.x;
    const CT chi = scalar_sum<LS>(ph);
    static_for<0, LS::Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      stash[q][tid] = ph[q];
      stash[LS::Q + q][tid] = lp[0][q];
    });
    vjp_cumulant27_param<LS, CT>(
        fg, chi, lg[0],
        [&](CT* phr, CT* mpr) {
          // a compiler barrier: the values are read back from LDS here, not
          // forwarded from the registers that wrote them
          asm volatile("" ::: "memory");
          static_for<0, LS::Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            phr[q] = stash[q][tid];
            mpr[q] = stash[LS::Q + q][tid];
          });
        },
        p, gb, pb, bi);
  } else if constexpr (MODEL == 0 || MODEL == 2)
    vjp_cumulant27<LS, LES, CT>(fg, ph, lg[0], lp[0], p, gb, pb, bc, bi);
  else
    vjp_bgk_q19_q6<LES, CT>(fg, ph, lg[0], lp[0], p, gb, pb, bc, bi);
  // seed of the wall friction term at this step: d u_x / d g_q = (c_qx - u_x) / rho
  if (az != 0.0) {
    static_for<0, LF::Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      gb[q] += CT(az) * (CT(LF::cx[q]) - sd_ux) * sd_ir;
    });
  }
  double v[2] = {0.0, 0.0};
  if (active) {
    CT* orow = lam_out + (int64_t)row * g.nxb * (QT * kXB);
    static_for<0, LF::Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      orow[q * kXB + t.own[0]] = gb[q];
    });
    static_for<0, LS::Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      orow[(LF::Q + q) * kXB + t.own[0]] = pb[q];
    });
    if (a.dchi0) {
      double s = 0.0;
      static_for<0, LS::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        s += weight<LS>(q) * (double)pb[q];
      });
      a.dchi0[(int64_t)row * g.nx + x] = s;
    }
    v[0] = (double)bc * a.dcs_dc;
    v[1] = (double)bi * a.disct_dsct;
  }
  // block sums of the parameter gradients, added to this block's accumulator
  for (int o = 32; o > 0; o >>= 1) {
    v[0] += __shfl_xor(v[0], o, 64);
    v[1] += __shfl_xor(v[1], o, 64);
  }
  __shared__ double red[kBlock / 64][2];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    red[wid][0] = v[0];
    red[wid][1] = v[1];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w) {
      s0 += red[w][0];
      s1 += red[w][1];
    }
    a.gpart[2 * blockIdx.x] += s0;
    a.gpart[2 * blockIdx.x + 1] += s1;
  }
}

// Final-step adjoint lambda(n): wall-friction seed (z = 0, 1) and front seed
// at (i*, j, k0) and (i* + 1, j, k1) for every span position j.
template <int MODEL, typename ST, typename CT>
__global__ __launch_bounds__(kBlock) void k_adjoint_seed(const ST* __restrict__ state,
                                                         CT* __restrict__ lam, Grid g, double a0,
                                                         double a1, const double* __restrict__ fs,
                                                         int nbx) {
  using LF = typename AModel<MODEL>::LF;
  using LS = typename AModel<MODEL>::LS;
  const int b = blockIdx.x;
  const int row = b / nbx;
  const int x = (b - row * nbx) * blockDim.x + threadIdx.x;
  if (x >= g.nx) return;
  const int y = row % g.ny, z = row / g.ny;
  CT gb[LF::Q];
  static_for<0, LF::Q>([&](auto qc) { gb[decltype(qc)::value] = CT(0); });
  const double az = (z == 0) ? a0 : ((z == 1) ? a1 : 0.0);
  if (az != 0.0) {
    CT fg[LF::Q], ph[LS::Q];
    gather<LF, LS, ST, CT>(state, g, x, y, z, fg, ph);
    CT drho = CT(0), jx = CT(0);
    static_for<0, LF::Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      drho += fg[q];
      if (LF::cx[q]) jx += CT(LF::cx[q]) * fg[q];
    });
    const CT ir = CT(1) / (CT(1) + drho);
    const CT ux = jx * ir;
    static_for<0, LF::Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      gb[q] = CT(az) * (CT(LF::cx[q]) - ux) * ir;
    });
  }
  // fs = {i*, k0, k1, cA / ny, cB / ny}
  CT pb = CT(0);
  const int istar = (int)fs[0];
  if (istar >= 0) {
    if (x == istar && z == (int)fs[1]) pb += CT(fs[3]);
    if (x == istar + 1 && z == (int)fs[2]) pb += CT(fs[4]);
  }
  static_for<0, LF::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    lam[elem_index<LF::Q + LS::Q>(g, q, row, x)] = gb[q];
  });
  static_for<0, LS::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    lam[elem_index<LF::Q + LS::Q>(g, LF::Q + q, row, x)] = pb;
  });
}

// Front seed coefficients from the span-averaged concentration chibar
// (nz x nx): i* = last column whose depth maximum reaches 0.02; A = m(i*),
// B = m(i*+1); x_front = i* + 1/2 + (A - theta)/(A - B) has
// d/dA = (theta - B)/(A - B)^2 and d/dB = (A - theta)/(A - B)^2, passed to
// the first depth maximum of each column, divided by ny for the span mean.
// One block of 1024 threads: the columns are scanned in parallel, i* is a
// max-reduction (wave shuffles, then LDS), the rest is one thread's work.
__global__ __launch_bounds__(1024) void k_front_seed(const double* __restrict__ chibar, Grid g,
                                                     double w_front, double* __restrict__ out) {
  __shared__ int wbest[16];
  const double theta = 0.02;
  int best = -1;
  for (int i = threadIdx.x; i < g.nx; i += blockDim.x) {
    double m = -INFINITY;
    for (int k = 0; k < g.nz; ++k) m = fmax(m, chibar[(int64_t)k * g.nx + i]);
    if (m >= theta) best = i;
  }
  for (int o = 32; o > 0; o >>= 1) best = max(best, __shfl_xor(best, o, 64));
  if ((threadIdx.x & 63) == 0) wbest[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) best = max(best, wbest[w]);
  out[0] = -1.0;
  out[1] = out[2] = out[3] = out[4] = 0.0;
  if (best < 0 || best == g.nx - 1) return;
  int k0 = 0, k1 = 0;
  double A = -INFINITY, B = -INFINITY;
  for (int k = 0; k < g.nz; ++k) {
    const double a = chibar[(int64_t)k * g.nx + best], c = chibar[(int64_t)k * g.nx + best + 1];
    if (a > A) { A = a; k0 = k; }
    if (c > B) { B = c; k1 = k; }
  }
  const double d = A - B;
  out[0] = (double)best;
  out[1] = (double)k0;
  out[2] = (double)k1;
  out[3] = w_front * (theta - B) / (d * d) / g.ny;
  out[4] = w_front * (A - theta) / (d * d) / g.ny;
}

// sum over the bottom two layers of u_x: fw_partial[block] = {sum u_x(z=0), sum u_x(z=1)}
template <int MODEL, typename ST, typename CT>
__global__ __launch_bounds__(64) void k_fw_layers(const ST* __restrict__ state, Grid g,
                                                  double* __restrict__ part) {
  // one wavefront per (x-block, y, z) of the two wall layers z = 0, 1: the
  // block's z is uniform, its sum goes to slot z of the block's pair
  using LF = typename AModel<MODEL>::LF;
  constexpr int QT = LF::Q + AModel<MODEL>::LS::Q;
  const int b = blockIdx.x;
  const int xb = b % g.nxb, y = (b / g.nxb) % g.ny, z = b / (g.nxb * g.ny);
  const int x = xb * kXB + (int)threadIdx.x;
  double v = 0.0;
  if (x < g.nx) {
    CT fg[LF::Q];
    static_for<0, LF::Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      fg[q] = Conv<ST, CT>::load(*pull_ptr<LF, q, QT>(state, g, 0, x, y, z));
    });
    double drho = 0.0, jx = 0.0;
    static_for<0, LF::Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      drho += (double)fg[q];
      if (LF::cx[q]) jx += LF::cx[q] * (double)fg[q];
    });
    v = jx / (1.0 + drho);
  }
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (threadIdx.x == 0) {
    part[2 * b] = z == 0 ? v : 0.0;
    part[2 * b + 1] = z == 0 ? 0.0 : v;
  }
}

// single block: out[0] += nu0 (9 sum0 - sum1) / 3 (fixed order)
__global__ __launch_bounds__(1024) void k_fw_accumulate(const double* __restrict__ part,
                                                        int64_t nparts, double nu0,
                                                        double* __restrict__ out) {
  __shared__ double red[16][2];
  double v0 = 0.0, v1 = 0.0;
  for (int64_t b = threadIdx.x; b < nparts; b += blockDim.x) {
    v0 += part[2 * b];
    v1 += part[2 * b + 1];
  }
  for (int o = 32; o > 0; o >>= 1) {
    v0 += __shfl_xor(v0, o, 64);
    v1 += __shfl_xor(v1, o, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    red[wid][0] = v0;
    red[wid][1] = v1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      s0 += red[w][0];
      s1 += red[w][1];
    }
    out[0] += nu0 * (9.0 * s0 - s1) / 3.0;
  }
}

// single block: sum the per-block parameter accumulators
__global__ __launch_bounds__(1024) void k_sum_pairs(const double* __restrict__ part, int nparts,
                                                    double* __restrict__ out) {
  __shared__ double red[16][2];
  double v0 = 0.0, v1 = 0.0;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
    v0 += part[2 * b];
    v1 += part[2 * b + 1];
  }
  for (int o = 32; o > 0; o >>= 1) {
    v0 += __shfl_xor(v0, o, 64);
    v1 += __shfl_xor(v1, o, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    red[wid][0] = v0;
    red[wid][1] = v1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      s0 += red[w][0];
      s1 += red[w][1];
    }
    out[0] = s0;
    out[1] = s1;
  }
}

__global__ void k_zero(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// ---------------------------------------------------------------- launchers
static Grid agrid(const lbm_handle* h) {
  return Grid{h->cfg.nx, h->cfg.ny, h->cfg.nz, h->n, xblocks(h->cfg.nx)};
}
static int ablock(const lbm_handle* h) {
  const int nx = h->cfg.nx;
  return nx >= kBlock ? kBlock : ((nx + 63) / 64) * 64;
}

int adjoint_blocks(const lbm_handle* h) {
  const int bx = ablock(h);
  const int nbx = (h->cfg.nx + bx - 1) / bx;
  return nbx * h->cfg.ny * h->cfg.nz;
}
int fw_blocks(const lbm_handle* h) {
  return xblocks(h->cfg.nx) * h->cfg.ny * std::min(h->cfg.nz, 2);
}

template <typename CT>
static Phys<CT> aphys(const lbm_handle* h) {
  const lbm_params& q = h->prm;
  const lbm_config& c = h->cfg;
  Phys<CT> r;
  r.g = (CT)q.g_prime;
  r.tau0 = (CT)q.tau0;
  r.tau_phi0 = (CT)q.tau_phi0;
  r.c_les = (CT)(18.0 * sqrt(2.0) * (c.smag_paper_form ? c.cs_smag : c.cs_smag * c.cs_smag));
  r.d0 = (CT)q.d0;
  r.inv_sct = (CT)(1.0 / c.sc_t);
  r.inv_cs2phi = (CT)(1.0 / q.cs2_phi);
  r.omega2 = (CT)c.omega_bulk;
  r.omega3 = (CT)c.omega3;
  r.omega4 = (CT)c.omega4;
  r.omega5 = (CT)c.omega5;
  r.omega6 = (CT)c.omega6;
  // parametrised cumulant (as for the forward step)
  const double h4 = q.tau0 - 0.5;  // 1/omega1 - 1/2
  r.w_plus = (CT)q.w_plus;
  r.w_minus = (CT)q.w_minus;
  r.w_111 = (CT)q.w_111;
  r.a4 = (CT)(-2.0 / 3.0 * h4 * q.coef_a);
  r.b4 = (CT)(-1.0 / 3.0 * h4 * q.coef_b);
  r.lam = c.limiter > 0.0 ? (CT)c.limiter : (CT)INFINITY;
  return r;
}

template <class F>
static hipError_t adj_dispatch(const lbm_handle* h, F&& f) {
  const bool f64 = h->cfg.storage == LBM_F64;
  auto by_type = [&](auto mc) {
    return f64 ? f(mc, double{}) : f(mc, float{});
  };
  switch (h->cfg.model) {
    case LBM_CUMULANT27_Q7: return by_type(std::integral_constant<int, 0>{});
    case LBM_BGK19_SMAG_Q6: return by_type(std::integral_constant<int, 1>{});
    case LBM_CUMULANT27_FCM27: return by_type(std::integral_constant<int, 2>{});
  }
  return hipErrorInvalidValue;
}

hipError_t launch_adjoint_step(lbm_handle* h, const void* state, const void* lam_next,
                               void* lam_out, double a0, double a1, double* gpart, double* dchi0) {
  const Grid g = agrid(h);
  const int bx = ablock(h);
  const int nbx = (g.nx + bx - 1) / bx;
  const unsigned blocks = (unsigned)((int64_t)nbx * g.ny * g.nz);
  AdjStep a;
  a.a0 = a0;
  a.a1 = a1;
  a.dcs_dc = h->cfg.smag_paper_form ? 18.0 * sqrt(2.0) : 36.0 * sqrt(2.0) * h->cfg.cs_smag;
  a.disct_dsct = -1.0 / (h->cfg.sc_t * h->cfg.sc_t);
  a.gpart = gpart;
  a.dchi0 = dchi0;
  const bool les = h->cfg.cs_smag > 0.0;
  return adj_dispatch(h, [&](auto mc, auto ct) {
    constexpr int M = decltype(mc)::value;
    using CT = decltype(ct);
    using ST = CT;
    const Phys<CT> p = aphys<CT>(h);
    if (M != 1 && h->cfg.parametrized)  // never with the LES
      hipLaunchKernelGGL((k_adjoint_step<M, ST, CT, false, true>), dim3(blocks), dim3(bx), 0, h->stream,
                         static_cast<const ST*>(state), static_cast<const CT*>(lam_next),
                         static_cast<CT*>(lam_out), g, p, a, nbx);
    else if (les)
      hipLaunchKernelGGL((k_adjoint_step<M, ST, CT, true>), dim3(blocks), dim3(bx), 0, h->stream,
                         static_cast<const ST*>(state), static_cast<const CT*>(lam_next),
                         static_cast<CT*>(lam_out), g, p, a, nbx);
    else
      hipLaunchKernelGGL((k_adjoint_step<M, ST, CT, false>), dim3(blocks), dim3(bx), 0, h->stream,
                         static_cast<const ST*>(state), static_cast<const CT*>(lam_next),
                         static_cast<CT*>(lam_out), g, p, a, nbx);
    return hipGetLastError();
  });
}

hipError_t launch_adjoint_seed(lbm_handle* h, const void* state, void* lam, double a0, double a1,
                               const double* fs) {
  const Grid g = agrid(h);
  const int bx = ablock(h);
  const int nbx = (g.nx + bx - 1) / bx;
  const unsigned blocks = (unsigned)((int64_t)nbx * g.ny * g.nz);
  return adj_dispatch(h, [&](auto mc, auto ct) {
    constexpr int M = decltype(mc)::value;
    using CT = decltype(ct);
    hipLaunchKernelGGL((k_adjoint_seed<M, CT, CT>), dim3(blocks), dim3(bx), 0, h->stream,
                       static_cast<const CT*>(state), static_cast<CT*>(lam), g, a0, a1, fs, nbx);
    return hipGetLastError();
  });
}

hipError_t launch_front_seed(lbm_handle* h, double w_front, double* out) {
  hipLaunchKernelGGL(k_front_seed, dim3(1), dim3(1024), 0, h->stream, h->chibar, agrid(h), w_front,
                     out);
  return hipGetLastError();
}

hipError_t launch_fw_layers(lbm_handle* h, const void* state, double* part) {
  const Grid g = agrid(h);
  const int nb = fw_blocks(h);
  return adj_dispatch(h, [&](auto mc, auto ct) {
    constexpr int M = decltype(mc)::value;
    using CT = decltype(ct);
    hipLaunchKernelGGL((k_fw_layers<M, CT, CT>), dim3(nb), dim3(64), 0, h->stream,
                       static_cast<const CT*>(state), g, part);
    return hipGetLastError();
  });
}

hipError_t launch_fw_reduce(lbm_handle* h, const double* part, int64_t nparts, double* out) {
  hipLaunchKernelGGL(k_fw_accumulate, dim3(1), dim3(1024), 0, h->stream, part, nparts,
                     h->prm.nu0, out);
  return hipGetLastError();
}

hipError_t launch_sum_pairs(lbm_handle* h, const double* part, int nparts, double* out) {
  hipLaunchKernelGGL(k_sum_pairs, dim3(1), dim3(1024), 0, h->stream, part, nparts, out);
  return hipGetLastError();
}

hipError_t launch_zero(lbm_handle* h, double* p, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->stream, p, n);
  return hipGetLastError();
}

}  // namespace lbm

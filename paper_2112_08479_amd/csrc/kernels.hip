// Forward kernels: fused gather + collide + store step, initial states,
// moment export, FP64 diagnostics, test hooks.
//
// State convention. A population buffer holds post-collision values at the
// node where they were produced. One step pulls them (the gather with
// half-way bounce-back and periodic span, i.e. streaming of Eq. 17), collides
// at the node and writes the result to the other buffer. The pre-collision
// populations at step n are therefore gather(buffer). The gather is a
// permutation of the (population, node) slots, so every state has exactly one
// buffer representation; the init kernels and the set hook write the inverse
// permutation.
#include <math.h>

#include <algorithm>
#include <mutex>

#include "collide.h"
#include "lattice.h"
#include "runtime.h"

namespace lbm {

template <int MODEL>
struct ModelT;
template <>
struct ModelT<0> {
  using LF = Q27;
  using LS = Q7;
};
template <>
struct ModelT<1> {
  using LF = Q19;
  using LS = Q6;
};
template <>
struct ModelT<2> {
  using LF = Q27;
  using LS = Q27;
};

template <typename T>
LBM_HD double to_d(T v);
template <>
LBM_HD double to_d<double>(double v) { return v; }
template <>
LBM_HD double to_d<float>(float v) { return (double)v; }

// Post-collision values are not read again before the next launch, so they
// may bypass the caches on the way to HBM (plain stores measured 5 % slower).
template <typename ST>
__device__ __forceinline__ void store_val(ST* p, ST v) {
  if constexpr (std::is_same<ST, double>::value || std::is_same<ST, float>::value) {
    __builtin_nontemporal_store(v, p);
  } else {
    uint16_t bits;
    __builtin_memcpy(&bits, &v, 2);
    __builtin_nontemporal_store(bits, reinterpret_cast<uint16_t*>(p));
  }
}

// ------------------------------------------------------------------- step
// collision kinds of the cumulant models
enum { kCumFast = 0, kCumGeneral = 1, kCumParam = 2 };

// one tile: NPT * blockDim.x consecutive nodes of one row; KIND: kCumFast
// (omega3..omega6 = 1), kCumGeneral (given rates), kCumParam (parametrised).
// FW (the adjoint's forward pass): the tiles of the wall layers z = 0, 1 also
// write the x-velocity sums of their x-blocks that F_w (Eq. 62, 64) needs for
// the state they gather, as the separate wall-layer kernel does: per x-block
// the wave sum of u_x = j_x / rho (FP64, populations in order) into
// fwp[2 b + z], with b = xb + nxb (y + ny z), and 0 into the other slot.
template <int MODEL, typename ST, typename SS, typename CT, bool LES, int KIND, int NPT,
          bool FW = false>
__device__ __forceinline__ void step_tile(const ST* __restrict__ src, ST* __restrict__ dst,
                                          const Grid& g, const Phys<CT>& p, int nbx, int b,
                                          double* __restrict__ fwp) {
  using LF = typename ModelT<MODEL>::LF;
  using LS = typename ModelT<MODEL>::LS;
  const int row = b / nbx;
  const int x0 = (b - row * nbx) * (int)blockDim.x * NPT;
  // lanes with no node at all; the wave sums of FW need every lane of a wave
  if (!FW && x0 + (int)threadIdx.x >= g.nx) return;
  const int y = row % g.ny, z = row / g.ny;
  constexpr int QT = LF::Q + LS::Q;
  const TileLanes<QT, NPT> t = tile_lanes<QT, NPT>(g, x0, (int)threadIdx.x, (int)blockDim.x);
  CT fg[NPT][LF::Q], ph[NPT][LS::Q];
  gather_rows<LF, LS, NPT, ST, CT, SS>(src, g, t, y, z, fg, ph);
  if constexpr (FW) {
    if (z < 2) {  // uniform per block
      const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
#pragma unroll
      for (int k = 0; k < NPT; ++k) {
        double v = 0.0;
        if (t.x[k] < g.nx) {
          double drho = 0.0, jx = 0.0;
          static_for<0, LF::Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            drho += (double)fg[k][q];
            if (LF::cx[q]) jx += LF::cx[q] * (double)fg[k][q];
          });
          v = jx / (1.0 + drho);
        }
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        const int xb = ((x0 + k * (int)blockDim.x) >> kXBShift) + wave;
        if (lane == 0 && xb < g.nxb) {
          const int64_t fb = xb + (int64_t)g.nxb * (y + (int64_t)g.ny * z);
          fwp[2 * fb] = z == 0 ? v : 0.0;
          fwp[2 * fb + 1] = z == 0 ? 0.0 : v;
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    if constexpr (MODEL == 0 || MODEL == 2) {
      if constexpr (KIND == kCumParam)
        collide_cumulant27_param<LS, CT>(fg[k], ph[k], p);
      else if constexpr (KIND == kCumGeneral)
        collide_cumulant27_general<LS, LES, CT>(fg[k], ph[k], p);
      else
        collide_cumulant27<LS, LES, CT>(fg[k], ph[k], p);
    } else {
      collide_bgk_q19_q6<LES, CT>(fg[k], ph[k], p);
    }
  }
  // block-uniform segment pointers + the lane's own offset, as for the loads
  ST* drow = dst + (int64_t)row * g.nxb * (QT * kXB);
  static_for<0, QT>([&](auto qc) {
    constexpr int a = decltype(qc)::value;
    ST* pa = drow + a * kXB;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      if ((k == 0 && !FW) || t.x[k] < g.nx) {
        if constexpr (a < LF::Q)
          store_val(&pa[t.own[k]], Conv<ST, CT>::store(fg[k][a]));
        else
          store_val(&reinterpret_cast<SS*>(pa)[t.own[k]], Conv<SS, CT>::store(ph[k][a - LF::Q]));
      }
    }
  });
}

template <int MODEL, typename ST, typename SS, typename CT, bool LES, int KIND, int NPT,
          bool FW = false>
__global__ __launch_bounds__(kBlock) void k_step(const ST* __restrict__ src, ST* __restrict__ dst,
                                                 Grid g, Phys<CT> p, int nbx,
                                                 double* __restrict__ fwp) {
  step_tile<MODEL, ST, SS, CT, LES, KIND, NPT, FW>(src, dst, g, p, nbx,
                                                   xcd_row_order(blockIdx.x, gridDim.x, nbx), fwp);
}

// ------------------------------------------------------------ init states
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct LockInit {
  int gate;
  double amp;
  uint64_t seed;
  __device__ double chi0(const Grid& g, int i, int j, int k) const {
    double c = (i < gate) ? 1.0 : 0.0;
    if (amp != 0.0 && (i == gate - 1 || i == gate)) {
      const uint64_t lin = (uint64_t)i + (uint64_t)g.nx * ((uint64_t)j + (uint64_t)g.ny * (uint64_t)k);
      const uint64_t r = splitmix64(seed ^ (lin * 0x9E3779B97F4A7C15ull));
      const double U = (double)(r >> 11) * 0x1.0p-53;
      c += amp * (2.0 * U - 1.0);
    }
    return c;
  }
};
struct FieldInit {
  const double* chi;
  __device__ double chi0(const Grid& g, int i, int j, int k) const {
    return chi[((int64_t)k * g.ny + j) * g.nx + i];
  }
};

// Buffer slot (q, node) is read by node + c_q when that node is fluid, else by
// the node itself for population opp(q) (bounce-back). Initial populations:
// flow f = w (stored deviation 0), scalar phi_p = w_p chi0.
template <int MODEL, typename ST, typename SS, class Init>
__global__ __launch_bounds__(kBlock) void k_init(ST* __restrict__ dst, Grid g, Init init, int nbx) {
  using LF = typename ModelT<MODEL>::LF;
  using LS = typename ModelT<MODEL>::LS;
  using CT = typename std::conditional<std::is_same<ST, double>::value, double, float>::type;
  const int b = blockIdx.x;
  const int row = b / nbx;
  const int x = (b - row * nbx) * blockDim.x + threadIdx.x;
  if (x >= g.nx) return;
  const int y = row % g.ny, z = row / g.ny;
  constexpr int QT = LF::Q + LS::Q;
  static_for<0, LF::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    dst[elem_index<QT>(g, q, row, x)] = Conv<ST, CT>::store(CT(0));
  });
  static_for<0, LS::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    const int xn = x + LS::cx[q], zn = z + LS::cz[q];
    int yn = y + LS::cy[q];
    yn = yn < 0 ? g.ny - 1 : (yn >= g.ny ? 0 : yn);
    const bool fluid = (unsigned)xn < (unsigned)g.nx && (unsigned)zn < (unsigned)g.nz;
    const double c = fluid ? init.chi0(g, xn, yn, zn) : init.chi0(g, x, y, z);
    reinterpret_cast<SS*>(dst)[elem_index<QT>(g, LF::Q + q, row, x)] =
        Conv<SS, CT>::store(CT(weight<LS>(q) * c));
  });
}

// ----------------------------------------------------------------- moments
template <typename OT>
__device__ __forceinline__ void put_out(void* p, int64_t i, double v) {
  if (p) static_cast<OT*>(p)[i] = (OT)v;
}

template <int MODEL, typename ST, typename SS, typename CT, typename OT>
__global__ __launch_bounds__(kBlock) void k_moments(const ST* __restrict__ src, Grid g, double gp,
                                                    int nbx, void* rho, void* ux, void* uy,
                                                    void* uz, void* chi) {
  using LF = typename ModelT<MODEL>::LF;
  using LS = typename ModelT<MODEL>::LS;
  const int b = blockIdx.x;
  const int row = b / nbx;
  const int x = (b - row * nbx) * blockDim.x + threadIdx.x;
  if (x >= g.nx) return;
  const int y = row % g.ny, z = row / g.ny;
  const int64_t node = (int64_t)row * g.nx + x;
  CT fg[LF::Q], ph[LS::Q];
  gather<LF, LS, ST, CT, SS>(src, g, x, y, z, fg, ph);
  double drho = 0, jx = 0, jy = 0, jz = 0, c = 0;
  static_for<0, LF::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    const double v = to_d(fg[q]);
    drho += v;
    if (LF::cx[q]) jx += LF::cx[q] * v;
    if (LF::cy[q]) jy += LF::cy[q] * v;
    if (LF::cz[q]) jz += LF::cz[q] * v;
  });
  static_for<0, LS::Q>([&](auto qc) { c += to_d(ph[decltype(qc)::value]); });
  const double r = 1.0 + drho;
  put_out<OT>(rho, node, r);
  put_out<OT>(ux, node, jx / r);
  put_out<OT>(uy, node, jy / r);
  put_out<OT>(uz, node, (jz - 0.5 * gp * c) / r);
  put_out<OT>(chi, node, c);
}

// streamwise velocity u_x = j_x / rho of the pre-collision state at a node
template <class LF, class LS, typename ST, typename SS, typename CT>
__device__ __forceinline__ double ux_at(const ST* __restrict__ src, const Grid& g, int x, int y,
                                        int z) {
  CT fg[LF::Q], ph[LS::Q];
  gather<LF, LS, ST, CT, SS>(src, g, x, y, z, fg, ph);
  double drho = 0, jx = 0;
  static_for<0, LF::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    const double v = to_d(fg[q]);
    drho += v;
    if (LF::cx[q]) jx += LF::cx[q] * v;
  });
  return jx / (1.0 + drho);
}

// Bottom-wall shear stress (Eq. 62, lattice units, rho_bar = 1): the slope at
// the half-way wall of the quadratic through u = 0 at the wall and the nodes at
// distances 1/2 and 3/2, tau_w = nu0 (9 u_x(z=0) - u_x(z=1)) / 3. One thread
// per x loops over the span: tau (ny x nx, row y) and its span mean tau_bar
// (nx, the integrand of Eq. 66); NULL skips either.
template <int MODEL, typename ST, typename SS, typename CT, typename OT>
__global__ __launch_bounds__(kBlock) void k_wall_shear(const ST* __restrict__ src, Grid g,
                                                       double nu0, void* tau, void* tau_bar) {
  using LF = typename ModelT<MODEL>::LF;
  using LS = typename ModelT<MODEL>::LS;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= g.nx) return;
  double s = 0;
  for (int y = 0; y < g.ny; ++y) {
    const double u0 = ux_at<LF, LS, ST, SS, CT>(src, g, x, y, 0);
    const double u1 = ux_at<LF, LS, ST, SS, CT>(src, g, x, y, 1);
    const double t = nu0 * (9.0 * u0 - u1) / 3.0;
    put_out<OT>(tau, (int64_t)y * g.nx + x, t);
    s += t;
  }
  put_out<OT>(tau_bar, x, s / g.ny);
}

// ------------------------------------------------------------- diagnostics
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// block-wide reduction of NV values (sum, except index imax: max); result in
// thread 0. Fixed order, so the result is reproducible.
template <int NV>
__device__ void block_reduce(double (&v)[NV], int imax) {
  __shared__ double red[kBlock / 64 * NV];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = (k == imax) ? wave_max(v[k]) : wave_sum(v[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) red[wid * NV + k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < nw; ++w)
#pragma unroll
      for (int k = 0; k < NV; ++k)
        v[k] = (k == imax) ? fmax(v[k], red[w * NV + k]) : v[k] + red[w * NV + k];
  }
  __syncthreads();
}

// one thread per (x, z) column, looping over the span
template <int MODEL, typename ST, typename SS, typename CT>
__global__ __launch_bounds__(kBlock) void k_diag_columns(const ST* __restrict__ src, Grid g,
                                                         double gp, double* __restrict__ chibar,
                                                         double* __restrict__ partials, int nbx) {
  using LF = typename ModelT<MODEL>::LF;
  using LS = typename ModelT<MODEL>::LS;
  const int z = blockIdx.x / nbx;
  const int x = (blockIdx.x - z * nbx) * blockDim.x + threadIdx.x;
  double v[6] = {0, 0, 0, 0, 0, 0};  // drho, chi, u_x(z=0), u_x(z=1), umax, nonfinite
  if (x < g.nx) {
    double col = 0;
    for (int y = 0; y < g.ny; ++y) {
      CT fg[LF::Q], ph[LS::Q];
      gather<LF, LS, ST, CT, SS>(src, g, x, y, z, fg, ph);
      double drho = 0, jx = 0, jy = 0, jz = 0, c = 0;
      static_for<0, LF::Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const double t = to_d(fg[q]);
        drho += t;
        if (LF::cx[q]) jx += LF::cx[q] * t;
        if (LF::cy[q]) jy += LF::cy[q] * t;
        if (LF::cz[q]) jz += LF::cz[q] * t;
      });
      static_for<0, LS::Q>([&](auto qc) { c += to_d(ph[decltype(qc)::value]); });
      const double r = 1.0 + drho;
      const double ux = jx / r, uy = jy / r, uz = (jz - 0.5 * gp * c) / r;
      const bool fin = isfinite(r) && isfinite(c) && isfinite(ux) && isfinite(uy) && isfinite(uz);
      v[0] += drho;
      col += c;
      if (z == 0) v[2] += ux;
      if (z == 1) v[3] += ux;
      if (fin)
        v[4] = fmax(v[4], sqrt(ux * ux + uy * uy + uz * uz));
      else
        v[5] += 1.0;
    }
    v[1] = col;
    chibar[(int64_t)z * g.nx + x] = col / g.ny;
  }
  block_reduce<6>(v, 4);
  if (threadIdx.x == 0) {
    double* o = partials + (int64_t)blockIdx.x * kDiagSlots;
    for (int k = 0; k < 6; ++k) o[k] = v[k];
  }
}

// single block: reduce the partials, locate the front, write out[8] =
// {mass, chi_mass, fw, x_front, umax, nonfinite, i_star, 0}
__global__ __launch_bounds__(1024) void k_diag_final(const double* __restrict__ partials, int nparts,
                                                     const double* __restrict__ chibar, Grid g,
                                                     double nu0, double* __restrict__ out) {
  __shared__ double red[16 * 6];
  __shared__ int ired[16];
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int b = t; b < nparts; b += blockDim.x) {
    const double* p = partials + (int64_t)b * kDiagSlots;
    for (int k = 0; k < 6; ++k) v[k] = (k == 4) ? fmax(v[k], p[k]) : v[k] + p[k];
  }
  const double theta = 0.02;
  int best = -1;
  for (int i = t; i < g.nx; i += blockDim.x) {
    // the depth maximum of column i, in four independent chains so that
    // the loads overlap (max is exact: the order does not matter)
    double m[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
    int k = 0;
    for (; k + 3 < g.nz; k += 4)
#pragma unroll
      for (int j = 0; j < 4; ++j) m[j] = fmax(m[j], chibar[(int64_t)(k + j) * g.nx + i]);
    for (; k < g.nz; ++k) m[0] = fmax(m[0], chibar[(int64_t)k * g.nx + i]);
    if (fmax(fmax(m[0], m[1]), fmax(m[2], m[3])) >= theta) best = i;
  }
  for (int k = 0; k < 6; ++k) v[k] = (k == 4) ? wave_max(v[k]) : wave_sum(v[k]);
  for (int o = 32; o > 0; o >>= 1) best = max(best, __shfl_xor(best, o, 64));
  if (lane == 0) {
    for (int k = 0; k < 6; ++k) red[wid * 6 + k] = v[k];
    ired[wid] = best;
  }
  __syncthreads();
  if (wid != 0) return;
  // wave 0: the sums in fixed order (lane 0), then the depth maxima of the
  // front column and its neighbour across the wave
  const int nw = blockDim.x >> 6;
  for (int w = 1; w < nw; ++w) {
    for (int k = 0; k < 6; ++k) v[k] = (k == 4) ? fmax(v[k], red[w * 6 + k]) : v[k] + red[w * 6 + k];
    best = max(best, ired[w]);
  }
  double m0 = -INFINITY, m1 = -INFINITY;
  if (best >= 0 && best < g.nx - 1) {
    for (int k = lane; k < g.nz; k += 64) {
      m0 = fmax(m0, chibar[(int64_t)k * g.nx + best]);
      m1 = fmax(m1, chibar[(int64_t)k * g.nx + best + 1]);
    }
  }
  m0 = wave_max(m0);
  m1 = wave_max(m1);
  if (lane == 0) {
    double xf;
    if (best < 0) {
      xf = 0.0;
    } else if (best == g.nx - 1) {
      xf = (double)g.nx;
    } else {
      xf = best + 0.5 + (m0 - theta) / (m0 - m1);
    }
    out[0] = (double)g.n + v[0];
    out[1] = v[1];
    out[2] = g.nz >= 2 ? nu0 * (9.0 * v[2] - v[3]) / 3.0 : 0.0;
    out[3] = xf;
    out[4] = v[4];
    out[5] = v[5];
    out[6] = (double)best;
    out[7] = 0.0;
  }
}

// -------------------------------------------------------------- test hooks
template <class L>
__device__ __forceinline__ void vel(int q, int& cx, int& cy, int& cz) {
  cx = L::cx[q];
  cy = L::cy[q];
  cz = L::cz[q];
}

// pre-collision population a (0..qt-1) at every node, full value, float64
template <int MODEL, typename ST, typename SS>
__global__ __launch_bounds__(kBlock) void k_get_pop(const ST* __restrict__ src, Grid g, int a,
                                                    int nbx, double* __restrict__ out) {
  using LF = typename ModelT<MODEL>::LF;
  using LS = typename ModelT<MODEL>::LS;
  using CT = typename std::conditional<std::is_same<ST, double>::value, double, float>::type;
  const int b = blockIdx.x;
  const int row = b / nbx;
  const int x = (b - row * nbx) * blockDim.x + threadIdx.x;
  if (x >= g.nx) return;
  const int y = row % g.ny, z = row / g.ny;
  const int64_t node = (int64_t)row * g.nx + x;
  const bool flow = a < LF::Q;
  const int q = flow ? a : a - LF::Q;
  int cx, cy, cz, o;
  double w;
  if (flow) {
    vel<LF>(q, cx, cy, cz);
    o = opp<LF>(q);
    w = weight<LF>(q);
  } else {
    vel<LS>(q, cx, cy, cz);
    o = opp<LS>(q);
    w = 0.0;
  }
  const int base = flow ? 0 : LF::Q;
  const int xs = x - cx, zs = z - cz;
  int ys = y - cy;
  ys = ys < 0 ? g.ny - 1 : (ys >= g.ny ? 0 : ys);
  const bool wall = (unsigned)xs >= (unsigned)g.nx || (unsigned)zs >= (unsigned)g.nz;
  constexpr int QT = LF::Q + LS::Q;
  const int64_t off = wall ? elem_index<QT>(g, base + o, row, x)
                           : elem_index<QT>(g, base + q, (int64_t)zs * g.ny + ys, xs);
  out[node] = (flow ? to_d(Conv<ST, CT>::load(src[off]))
                    : to_d(Conv<SS, CT>::load(reinterpret_cast<const SS*>(src)[off]))) + w;
}

// inverse of the gather for population a given its pre-collision values v
// (full values, float64): slot (a, y) <- v(y + c_a) when that node is fluid;
// slot (opp a, y) <- v(y) when y - c_a is outside.
template <int MODEL, typename ST, typename SS>
__global__ __launch_bounds__(kBlock) void k_set_pop(ST* __restrict__ dst, Grid g, int a, int nbx,
                                                    const double* __restrict__ v) {
  using LF = typename ModelT<MODEL>::LF;
  using LS = typename ModelT<MODEL>::LS;
  using CT = typename std::conditional<std::is_same<ST, double>::value, double, float>::type;
  const int b = blockIdx.x;
  const int row = b / nbx;
  const int x = (b - row * nbx) * blockDim.x + threadIdx.x;
  if (x >= g.nx) return;
  const int y = row % g.ny, z = row / g.ny;
  const int64_t node = (int64_t)row * g.nx + x;
  const bool flow = a < LF::Q;
  const int q = flow ? a : a - LF::Q;
  int cx, cy, cz, o;
  double w;
  if (flow) {
    vel<LF>(q, cx, cy, cz);
    o = opp<LF>(q);
    w = weight<LF>(q);
  } else {
    vel<LS>(q, cx, cy, cz);
    o = opp<LS>(q);
    w = 0.0;
  }
  const int base = flow ? 0 : LF::Q;
  auto put = [&](int64_t i, double val) {
    if (flow)
      dst[i] = Conv<ST, CT>::store(CT(val));
    else
      reinterpret_cast<SS*>(dst)[i] = Conv<SS, CT>::store(CT(val));
  };
  {
    const int xn = x + cx, zn = z + cz;
    int yn = y + cy;
    yn = yn < 0 ? g.ny - 1 : (yn >= g.ny ? 0 : yn);
    if ((unsigned)xn < (unsigned)g.nx && (unsigned)zn < (unsigned)g.nz)
      put(elem_index<LF::Q + LS::Q>(g, base + q, row, x), v[((int64_t)zn * g.ny + yn) * g.nx + xn] - w);
  }
  {
    const int xs = x - cx, zs = z - cz;
    if ((unsigned)xs >= (unsigned)g.nx || (unsigned)zs >= (unsigned)g.nz)
      put(elem_index<LF::Q + LS::Q>(g, base + o, row, x), v[node] - w);
  }
}

// ------------------------------------------- allocation-free diagnostics
// Scratch of lbm_checkpoint_diagnostics: the span-averaged concentration, the
// per-block partial sums and the result slot of the diagnostics kernels,
// which a handle keeps in its workspace. A file-scope device array, so that
// the entry point allocates nothing; every GPU the library runs on holds its
// own copy until the process ends. In host code its name is only a stand-in
// for the symbol: its device address comes from hipGetSymbolAddress, taken
// once per device with that device current, and only that address is used.
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

hipError_t static_scratch(double** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double* addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<double*>(p);
  }
  *ptr = addr[dev];
  return hipSuccess;
}

// ---------------------------------------------------------------- dispatch
static Grid grid_of(const lbm_handle* h) {
  return Grid{h->cfg.nx, h->cfg.ny, h->cfg.nz, h->n, xblocks(h->cfg.nx)};
}

static int block_x(const lbm_handle* h) {
  const int nx = h->cfg.nx;
  return nx >= kBlock ? kBlock : ((nx + 63) / 64) * 64;
}

template <typename CT>
static Phys<CT> phys_of(const lbm_handle* h) {
  const lbm_params& p = h->prm;
  const lbm_config& c = h->cfg;
  Phys<CT> r;
  r.g = (CT)p.g_prime;
  r.tau0 = (CT)p.tau0;
  r.tau_phi0 = (CT)p.tau_phi0;
  // 18 sqrt(2) C_s^2 (standard closure) or 18 sqrt(2) C_s (as printed in Eq. 32)
  r.c_les = (CT)(18.0 * sqrt(2.0) * (c.smag_paper_form ? c.cs_smag : c.cs_smag * c.cs_smag));
  r.d0 = (CT)p.d0;
  r.inv_sct = (CT)(1.0 / c.sc_t);
  r.inv_cs2phi = (CT)(1.0 / p.cs2_phi);
  r.omega2 = (CT)c.omega_bulk;
  r.omega3 = (CT)c.omega3;
  r.omega4 = (CT)c.omega4;
  r.omega5 = (CT)c.omega5;
  r.omega6 = (CT)c.omega6;
  const double h4 = p.tau0 - 0.5;  // 1/omega1 - 1/2
  r.w_plus = (CT)p.w_plus;
  r.w_minus = (CT)p.w_minus;
  r.w_111 = (CT)p.w_111;
  r.a4 = (CT)(-2.0 / 3.0 * h4 * p.coef_a);
  r.b4 = (CT)(-1.0 / 3.0 * h4 * p.coef_b);
  r.lam = c.limiter > 0.0 ? (CT)c.limiter : (CT)INFINITY;
  return r;
}

// calls f(ST{}, SS{}, CT{}) for the handle's storage mode: flow element
// type, scalar element type, arithmetic type
template <class F>
static hipError_t with_storage(const lbm_handle* h, F&& f) {
  switch (h->cfg.storage) {
    case LBM_F64: return f(double{}, double{}, double{});
    case LBM_F32: return f(float{}, float{}, float{});
    case LBM_F16: return f(__half{}, __half{}, float{});
    case LBM_BF16: return f(bf16_t{}, bf16_t{}, float{});
    case LBM_BF16_F16S: return f(bf16_t{}, __half{}, float{});
  }
  return hipErrorInvalidValue;
}
template <class F>
static hipError_t with_model(const lbm_handle* h, F&& f) {
  switch (h->cfg.model) {
    case LBM_CUMULANT27_Q7: return f(std::integral_constant<int, 0>{});
    case LBM_BGK19_SMAG_Q6: return f(std::integral_constant<int, 1>{});
    case LBM_CUMULANT27_FCM27: return f(std::integral_constant<int, 2>{});
  }
  return hipErrorInvalidValue;
}

static int cumulant_kind(const lbm_handle* h) {
  const lbm_config& c = h->cfg;
  if (c.parametrized) return kCumParam;
  return (c.omega3 != 1.0 || c.omega4 != 1.0 || c.omega5 != 1.0 || c.omega6 != 1.0) ? kCumGeneral
                                                                                   : kCumFast;
}

template <int M, typename ST, typename SS, typename CT, int NPT>
static hipError_t launch_step_npt(lbm_handle* h, const Grid& g, const void* src, void* dst,
                                  double* fw, hipStream_t st) {
  const bool les = h->cfg.cs_smag > 0.0;
  const int per_thread_x = (g.nx + NPT - 1) / NPT;  // x-extent in threads if one block
  const int bx = per_thread_x >= kBlock ? kBlock : ((per_thread_x + 63) / 64) * 64;
  const int nbx = (g.nx + bx * NPT - 1) / (bx * NPT);
  const unsigned blocks = (unsigned)((int64_t)nbx * g.ny * g.nz);
  const Phys<CT> p = phys_of<CT>(h);
  const ST* s = static_cast<const ST*>(src);
  ST* d = static_cast<ST*>(dst);
  if (fw) {  // the adjoint's forward pass: FP32 / FP64 storage
    if constexpr (std::is_same<ST, CT>::value && std::is_same<SS, ST>::value) {
      const int kind = M == 1 ? kCumFast : cumulant_kind(h);
      if (kind == kCumGeneral) return hipErrorInvalidValue;
      if constexpr (M != 1) {
        if (kind == kCumParam) {
          hipLaunchKernelGGL((k_step<M, ST, SS, CT, false, kCumParam, NPT, true>), dim3(blocks), dim3(bx), 0, st, s, d, g, p, nbx, fw);
          return hipGetLastError();
        }
      }
      if (les)
        hipLaunchKernelGGL((k_step<M, ST, SS, CT, true, kCumFast, NPT, true>), dim3(blocks), dim3(bx), 0, st, s, d, g, p, nbx, fw);
      else
        hipLaunchKernelGGL((k_step<M, ST, SS, CT, false, kCumFast, NPT, true>), dim3(blocks), dim3(bx), 0, st, s, d, g, p, nbx, fw);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  if constexpr (M == 1) {  // BGK: one collision kind
    if (les)
      hipLaunchKernelGGL((k_step<M, ST, SS, CT, true, kCumFast, NPT>), dim3(blocks), dim3(bx), 0, st, s, d, g, p, nbx, nullptr);
    else
      hipLaunchKernelGGL((k_step<M, ST, SS, CT, false, kCumFast, NPT>), dim3(blocks), dim3(bx), 0, st, s, d, g, p, nbx, nullptr);
  } else {
    // the parametrised kind never has the LES (rejected when the handle is made)
    const int kind = cumulant_kind(h);
    if (les && kind == kCumGeneral)
      hipLaunchKernelGGL((k_step<M, ST, SS, CT, true, kCumGeneral, NPT>), dim3(blocks), dim3(bx), 0, st, s, d, g, p, nbx, nullptr);
    else if (les)
      hipLaunchKernelGGL((k_step<M, ST, SS, CT, true, kCumFast, NPT>), dim3(blocks), dim3(bx), 0, st, s, d, g, p, nbx, nullptr);
    else if (kind == kCumParam)
      hipLaunchKernelGGL((k_step<M, ST, SS, CT, false, kCumParam, NPT>), dim3(blocks), dim3(bx), 0, st, s, d, g, p, nbx, nullptr);
    else if (kind == kCumGeneral)
      hipLaunchKernelGGL((k_step<M, ST, SS, CT, false, kCumGeneral, NPT>), dim3(blocks), dim3(bx), 0, st, s, d, g, p, nbx, nullptr);
    else
      hipLaunchKernelGGL((k_step<M, ST, SS, CT, false, kCumFast, NPT>), dim3(blocks), dim3(bx), 0, st, s, d, g, p, nbx, nullptr);
  }
  return hipGetLastError();
}

// Grids too small to give every SIMD four waves at the preferred nodes per
// thread (cache-resident, latency-bound runs such as a 256 x 16 x 32
// adjoint) take one node per thread: twice the waves.
static bool few_waves(const lbm_handle* h, int npt) {
  const int64_t waves = (h->n + (int64_t)64 * npt - 1) / ((int64_t)64 * npt);
  return waves < (int64_t)16 * h->cu_count;
}

hipError_t launch_step(lbm_handle* h, const void* src, void* dst, double* fw,
                       hipStream_t stream) {
  const Grid g = grid_of(h);
  if (!stream) stream = h->stream;
  return with_model(h, [&](auto mc) {
    constexpr int M = decltype(mc)::value;
    return with_storage(h, [&](auto st, auto ss, auto ct) {
      using ST = decltype(st);
      using SS = decltype(ss);
      using CT = decltype(ct);
      constexpr int NPT = nodes_per_thread<M, ST>();
      if constexpr (NPT > 1) {
        if (few_waves(h, NPT)) return launch_step_npt<M, ST, SS, CT, 1>(h, g, src, dst, fw, stream);
      }
      return launch_step_npt<M, ST, SS, CT, NPT>(h, g, src, dst, fw, stream);
    });
  });
}

template <class Init>
static hipError_t launch_init_any(lbm_handle* h, Init init) {
  const Grid g = grid_of(h);
  const int bx = block_x(h);
  const int nbx = (g.nx + bx - 1) / bx;
  const unsigned blocks = (unsigned)((int64_t)nbx * g.ny * g.nz);
  return with_model(h, [&](auto mc) {
    constexpr int M = decltype(mc)::value;
    return with_storage(h, [&](auto st, auto ss, auto) {
      using ST = decltype(st);
      using SS = decltype(ss);
      hipLaunchKernelGGL((k_init<M, ST, SS, Init>), dim3(blocks), dim3(bx), 0, h->stream,
                         static_cast<ST*>(h->buf[h->cur]), g, init, nbx);
      return hipGetLastError();
    });
  });
}

hipError_t launch_init_lock(lbm_handle* h, double lock_fraction, double amp, uint64_t seed) {
  LockInit init{(int)floor(lock_fraction * h->cfg.nx), amp, seed};
  return launch_init_any(h, init);
}

hipError_t launch_init_field(lbm_handle* h, const double* chi0) {
  return launch_init_any(h, FieldInit{chi0});
}

hipError_t launch_moments(lbm_handle* h, int dtype, void* rho, void* ux, void* uy, void* uz,
                          void* chi) {
  const Grid g = grid_of(h);
  const int bx = block_x(h);
  const int nbx = (g.nx + bx - 1) / bx;
  const unsigned blocks = (unsigned)((int64_t)nbx * g.ny * g.nz);
  const double gp = h->prm.g_prime;
  return with_model(h, [&](auto mc) {
    constexpr int M = decltype(mc)::value;
    return with_storage(h, [&](auto st, auto ss, auto ct) {
      using ST = decltype(st);
      using SS = decltype(ss);
      using CT = decltype(ct);
      const ST* s = static_cast<const ST*>(h->buf[h->cur]);
      if (dtype == LBM_OUT_F64)
        hipLaunchKernelGGL((k_moments<M, ST, SS, CT, double>), dim3(blocks), dim3(bx), 0, h->stream, s, g, gp, nbx, rho, ux, uy, uz, chi);
      else
        hipLaunchKernelGGL((k_moments<M, ST, SS, CT, float>), dim3(blocks), dim3(bx), 0, h->stream, s, g, gp, nbx, rho, ux, uy, uz, chi);
      return hipGetLastError();
    });
  });
}

hipError_t launch_wall_shear(lbm_handle* h, int dtype, void* tau, void* tau_bar) {
  const Grid g = grid_of(h);
  const int bx = block_x(h);
  const unsigned blocks = (unsigned)((g.nx + bx - 1) / bx);
  const double nu0 = h->prm.nu0;
  return with_model(h, [&](auto mc) {
    constexpr int M = decltype(mc)::value;
    return with_storage(h, [&](auto st, auto ss, auto ct) {
      using ST = decltype(st);
      using SS = decltype(ss);
      using CT = decltype(ct);
      const ST* s = static_cast<const ST*>(h->buf[h->cur]);
      if (dtype == LBM_OUT_F64)
        hipLaunchKernelGGL((k_wall_shear<M, ST, SS, CT, double>), dim3(blocks), dim3(bx), 0, h->stream, s, g, nu0, tau, tau_bar);
      else
        hipLaunchKernelGGL((k_wall_shear<M, ST, SS, CT, float>), dim3(blocks), dim3(bx), 0, h->stream, s, g, nu0, tau, tau_bar);
      return hipGetLastError();
    });
  });
}

hipError_t launch_diag(lbm_handle* h, double* out) {
  const Grid g = grid_of(h);
  const int bx = block_x(h);
  const int nbx = (g.nx + bx - 1) / bx;
  const double gp = h->prm.g_prime;
  hipError_t e = with_model(h, [&](auto mc) {
    constexpr int M = decltype(mc)::value;
    return with_storage(h, [&](auto st, auto ss, auto ct) {
      using ST = decltype(st);
      using SS = decltype(ss);
      using CT = decltype(ct);
      hipLaunchKernelGGL((k_diag_columns<M, ST, SS, CT>), dim3(nbx * g.nz), dim3(bx), 0, h->stream,
                         static_cast<const ST*>(h->buf[h->cur]), g, gp, h->chibar, h->partials,
                         nbx);
      return hipGetLastError();
    });
  });
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(1024), 0, h->stream, h->partials, nbx * g.nz,
                     h->chibar, g, h->prm.nu0, out);
  return hipGetLastError();
}

hipError_t launch_get_pop(lbm_handle* h, int a, double* dst) {
  const Grid g = grid_of(h);
  const int bx = block_x(h);
  const int nbx = (g.nx + bx - 1) / bx;
  const unsigned blocks = (unsigned)((int64_t)nbx * g.ny * g.nz);
  return with_model(h, [&](auto mc) {
    constexpr int M = decltype(mc)::value;
    return with_storage(h, [&](auto st, auto ss, auto) {
      using ST = decltype(st);
      using SS = decltype(ss);
      hipLaunchKernelGGL((k_get_pop<M, ST, SS>), dim3(blocks), dim3(bx), 0, h->stream,
                         static_cast<const ST*>(h->buf[h->cur]), g, a, nbx, dst);
      return hipGetLastError();
    });
  });
}

hipError_t launch_set_pop(lbm_handle* h, int a, const double* src) {
  const Grid g = grid_of(h);
  const int bx = block_x(h);
  const int nbx = (g.nx + bx - 1) / bx;
  const unsigned blocks = (unsigned)((int64_t)nbx * g.ny * g.nz);
  return with_model(h, [&](auto mc) {
    constexpr int M = decltype(mc)::value;
    return with_storage(h, [&](auto st, auto ss, auto) {
      using ST = decltype(st);
      using SS = decltype(ss);
      hipLaunchKernelGGL((k_set_pop<M, ST, SS>), dim3(blocks), dim3(bx), 0, h->stream,
                         static_cast<ST*>(h->buf[h->cur]), g, a, nbx, src);
      return hipGetLastError();
    });
  });
}

hipError_t launch_copy_state(lbm_handle* h, const void* src, void* dst) {
  return hipMemcpyAsync(dst, src, h->state_bytes, hipMemcpyDeviceToDevice, h->stream);
}

}  // namespace lbm

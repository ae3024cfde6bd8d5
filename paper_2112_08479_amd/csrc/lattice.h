// Velocity sets, weights, storage conversions and the pull gather with
// half-way bounce-back used by every kernel of the library.
//
// Velocity sets: D3Q19 in the order of Eq. 23, D3Q27 = D3Q19 + the eight
// corners (Eq. 36 lists only seven; (1,-1,1) is added), D3Q6 in the order of
// Eq. 31, D3Q7 = rest + D3Q6. Moving velocities come in +/- pairs, so the
// opposite of q is q+1 / q-1.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#define LBM_HD __host__ __device__ __forceinline__

namespace lbm {

struct Q27 {
  static constexpr int Q = 27;
  static constexpr bool has_rest = true;
  static constexpr int cx[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                                 1, -1, 1, -1, 1, -1, 1, -1};
  static constexpr int cy[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                                 1, -1, 1, -1, -1, 1, -1, 1};
  static constexpr int cz[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                                 1, -1, -1, 1, 1, -1, -1, 1};
};
struct Q19 {
  static constexpr int Q = 19;
  static constexpr bool has_rest = true;
  static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
};
struct Q7 {
  static constexpr int Q = 7;
  static constexpr bool has_rest = true;
  static constexpr int cx[7] = {0, 1, -1, 0, 0, 0, 0};
  static constexpr int cy[7] = {0, 0, 0, 1, -1, 0, 0};
  static constexpr int cz[7] = {0, 0, 0, 0, 0, 1, -1};
};
struct Q6 {
  static constexpr int Q = 6;
  static constexpr bool has_rest = false;
  static constexpr int cx[6] = {1, -1, 0, 0, 0, 0};
  static constexpr int cy[6] = {0, 0, 1, -1, 0, 0};
  static constexpr int cz[6] = {0, 0, 0, 0, 1, -1};
};

template <class L>
constexpr int opp(int q) {
  return L::has_rest ? (q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1)) : ((q & 1) ? q - 1 : q + 1);
}

// Weights. D3Q19 (Eq. 24): 1/3, 1/18, 1/36 by |c|^2 = 0, 1, 2. D3Q27: tensor
// product of the one-dimensional weights 2/3 (c = 0) and 1/6 (c = +-1).
// D3Q6: 1/6 (Eq. 31). D3Q7: 1/4 rest, 1/8 moving.
template <class L>
constexpr double weight(int q);
template <>
constexpr double weight<Q27>(int q) {
  return (Q27::cx[q] ? 1.0 / 6.0 : 2.0 / 3.0) * (Q27::cy[q] ? 1.0 / 6.0 : 2.0 / 3.0) *
         (Q27::cz[q] ? 1.0 / 6.0 : 2.0 / 3.0);
}
template <>
constexpr double weight<Q19>(int q) {
  return q == 0 ? 1.0 / 3.0 : (q < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}
template <>
constexpr double weight<Q7>(int q) {
  return q == 0 ? 0.25 : 0.125;
}
template <>
constexpr double weight<Q6>(int q) {
  return 1.0 / 6.0;
}

// population index of velocity (a, b, c) in D3Q27
constexpr int idx27(int a, int b, int c) {
  for (int q = 0; q < 27; ++q)
    if (Q27::cx[q] == a && Q27::cy[q] == b && Q27::cz[q] == c) return q;
  return -1;
}

// ---------------------------------------------------------------- storage
struct bf16_t {
  uint16_t bits;
};

template <typename ST, typename CT>
struct Conv;
template <>
struct Conv<double, double> {
  static LBM_HD double load(double v) { return v; }
  static LBM_HD double store(double v) { return v; }
};
template <>
struct Conv<float, float> {
  static LBM_HD float load(float v) { return v; }
  static LBM_HD float store(float v) { return v; }
};
template <>
struct Conv<__half, float> {
  static LBM_HD float load(__half v) { return __half2float(v); }
  static LBM_HD __half store(float v) { return __float2half_rn(v); }
};
template <>
struct Conv<bf16_t, float> {
  static LBM_HD float load(bf16_t v) {
    uint32_t u = (uint32_t)v.bits << 16;
    return __uint_as_float(u);
  }
  // round to nearest even on the 16 dropped bits; NaN stays NaN
  static LBM_HD bf16_t store(float v) {
    uint32_t u = __float_as_uint(v);
    bf16_t r;
    if ((u & 0x7fffffffu) > 0x7f800000u) {
      r.bits = (uint16_t)((u >> 16) | 0x40u);
    } else {
      u += 0x7fffu + ((u >> 16) & 1u);
      r.bits = (uint16_t)(u >> 16);
    }
    return r;
  }
};

// Every population buffer is allocated with at least this many bytes of the
// same allocation after its end: a lattice whose last array is x-shifted
// (D3Q27 ends with a corner) makes the never-used first load of the lane at
// x = nx - 1 read one element past the buffer.
constexpr int kBufferGuardBytes = 256;

// ---------------------------------------------------------------- geometry
struct Grid {
  int nx, ny, nz;
  int64_t n;  // nodes
};

// Source element (array index, node index) that population q of lattice L at
// node (x, y, z) pulls from: the neighbour x - c_q when it is a fluid node
// (y taken modulo ny), else -- half-way bounce-back -- population opp(q) of
// the node itself.
// The array base pointers depend only on q and the launch (scalar registers);
// node indices fit in 32 bits (n < 2^31), computed unsigned so that the
// unselected out-of-range candidate at a wall is harmless.
template <class L, int q, typename ST>
LBM_HD const ST* pull_ptr(const ST* __restrict__ src, const Grid& g, int base, int x, int y, int z,
                          uint32_t node) {
  constexpr int cx = L::cx[q], cy = L::cy[q], cz = L::cz[q];
  const ST* pq = src + (int64_t)(base + q) * g.n;
  const ST* po = src + (int64_t)(base + opp<L>(q)) * g.n;
  const int xs = x - cx;
  const int zs = z - cz;
  int ys = y - cy;
  if (cy == 1) ys = (y == 0) ? g.ny - 1 : ys;
  if (cy == -1) ys = (y == g.ny - 1) ? 0 : ys;
  bool wall = false;
  if (cx != 0) wall = wall || ((unsigned)xs >= (unsigned)g.nx);
  if (cz != 0) wall = wall || ((unsigned)zs >= (unsigned)g.nz);
  const uint32_t s = ((uint32_t)zs * (uint32_t)g.ny + (uint32_t)ys) * (uint32_t)g.nx + (uint32_t)xs;
  return wall ? po + node : pq + s;
}

template <int I, int N, class F>
LBM_HD void static_for(F&& f);

// Gather for a thread block that covers NPT * blockDim.x consecutive nodes
// x0 .. of one row (y, z); thread `lane` handles x0 + lane + k blockDim.x,
// k < NPT. Every pull address is a block-uniform row pointer (scalar
// registers, advanced by one array per population) plus the lane index, so
// the gather costs no per-lane address arithmetic:
//   - y is periodic: the source row is chosen per block;
//   - a source beyond a z wall (uniform per block) selects the bounce-back
//     pointer, the node's own opposite population;
//   - lanes at an x wall first load a neighbouring element of the buffer
//     (never used) and, in the waves that hold such a lane only, take the
//     bounce-back value afterwards. That first load stays inside the
//     allocation because the buffer's first array is a rest population (no x
//     shift reads below it) and either its last array has c_x = 0 (nothing
//     reads past its end) or the guard bytes follow it -- checked by the
//     static_asserts. Lane offsets are clamped to the row so
//     that tail lanes of a ragged row never read past it.
template <class L, int base, int NPT, typename ST, typename CT>
__device__ __forceinline__ void pull_lattice(const ST* __restrict__ src, const Grid& g,
                                             int64_t row0, int y, int z, const unsigned* li,
                                             bool wave_at_wall, const int* xk,
                                             CT (&out)[NPT][L::Q]) {
  const int dy_m = (y == g.ny - 1) ? -(g.ny - 1) : 1;  // c_y = -1: source row y + 1
  const int dy_p = (y == 0) ? g.ny - 1 : -1;           // c_y = +1: source row y - 1
  const ST* arr0 = src + (int64_t)base * g.n + row0;
  {
    const ST* arr = arr0;
    static_for<0, L::Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      constexpr int cx = L::cx[q], cy = L::cy[q], cz = L::cz[q];
      constexpr int o = opp<L>(q);
      const bool zwall = cz != 0 && (unsigned)(z - cz) >= (unsigned)g.nz;
      const int dy = cy == 0 ? 0 : (cy == 1 ? dy_p : dy_m);
      const int64_t sh = zwall ? (int64_t)(o - q) * g.n : ((int64_t)(-cz) * g.ny + dy) * g.nx - cx;
      const ST* p = arr + sh;
#pragma unroll
      for (int k = 0; k < NPT; ++k) out[k][q] = Conv<ST, CT>::load(p[li[k]]);
      arr += g.n;
    });
  }
  if (wave_at_wall) {  // wave-uniform: this wave holds x = 0 or x = nx - 1
    const ST* arr = arr0;
    static_for<0, L::Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      constexpr int cx = L::cx[q], cz = L::cz[q];
      constexpr int o = opp<L>(q);
      if constexpr (cx != 0) {
        const bool zwall = cz != 0 && (unsigned)(z - cz) >= (unsigned)g.nz;
        const ST* po = arr + (int64_t)(o - q) * g.n;
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
          const bool wall = !zwall && (unsigned)(xk[k] - cx) >= (unsigned)g.nx;
          const CT b = Conv<ST, CT>::load(po[li[k]]);
          out[k][q] = wall ? b : out[k][q];
        }
      }
      arr += g.n;
    });
  }
}

// ST: element type of the flow arrays; SS: of the scalar arrays, which follow
// the flow arrays in the same buffer (same element size, so the array
// geometry and the over-read argument above are unchanged).
template <class LF, class LS, int NPT, typename ST, typename CT, typename SS = ST>
__device__ __forceinline__ void gather_rows(const ST* __restrict__ src, const Grid& g, int x0, int y,
                                            int z, CT (&fg)[NPT][LF::Q], CT (&ph)[NPT][LS::Q]) {
  static_assert(sizeof(SS) == sizeof(ST), "flow and scalar elements must have one size");
  static_assert(LF::cx[0] == 0 && LF::cy[0] == 0 && LF::cz[0] == 0, "buffer must start at rest");
  static_assert(LS::cx[LS::Q - 1] == 0 || kBufferGuardBytes >= (int)sizeof(ST),
                "an x-shifted last array reads one element past the buffer: needs the guard");
  const int64_t row0 = ((int64_t)z * g.ny + y) * g.nx + x0;
  unsigned li[NPT];
  int xk[NPT];
  const unsigned last = (unsigned)(g.nx - 1 - x0);  // >= 0: the block holds a node
  bool at_wall = false;
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const unsigned o = threadIdx.x + (unsigned)k * blockDim.x;
    li[k] = o < last ? o : last;
    xk[k] = x0 + (int)o;
    at_wall = at_wall || xk[k] == 0 || xk[k] == g.nx - 1;
  }
  const bool wave_at_wall = __builtin_amdgcn_ballot_w64(at_wall) != 0;
  pull_lattice<LF, 0, NPT, ST, CT>(src, g, row0, y, z, li, wave_at_wall, xk, fg);
  pull_lattice<LS, LF::Q, NPT, SS, CT>(reinterpret_cast<const SS*>(src), g, row0, y, z, li,
                                       wave_at_wall, xk, ph);
}

template <int I, int N, class F>
LBM_HD void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// Gathers the pre-collision populations of node (x, y, z): flow populations
// as deviations f - w into fg[], scalar populations into ph[] (scalar arrays
// of element type SS, as in gather_rows).
template <class LF, class LS, typename ST, typename CT, typename SS = ST>
LBM_HD void gather(const ST* __restrict__ src, const Grid& g, int x, int y, int z, int64_t node,
                   CT* fg, CT* ph) {
  static_assert(sizeof(SS) == sizeof(ST), "flow and scalar elements must have one size");
  static_for<0, LF::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    fg[q] = Conv<ST, CT>::load(*pull_ptr<LF, q>(src, g, 0, x, y, z, (uint32_t)node));
  });
  static_for<0, LS::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    ph[q] = Conv<SS, CT>::load(
        *reinterpret_cast<const SS*>(pull_ptr<LS, q>(src, g, LF::Q, x, y, z, (uint32_t)node)));
  });
}

}  // namespace lbm

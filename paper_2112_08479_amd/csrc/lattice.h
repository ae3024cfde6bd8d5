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

// The velocity set L with every velocity reversed (same indices, so the same
// opposite of each index). A pull on Rev<L> reads population q from x + c_q,
// or, beyond a wall, population opp(q) of the node itself: the transpose of
// the pull on L, which the adjoint applies to its lambda field.
template <class L>
struct Rev {
  static constexpr int Q = L::Q;
  static constexpr bool has_rest = L::has_rest;
  struct Neg {
    int v[L::Q];
    constexpr int operator[](int i) const { return v[i]; }
  };
  static constexpr Neg neg(const int (&c)[L::Q]) {
    Neg r{};
    for (int i = 0; i < L::Q; ++i) r.v[i] = -c[i];
    return r;
  }
  static constexpr Neg cx = neg(L::cx), cy = neg(L::cy), cz = neg(L::cz);
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
  // round to nearest even (gfx950 converts in hardware, v_cvt_pk_bf16_f32);
  // NaN stays NaN
  static LBM_HD bf16_t store(float v) {
    bf16_t r;
    r.bits = __builtin_bit_cast(uint16_t, (__bf16)v);
    return r;
  }
};

// ---------------------------------------------------------------- geometry
// Population buffer layout (x-blocked). Rows (y, z) follow one another; each
// row is cut into blocks of kXB = 64 consecutive x (one wavefront), and an
// x-block holds the QT populations one after the other, 64 values each:
//   element(a, x, row) = (row nxb + x / 64) QT 64 + 64 a + x % 64,
// with nxb = ceil(nx / 64) x-blocks per row (the last one padded when 64 does
// not divide nx; padding is never read as fluid data). A wavefront loads or
// stores one population as one contiguous 64-element segment, and the QT
// populations of a tile are one contiguous span: a tile reads from the nine
// rows (y - c_y, z - c_z) and writes one span, where a population-major
// layout has every tile touch 2 QT separate arrays.
constexpr int kXB = 64;
constexpr int kXBShift = 6;

// Spare bytes after every population buffer in its allocation (none are read
// by the kernels; kept as a margin).
constexpr int kBufferGuardBytes = 256;

struct Grid {
  int nx, ny, nz;
  int64_t n;  // nodes
  int nxb;    // x-blocks per row, ceil(nx / 64)
};

LBM_HD int xblocks(int nx) { return (nx + kXB - 1) / kXB; }

// element index of population a at (x, row), row = z ny + y
template <int QT>
LBM_HD int64_t elem_index(const Grid& g, int a, int64_t row, int x) {
  return (row * g.nxb + (x >> kXBShift)) * (int64_t)(QT * kXB) + (int64_t)a * kXB + (x & (kXB - 1));
}

// Source element of population q (lattice L, arrays base.. of a buffer with
// QT populations) at node (x, y, z): the neighbour x - c_q when it is a fluid
// node (y taken modulo ny), else -- half-way bounce-back -- population opp(q)
// of the node itself.
template <class L, int q, int QT, typename ST>
LBM_HD const ST* pull_ptr(const ST* __restrict__ src, const Grid& g, int base, int x, int y, int z) {
  constexpr int cx = L::cx[q], cy = L::cy[q], cz = L::cz[q];
  const int xs = x - cx;
  const int zs = z - cz;
  int ys = y - cy;
  if (cy == 1) ys = (y == 0) ? g.ny - 1 : ys;
  if (cy == -1) ys = (y == g.ny - 1) ? 0 : ys;
  bool wall = false;
  if (cx != 0) wall = wall || ((unsigned)xs >= (unsigned)g.nx);
  if (cz != 0) wall = wall || ((unsigned)zs >= (unsigned)g.nz);
  const int64_t e = wall ? elem_index<QT>(g, base + opp<L>(q), (int64_t)z * g.ny + y, x)
                         : elem_index<QT>(g, base + q, (int64_t)zs * g.ny + ys, xs);
  return src + e;
}

template <int I, int N, class F>
LBM_HD void static_for(F&& f);

// Block order of the row-tiled kernels. Consecutive block ids are dealt
// round-robin to the 8 XCDs, each with its own L2, and the tiles of one row
// share a cache line at each tile edge (the x-shifted pulls read one element
// across it). Rows are taken in groups of eight; within a group, block b
// takes row b % 8 and tile b / 8 of it, so a whole row runs on one XCD with
// its tiles dispatched eight blocks apart, while consecutive blocks still go
// to different rows (a tail group of fewer rows is dealt the same way).
// Returns the tile index row * nbx + tile for block b of nblocks, nbx tiles
// per row. Measured against plain order on the step kernel: FP16 +3.7 %,
// FP32 within 1 %, and less read traffic at tile edges.
LBM_HD int xcd_row_order(int b, int nblocks, int nbx) {
  constexpr int kXcd = 8;
  const int group = kXcd * nbx;
  const int g0 = b / group, rem = b - g0 * group;
  const int nrows = nblocks / nbx;
  const int rows = (nrows - g0 * kXcd) < kXcd ? (nrows - g0 * kXcd) : kXcd;
  const int i = rem / rows, r = g0 * kXcd + (rem - (rem / rows) * rows);
  return r * nbx + i;
}

// Lane geometry of a tile for the x-blocked layout. Thread t handles nodes
// x = x0 + t + k blockDim.x (k < NPT); x0 and blockDim.x are multiples of 64,
// so t % 64 is the node's place in its x-block. Offsets are element offsets
// inside a row (all populations of the row), taken at x clamped to nx - 1 so
// that tail lanes of a ragged row read a real node (their results are never
// stored):
//   own:  the node itself;
//   srcp: its x - 1 neighbour (pull of c_x = +1), the node itself at x = 0;
//   srcm: its x + 1 neighbour (pull of c_x = -1), the node itself at x = nx - 1.
// At the walls the neighbour is replaced by bounce-back afterwards, so every
// address stays inside the row.
template <int QT, int NPT>
struct TileLanes {
  int own[NPT], srcp[NPT], srcm[NPT], x[NPT];
};

template <int QT, int NPT>
LBM_HD TileLanes<QT, NPT> tile_lanes(const Grid& g, int x0, int tid, int bdim) {
  TileLanes<QT, NPT> t;
  constexpr int XBLK = QT * kXB;
#pragma unroll
  for (int k = 0; k < NPT; ++k) {
    const int x = x0 + tid + k * bdim;
    const int xe = x < g.nx ? x : g.nx - 1;
    const int xl = xe & (kXB - 1);
    const int own = (xe >> kXBShift) * XBLK + xl;
    t.x[k] = x;
    t.own[k] = own;
    t.srcp[k] = xe == 0 ? own : (xl == 0 ? own - XBLK + (kXB - 1) : own - 1);
    t.srcm[k] = xe == g.nx - 1 ? own : (xl == kXB - 1 ? own + XBLK - (kXB - 1) : own + 1);
  }
  return t;
}

// Gather of one lattice (arrays base.. of the buffer) for a tile of row
// (y, z). Each pull is a block-uniform pointer (scalar registers: the source
// row, or the node's own row at a z wall, plus the population's segment) and a
// per-lane offset from TileLanes, chosen by c_x:
//   - y is periodic: the source row is chosen per block;
//   - a source beyond a z wall (uniform per block) selects the bounce-back
//     segment of the node's own row;
//   - lanes at an x wall first load their own node's element (never used)
//     and, in the waves that hold such a lane only, take the bounce-back
//     value afterwards.
// Block-uniform part of the pull of population q (lattice L, arrays base..):
// the element index of its 64-value segment in the source row, or in the
// node's own row (population opp(q)) when the source is beyond a z wall.
template <class L, int q, int base, int QT>
LBM_HD int64_t pull_segment(const Grid& g, int y, int z, bool& zwall) {
  constexpr int cy = L::cy[q], cz = L::cz[q];
  const int64_t rowlen = (int64_t)g.nxb * (QT * kXB);
  zwall = cz != 0 && (unsigned)(z - cz) >= (unsigned)g.nz;
  int ys = y;
  if (cy == 1) ys = (y == 0) ? g.ny - 1 : y - 1;
  if (cy == -1) ys = (y == g.ny - 1) ? 0 : y + 1;
  return zwall ? ((int64_t)z * g.ny + y) * rowlen + (base + opp<L>(q)) * kXB
               : ((int64_t)(z - cz) * g.ny + ys) * rowlen + (base + q) * kXB;
}

// Per-lane part: the offset of node k's source inside the row, by c_x (the
// node itself at a z wall).
template <class L, int q, int QT, int NPT>
LBM_HD int pull_lane(const TileLanes<QT, NPT>& t, int k, bool zwall) {
  constexpr int cx = L::cx[q];
  return zwall ? t.own[k] : (cx == 1 ? t.srcp[k] : (cx == -1 ? t.srcm[k] : t.own[k]));
}

// Bounce-back at an x wall: population opp(q) of the node itself.
template <class L, int q, int base, int QT>
LBM_HD int64_t bounce_segment(const Grid& g, int y, int z) {
  return ((int64_t)z * g.ny + y) * ((int64_t)g.nxb * (QT * kXB)) + (base + opp<L>(q)) * kXB;
}

template <class L, int q>
LBM_HD bool x_wall(const Grid& g, int x, bool zwall) {
  constexpr int cx = L::cx[q];
  return cx != 0 && !zwall && (unsigned)(x - cx) >= (unsigned)g.nx;
}

template <class L, int base, int QT, int NPT, typename ST, typename CT>
__device__ __forceinline__ void pull_lattice(const ST* __restrict__ src, const Grid& g, int y,
                                             int z, const TileLanes<QT, NPT>& t,
                                             bool wave_at_wall, CT (&out)[NPT][L::Q]) {
  static_for<0, L::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    bool zwall;
    const ST* p = src + pull_segment<L, q, base, QT>(g, y, z, zwall);
#pragma unroll
    for (int k = 0; k < NPT; ++k) out[k][q] = Conv<ST, CT>::load(p[pull_lane<L, q, QT, NPT>(t, k, zwall)]);
  });
  if (wave_at_wall) {  // wave-uniform: this wave holds x = 0 or x = nx - 1
    static_for<0, L::Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      if constexpr (L::cx[q] != 0) {
        bool zwall;
        (void)pull_segment<L, q, base, QT>(g, y, z, zwall);
        const ST* po = src + bounce_segment<L, q, base, QT>(g, y, z);
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
          const CT b = Conv<ST, CT>::load(po[t.own[k]]);
          out[k][q] = x_wall<L, q>(g, t.x[k], zwall) ? b : out[k][q];
        }
      }
    });
  }
}

// ST: element type of the flow arrays; SS: of the scalar arrays (same
// element size, so one layout holds both).
template <class LF, class LS, int NPT, typename ST, typename CT, typename SS = ST>
__device__ __forceinline__ void gather_rows(const ST* __restrict__ src, const Grid& g,
                                            const TileLanes<LF::Q + LS::Q, NPT>& t, int y, int z,
                                            CT (&fg)[NPT][LF::Q], CT (&ph)[NPT][LS::Q]) {
  static_assert(sizeof(SS) == sizeof(ST), "flow and scalar elements must have one size");
  constexpr int QT = LF::Q + LS::Q;
  bool at_wall = false;
#pragma unroll
  for (int k = 0; k < NPT; ++k) at_wall = at_wall || t.x[k] == 0 || t.x[k] == g.nx - 1;
  const bool wave_at_wall = __builtin_amdgcn_ballot_w64(at_wall) != 0;
  pull_lattice<LF, 0, QT, NPT, ST, CT>(src, g, y, z, t, wave_at_wall, fg);
  pull_lattice<LS, LF::Q, QT, NPT, SS, CT>(reinterpret_cast<const SS*>(src), g, y, z, t,
                                           wave_at_wall, ph);
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
LBM_HD void gather(const ST* __restrict__ src, const Grid& g, int x, int y, int z, CT* fg, CT* ph) {
  static_assert(sizeof(SS) == sizeof(ST), "flow and scalar elements must have one size");
  constexpr int QT = LF::Q + LS::Q;
  static_for<0, LF::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    fg[q] = Conv<ST, CT>::load(*pull_ptr<LF, q, QT>(src, g, 0, x, y, z));
  });
  static_for<0, LS::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    ph[q] = Conv<SS, CT>::load(
        *reinterpret_cast<const SS*>(pull_ptr<LS, q, QT>(src, g, LF::Q, x, y, z)));
  });
}

}  // namespace lbm

// Host check of the x-blocked pull addressing of the step kernel: bounds of every load
// and store of the step kernel's tile geometry, and that the fix-up result
// equals the reference pull (pull_ptr) for every real node.
#include "lattice.h"
#include <cstdio>
#include <vector>
#include <set>
using namespace lbm;
static long fails = 0;
template <class LF, class LS, int NPT>
void check(int nx, int ny, int nz, int kBlock) {
  constexpr int QT = LF::Q + LS::Q;
  Grid g{nx, ny, nz, (int64_t)nx * ny * nz, xblocks(nx)};
  const int64_t total = (int64_t)ny * nz * g.nxb * QT * kXB;
  const int per_thread_x = (nx + NPT - 1) / NPT;
  const int bx = per_thread_x >= kBlock ? kBlock : ((per_thread_x + 63) / 64) * 64;
  const int nbx = (nx + bx * NPT - 1) / (bx * NPT);
  std::vector<char> stored(total, 0);
  // base of the reference pull's pointer arithmetic (never dereferenced)
  std::vector<float> buf(total + 1);
  const float* base0 = buf.data();
  for (int row = 0; row < ny * nz; ++row) {
    const int y = row % ny, z = row / ny;
    for (int tb = 0; tb < nbx; ++tb) {
      const int x0 = tb * bx * NPT;
      for (int tid = 0; tid < bx; ++tid) {
        if (x0 + tid >= nx) continue;  // early return
        auto t = tile_lanes<QT, NPT>(g, x0, tid, bx);
        auto pull = [&](auto lat_tag, auto base_tag) {
          using L = decltype(lat_tag);
          constexpr int base = decltype(base_tag)::value;
          static_for<0, L::Q>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            bool zw;
            const int64_t seg = pull_segment<L, q, base, QT>(g, y, z, zw);
            for (int k = 0; k < NPT; ++k) {
              int64_t idx = seg + pull_lane<L, q, QT, NPT>(t, k, zw);
              if (idx < 0 || idx >= total) { ++fails; if (fails < 10) printf("load OOB %d %d %d q%d k%d idx %lld\n", nx, ny, nz, q, k, (long long)idx); }
              const int64_t bidx = bounce_segment<L, q, base, QT>(g, y, z) + t.own[k];
              if (L::cx[q] != 0 && (bidx < 0 || bidx >= total)) { ++fails; printf("fixup OOB\n"); }
              if (t.x[k] < nx) {
                const int64_t eff = x_wall<L, q>(g, t.x[k], zw) ? bidx : idx;
                const float* ref = pull_ptr<L, q, QT>(base0, g, base, t.x[k], y, z);
                if ((int64_t)(ref - base0) != eff) { ++fails; if (fails < 10) printf("mismatch %d %d %d row %d x %d q %d\n", nx, ny, nz, row, t.x[k], q); }
              }
            }
          });
        };
        pull(LF{}, std::integral_constant<int, 0>{});
        pull(LS{}, std::integral_constant<int, LF::Q>{});
        // stores
        const int64_t rowbase = (int64_t)row * g.nxb * QT * kXB;
        for (int a = 0; a < QT; ++a)
          for (int k = 0; k < NPT; ++k) {
            if (!(k == 0 || t.x[k] < nx)) continue;
            const int64_t s = rowbase + a * kXB + t.own[k];
            if (s < 0 || s >= total) { ++fails; printf("store OOB\n"); continue; }
            if (s != elem_index<QT>(g, a, row, t.x[k])) { ++fails; printf("store index mismatch\n"); }
            if (stored[s]) { ++fails; if (fails < 10) printf("double store %d %d %d row %d x %d a %d\n", nx, ny, nz, row, t.x[k], a); }
            stored[s] = 1;
          }
      }
    }
  }
  // every real (a, node) stored exactly once
  long cnt = 0;
  for (char c : stored) cnt += c;
  if (cnt != (long)QT * nx * ny * nz) { ++fails; printf("store count %ld vs %ld (%d %d %d)\n", cnt, (long)QT * nx * ny * nz, nx, ny, nz); }
}
// The adjoint's reverse pull of lambda: pull_lattice on Rev<L> (the step
// kernel's segments and lane offsets with the velocities reversed) in the
// adjoint step's geometry (one node per thread), against the reverse pull
// written out here: population q at node x receives slot (q, x + c_q) when
// x + c_q is a fluid node (y periodic), else slot (opp q, x).
template <class L, int base, int QT>
void check_rev(int nx, int ny, int nz, int bx) {
  Grid g{nx, ny, nz, (int64_t)nx * ny * nz, xblocks(nx)};
  const int64_t total = (int64_t)ny * nz * g.nxb * QT * kXB;
  const int nbx = (nx + bx - 1) / bx;
  for (int row = 0; row < ny * nz; ++row) {
    const int y = row % ny, z = row / ny;
    for (int tb = 0; tb < nbx; ++tb)
      for (int tid = 0; tid < bx; ++tid) {
        const int x0 = tb * bx;
        auto t = tile_lanes<QT, 1>(g, x0, tid, bx);
        static_for<0, L::Q>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          bool zw;
          const int64_t seg = pull_segment<Rev<L>, q, base, QT>(g, y, z, zw);
          const int64_t idx = seg + pull_lane<Rev<L>, q, QT, 1>(t, 0, zw);
          const int64_t bidx = bounce_segment<Rev<L>, q, base, QT>(g, y, z) + t.own[0];
          if (idx < 0 || idx >= total || bidx < 0 || bidx >= total) {
            ++fails;
            if (fails < 10) printf("rev OOB %d %d %d q%d\n", nx, ny, nz, q);
          }
          const int x = t.x[0];
          if (x >= nx) return;  // lane past the row's end: result dropped
          const int64_t eff = x_wall<Rev<L>, q>(g, x, zw) ? bidx : idx;
          const int xn = x + L::cx[q], zn = z + L::cz[q];
          const int yn = ((y + L::cy[q]) % ny + ny) % ny;
          const bool fluid = xn >= 0 && xn < nx && zn >= 0 && zn < nz;
          const int64_t ref = fluid ? elem_index<QT>(g, base + q, (int64_t)zn * ny + yn, xn)
                                    : elem_index<QT>(g, base + opp<L>(q), (int64_t)row, x);
          if (eff != ref) {
            ++fails;
            if (fails < 10) printf("rev mismatch %d %d %d row %d x %d q %d\n", nx, ny, nz, row, x, q);
          }
        });
      }
  }
}

int main() {
  const int nxs[] = {1, 2, 5, 63, 64, 65, 127, 128, 129, 300, 513, 1024};
  const int ns[] = {1, 2, 3, 4};
  for (int nx : nxs)
    for (int ny : ns)
      for (int nz : ns) {
        check<Q27, Q7, 2>(nx, ny, nz, 256);
        check<Q19, Q6, 2>(nx, ny, nz, 256);
        check<Q19, Q6, 1>(nx, ny, nz, 256);
        check<Q27, Q27, 1>(nx, ny, nz, 256);
        check<Q27, Q7, 1>(nx, ny, nz, 64);
        for (int bx : {64, 256}) {
          check_rev<Q27, 0, 34>(nx, ny, nz, bx);
          check_rev<Q7, 27, 34>(nx, ny, nz, bx);
          check_rev<Q19, 0, 25>(nx, ny, nz, bx);
          check_rev<Q6, 19, 25>(nx, ny, nz, bx);
          check_rev<Q27, 27, 54>(nx, ny, nz, bx);
        }
      }
  printf("fails %ld\n", fails);
  return fails != 0;
}

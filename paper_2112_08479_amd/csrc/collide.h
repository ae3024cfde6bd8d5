// Local collision operators, written on deviations from the lattice rest
// state so that FP32 keeps the small quantities that drive the flow.
//
// Inputs per node: flow deviations g_q = f_q - w_q (g[]), scalar populations
// phi_p (ph[]). Outputs overwrite them with the post-collision values.
//
// Moments (Eq. 18-20, 27): drho = sum g (Eq. 52-53), rho = 1 + drho,
// j = sum c g, chi = sum phi, Boussinesq force F = (0, 0, -g' chi) (Eq. 11),
// velocity u = (j + F/2) / rho (Eq. 20).
//
// Cumulant model (Eq. 54-58): the cumulants of f / rho are those of its
// moment generating function; the first-order ones are the mean velocity
// j / rho (Eq. 57) and those of order >= 2 do not depend on the frame. The
// pre-collision cumulants are taken about the pre-collision mean j / rho, the
// post-collision populations are rebuilt about the post-collision mean
// (j + F) / rho, so density is conserved (Eq. 56) and the force enters as a
// momentum change of F. Second-order deviatoric cumulants relax with
// w1 = 1/tau_f (Eq. 58), the trace with omega_bulk towards 1 (= 3 cs^2),
// orders 3..6 with omega3..omega6 towards 0 (Eq. 55).
//
// The moment <-> population maps are done as three one-dimensional
// transforms (z, y, x) on quantities measured from their rest values
// K (1, 0, 1/3) so that nothing of size 1/3 is subtracted in FP32.
#pragma once

#include "lattice.h"

namespace lbm {

template <typename CT>
struct Phys {
  CT g;           // g'
  CT tau0;        // 3 nu0 + 1/2
  CT tau_phi0;    // 1/2 + D0 / cs_phi^2
  CT c_les;       // 18 sqrt(2) C_s^2 (18 sqrt(2) C_s for the closure as printed)
  CT d0;          // nu0 / Sc
  CT inv_sct;     // 1 / Sc_T
  CT inv_cs2phi;  // 1 / cs_phi^2
  CT omega2, omega3, omega4, omega5, omega6;
  // parametrised cumulant: third-order rates, fourth-order equilibrium
  // factors -(2/3)(1/omega1 - 1/2) A and -(1/3)(1/omega1 - 1/2) B, limiter
  // lambda (+inf: none)
  CT w_plus, w_minus, w_111, a4, b4, lam;
};

// one-dimensional rest central moments k_c and weights w(c), c = -1, 0, 1
LBM_HD constexpr double k1d(int a) { return a == 0 ? 1.0 : (a == 1 ? 0.0 : 1.0 / 3.0); }
LBM_HD constexpr double w1d(int i) { return i == 1 ? 2.0 / 3.0 : 1.0 / 6.0; }
// rest value of the central moment m[9a + 3b + c]: k_a k_b k_c
LBM_HD constexpr double rest_moment(int i) { return k1d(i / 9) * k1d((i / 3) % 3) * k1d(i % 3); }

// values t(-1), t(0), t(+1) of a triple whose rest values are K (1/6, 2/3, 1/6)
// -> central moments of order 0, 1, 2 about u, minus their rest values K (1, 0, 1/3)
template <typename CT>
LBM_HD void fwd1d(CT tm, CT t0, CT tp, CT u, CT K, CT& o0, CT& o1, CT& o2) {
  o0 = tm + t0 + tp;
  const CT A = K + o0;
  const CT d = tp - tm;
  o1 = d - u * A;
  o2 = (tp + tm) - CT(2) * u * d + u * u * A;
}

// inverse of fwd1d
template <typename CT>
LBM_HD void inv1d(CT o0, CT o1, CT o2, CT u, CT K, CT& tm, CT& t0, CT& tp) {
  const CT A = K + o0;
  const CT uu = u * u;
  t0 = o0 - o2 - CT(2) * u * o1 - uu * A;
  tp = CT(0.5) * (o2 + o1 * (CT(1) + CT(2) * u) + (uu + u) * A);
  tm = CT(0.5) * (o2 + o1 * (CT(2) * u - CT(1)) + (uu - u) * A);
}

// deviations g (population order) -> central-moment deviations m[9a+3b+c]
// about (ux, uy, uz)
template <typename CT>
LBM_HD void forward_chimera(const CT* g, CT ux, CT uy, CT uz, CT* m) {
  CT A[27], B[27];
  static_for<0, 9>([&](auto ic) {  // z: groups (cx, cy)
    constexpr int i = decltype(ic)::value, cxi = i / 3, cyi = i % 3;
    constexpr double K = w1d(cxi) * w1d(cyi);
    fwd1d<CT>(g[idx27(cxi - 1, cyi - 1, -1)], g[idx27(cxi - 1, cyi - 1, 0)],
              g[idx27(cxi - 1, cyi - 1, 1)], uz, CT(K), A[cxi * 9 + cyi * 3 + 0],
              A[cxi * 9 + cyi * 3 + 1], A[cxi * 9 + cyi * 3 + 2]);
  });
  static_for<0, 9>([&](auto ic) {  // y: groups (cx, c)
    constexpr int i = decltype(ic)::value, cxi = i / 3, c = i % 3;
    constexpr double K = w1d(cxi) * k1d(c);
    fwd1d<CT>(A[cxi * 9 + 0 + c], A[cxi * 9 + 3 + c], A[cxi * 9 + 6 + c], uy, CT(K),
              B[cxi * 9 + 0 + c], B[cxi * 9 + 3 + c], B[cxi * 9 + 6 + c]);
  });
  static_for<0, 9>([&](auto ic) {  // x: groups (b, c)
    constexpr int i = decltype(ic)::value, b = i / 3, c = i % 3;
    constexpr double K = k1d(b) * k1d(c);
    fwd1d<CT>(B[0 + b * 3 + c], B[9 + b * 3 + c], B[18 + b * 3 + c], ux, CT(K),
              m[0 + b * 3 + c], m[9 + b * 3 + c], m[18 + b * 3 + c]);
  });
}

// central-moment deviations m[9a+3b+c] about (ux, uy, uz) -> deviations g
template <typename CT>
LBM_HD void inverse_chimera(const CT* m, CT ux, CT uy, CT uz, CT* g) {
  CT A[27], B[27];
  static_for<0, 9>([&](auto ic) {  // x: groups (b, c)
    constexpr int i = decltype(ic)::value, b = i / 3, c = i % 3;
    constexpr double K = k1d(b) * k1d(c);
    inv1d<CT>(m[0 + b * 3 + c], m[9 + b * 3 + c], m[18 + b * 3 + c], ux, CT(K),
              B[0 + b * 3 + c], B[9 + b * 3 + c], B[18 + b * 3 + c]);
  });
  static_for<0, 9>([&](auto ic) {  // y: groups (cx, c)
    constexpr int i = decltype(ic)::value, cxi = i / 3, c = i % 3;
    constexpr double K = w1d(cxi) * k1d(c);
    inv1d<CT>(B[cxi * 9 + 0 + c], B[cxi * 9 + 3 + c], B[cxi * 9 + 6 + c], uy, CT(K),
              A[cxi * 9 + 0 + c], A[cxi * 9 + 3 + c], A[cxi * 9 + 6 + c]);
  });
  static_for<0, 9>([&](auto ic) {  // z: groups (cx, cy)
    constexpr int i = decltype(ic)::value, cxi = i / 3, cyi = i % 3;
    constexpr double K = w1d(cxi) * w1d(cyi);
    inv1d<CT>(A[cxi * 9 + cyi * 3 + 0], A[cxi * 9 + cyi * 3 + 1], A[cxi * 9 + cyi * 3 + 2], uz,
              CT(K), g[idx27(cxi - 1, cyi - 1, -1)], g[idx27(cxi - 1, cyi - 1, 0)],
              g[idx27(cxi - 1, cyi - 1, 1)]);
  });
}

// Smagorinsky total relaxation time from q2 = |Pi_neq|^2 / rho^2:
// tau_f = (tau0 + sqrt(tau0^2 + 18 sqrt(2) C_s^2 sqrt(Q) / rho)) / 2
// (Eq. 32-34 in the standard form nu_T = (C_s Delta)^2 |S|, Delta = 1).
template <typename CT>
LBM_HD CT smagorinsky_tau(CT q2, const Phys<CT>& p) {
  return CT(0.5) * (p.tau0 + sqrt(p.tau0 * p.tau0 + p.c_les * sqrt(q2)));
}

// v[B] + ... + v[E-1] summed as a balanced binary tree: the rounding error of
// the sum grows with log2(E - B) instead of E - B.
template <int B, int E, typename CT>
LBM_HD CT tree_sum(const CT* v) {
  if constexpr (E - B == 1) {
    return v[B];
  } else {
    constexpr int M = (B + E) / 2;
    return tree_sum<B, M>(v) + tree_sum<M, E>(v);
  }
}

// Scalar BGK (Eq. 28-29): phi* = phi - (phi - w chi (1 + c.u / cs_phi^2)) / tau_phi,
// tau_phi = 1/2 + (D0 + nu_T / Sc_T) / cs_phi^2 (Eq. 30, 35), nu_T = (tau_f - tau0)/3.
template <class LS, bool LES, typename CT>
LBM_HD void collide_scalar(CT* ph, CT chi, CT ux, CT uy, CT uz, CT tau, const Phys<CT>& p) {
  CT tau_phi = p.tau_phi0;
  if constexpr (LES) {
    const CT nu_t = (tau - p.tau0) * CT(1.0 / 3.0);
    tau_phi = CT(0.5) + (p.d0 + nu_t * p.inv_sct) * p.inv_cs2phi;
  }
  const CT wphi = CT(1) / tau_phi;
  CT neq[LS::Q];
  static_for<0, LS::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int cx = LS::cx[q], cy = LS::cy[q], cz = LS::cz[q];
    CT cu = CT(0);
    if (cx) cu += CT(cx) * ux;
    if (cy) cu += CT(cy) * uy;
    if (cz) cu += CT(cz) * uz;
    const CT peq = CT(weight<LS>(q)) * chi * (CT(1) + cu * p.inv_cs2phi);
    neq[q] = ph[q] - peq;
  });
  // D3Q6 weights of 1/6 are not exact in binary: rounded, they sum to
  // 1 + 3e-8 in FP32, and with 1/tau_phi near 2 every collision would raise chi
  // by about 6e-8 of itself. The non-equilibrium parts sum to zero exactly
  // (the equilibria sum to chi), so their mean is removed; it leaves the
  // flux (sum c neq, c in +- pairs) and, before rounding, every value
  // unchanged. (D3Q7's weights 1/4 and 1/8 are exact.)
  if constexpr (!LS::has_rest) {
    const CT mean = tree_sum<0, LS::Q>(neq) * CT(1.0 / LS::Q);
    static_for<0, LS::Q>([&](auto qc) { neq[decltype(qc)::value] -= mean; });
  }
  static_for<0, LS::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    ph[q] = ph[q] - wphi * neq[q];
  });
}

// Factorized-central-moment scalar on D3Q27 (Eq. 37-51). The moments of Eq. 39
// are taken about the fluid velocity u; chi (Eq. 40) is conserved, the
// first-order moments relax with omega_100 = 1/tau_phi (Eq. 50-51:
// D = (1/omega_100 - 1/2)/3, tau_phi as for the BGK scalar), and every other
// factorized moment is relaxed with rate 1 to its zero equilibrium. Undoing
// the factorization (Eq. 44-49) then leaves the post-collision central moments
//   chi E + K_x F_x + K_y F_y + K_z F_z,
// with E = e (x) e (x) e, e = (1, 0, 1/3) per axis, F_x = f (x) e (x) e,
// f = (0, 1, 0), and K = (1 - omega_100)(j_phi - chi u) the relaxed first
// moments. The inverse of Eq. 39 is a product of one-dimensional inverses, so
//   phi*_ijk = chi P_x(i) P_y(j) P_z(k) + K_x Q_x(i) P_y(j) P_z(k) + ...
// where P (central moments e about u) and Q (central moments f about u) are
//   P(-1) = (1/3 + u^2 - u)/2, P(0) = 2/3 - u^2, P(+1) = (1/3 + u^2 + u)/2,
//   Q(-1) = u - 1/2,           Q(0) = -2u,       Q(+1) = u + 1/2.
template <bool LES, typename CT>
LBM_HD void collide_fcm27(CT* ph, CT chi, CT ux, CT uy, CT uz, CT tau, const Phys<CT>& p) {
  CT tau_phi = p.tau_phi0;
  if constexpr (LES) {
    const CT nu_t = (tau - p.tau0) * CT(1.0 / 3.0);
    tau_phi = CT(0.5) + (p.d0 + nu_t * p.inv_sct) * p.inv_cs2phi;
  }
  const CT a1 = CT(1) - CT(1) / tau_phi;
  CT jx = CT(0), jy = CT(0), jz = CT(0);
  static_for<0, 27>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    if (Q27::cx[q]) jx += CT(Q27::cx[q]) * ph[q];
    if (Q27::cy[q]) jy += CT(Q27::cy[q]) * ph[q];
    if (Q27::cz[q]) jz += CT(Q27::cz[q]) * ph[q];
  });
  const CT kx = a1 * (jx - chi * ux), ky = a1 * (jy - chi * uy), kz = a1 * (jz - chi * uz);
  CT P[3][3], Qv[3][3];  // [axis][c + 1]
  const CT uu[3] = {ux, uy, uz};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const CT u = uu[d];
    const CT s = CT(1.0 / 3.0) + u * u;
    P[d][0] = CT(0.5) * (s - u);
    P[d][1] = CT(1) - s;
    P[d][2] = CT(0.5) * (s + u);
    Qv[d][0] = u - CT(0.5);
    Qv[d][1] = CT(-2) * u;
    Qv[d][2] = u + CT(0.5);
  }
  // The moving populations from the closed form; the rest population takes
  // what the others leave of chi (their tree sum), so that the sum is chi up
  // to a few unbiased roundings. In FP32 the rounded factors do not sum to
  // exactly 1 -- at u = 0, fl(1 - fl(1/3)) + 2 fl(1/6) = 1 - 3e-8 -- and the
  // closed-form rest value would lose about 1e-7 of chi per step near rest.
  static_for<1, 27>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int i = Q27::cx[q] + 1, j = Q27::cy[q] + 1, k = Q27::cz[q] + 1;
    ph[q] = P[1][j] * P[2][k] * (chi * P[0][i] + kx * Qv[0][i]) +
            P[0][i] * (ky * Qv[1][j] * P[2][k] + kz * P[1][j] * Qv[2][k]);
  });
  static_assert(Q27::cx[0] == 0 && Q27::cy[0] == 0 && Q27::cz[0] == 0, "rest population first");
  ph[0] = chi - tree_sum<1, 27>(ph);
}

// scalar collision of the scalar lattice LS: BGK on D3Q7 / D3Q6, factorized
// central moments on D3Q27
template <class LS, bool LES, typename CT>
LBM_HD void scalar_collision(CT* ph, CT chi, CT ux, CT uy, CT uz, CT tau, const Phys<CT>& p) {
  if constexpr (LS::Q == 27)
    collide_fcm27<LES, CT>(ph, chi, ux, uy, uz, tau, p);
  else
    collide_scalar<LS, LES, CT>(ph, chi, ux, uy, uz, tau, p);
}

// Flow moments of the deviations: drho, j, and raw second moments Pi^g.
// drho and j are tree sums (their rounding feeds the stored state every step;
// adding the exact zeros of the c = 0 terms changes nothing).
template <class L, typename CT>
LBM_HD void flow_moments(const CT* g, CT& drho, CT& jx, CT& jy, CT& jz, CT& pxx, CT& pyy,
                         CT& pzz, CT& pxy, CT& pxz, CT& pyz) {
  CT tx[L::Q], ty[L::Q], tz[L::Q];
  pxx = pyy = pzz = pxy = pxz = pyz = CT(0);
  static_for<0, L::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int cx = L::cx[q], cy = L::cy[q], cz = L::cz[q];
    const CT v = g[q];
    tx[q] = cx == 0 ? CT(0) : (cx > 0 ? v : -v);
    ty[q] = cy == 0 ? CT(0) : (cy > 0 ? v : -v);
    tz[q] = cz == 0 ? CT(0) : (cz > 0 ? v : -v);
    if (cx) pxx += v;
    if (cy) pyy += v;
    if (cz) pzz += v;
    if (cx * cy) pxy += CT(cx * cy) * v;
    if (cx * cz) pxz += CT(cx * cz) * v;
    if (cy * cz) pyz += CT(cy * cz) * v;
  });
  drho = tree_sum<0, L::Q>(g);
  jx = tree_sum<0, L::Q>(tx);
  jy = tree_sum<0, L::Q>(ty);
  jz = tree_sum<0, L::Q>(tz);
}

template <class L, typename CT>
LBM_HD CT scalar_sum(const CT* ph) {
  return tree_sum<0, L::Q>(ph);
}

// Relaxation of the second-order cumulant deviations D = C - delta/3
// (deviatoric part with w1, trace with omega2 towards 0).
template <typename CT>
LBM_HD void relax_second(CT a1, CT omega2, CT& xx, CT& yy, CT& zz, CT& xy, CT& xz, CT& yz) {
  const CT T3 = (xx + yy + zz) * CT(1.0 / 3.0);
  const CT Ts3 = (CT(1) - omega2) * T3;
  xx = Ts3 + a1 * (xx - T3);
  yy = Ts3 + a1 * (yy - T3);
  zz = Ts3 + a1 * (zz - T3);
  xy = a1 * xy;
  xz = a1 * xz;
  yz = a1 * yz;
}

// ---- cumulant collision, omega3..omega6 = 1 (every cumulant above second
// order is reset to its equilibrium value 0): only the second-order
// cumulants are needed; they come from the raw second moments. LS: the
// scalar lattice (D3Q7 BGK or D3Q27 factorized central moments).
template <class LS, bool LES, typename CT>
LBM_HD void collide_cumulant27(CT* g, CT* ph, const Phys<CT>& p, CT* tau_out = nullptr) {
  CT drho, jx, jy, jz, pxx, pyy, pzz, pxy, pxz, pyz;
  flow_moments<Q27>(g, drho, jx, jy, jz, pxx, pyy, pzz, pxy, pxz, pyz);
  const CT chi = scalar_sum<LS>(ph);
  const CT rho = CT(1) + drho;
  const CT irho = CT(1) / rho;
  const CT Fz = -p.g * chi;
  const CT ux = jx * irho, uy = jy * irho, uz = jz * irho;  // pre-collision mean
  const CT third = CT(1.0 / 3.0);
  // D = C - delta/3, C = Pi / rho - mean mean (Pi = delta/3 + Pi^g)
  CT dxx = (pxx - drho * third) * irho - ux * ux;
  CT dyy = (pyy - drho * third) * irho - uy * uy;
  CT dzz = (pzz - drho * third) * irho - uz * uz;
  CT dxy = pxy * irho - ux * uy;
  CT dxz = pxz * irho - ux * uz;
  CT dyz = pyz * irho - uy * uz;
  CT tau = p.tau0;
  if constexpr (LES) {
    const CT q2 = dxx * dxx + dyy * dyy + dzz * dzz + CT(2) * (dxy * dxy + dxz * dxz + dyz * dyz);
    tau = smagorinsky_tau(q2, p);
  }
  if (tau_out) *tau_out = tau;
  const CT a1 = CT(1) - CT(1) / tau;
  relax_second(a1, p.omega2, dxx, dyy, dzz, dxy, dxz, dyz);
  // post-collision central moments about the post-collision mean: Gaussian
  // (Wick) moments of the relaxed covariance, as deviations from rest
  CT m[27];
  static_for<0, 27>([&](auto ic) { m[decltype(ic)::value] = CT(0); });
  const CT ninth = CT(1.0 / 9.0);
  m[0] = drho;
  m[18] = rho * dxx + drho * third;
  m[6] = rho * dyy + drho * third;
  m[2] = rho * dzz + drho * third;
  m[12] = rho * dxy;
  m[10] = rho * dxz;
  m[4] = rho * dyz;
  m[24] = rho * ((dxx + dyy) * third + dxx * dyy + CT(2) * dxy * dxy) + drho * ninth;
  m[20] = rho * ((dxx + dzz) * third + dxx * dzz + CT(2) * dxz * dxz) + drho * ninth;
  m[8] = rho * ((dyy + dzz) * third + dyy * dzz + CT(2) * dyz * dyz) + drho * ninth;
  m[22] = rho * ((third + dxx) * dyz + CT(2) * dxy * dxz);
  m[16] = rho * ((third + dyy) * dxz + CT(2) * dxy * dyz);
  m[14] = rho * ((third + dzz) * dxy + CT(2) * dxz * dyz);
  m[26] = rho * ((dxx + dyy + dzz) * ninth + (dxx * dyy + dxx * dzz + dyy * dzz) * third +
                 dxx * dyy * dzz +
                 CT(2) * ((third + dxx) * dyz * dyz + (third + dyy) * dxz * dxz +
                          (third + dzz) * dxy * dxy) +
                 CT(8) * dxy * dxz * dyz) +
          drho * CT(1.0 / 27.0);
  inverse_chimera<CT>(m, ux, uy, (jz + Fz) * irho, g);
  scalar_collision<LS, LES>(ph, chi, ux, uy, (jz + CT(0.5) * Fz) * irho, tau, p);
}

// Third-order limiter of the parametrised cumulant: 1 - (limited rate) for
// the quantity X, (1 - w)(1 - q) with q = |X| / (|X| + lambda) (also
// returned); lambda = +inf gives q = 0. In FP32 the quotient takes the
// hardware reciprocal (1 ulp), which only scales a small third-order
// quantity.
template <typename CT>
LBM_HD CT third_order_keep(CT w, CT X, CT lam, CT& q) {
  const CT a = X < CT(0) ? -X : X;
  if constexpr (sizeof(CT) == 4)
    q = a * __builtin_amdgcn_rcpf(a + lam);
  else
    q = a / (a + lam);
  return (CT(1) - w) * (CT(1) - q);
}

// Third-order central moments (= cumulants) of f / rho from the deviations g,
// for the parametrised cumulant: raw sums r_abc = sum_q cx^a cy^b cz^c g_q
// (the rest state's vanish), then E[(X-a)(Y-b)^2] = E[X Y^2] - a var(Y)
// - 2 b cov(X,Y) - a b^2 with var(Y) = 1/3 + D_yy, and
// E[(X-a)(Y-b)(Z-c)] = E[XYZ] - a cov(Y,Z) - b cov(X,Z) - c cov(X,Y) - abc.
// Order of r and k: 120, 102, 210, 012, 201, 021, 111.
template <typename CT>
LBM_HD void third_raw_sums(const CT* g, CT (&r)[7]) {
#pragma unroll
  for (int i = 0; i < 7; ++i) r[i] = CT(0);
  static_for<0, 27>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int cx = Q27::cx[q], cy = Q27::cy[q], cz = Q27::cz[q];
    const CT v = g[q];
    if (cx && cy) r[0] += cx > 0 ? v : -v;
    if (cx && cz) r[1] += cx > 0 ? v : -v;
    if (cx && cy) r[2] += cy > 0 ? v : -v;
    if (cy && cz) r[3] += cy > 0 ? v : -v;
    if (cx && cz) r[4] += cz > 0 ? v : -v;
    if (cy && cz) r[5] += cz > 0 ? v : -v;
    if (cx && cy && cz) r[6] += (cx * cy * cz) > 0 ? v : -v;
  });
}

template <typename CT>
LBM_HD void third_central(const CT (&r)[7], CT ir, CT ux, CT uy, CT uz, CT dxx, CT dyy, CT dzz,
                          CT dxy, CT dxz, CT dyz, CT (&k)[7]) {
  const CT third = CT(1.0 / 3.0);
  k[0] = r[0] * ir - ux * (third + dyy) - CT(2) * uy * dxy - ux * uy * uy;
  k[1] = r[1] * ir - ux * (third + dzz) - CT(2) * uz * dxz - ux * uz * uz;
  k[2] = r[2] * ir - uy * (third + dxx) - CT(2) * ux * dxy - uy * ux * ux;
  k[3] = r[3] * ir - uy * (third + dzz) - CT(2) * uz * dyz - uy * uz * uz;
  k[4] = r[4] * ir - uz * (third + dxx) - CT(2) * ux * dxz - uz * ux * ux;
  k[5] = r[5] * ir - uz * (third + dyy) - CT(2) * uy * dyz - uz * uy * uy;
  k[6] = r[6] * ir - ux * dyz - uy * dxz - uz * dxy - ux * uy * uz;
}

// post-collision cumulants of orders 3..6 (of f / rho, zero mean)
template <typename CT>
struct HighCumulants {
  CT c210, c201, c120, c021, c102, c012, c111;
  CT c220, c202, c022, c211, c121, c112;
  CT c221, c212, c122, c222;
};

// Post-collision populations from the relaxed second-order deviations
// D = C - delta/3 (dxx..dyz) and the cumulants of orders 3..6: moments about
// the post-collision mean from cumulants (zero mean), as deviations from the
// rest values, then the inverse chimera transform.
template <typename CT>
LBM_HD void rebuild_from_cumulants(CT* g, CT drho, CT rho, CT dxx, CT dyy, CT dzz, CT dxy, CT dxz,
                                   CT dyz, const HighCumulants<CT>& c, CT ux, CT uy, CT uz) {
  const CT third = CT(1.0 / 3.0), ninth = CT(1.0 / 9.0);
  CT m[27];
  m[0] = drho;
  m[1] = m[3] = m[9] = CT(0);
  auto put = [&](int i, CT dev, double K) { m[i] = rho * dev + drho * CT(K); };
  put(18, dxx, 1.0 / 3.0);
  put(6, dyy, 1.0 / 3.0);
  put(2, dzz, 1.0 / 3.0);
  put(12, dxy, 0);
  put(10, dxz, 0);
  put(4, dyz, 0);
  put(21, c.c210, 0);
  put(19, c.c201, 0);
  put(15, c.c120, 0);
  put(7, c.c021, 0);
  put(11, c.c102, 0);
  put(5, c.c012, 0);
  put(13, c.c111, 0);
  put(24, c.c220 + (dxx + dyy) * third + dxx * dyy + CT(2) * dxy * dxy, 1.0 / 9.0);
  put(20, c.c202 + (dxx + dzz) * third + dxx * dzz + CT(2) * dxz * dxz, 1.0 / 9.0);
  put(8, c.c022 + (dyy + dzz) * third + dyy * dzz + CT(2) * dyz * dyz, 1.0 / 9.0);
  put(22, c.c211 + (third + dxx) * dyz + CT(2) * dxy * dxz, 0);
  put(16, c.c121 + (third + dyy) * dxz + CT(2) * dxy * dyz, 0);
  put(14, c.c112 + (third + dzz) * dxy + CT(2) * dxz * dyz, 0);
  put(25, c.c221 + (third + dxx) * c.c021 + (third + dyy) * c.c201 + CT(4) * dxy * c.c111 +
              CT(2) * dxz * c.c120 + CT(2) * dyz * c.c210,
      0);
  put(23, c.c212 + (third + dxx) * c.c012 + (third + dzz) * c.c210 + CT(4) * dxz * c.c111 +
              CT(2) * dxy * c.c102 + CT(2) * dyz * c.c201,
      0);
  put(17, c.c122 + (third + dyy) * c.c102 + (third + dzz) * c.c120 + CT(4) * dyz * c.c111 +
              CT(2) * dxy * c.c012 + CT(2) * dxz * c.c021,
      0);
  const CT m222s =
      c.c222 + (third + dxx) * c.c022 + (third + dyy) * c.c202 + (third + dzz) * c.c220 +
      CT(4) * (dxy * c.c112 + dxz * c.c121 + dyz * c.c211) +
      CT(2) * (c.c210 * c.c012 + c.c201 * c.c021 + c.c120 * c.c102) + CT(4) * c.c111 * c.c111 +
      (dxx + dyy + dzz) * ninth + (dxx * dyy + dxx * dzz + dyy * dzz) * third + dxx * dyy * dzz +
      CT(2) * ((third + dxx) * dyz * dyz + (third + dyy) * dxz * dxz + (third + dzz) * dxy * dxy) +
      CT(8) * dxy * dxz * dyz;
  put(26, m222s, 1.0 / 27.0);
  inverse_chimera<CT>(m, ux, uy, uz, g);
}

// ---- cumulant collision with general rates omega3..omega6.
template <class LS, bool LES, typename CT>
LBM_HD void collide_cumulant27_general(CT* g, CT* ph, const Phys<CT>& p) {
  CT drho = CT(0), jx = CT(0), jy = CT(0), jz = CT(0);
  static_for<0, 27>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    const CT v = g[q];
    drho += v;
    if (Q27::cx[q]) jx += CT(Q27::cx[q]) * v;
    if (Q27::cy[q]) jy += CT(Q27::cy[q]) * v;
    if (Q27::cz[q]) jz += CT(Q27::cz[q]) * v;
  });
  const CT chi = scalar_sum<LS>(ph);
  const CT rho = CT(1) + drho;
  const CT irho = CT(1) / rho;
  const CT Fz = -p.g * chi;
  const CT ux = jx * irho, uy = jy * irho, uz = jz * irho;
  CT k[27];
  forward_chimera<CT>(g, ux, uy, uz, k);
  // mu = m - K: normalised central moments about the mean minus rest values;
  // the first-order central moments about the mean vanish
  const CT third = CT(1.0 / 3.0), ninth = CT(1.0 / 9.0);
  auto mu = [&](int i, double K) { return (k[i] - drho * CT(K)) * irho; };
  const CT m200 = mu(18, 1.0 / 3.0), m020 = mu(6, 1.0 / 3.0), m002 = mu(2, 1.0 / 3.0);
  const CT m110 = mu(12, 0), m101 = mu(10, 0), m011 = mu(4, 0);
  const CT m210 = mu(21, 0), m201 = mu(19, 0), m120 = mu(15, 0), m021 = mu(7, 0);
  const CT m102 = mu(11, 0), m012 = mu(5, 0), m111 = mu(13, 0);
  const CT m220 = mu(24, 1.0 / 9.0), m202 = mu(20, 1.0 / 9.0), m022 = mu(8, 1.0 / 9.0);
  const CT m211 = mu(22, 0), m121 = mu(16, 0), m112 = mu(14, 0);
  const CT m221 = mu(25, 0), m212 = mu(23, 0), m122 = mu(17, 0);
  const CT m222 = mu(26, 1.0 / 27.0);
  // cumulants (zero mean) from moments, as deviations from the rest values
  CT dxx = m200, dyy = m020, dzz = m002, dxy = m110, dxz = m101, dyz = m011;
  const CT c220 = m220 - (m200 + m020) * third - m200 * m020 - CT(2) * m110 * m110;
  const CT c202 = m202 - (m200 + m002) * third - m200 * m002 - CT(2) * m101 * m101;
  const CT c022 = m022 - (m020 + m002) * third - m020 * m002 - CT(2) * m011 * m011;
  const CT c211 = m211 - (third + m200) * m011 - CT(2) * m110 * m101;
  const CT c121 = m121 - (third + m020) * m101 - CT(2) * m110 * m011;
  const CT c112 = m112 - (third + m002) * m110 - CT(2) * m101 * m011;
  const CT c221 = m221 - (third + m200) * m021 - (third + m020) * m201 - CT(4) * m110 * m111 -
                  CT(2) * m101 * m120 - CT(2) * m011 * m210;
  const CT c212 = m212 - (third + m200) * m012 - (third + m002) * m210 - CT(4) * m101 * m111 -
                  CT(2) * m110 * m102 - CT(2) * m011 * m201;
  const CT c122 = m122 - (third + m020) * m102 - (third + m002) * m120 - CT(4) * m011 * m111 -
                  CT(2) * m110 * m012 - CT(2) * m101 * m021;
  const CT s1 = m200 + m020 + m002;
  const CT c222 =
      m222 + s1 * ninth - (m022 + m202 + m220) * third -
      (m200 * m022 + m020 * m202 + m002 * m220) -
      CT(4) * (m110 * m112 + m101 * m121 + m011 * m211) -
      CT(2) * (m210 * m012 + m201 * m021 + m120 * m102) - CT(4) * m111 * m111 +
      CT(2.0 / 3.0) * (m200 * m020 + m200 * m002 + m020 * m002) + CT(2) * m200 * m020 * m002 +
      CT(4) * ((third + m200) * m011 * m011 + (third + m020) * m101 * m101 +
               (third + m002) * m110 * m110) +
      CT(16) * m110 * m101 * m011;
  CT tau = p.tau0;
  if constexpr (LES) {
    const CT q2 = dxx * dxx + dyy * dyy + dzz * dzz + CT(2) * (dxy * dxy + dxz * dxz + dyz * dyz);
    tau = smagorinsky_tau(q2, p);
  }
  const CT a1 = CT(1) - CT(1) / tau;
  relax_second(a1, p.omega2, dxx, dyy, dzz, dxy, dxz, dyz);
  const CT a3 = CT(1) - p.omega3, a4 = CT(1) - p.omega4, a5 = CT(1) - p.omega5,
           a6 = CT(1) - p.omega6;
  HighCumulants<CT> c;
  c.c210 = a3 * m210, c.c201 = a3 * m201, c.c120 = a3 * m120, c.c021 = a3 * m021;
  c.c102 = a3 * m102, c.c012 = a3 * m012, c.c111 = a3 * m111;
  c.c220 = a4 * c220, c.c202 = a4 * c202, c.c022 = a4 * c022;
  c.c211 = a4 * c211, c.c121 = a4 * c121, c.c112 = a4 * c112;
  c.c221 = a5 * c221, c.c212 = a5 * c212, c.c122 = a5 * c122;
  c.c222 = a6 * c222;
  rebuild_from_cumulants<CT>(g, drho, rho, dxx, dyy, dzz, dxy, dxz, dyz, c, ux, uy, (jz + Fz) * irho);
  scalar_collision<LS, LES>(ph, chi, ux, uy, (jz + CT(0.5) * Fz) * irho, tau, p);
}

// ---- the parametrised cumulant of Geier, Pasquali and Schoenherr (2017) that
// the paper's VirtualFluids runs apply (Sec. 2.3), without the LES:
//   third order: the sums C_120 + C_102 (and permutations) relax with w_plus,
//     the differences with w_minus, C_111 with w_111, each limited to
//     w + (1 - w)|X| / (|X| + lambda) for its own quantity X;
//   fourth order: rate 1 onto equilibria proportional to the velocity
//     gradients, estimated from the pre-collision second-order cumulants at
//     first Chapman-Enskog order (non-equilibrium part of C_ab =
//     -(d_a u_b + d_b u_a) / (3 w), w = omega1 deviatoric, omega_bulk trace);
//   fifth and sixth order: rate 1 towards 0.
// Only the second- and third-order pre-collision cumulants are needed; they
// come from raw sums of the deviations (the third-order raw moments of the
// rest state vanish) instead of the full forward transform.
template <class LS, typename CT>
LBM_HD void collide_cumulant27_param(CT* g, CT* ph, const Phys<CT>& p) {
  CT drho, jx, jy, jz, pxx, pyy, pzz, pxy, pxz, pyz;
  flow_moments<Q27>(g, drho, jx, jy, jz, pxx, pyy, pzz, pxy, pxz, pyz);
  CT r3[7];
  third_raw_sums<CT>(g, r3);
  const CT chi = scalar_sum<LS>(ph);
  const CT rho = CT(1) + drho;
  const CT irho = CT(1) / rho;
  const CT Fz = -p.g * chi;
  const CT ux = jx * irho, uy = jy * irho, uz = jz * irho;  // pre-collision mean
  const CT third = CT(1.0 / 3.0);
  // second-order central deviations D = C - delta/3 (normalised by rho)
  CT dxx = (pxx - drho * third) * irho - ux * ux;
  CT dyy = (pyy - drho * third) * irho - uy * uy;
  CT dzz = (pzz - drho * third) * irho - uz * uz;
  CT dxy = pxy * irho - ux * uy;
  CT dxz = pxz * irho - ux * uz;
  CT dyz = pyz * irho - uy * uz;
  // third-order central moments (= cumulants)
  CT k3[7];
  third_central<CT>(r3, irho, ux, uy, uz, dxx, dyy, dzz, dxy, dxz, dyz, k3);
  const CT k120 = k3[0], k102 = k3[1], k210 = k3[2], k012 = k3[3], k201 = k3[4], k021 = k3[5],
           k111 = k3[6];
  // velocity gradients from the pre-collision second-order cumulants
  const CT w1 = CT(1) / p.tau0;
  const CT div = CT(-1.5) * p.omega2 * (dxx + dyy + dzz);
  const CT dxy_d = CT(-1.5) * w1 * (dxx - dyy), dxz_d = CT(-1.5) * w1 * (dxx - dzz);
  const CT dxux = (div + dxy_d + dxz_d) * third;
  const CT dyuy = dxux - dxy_d, dzuz = dxux - dxz_d;
  HighCumulants<CT> c;
  c.c220 = p.a4 * (dxux + dyuy);
  c.c202 = p.a4 * (dxux + dzuz);
  c.c022 = p.a4 * (dyuy + dzuz);
  c.c112 = p.b4 * (CT(-3) * w1 * dxy);
  c.c121 = p.b4 * (CT(-3) * w1 * dxz);
  c.c211 = p.b4 * (CT(-3) * w1 * dyz);
  c.c221 = c.c212 = c.c122 = c.c222 = CT(0);
  // third order, limited
  auto keep = [&](CT w, CT X) {
    CT q;
    return third_order_keep(w, X, p.lam, q);
  };
  auto pair = [&](CT a, CT b, CT& oa, CT& ob) {
    CT s = a + b, d = a - b;
    s *= keep(p.w_plus, s);
    d *= keep(p.w_minus, d);
    oa = CT(0.5) * (s + d);
    ob = CT(0.5) * (s - d);
  };
  pair(k120, k102, c.c120, c.c102);
  pair(k210, k012, c.c210, c.c012);
  pair(k201, k021, c.c201, c.c021);
  c.c111 = keep(p.w_111, k111) * k111;
  relax_second(CT(1) - w1, p.omega2, dxx, dyy, dzz, dxy, dxz, dyz);
  rebuild_from_cumulants<CT>(g, drho, rho, dxx, dyy, dzz, dxy, dxz, dyz, c, ux, uy, (jz + Fz) * irho);
  scalar_collision<LS, false>(ph, chi, ux, uy, (jz + CT(0.5) * Fz) * irho, p.tau0, p);
}

// ---- D3Q19 BGK with Guo forcing (Eq. 21-26), Smagorinsky (Eq. 32-35),
// D3Q6 scalar. Pi_neq = sum c c (f - f_eq) = Pi^g - drho I/3 - rho u u.
template <bool LES, typename CT>
LBM_HD void collide_bgk_q19_q6(CT* g, CT* ph, const Phys<CT>& p, CT* tau_out = nullptr) {
  CT drho, jx, jy, jz, pxx, pyy, pzz, pxy, pxz, pyz;
  flow_moments<Q19>(g, drho, jx, jy, jz, pxx, pyy, pzz, pxy, pxz, pyz);
  const CT chi = scalar_sum<Q6>(ph);
  const CT rho = CT(1) + drho;
  const CT irho = CT(1) / rho;
  const CT Fz = -p.g * chi;
  const CT ux = jx * irho, uy = jy * irho, uz = (jz + CT(0.5) * Fz) * irho;
  CT tau = p.tau0;
  if constexpr (LES) {
    const CT t3 = drho * CT(1.0 / 3.0);
    const CT nxx = pxx - t3 - rho * ux * ux, nyy = pyy - t3 - rho * uy * uy,
             nzz = pzz - t3 - rho * uz * uz;
    const CT nxy = pxy - rho * ux * uy, nxz = pxz - rho * ux * uz, nyz = pyz - rho * uy * uz;
    const CT Q = nxx * nxx + nyy * nyy + nzz * nzz + CT(2) * (nxy * nxy + nxz * nxz + nyz * nyz);
    tau = CT(0.5) * (p.tau0 + sqrt(p.tau0 * p.tau0 + p.c_les * sqrt(Q) * irho));
  }
  if (tau_out) *tau_out = tau;
  const CT w = CT(1) / tau;
  const CT usq = ux * ux + uy * uy + uz * uz;
  const CT sfac = CT(1) - CT(0.5) * w;
  static_for<0, 19>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int cx = Q19::cx[q], cy = Q19::cy[q], cz = Q19::cz[q];
    constexpr double W = weight<Q19>(q);
    CT cu = CT(0);
    if (cx) cu += CT(cx) * ux;
    if (cy) cu += CT(cy) * uy;
    if (cz) cu += CT(cz) * uz;
    const CT geq = CT(W) * (drho + rho * (CT(3) * cu + CT(4.5) * cu * cu - CT(1.5) * usq));
    const CT S = sfac * CT(W) * (CT(3) * (CT(cz) - uz) * Fz + CT(9) * cu * CT(cz) * Fz);
    g[q] = g[q] - w * (g[q] - geq) + S;
  });
  collide_scalar<Q6, LES>(ph, chi, ux, uy, uz, tau, p);
}

}  // namespace lbm

// Reverse-mode derivative (vector-Jacobian product) of the local collisions
// in collide.h, written out by hand: given the pre-collision deviations g,
// scalar populations ph and the adjoints mg, mp of the post-collision values,
// return the adjoints gb, pb of the inputs and accumulate the adjoints of the
// parameters c_les = 18 sqrt(2) C_s^2 (18 sqrt(2) C_s for the Smagorinsky
// closure as printed) and inv_sct = 1 / Sc_T.
//
// Each function first recomputes the forward quantities it needs, in the
// order of the forward code, then runs the chain rule backwards through them.
// The cumulant version covers omega3..omega6 = 1 (every cumulant above
// second order reset to 0). Non-smooth points: sqrt(Q) at Q = 0 takes the
// zero subgradient.
#pragma once

#include "collide.h"

namespace lbm {


// adjoint of inv1d (linear in o2, so o2's own value is not needed)
template <typename CT>
LBM_HD void inv1d_vjp(CT o0, CT o1, CT /*o2*/, CT u, CT K, CT btm, CT bt0, CT btp, CT& bo0, CT& bo1,
                      CT& bo2, CT& bu) {
  const CT A = K + o0, uu = u * u;
  bo0 = bt0 * (CT(1) - uu) + CT(0.5) * (btp * (uu + u) + btm * (uu - u));
  bo1 = -CT(2) * u * bt0 + CT(0.5) * (btp * (CT(1) + CT(2) * u) + btm * (CT(2) * u - CT(1)));
  bo2 = -bt0 + CT(0.5) * (btp + btm);
  bu += bt0 * (-CT(2) * o1 - CT(2) * u * A) + CT(0.5) * btp * (CT(2) * o1 + (CT(2) * u + CT(1)) * A) +
        CT(0.5) * btm * (CT(2) * o1 + (CT(2) * u - CT(1)) * A);
}

// output S of inv1d alone (0: t(-1), 1: t(0), 2: t(+1))
template <int S, typename CT>
LBM_HD CT inv1d_one(CT o0, CT o1, CT o2, CT u, CT K) {
  const CT A = K + o0, uu = u * u;
  if constexpr (S == 1)
    return o0 - o2 - CT(2) * u * o1 - uu * A;
  else if constexpr (S == 2)
    return CT(0.5) * (o2 + o1 * (CT(1) + CT(2) * u) + (uu + u) * A);
  else
    return CT(0.5) * (o2 + o1 * (CT(2) * u - CT(1)) + (uu - u) * A);
}

// adjoint of output S of inv1d alone: adds bt's contribution to bo0, bo1,
// bo2 and bu (the three outputs' terms of inv1d_vjp, one at a time)
template <int S, typename CT>
LBM_HD void inv1d_one_vjp(CT o0, CT o1, CT u, CT K, CT bt, CT& bo0, CT& bo1, CT& bo2, CT& bu) {
  const CT A = K + o0, uu = u * u;
  if constexpr (S == 1) {
    bo0 += bt * (CT(1) - uu);
    bo1 += -CT(2) * u * bt;
    bo2 += -bt;
    bu += bt * (-CT(2) * o1 - CT(2) * u * A);
  } else if constexpr (S == 2) {
    bo0 += CT(0.5) * bt * (uu + u);
    bo1 += CT(0.5) * bt * (CT(1) + CT(2) * u);
    bo2 += CT(0.5) * bt;
    bu += CT(0.5) * bt * (CT(2) * o1 + (CT(2) * u + CT(1)) * A);
  } else {
    bo0 += CT(0.5) * bt * (uu - u);
    bo1 += CT(0.5) * bt * (CT(2) * u - CT(1));
    bo2 += CT(0.5) * bt;
    bu += CT(0.5) * bt * (CT(2) * o1 + (CT(2) * u - CT(1)) * A);
  }
}

// adjoint of inverse_chimera: gb (population order) -> mb[9a+3b+c] and the
// adjoints of the three velocity components. The transform is taken one
// x-velocity slab (c_x = -1, 0, +1) at a time: the slab's nine x-pass values
// and its y pass are recomputed from m, its z and y passes are reversed, and
// its share of the reversed x pass is added to mb. Only one slab's
// intermediates are live at once (the x pass is linear in each output).
template <typename CT>
LBM_HD void inverse_chimera_vjp(const CT* m, CT ux, CT uy, CT uz, const CT* gbar, CT* mb, CT& bux,
                                CT& buy, CT& buz) {
  static_for<0, 27>([&](auto ic) { mb[decltype(ic)::value] = CT(0); });
  static_for<0, 3>([&](auto sc) {
    constexpr int cxi = decltype(sc)::value;
    CT Bs[9], As[9], Abs[9], Bbs[9];
    static_for<0, 9>([&](auto ic) {  // forward x pass, this slab's output
      constexpr int i = decltype(ic)::value, b = i / 3, c = i % 3;
      constexpr double K = k1d(b) * k1d(c);
      Bs[i] = inv1d_one<cxi, CT>(m[i], m[9 + i], m[18 + i], ux, CT(K));
    });
    static_for<0, 3>([&](auto cc) {  // forward y pass
      constexpr int c = decltype(cc)::value;
      constexpr double K = w1d(cxi) * k1d(c);
      inv1d<CT>(Bs[c], Bs[3 + c], Bs[6 + c], uy, CT(K), As[c], As[3 + c], As[6 + c]);
    });
    static_for<0, 3>([&](auto yc) {  // reverse z pass
      constexpr int cyi = decltype(yc)::value;
      constexpr double K = w1d(cxi) * w1d(cyi);
      const int o = cyi * 3;
      inv1d_vjp<CT>(As[o], As[o + 1], As[o + 2], uz, CT(K), gbar[idx27(cxi - 1, cyi - 1, -1)],
                    gbar[idx27(cxi - 1, cyi - 1, 0)], gbar[idx27(cxi - 1, cyi - 1, 1)], Abs[o],
                    Abs[o + 1], Abs[o + 2], buz);
    });
    static_for<0, 3>([&](auto cc) {  // reverse y pass
      constexpr int c = decltype(cc)::value;
      constexpr double K = w1d(cxi) * k1d(c);
      inv1d_vjp<CT>(Bs[c], Bs[3 + c], Bs[6 + c], uy, CT(K), Abs[c], Abs[3 + c], Abs[6 + c], Bbs[c],
                    Bbs[3 + c], Bbs[6 + c], buy);
    });
    static_for<0, 9>([&](auto ic) {  // this slab's share of the reverse x pass
      constexpr int i = decltype(ic)::value, b = i / 3, c = i % 3;
      constexpr double K = k1d(b) * k1d(c);
      inv1d_one_vjp<cxi, CT>(m[i], m[9 + i], ux, CT(K), Bbs[i], mb[i], mb[9 + i], mb[18 + i], bux);
    });
  });
}

// adjoint of collide_scalar. Inputs: forward values; mp = adjoint of phi*.
// Outputs: pb (set), and accumulates bchi, bu*, btau and b_isct.
template <class LS, bool LES, typename CT>
LBM_HD void scalar_vjp(const CT* ph, CT chi, CT ux, CT uy, CT uz, CT tau, const Phys<CT>& p,
                       const CT* mp, CT* pb, CT& bchi, CT& bux, CT& buy, CT& buz, CT& btau,
                       CT& b_isct) {
  CT tau_phi = p.tau_phi0;
  if constexpr (LES) {
    const CT nu_t = (tau - p.tau0) * CT(1.0 / 3.0);
    tau_phi = CT(0.5) + (p.d0 + nu_t * p.inv_sct) * p.inv_cs2phi;
  }
  const CT wphi = CT(1) / tau_phi;
  CT bwphi = CT(0);
  static_for<0, LS::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int cx = LS::cx[q], cy = LS::cy[q], cz = LS::cz[q];
    constexpr double W = weight<LS>(q);
    CT cu = CT(0);
    if (cx) cu += CT(cx) * ux;
    if (cy) cu += CT(cy) * uy;
    if (cz) cu += CT(cz) * uz;
    const CT e = CT(W) * (CT(1) + cu * p.inv_cs2phi);
    pb[q] = (CT(1) - wphi) * mp[q];
    bwphi += mp[q] * (e * chi - ph[q]);
    bchi += mp[q] * wphi * e;
    const CT t = mp[q] * wphi * CT(W) * chi * p.inv_cs2phi;
    if (cx) bux += CT(cx) * t;
    if (cy) buy += CT(cy) * t;
    if (cz) buz += CT(cz) * t;
  });
  if constexpr (LES) {
    const CT btp = -bwphi / (tau_phi * tau_phi);
    btau += btp * p.inv_cs2phi * p.inv_sct * CT(1.0 / 3.0);
    b_isct += btp * p.inv_cs2phi * (tau - p.tau0) * CT(1.0 / 3.0);
  }
}

// adjoint of collide_fcm27 (the closed form with the rest closure). Inputs:
// forward values; mp = adjoint of phi*. Outputs: pb (set), and accumulates
// bchi, bu*, btau and b_isct.
template <bool LES, typename CT>
LBM_HD void fcm27_vjp(const CT* ph, CT chi, CT ux, CT uy, CT uz, CT tau, const Phys<CT>& p,
                      const CT* mp, CT* pb, CT& bchi, CT& bux, CT& buy, CT& buz, CT& btau,
                      CT& b_isct) {
  // forward recompute
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
  const CT uu[3] = {ux, uy, uz};
  const CT dj[3] = {jx - chi * ux, jy - chi * uy, jz - chi * uz};
  const CT k[3] = {a1 * dj[0], a1 * dj[1], a1 * dj[2]};
  CT P[3][3], Qv[3][3];
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
  // reverse: phi*_0 = chi - sum of the others
  const CT m0 = mp[0];
  bchi += m0;
  CT bP[3][3], bQ[3][3], bk[3] = {CT(0), CT(0), CT(0)};
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int c = 0; c < 3; ++c) bP[d][c] = bQ[d][c] = CT(0);
  static_for<1, 27>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int i = Q27::cx[q] + 1, j = Q27::cy[q] + 1, l = Q27::cz[q] + 1;
    const CT m = mp[q] - m0;
    const CT px = P[0][i], py = P[1][j], pz = P[2][l];
    const CT qx = Qv[0][i], qy = Qv[1][j], qz = Qv[2][l];
    bchi += m * px * py * pz;
    bk[0] += m * qx * py * pz;
    bk[1] += m * px * qy * pz;
    bk[2] += m * px * py * qz;
    bP[0][i] += m * (chi * py * pz + k[1] * qy * pz + k[2] * py * qz);
    bP[1][j] += m * (chi * px * pz + k[0] * qx * pz + k[2] * px * qz);
    bP[2][l] += m * (chi * px * py + k[0] * qx * py + k[1] * px * qy);
    bQ[0][i] += m * k[0] * py * pz;
    bQ[1][j] += m * k[1] * px * pz;
    bQ[2][l] += m * k[2] * px * py;
  });
  // P(c) and Q(c) as functions of u: dP/du = (u - 1/2, -2u, u + 1/2), dQ/du = (1, -2, 1)
  CT bu[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const CT u = uu[d];
    bu[d] = bP[d][0] * (u - CT(0.5)) + bP[d][1] * (CT(-2) * u) + bP[d][2] * (u + CT(0.5)) +
            bQ[d][0] - CT(2) * bQ[d][1] + bQ[d][2];
  }
  // k_d = a1 (j_d - chi u_d)
  CT ba1 = CT(0), bj[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    ba1 += bk[d] * dj[d];
    bj[d] = a1 * bk[d];
    bchi += -a1 * uu[d] * bk[d];
    bu[d] += -a1 * chi * bk[d];
  }
  bux += bu[0];
  buy += bu[1];
  buz += bu[2];
  static_for<0, 27>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    CT v = CT(0);
    if (Q27::cx[q]) v += CT(Q27::cx[q]) * bj[0];
    if (Q27::cy[q]) v += CT(Q27::cy[q]) * bj[1];
    if (Q27::cz[q]) v += CT(Q27::cz[q]) * bj[2];
    pb[q] = v;
  });
  if constexpr (LES) {
    const CT btp = ba1 / (tau_phi * tau_phi);
    btau += btp * p.inv_cs2phi * p.inv_sct * CT(1.0 / 3.0);
    b_isct += btp * p.inv_cs2phi * (tau - p.tau0) * CT(1.0 / 3.0);
  }
}

// scalar collision adjoint of the scalar lattice LS (BGK or FCM)
template <class LS, bool LES, typename CT>
LBM_HD void scalar_collision_vjp(const CT* ph, CT chi, CT ux, CT uy, CT uz, CT tau,
                                 const Phys<CT>& p, const CT* mp, CT* pb, CT& bchi, CT& bux,
                                 CT& buy, CT& buz, CT& btau, CT& b_isct) {
  if constexpr (LS::Q == 27)
    fcm27_vjp<LES, CT>(ph, chi, ux, uy, uz, tau, p, mp, pb, bchi, bux, buy, buz, btau, b_isct);
  else
    scalar_vjp<LS, LES, CT>(ph, chi, ux, uy, uz, tau, p, mp, pb, bchi, bux, buy, buz, btau, b_isct);
}

template <class L, typename CT>
LBM_HD void flow_moments_vjp(CT bdrho, CT bjx, CT bjy, CT bjz, CT bpxx, CT bpyy, CT bpzz, CT bpxy,
                             CT bpxz, CT bpyz, CT* gb) {
  static_for<0, L::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int cx = L::cx[q], cy = L::cy[q], cz = L::cz[q];
    CT v = bdrho;
    if (cx) v += CT(cx) * bjx + bpxx;
    if (cy) v += CT(cy) * bjy + bpyy;
    if (cz) v += CT(cz) * bjz + bpzz;
    if (cx * cy) v += CT(cx * cy) * bpxy;
    if (cx * cz) v += CT(cx * cz) * bpxz;
    if (cy * cz) v += CT(cy * cz) * bpyz;
    gb[q] += v;
  });
}

// ---- cumulant D3Q27 + scalar lattice LS (D3Q7 BGK or D3Q27 FCM),
// omega3..omega6 = 1
template <class LS, bool LES, typename CT>
LBM_HD void vjp_cumulant27(const CT* g, const CT* ph, const CT* mg, const CT* mp,
                           const Phys<CT>& p, CT* gb, CT* pb, CT& b_cles, CT& b_isct) {
  // ---- forward recompute
  CT drho, jx, jy, jz, pxx, pyy, pzz, pxy, pxz, pyz;
  flow_moments<Q27>(g, drho, jx, jy, jz, pxx, pyy, pzz, pxy, pxz, pyz);
  const CT chi = scalar_sum<LS>(ph);
  const CT rho = CT(1) + drho;
  const CT ir = CT(1) / rho;
  const CT Fz = -p.g * chi;
  const CT ux = jx * ir, uy = jy * ir, uz = jz * ir;
  const CT third = CT(1.0 / 3.0), ninth = CT(1.0 / 9.0);
  const CT dxx = (pxx - drho * third) * ir - ux * ux;
  const CT dyy = (pyy - drho * third) * ir - uy * uy;
  const CT dzz = (pzz - drho * third) * ir - uz * uz;
  const CT dxy = pxy * ir - ux * uy;
  const CT dxz = pxz * ir - ux * uz;
  const CT dyz = pyz * ir - uy * uz;
  CT tau = p.tau0, s = CT(0), R = CT(0);
  if constexpr (LES) {
    const CT q2 = dxx * dxx + dyy * dyy + dzz * dzz + CT(2) * (dxy * dxy + dxz * dxz + dyz * dyz);
    s = sqrt(q2);
    R = sqrt(p.tau0 * p.tau0 + p.c_les * s);
    tau = CT(0.5) * (p.tau0 + R);
  }
  const CT a1 = CT(1) - CT(1) / tau;
  // d tau / d s = c_les / (4 R) (zero subgradient of sqrt(Q) at Q = 0), over s:
  // formed here, unconditionally, so that the reverse sweep has no branch
  const CT cbs = (LES && s > CT(0)) ? p.c_les / (CT(4) * R * s) : CT(0);
  CT exx = dxx, eyy = dyy, ezz = dzz, exy = dxy, exz = dxz, eyz = dyz;
  relax_second(a1, p.omega2, exx, eyy, ezz, exy, exz, eyz);
  const CT T3 = (dxx + dyy + dzz) * third;
  const CT vz = (jz + Fz) * ir;
  CT m[27];
  static_for<0, 27>([&](auto ic) { m[decltype(ic)::value] = CT(0); });
  const CT W24 = (exx + eyy) * third + exx * eyy + CT(2) * exy * exy;
  const CT W20 = (exx + ezz) * third + exx * ezz + CT(2) * exz * exz;
  const CT W8 = (eyy + ezz) * third + eyy * ezz + CT(2) * eyz * eyz;
  const CT W22 = (third + exx) * eyz + CT(2) * exy * exz;
  const CT W16 = (third + eyy) * exz + CT(2) * exy * eyz;
  const CT W14 = (third + ezz) * exy + CT(2) * exz * eyz;
  const CT W26 = (exx + eyy + ezz) * ninth + (exx * eyy + exx * ezz + eyy * ezz) * third +
                 exx * eyy * ezz +
                 CT(2) * ((third + exx) * eyz * eyz + (third + eyy) * exz * exz +
                          (third + ezz) * exy * exy) +
                 CT(8) * exy * exz * eyz;
  m[0] = drho;
  m[18] = rho * exx + drho * third;
  m[6] = rho * eyy + drho * third;
  m[2] = rho * ezz + drho * third;
  m[12] = rho * exy;
  m[10] = rho * exz;
  m[4] = rho * eyz;
  m[24] = rho * W24 + drho * ninth;
  m[20] = rho * W20 + drho * ninth;
  m[8] = rho * W8 + drho * ninth;
  m[22] = rho * W22;
  m[16] = rho * W16;
  m[14] = rho * W14;
  m[26] = rho * W26 + drho * CT(1.0 / 27.0);
  const CT uzs = (jz + CT(0.5) * Fz) * ir;  // scalar velocity (Eq. 20)

  // ---- reverse
  CT bchi = CT(0), bux = CT(0), buy = CT(0), buz = CT(0), btau = CT(0);
  CT buzs = CT(0);
  scalar_collision_vjp<LS, LES, CT>(ph, chi, ux, uy, uzs, tau, p, mp, pb, bchi, bux, buy, buzs, btau,
                                    b_isct);
  CT mb[27];
  CT bvz = CT(0);
  inverse_chimera_vjp<CT>(m, ux, uy, vz, mg, mb, bux, buy, bvz);
  CT brho = CT(0), bdrho = CT(0);
  CT bexx = CT(0), beyy = CT(0), bezz = CT(0), bexy = CT(0), bexz = CT(0), beyz = CT(0);
  bdrho += mb[0];
  brho += mb[18] * exx + mb[6] * eyy + mb[2] * ezz + mb[12] * exy + mb[10] * exz + mb[4] * eyz;
  bdrho += (mb[18] + mb[6] + mb[2]) * third;
  bexx += mb[18] * rho;
  beyy += mb[6] * rho;
  bezz += mb[2] * rho;
  bexy += mb[12] * rho;
  bexz += mb[10] * rho;
  beyz += mb[4] * rho;
  brho += mb[24] * W24 + mb[20] * W20 + mb[8] * W8 + mb[22] * W22 + mb[16] * W16 + mb[14] * W14 +
          mb[26] * W26;
  bdrho += (mb[24] + mb[20] + mb[8]) * ninth + mb[26] * CT(1.0 / 27.0);
  {
    const CT r24 = mb[24] * rho, r20 = mb[20] * rho, r8 = mb[8] * rho;
    bexx += r24 * (third + eyy) + r20 * (third + ezz);
    beyy += r24 * (third + exx) + r8 * (third + ezz);
    bezz += r20 * (third + exx) + r8 * (third + eyy);
    bexy += r24 * CT(4) * exy;
    bexz += r20 * CT(4) * exz;
    beyz += r8 * CT(4) * eyz;
    const CT r22 = mb[22] * rho, r16 = mb[16] * rho, r14 = mb[14] * rho;
    bexx += r22 * eyz;
    beyz += r22 * (third + exx);
    bexy += r22 * CT(2) * exz;
    bexz += r22 * CT(2) * exy;
    beyy += r16 * exz;
    bexz += r16 * (third + eyy);
    bexy += r16 * CT(2) * eyz;
    beyz += r16 * CT(2) * exy;
    bezz += r14 * exy;
    bexy += r14 * (third + ezz);
    bexz += r14 * CT(2) * eyz;
    beyz += r14 * CT(2) * exz;
    const CT r26 = mb[26] * rho;
    bexx += r26 * (ninth + (eyy + ezz) * third + eyy * ezz + CT(2) * eyz * eyz);
    beyy += r26 * (ninth + (exx + ezz) * third + exx * ezz + CT(2) * exz * exz);
    bezz += r26 * (ninth + (exx + eyy) * third + exx * eyy + CT(2) * exy * exy);
    bexy += r26 * (CT(4) * (third + ezz) * exy + CT(8) * exz * eyz);
    bexz += r26 * (CT(4) * (third + eyy) * exz + CT(8) * exy * eyz);
    beyz += r26 * (CT(4) * (third + exx) * eyz + CT(8) * exy * exz);
  }
  // relaxation
  const CT ba1 = bexx * (dxx - T3) + beyy * (dyy - T3) + bezz * (dzz - T3) + bexy * dxy + bexz * dxz +
                 beyz * dyz;
  const CT bT3 = ((CT(1) - p.omega2) - a1) * (bexx + beyy + bezz);
  CT bdxx = a1 * bexx + bT3 * third, bdyy = a1 * beyy + bT3 * third, bdzz = a1 * bezz + bT3 * third;
  CT bdxy = a1 * bexy, bdxz = a1 * bexz, bdyz = a1 * beyz;
  btau += ba1 / (tau * tau);
  if constexpr (LES) {
    b_cles += btau * s / (CT(4) * R);
    const CT bs = btau * cbs;
    bdxx += bs * dxx;
    bdyy += bs * dyy;
    bdzz += bs * dzz;
    bdxy += bs * CT(2) * dxy;
    bdxz += bs * CT(2) * dxz;
    bdyz += bs * CT(2) * dyz;
  }
  // D from raw moments
  CT bpxx = bdxx * ir, bpyy = bdyy * ir, bpzz = bdzz * ir;
  CT bpxy = bdxy * ir, bpxz = bdxz * ir, bpyz = bdyz * ir;
  bdrho -= (bdxx + bdyy + bdzz) * ir * third;
  CT bir = bdxx * (pxx - drho * third) + bdyy * (pyy - drho * third) + bdzz * (pzz - drho * third) +
           bdxy * pxy + bdxz * pxz + bdyz * pyz;
  bux -= CT(2) * ux * bdxx + uy * bdxy + uz * bdxz;
  buy -= CT(2) * uy * bdyy + ux * bdxy + uz * bdyz;
  buz -= CT(2) * uz * bdzz + ux * bdxz + uy * bdyz;
  // velocities
  CT bjx = bux * ir, bjy = buy * ir, bjz = buz * ir;
  bir += bux * jx + buy * jy + buz * jz;
  bjz += bvz * ir + buzs * ir;
  CT bFz = bvz * ir + buzs * ir * CT(0.5);
  bir += bvz * (jz + Fz) + buzs * (jz + CT(0.5) * Fz);
  bchi += -p.g * bFz;
  brho += -bir * ir * ir;
  bdrho += brho;
  static_for<0, LS::Q>([&](auto qc) { pb[decltype(qc)::value] += bchi; });
  static_for<0, 27>([&](auto qc) { gb[decltype(qc)::value] = CT(0); });
  flow_moments_vjp<Q27, CT>(bdrho, bjx, bjy, bjz, bpxx, bpyy, bpzz, bpxy, bpxz, bpyz, gb);
}

// ---- parametrised cumulant D3Q27 (no LES) + scalar lattice LS: the
// derivative of collide_cumulant27_param. The limited third-order map
// X -> X (1 - w)(1 - |X| / (|X| + lambda)) has the derivative
// (1 - w)(1 - q)^2, q = |X| / (|X| + lambda), which is smooth at X = 0.
// Without the LES the scalar collision's adjoint and the flow's reverse
// sweep meet only in additive accumulators (the velocity and chi adjoints),
// so the scalar part runs last: the caller passes chi = sum of ph, and
// reload(ph, mp) fills the scalar populations and their adjoints only when
// they are needed, so that they need not be held through the flow part.
template <class LS, typename CT, class Reload>
LBM_HD void vjp_cumulant27_param(const CT* g, CT chi, const CT* mg, Reload&& reload,
                                 const Phys<CT>& p, CT* gb, CT* pb, CT& b_isct) {
  // ---- forward recompute (as collide_cumulant27_param)
  CT drho, jx, jy, jz, pxx, pyy, pzz, pxy, pxz, pyz;
  flow_moments<Q27>(g, drho, jx, jy, jz, pxx, pyy, pzz, pxy, pxz, pyz);
  CT r3[7];
  third_raw_sums<CT>(g, r3);
  const CT r120 = r3[0], r102 = r3[1], r210 = r3[2], r012 = r3[3], r201 = r3[4], r021 = r3[5],
           r111 = r3[6];
  const CT rho = CT(1) + drho;
  const CT ir = CT(1) / rho;
  const CT Fz = -p.g * chi;
  const CT ux = jx * ir, uy = jy * ir, uz = jz * ir;
  const CT third = CT(1.0 / 3.0), ninth = CT(1.0 / 9.0);
  const CT dxx = (pxx - drho * third) * ir - ux * ux;
  const CT dyy = (pyy - drho * third) * ir - uy * uy;
  const CT dzz = (pzz - drho * third) * ir - uz * uz;
  const CT dxy = pxy * ir - ux * uy;
  const CT dxz = pxz * ir - ux * uz;
  const CT dyz = pyz * ir - uy * uz;
  CT kc[7];
  third_central<CT>(r3, ir, ux, uy, uz, dxx, dyy, dzz, dxy, dxz, dyz, kc);
  const CT k120 = kc[0], k102 = kc[1], k210 = kc[2], k012 = kc[3], k201 = kc[4], k021 = kc[5],
           k111 = kc[6];
  const CT w1 = CT(1) / p.tau0;
  const CT div = CT(-1.5) * p.omega2 * (dxx + dyy + dzz);
  const CT dxy_d = CT(-1.5) * w1 * (dxx - dyy), dxz_d = CT(-1.5) * w1 * (dxx - dzz);
  const CT dxux = (div + dxy_d + dxz_d) * third;
  const CT dyuy = dxux - dxy_d, dzuz = dxux - dxz_d;
  const CT C220 = p.a4 * (dxux + dyuy), C202 = p.a4 * (dxux + dzuz), C022 = p.a4 * (dyuy + dzuz);
  const CT C112 = p.b4 * (CT(-3) * w1 * dxy), C121 = p.b4 * (CT(-3) * w1 * dxz),
           C211 = p.b4 * (CT(-3) * w1 * dyz);
  // third-order pairs: keep factors and q of the sums and differences
  CT qs[3], qd[3], ks[3], kd[3], sv[3], dv[3];
  const CT ka[3] = {k120, k210, k201}, kb[3] = {k102, k012, k021};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    sv[i] = ka[i] + kb[i];
    dv[i] = ka[i] - kb[i];
    ks[i] = third_order_keep(p.w_plus, sv[i], p.lam, qs[i]);
    kd[i] = third_order_keep(p.w_minus, dv[i], p.lam, qd[i]);
  }
  CT q111;
  const CT k3 = third_order_keep(p.w_111, k111, p.lam, q111);
  const CT C120 = CT(0.5) * (sv[0] * ks[0] + dv[0] * kd[0]), C102 = CT(0.5) * (sv[0] * ks[0] - dv[0] * kd[0]);
  const CT C210 = CT(0.5) * (sv[1] * ks[1] + dv[1] * kd[1]), C012 = CT(0.5) * (sv[1] * ks[1] - dv[1] * kd[1]);
  const CT C201 = CT(0.5) * (sv[2] * ks[2] + dv[2] * kd[2]), C021 = CT(0.5) * (sv[2] * ks[2] - dv[2] * kd[2]);
  const CT C111 = k3 * k111;
  const CT a1 = CT(1) - w1;
  CT exx = dxx, eyy = dyy, ezz = dzz, exy = dxy, exz = dxz, eyz = dyz;
  relax_second(a1, p.omega2, exx, eyy, ezz, exy, exz, eyz);
  const CT W24 = (exx + eyy) * third + exx * eyy + CT(2) * exy * exy;
  const CT W20 = (exx + ezz) * third + exx * ezz + CT(2) * exz * exz;
  const CT W8 = (eyy + ezz) * third + eyy * ezz + CT(2) * eyz * eyz;
  const CT W22 = (third + exx) * eyz + CT(2) * exy * exz;
  const CT W16 = (third + eyy) * exz + CT(2) * exy * eyz;
  const CT W14 = (third + ezz) * exy + CT(2) * exz * eyz;
  const CT W26 = (exx + eyy + ezz) * ninth + (exx * eyy + exx * ezz + eyy * ezz) * third +
                 exx * eyy * ezz +
                 CT(2) * ((third + exx) * eyz * eyz + (third + eyy) * exz * exz +
                          (third + ezz) * exy * exy) +
                 CT(8) * exy * exz * eyz;
  // moments about the post-collision mean, as deviations from rest (the
  // same as rebuild_from_cumulants with orders 5 and 6 at 0)
  CT dev[27];
  static_for<0, 27>([&](auto ic) { dev[decltype(ic)::value] = CT(0); });
  dev[18] = exx, dev[6] = eyy, dev[2] = ezz, dev[12] = exy, dev[10] = exz, dev[4] = eyz;
  dev[21] = C210, dev[19] = C201, dev[15] = C120, dev[7] = C021, dev[11] = C102, dev[5] = C012;
  dev[13] = C111;
  dev[24] = C220 + W24, dev[20] = C202 + W20, dev[8] = C022 + W8;
  dev[22] = C211 + W22, dev[16] = C121 + W16, dev[14] = C112 + W14;
  dev[25] = (third + exx) * C021 + (third + eyy) * C201 + CT(4) * exy * C111 + CT(2) * exz * C120 +
            CT(2) * eyz * C210;
  dev[23] = (third + exx) * C012 + (third + ezz) * C210 + CT(4) * exz * C111 + CT(2) * exy * C102 +
            CT(2) * eyz * C201;
  dev[17] = (third + eyy) * C102 + (third + ezz) * C120 + CT(4) * eyz * C111 + CT(2) * exy * C012 +
            CT(2) * exz * C021;
  dev[26] = (third + exx) * C022 + (third + eyy) * C202 + (third + ezz) * C220 +
            CT(4) * (exy * C112 + exz * C121 + eyz * C211) +
            CT(2) * (C210 * C012 + C201 * C021 + C120 * C102) + CT(4) * C111 * C111 + W26;
  CT m[27];
  m[0] = drho;
  m[1] = m[3] = m[9] = CT(0);
  static_for<1, 27>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    if constexpr (i != 1 && i != 3 && i != 9) m[i] = rho * dev[i] + drho * CT(rest_moment(i));
  });
  const CT vz = (jz + Fz) * ir;
  const CT uzs = (jz + CT(0.5) * Fz) * ir;

  // ---- reverse
  CT bchi = CT(0), bux = CT(0), buy = CT(0), buz = CT(0), buzs = CT(0);
  CT mb[27];
  CT bvz = CT(0);
  inverse_chimera_vjp<CT>(m, ux, uy, vz, mg, mb, bux, buy, bvz);
  CT brho = CT(0), bdrho = mb[0];
  CT r[27];
  static_for<1, 27>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    if constexpr (i != 1 && i != 3 && i != 9) {
      brho += mb[i] * dev[i];
      bdrho += mb[i] * CT(rest_moment(i));
      r[i] = mb[i] * rho;
    }
  });
  // cumulants of orders 3 and 4
  const CT bC210 = r[21] + r[25] * CT(2) * eyz + r[23] * (third + ezz) + r[26] * CT(2) * C012;
  const CT bC201 = r[19] + r[25] * (third + eyy) + r[23] * CT(2) * eyz + r[26] * CT(2) * C021;
  const CT bC120 = r[15] + r[25] * CT(2) * exz + r[17] * (third + ezz) + r[26] * CT(2) * C102;
  const CT bC021 = r[7] + r[25] * (third + exx) + r[17] * CT(2) * exz + r[26] * CT(2) * C201;
  const CT bC102 = r[11] + r[23] * CT(2) * exy + r[17] * (third + eyy) + r[26] * CT(2) * C120;
  const CT bC012 = r[5] + r[23] * (third + exx) + r[17] * CT(2) * exy + r[26] * CT(2) * C210;
  const CT bC111 = r[13] + CT(4) * (r[25] * exy + r[23] * exz + r[17] * eyz) + r[26] * CT(8) * C111;
  const CT bC220 = r[24] + r[26] * (third + ezz), bC202 = r[20] + r[26] * (third + eyy),
           bC022 = r[8] + r[26] * (third + exx);
  const CT bC211 = r[22] + r[26] * CT(4) * eyz, bC121 = r[16] + r[26] * CT(4) * exz,
           bC112 = r[14] + r[26] * CT(4) * exy;
  // relaxed second order: from the Wick parts and the products with C
  CT bexx = r[18] + r[25] * C021 + r[23] * C012 + r[26] * C022;
  CT beyy = r[6] + r[25] * C201 + r[17] * C102 + r[26] * C202;
  CT bezz = r[2] + r[23] * C210 + r[17] * C120 + r[26] * C220;
  CT bexy = r[12] + r[25] * CT(4) * C111 + r[23] * CT(2) * C102 + r[17] * CT(2) * C012 +
            r[26] * CT(4) * C112;
  CT bexz = r[10] + r[25] * CT(2) * C120 + r[23] * CT(4) * C111 + r[17] * CT(2) * C021 +
            r[26] * CT(4) * C121;
  CT beyz = r[4] + r[25] * CT(2) * C210 + r[23] * CT(2) * C201 + r[17] * CT(4) * C111 +
            r[26] * CT(4) * C211;
  {
    const CT r24 = r[24], r20 = r[20], r8 = r[8];
    bexx += r24 * (third + eyy) + r20 * (third + ezz);
    beyy += r24 * (third + exx) + r8 * (third + ezz);
    bezz += r20 * (third + exx) + r8 * (third + eyy);
    bexy += r24 * CT(4) * exy;
    bexz += r20 * CT(4) * exz;
    beyz += r8 * CT(4) * eyz;
    const CT r22 = r[22], r16 = r[16], r14 = r[14];
    bexx += r22 * eyz;
    beyz += r22 * (third + exx);
    bexy += r22 * CT(2) * exz;
    bexz += r22 * CT(2) * exy;
    beyy += r16 * exz;
    bexz += r16 * (third + eyy);
    bexy += r16 * CT(2) * eyz;
    beyz += r16 * CT(2) * exy;
    bezz += r14 * exy;
    bexy += r14 * (third + ezz);
    bexz += r14 * CT(2) * eyz;
    beyz += r14 * CT(2) * exz;
    const CT r26 = r[26];
    bexx += r26 * (ninth + (eyy + ezz) * third + eyy * ezz + CT(2) * eyz * eyz);
    beyy += r26 * (ninth + (exx + ezz) * third + exx * ezz + CT(2) * exz * exz);
    bezz += r26 * (ninth + (exx + eyy) * third + exx * eyy + CT(2) * exy * exy);
    bexy += r26 * (CT(4) * (third + ezz) * exy + CT(8) * exz * eyz);
    bexz += r26 * (CT(4) * (third + eyy) * exz + CT(8) * exy * eyz);
    beyz += r26 * (CT(4) * (third + exx) * eyz + CT(8) * exy * exz);
  }
  // relaxation of the second order (a1 fixed: no LES)
  const CT bT3 = ((CT(1) - p.omega2) - a1) * (bexx + beyy + bezz);
  CT bdxx = a1 * bexx + bT3 * third, bdyy = a1 * beyy + bT3 * third, bdzz = a1 * bezz + bT3 * third;
  CT bdxy = a1 * bexy, bdxz = a1 * bexz, bdyz = a1 * beyz;
  // fourth-order equilibria through the gradient estimates
  {
    const CT bdxux = p.a4 * (bC220 + bC202), bdyuy = p.a4 * (bC220 + bC022),
             bdzuz = p.a4 * (bC202 + bC022);
    const CT bsum = bdxux + bdyuy + bdzuz;         // adjoint of dxux through all three
    const CT bdxy_d = bsum * third - bdyuy, bdxz_d = bsum * third - bdzuz;
    const CT bdiv = bsum * third;
    bdxx += CT(-1.5) * p.omega2 * bdiv + CT(-1.5) * w1 * (bdxy_d + bdxz_d);
    bdyy += CT(-1.5) * p.omega2 * bdiv + CT(1.5) * w1 * bdxy_d;
    bdzz += CT(-1.5) * p.omega2 * bdiv + CT(1.5) * w1 * bdxz_d;
    bdxy += CT(-3) * w1 * p.b4 * bC112;
    bdxz += CT(-3) * w1 * p.b4 * bC121;
    bdyz += CT(-3) * w1 * p.b4 * bC211;
  }
  // third order through the limited pairs
  CT bka[3], bkb[3];
  const CT bCa[3] = {bC120, bC210, bC201}, bCb[3] = {bC102, bC012, bC021};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const CT bsp = CT(0.5) * (bCa[i] + bCb[i]), bdp = CT(0.5) * (bCa[i] - bCb[i]);
    const CT bs = bsp * (CT(1) - p.w_plus) * (CT(1) - qs[i]) * (CT(1) - qs[i]);
    const CT bd = bdp * (CT(1) - p.w_minus) * (CT(1) - qd[i]) * (CT(1) - qd[i]);
    bka[i] = bs + bd;
    bkb[i] = bs - bd;
  }
  const CT bk111 = bC111 * (CT(1) - p.w_111) * (CT(1) - q111) * (CT(1) - q111);
  // third-order central moments from the raw sums
  CT bir = CT(0);
  const CT bk120 = bka[0], bk102 = bkb[0], bk210 = bka[1], bk012 = bkb[1], bk201 = bka[2],
           bk021 = bkb[2];
  const CT br120 = bk120 * ir, br102 = bk102 * ir, br210 = bk210 * ir, br012 = bk012 * ir,
           br201 = bk201 * ir, br021 = bk021 * ir, br111 = bk111 * ir;
  bir += bk120 * r120 + bk102 * r102 + bk210 * r210 + bk012 * r012 + bk201 * r201 + bk021 * r021 +
         bk111 * r111;
  bux -= bk120 * (third + dyy + uy * uy) + bk102 * (third + dzz + uz * uz) +
         bk210 * CT(2) * (dxy + uy * ux) + bk201 * CT(2) * (dxz + uz * ux) + bk111 * (dyz + uy * uz);
  buy -= bk210 * (third + dxx + ux * ux) + bk012 * (third + dzz + uz * uz) +
         bk120 * CT(2) * (dxy + ux * uy) + bk021 * CT(2) * (dyz + uz * uy) + bk111 * (dxz + ux * uz);
  buz -= bk201 * (third + dxx + ux * ux) + bk021 * (third + dyy + uy * uy) +
         bk102 * CT(2) * (dxz + ux * uz) + bk012 * CT(2) * (dyz + uy * uz) + bk111 * (dxy + ux * uy);
  bdxx -= bk210 * uy + bk201 * uz;
  bdyy -= bk120 * ux + bk021 * uz;
  bdzz -= bk102 * ux + bk012 * uy;
  bdxy -= CT(2) * (bk120 * uy + bk210 * ux) + bk111 * uz;
  bdxz -= CT(2) * (bk102 * uz + bk201 * ux) + bk111 * uy;
  bdyz -= CT(2) * (bk012 * uz + bk021 * uy) + bk111 * ux;
  // D from raw moments
  CT bpxx = bdxx * ir, bpyy = bdyy * ir, bpzz = bdzz * ir;
  CT bpxy = bdxy * ir, bpxz = bdxz * ir, bpyz = bdyz * ir;
  bdrho -= (bdxx + bdyy + bdzz) * ir * third;
  bir += bdxx * (pxx - drho * third) + bdyy * (pyy - drho * third) + bdzz * (pzz - drho * third) +
         bdxy * pxy + bdxz * pxz + bdyz * pyz;
  bux -= CT(2) * ux * bdxx + uy * bdxy + uz * bdxz;
  buy -= CT(2) * uy * bdyy + ux * bdxy + uz * bdyz;
  buz -= CT(2) * uz * bdzz + ux * bdxz + uy * bdyz;
  // the scalar collision
  {
    CT phr[LS::Q], mpr[LS::Q], btau = CT(0);
    reload(phr, mpr);
    scalar_collision_vjp<LS, false, CT>(phr, chi, ux, uy, uzs, p.tau0, p, mpr, pb, bchi, bux, buy,
                                        buzs, btau, b_isct);
  }
  // velocities
  CT bjx = bux * ir, bjy = buy * ir, bjz = buz * ir;
  bir += bux * jx + buy * jy + buz * jz;
  bjz += bvz * ir + buzs * ir;
  const CT bFz = bvz * ir + buzs * ir * CT(0.5);
  bir += bvz * (jz + Fz) + buzs * (jz + CT(0.5) * Fz);
  bchi += -p.g * bFz;
  brho += -bir * ir * ir;
  bdrho += brho;
  static_for<0, LS::Q>([&](auto qc) { pb[decltype(qc)::value] += bchi; });
  static_for<0, 27>([&](auto qc) { gb[decltype(qc)::value] = CT(0); });
  flow_moments_vjp<Q27, CT>(bdrho, bjx, bjy, bjz, bpxx, bpyy, bpzz, bpxy, bpxz, bpyz, gb);
  static_for<0, 27>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int cx = Q27::cx[q], cy = Q27::cy[q], cz = Q27::cz[q];
    CT t = CT(0);
    if (cx && cy) t += cx > 0 ? br120 : -br120;
    if (cx && cz) t += cx > 0 ? br102 : -br102;
    if (cx && cy) t += cy > 0 ? br210 : -br210;
    if (cy && cz) t += cy > 0 ? br012 : -br012;
    if (cx && cz) t += cz > 0 ? br201 : -br201;
    if (cy && cz) t += cz > 0 ? br021 : -br021;
    if (cx && cy && cz) t += (cx * cy * cz) > 0 ? br111 : -br111;
    gb[q] += t;
  });
}

// ---- BGK D3Q19 + Guo + Smagorinsky, D3Q6 scalar
template <bool LES, typename CT>
LBM_HD void vjp_bgk_q19_q6(const CT* g, const CT* ph, const CT* mg, const CT* mp, const Phys<CT>& p,
                           CT* gb, CT* pb, CT& b_cles, CT& b_isct) {
  CT drho, jx, jy, jz, pxx, pyy, pzz, pxy, pxz, pyz;
  flow_moments<Q19>(g, drho, jx, jy, jz, pxx, pyy, pzz, pxy, pxz, pyz);
  const CT chi = scalar_sum<Q6>(ph);
  const CT rho = CT(1) + drho;
  const CT ir = CT(1) / rho;
  const CT Fz = -p.g * chi;
  const CT ux = jx * ir, uy = jy * ir, uz = (jz + CT(0.5) * Fz) * ir;
  const CT t3 = drho * CT(1.0 / 3.0);
  const CT nxx = pxx - t3 - rho * ux * ux, nyy = pyy - t3 - rho * uy * uy,
           nzz = pzz - t3 - rho * uz * uz;
  const CT nxy = pxy - rho * ux * uy, nxz = pxz - rho * ux * uz, nyz = pyz - rho * uy * uz;
  CT tau = p.tau0, sq = CT(0), h = CT(0), R = CT(0);
  if constexpr (LES) {
    sq = sqrt(nxx * nxx + nyy * nyy + nzz * nzz + CT(2) * (nxy * nxy + nxz * nxz + nyz * nyz));
    h = sq * ir;
    R = sqrt(p.tau0 * p.tau0 + p.c_les * h);
    tau = CT(0.5) * (p.tau0 + R);
  }
  const CT w = CT(1) / tau;
  // 1 / sqrt(Q) with the zero subgradient at Q = 0, formed here so that the
  // reverse sweep has no branch
  const CT isq = (LES && sq > CT(0)) ? CT(1) / sq : CT(0);
  const CT usq = ux * ux + uy * uy + uz * uz;
  const CT sfac = CT(1) - CT(0.5) * w;

  CT bchi = CT(0), bux = CT(0), buy = CT(0), buz = CT(0), btau = CT(0);
  scalar_vjp<Q6, LES, CT>(ph, chi, ux, uy, uz, tau, p, mp, pb, bchi, bux, buy, buz, btau, b_isct);
  CT bw = CT(0), bsfac = CT(0), busq = CT(0), bdrho = CT(0), brho = CT(0), bFz = CT(0);
  static_for<0, 19>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int cx = Q19::cx[q], cy = Q19::cy[q], cz = Q19::cz[q];
    constexpr double W = weight<Q19>(q);
    CT cu = CT(0);
    if (cx) cu += CT(cx) * ux;
    if (cy) cu += CT(cy) * uy;
    if (cz) cu += CT(cz) * uz;
    const CT geq = CT(W) * (drho + rho * (CT(3) * cu + CT(4.5) * cu * cu - CT(1.5) * usq));
    const CT term = CT(3) * (CT(cz) - uz) * Fz + CT(9) * cu * CT(cz) * Fz;
    gb[q] = (CT(1) - w) * mg[q];
    bw += mg[q] * (geq - g[q]);
    const CT bgeq = w * mg[q];
    const CT bS = mg[q];
    bsfac += bS * CT(W) * term;
    buz += bS * sfac * CT(W) * (-CT(3) * Fz);
    CT bcu = bS * sfac * CT(W) * CT(9) * CT(cz) * Fz;
    bFz += bS * sfac * CT(W) * (CT(3) * (CT(cz) - uz) + CT(9) * cu * CT(cz));
    bdrho += bgeq * CT(W);
    brho += bgeq * CT(W) * (CT(3) * cu + CT(4.5) * cu * cu - CT(1.5) * usq);
    bcu += bgeq * CT(W) * rho * (CT(3) + CT(9) * cu);
    busq += bgeq * CT(W) * rho * (-CT(1.5));
    if (cx) bux += CT(cx) * bcu;
    if (cy) buy += CT(cy) * bcu;
    if (cz) buz += CT(cz) * bcu;
  });
  bw += -CT(0.5) * bsfac;
  bux += CT(2) * ux * busq;
  buy += CT(2) * uy * busq;
  buz += CT(2) * uz * busq;
  btau += -bw / (tau * tau);
  CT bpxx = CT(0), bpyy = CT(0), bpzz = CT(0), bpxy = CT(0), bpxz = CT(0), bpyz = CT(0);
  CT bir = CT(0);
  if constexpr (LES) {
    b_cles += btau * h / (CT(4) * R);
    const CT bh = btau * p.c_les / (CT(4) * R);
    bir += bh * sq;
    const CT bsq = bh * ir * isq;
    const CT bnxx = bsq * nxx, bnyy = bsq * nyy, bnzz = bsq * nzz;
    const CT bnxy = bsq * CT(2) * nxy, bnxz = bsq * CT(2) * nxz, bnyz = bsq * CT(2) * nyz;
    bpxx += bnxx;
    bpyy += bnyy;
    bpzz += bnzz;
    bpxy += bnxy;
    bpxz += bnxz;
    bpyz += bnyz;
    bdrho -= (bnxx + bnyy + bnzz) * CT(1.0 / 3.0);
    brho -= bnxx * ux * ux + bnyy * uy * uy + bnzz * uz * uz + bnxy * ux * uy + bnxz * ux * uz +
            bnyz * uy * uz;
    bux -= rho * (CT(2) * ux * bnxx + uy * bnxy + uz * bnxz);
    buy -= rho * (CT(2) * uy * bnyy + ux * bnxy + uz * bnyz);
    buz -= rho * (CT(2) * uz * bnzz + ux * bnxz + uy * bnyz);
  }
  CT bjx = bux * ir, bjy = buy * ir, bjz = buz * ir;
  bFz += buz * ir * CT(0.5);
  bir += bux * jx + buy * jy + buz * (jz + CT(0.5) * Fz);
  bchi += -p.g * bFz;
  brho += -bir * ir * ir;
  bdrho += brho;
  static_for<0, 6>([&](auto qc) { pb[decltype(qc)::value] += bchi; });
  flow_moments_vjp<Q19, CT>(bdrho, bjx, bjy, bjz, bpxx, bpyy, bpzz, bpxy, bpxz, bpyz, gb);
}

}  // namespace lbm

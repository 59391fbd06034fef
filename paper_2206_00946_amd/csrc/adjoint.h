// Per-cell reverse-mode (adjoint) arithmetic of the coupled step: the
// transposes of the linear maps and the Jacobians of the nonlinear ones in
// lattice.h.  Notation: xb is the adjoint (dJ/dx) of a forward quantity x.
// Method: Huang, Wang, He & Huang, arXiv 2206.00946, Sec. 2 and 3.3.
#pragma once

#include "lattice.h"

namespace lbm {

// Column i of the transform (A.1): the moment monomials 1, x, y, z, |c|^2,
// 2x^2-y^2-z^2, y^2-z^2, xy, xz, yz, x^2y, xy^2, x^2z, xz^2, y^2z, yz^2,
// x^2y^2, x^2z^2, y^2z^2 evaluated at c_i.
__host__ __device__ constexpr int mono19(int k, int i) {
  const int x = CX[i], y = CY[i], z = CZ[i];
  switch (k) {
    case 0: return 1;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * x + y * y + z * z;
    case 5: return 2 * x * x - y * y - z * z;
    case 6: return y * y - z * z;
    case 7: return x * y;
    case 8: return x * z;
    case 9: return y * z;
    case 10: return x * x * y;
    case 11: return x * y * y;
    case 12: return x * x * z;
    case 13: return x * z * z;
    case 14: return y * y * z;
    case 15: return y * z * z;
    case 16: return x * x * y * y;
    case 17: return x * x * z * z;
    default: return y * y * z * z;
  }
}

// fb = M^T mb
template <typename C>
__host__ __device__ __forceinline__ void moments19_T(const C* mb, C* fb) {
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    C s = C(0);
#pragma unroll
    for (int k = 0; k < 19; ++k) {
      const int c = mono19(k, i);
      if (c != 0) s += C(c) * mb[k];
    }
    fb[i] = s;
  }
}

// mb = M^-T fb: the reverse of populations19, stage by stage.
template <typename C>
__host__ __device__ __forceinline__ void populations19_T(const C* fb, C* mb) {
  const C q = C(0.25);
  const C dxb = C(0.5) * (fb[1] - fb[2]);
  const C dyb = C(0.5) * (fb[3] - fb[4]);
  const C dzb = C(0.5) * (fb[5] - fb[6]);
  const C Bb = C(0.5) * (fb[3] + fb[4]);
  const C Cb = C(0.5) * (fb[5] + fb[6]);
  // B = (S - A + Q)/2 and C = (S - A - Q)/2
  const C Ab = C(0.5) * (fb[1] + fb[2]) - C(0.5) * (Bb + Cb);
  const C Qb = C(0.5) * (Bb - Cb);
  // A = (S + P)/3
  const C Sb = C(0.5) * (Bb + Cb) + cdiv<3>(Ab);
  const C Pb = cdiv<3>(Ab);
  const C sxy = fb[7] + fb[8] + fb[9] + fb[10];
  const C sxz = fb[11] + fb[12] + fb[13] + fb[14];
  const C syz = fb[15] + fb[16] + fb[17] + fb[18];
  mb[0] = fb[0];
  mb[1] = dxb;
  mb[2] = dyb;
  mb[3] = dzb;
  mb[4] = Sb - fb[0];
  mb[5] = Pb;
  mb[6] = Qb;
  mb[7] = q * (fb[7] + fb[8] - fb[9] - fb[10]);
  mb[8] = q * (fb[11] + fb[12] - fb[13] - fb[14]);
  mb[9] = q * (fb[15] + fb[16] - fb[17] - fb[18]);
  mb[10] = q * (fb[7] - fb[8] - fb[9] + fb[10]) - dyb;
  mb[11] = q * (fb[7] - fb[8] + fb[9] - fb[10]) - dxb;
  mb[12] = q * (fb[11] - fb[12] - fb[13] + fb[14]) - dzb;
  mb[13] = q * (fb[11] - fb[12] + fb[13] - fb[14]) - dxb;
  mb[14] = q * (fb[15] - fb[16] - fb[17] + fb[18]) - dzb;
  mb[15] = q * (fb[15] - fb[16] + fb[17] - fb[18]) - dyb;
  mb[16] = fb[0] - C(2) * Sb - Pb - Qb + q * sxy;
  mb[17] = fb[0] - C(2) * Sb - Pb + Qb + q * sxz;
  mb[18] = fb[0] - C(2) * Sb + C(2) * Pb + q * syz;
}

// Equilibrium moments of eq. (10) per unit density, h(u) = m^eq(1, u), and
// the adjoint of m^eq(rho, u) = rho h(u): rb += ab . h(u),
// ub += rho (dh/du)^T ab.
template <typename C>
__host__ __device__ __forceinline__ void meq19_adj(const C* ab, C rho, C ux, C uy, C uz, C& rb, C& uxb, C& uyb,
                                                   C& uzb) {
  const C t = C(1) / C(3);
  const C xx = ux * ux, yy = uy * uy, zz = uz * uz, s = xx + yy + zz;
  const C rest = C(1) / C(9) - s / C(6);
  rb += ab[0] + ab[1] * ux + ab[2] * uy + ab[3] * uz + ab[4] * (C(1) + s) + ab[5] * (C(2) * xx - yy - zz) +
        ab[6] * (yy - zz) + ab[7] * ux * uy + ab[8] * ux * uz + ab[9] * uy * uz +
        t * (ab[10] * uy + ab[11] * ux + ab[12] * uz + ab[13] * ux + ab[14] * uz + ab[15] * uy) +
        ab[16] * (rest + t * (xx + yy)) + ab[17] * (rest + t * (xx + zz)) + ab[18] * (rest + t * (yy + zz));
  // d h_16..18 / d u_a: -u_a/3 from the rest term, +2 u_a/3 where u_a^2 appears
  const C gx = ab[1] + C(2) * ux * ab[4] + C(4) * ux * ab[5] + uy * ab[7] + uz * ab[8] + t * (ab[11] + ab[13]) +
               t * ux * (ab[16] + ab[17] - ab[18]);
  const C gy = ab[2] + C(2) * uy * ab[4] - C(2) * uy * ab[5] + C(2) * uy * ab[6] + ux * ab[7] + uz * ab[9] +
               t * (ab[10] + ab[15]) + t * uy * (ab[16] - ab[17] + ab[18]);
  const C gz = ab[3] + C(2) * uz * ab[4] - C(2) * uz * ab[5] - C(2) * uz * ab[6] + ux * ab[8] + uy * ab[9] +
               t * (ab[12] + ab[14]) + t * uz * (-ab[16] + ab[17] + ab[18]);
  uxb += rho * gx;
  uyb += rho * gy;
  uzb += rho * gz;
}

template <typename C>
__host__ __device__ __forceinline__ C rate19(int k, const Phys<C>& ph) {
  return k < 4 ? C(1) : (k == 4 ? ph.s_e : (k < 10 ? ph.s_nu : (k < 16 ? ph.s_q : ph.s_pi)));
}

// Adjoint of collide19 (eq. (8)): f* = M^-1 [(I - L) m + (L - I) meq(u_eq) +
// meq(u_eq + du)], m = M f.  Input fsb = adjoint of f*; outputs the adjoint
// of the pre-collision f (overwrites fb) and adds to rb, ub (of u_eq), dub.
template <typename C>
__host__ __device__ __forceinline__ void collide19_adj(const C* fsb, C rho, C ux, C uy, C uz, C dux, C duy, C duz,
                                                       const Phys<C>& ph, C* fb, C& rb, C* ub, C* dub) {
  C mb[19];
  populations19_T(fsb, mb);
  C a0[19], keep[19];
#pragma unroll
  for (int k = 0; k < 19; ++k) {
    const C om = C(1) - rate19<C>(k, ph);
    keep[k] = om * mb[k];
    a0[k] = -om * mb[k];
  }
  moments19_T(keep, fb);
  C vxb = C(0), vyb = C(0), vzb = C(0);
  meq19_adj(mb, rho, ux + dux, uy + duy, uz + duz, rb, vxb, vyb, vzb);
  meq19_adj(a0, rho, ux, uy, uz, rb, ub[0], ub[1], ub[2]);
  ub[0] += vxb;
  ub[1] += vyb;
  ub[2] += vzb;
  dub[0] += vxb;
  dub[1] += vyb;
  dub[2] += vzb;
}

// Adjoint of collide7 (eq. (13) collision with the source of eq. (15)):
// input gsb = adjoint of g*; outputs the adjoint of the pre-collision g and
// of Fbar.
template <typename C>
__host__ __device__ __forceinline__ void collide7_adj(const C* gsb, const Phys<C>& ph, C* gb, C& Fbarb) {
  Fbarb = -ph.w0 * gsb[0] - ph.w1 * (gsb[1] + gsb[2] + gsb[3] + gsb[4] + gsb[5] + gsb[6]);
  const C om = C(1) - ph.vother;
  const C of = C(1) - ph.vflux;
  C n0b = gsb[0];
  const C n4sb = -gsb[0] + cdiv<6>(gsb[1] + gsb[2] + gsb[3] + gsb[4] + gsb[5] + gsb[6]);
  const C ab = cdiv<6>(gsb[1] + gsb[2]);
  const C n1sb = C(0.5) * (gsb[1] - gsb[2]);
  const C n2sb = C(0.5) * (gsb[3] - gsb[4]);
  const C n3sb = C(0.5) * (gsb[5] - gsb[6]);
  const C n5sb = ab - cdiv<3>(gsb[3] + gsb[4]) + cdiv<6>(gsb[5] + gsb[6]);
  const C n6sb = ab + cdiv<6>(gsb[3] + gsb[4]) - cdiv<3>(gsb[5] + gsb[6]);
  const C n1b = of * n1sb, n2b = of * n2sb, n3b = of * n3sb;
  const C n4b = (C(1) - ph.vother) * n4sb;
  n0b += ph.vother * ph.wbar * n4sb;
  const C n5b = om * n5sb, n6b = om * n6sb;
  gb[0] = n0b;
  gb[1] = n0b + n1b + n4b + n5b + n6b;
  gb[2] = n0b - n1b + n4b + n5b + n6b;
  gb[3] = n0b + n2b + n4b - n5b;
  gb[4] = n0b - n2b + n4b - n5b;
  gb[5] = n0b + n3b + n4b - n6b;
  gb[6] = n0b - n3b + n4b - n6b;
}

// Peng-Robinson partial derivatives (eqs. (54)-(55)): dp/drho, and the
// derivatives of dp/dT with respect to rho and T.
template <typename C>
__host__ __device__ __forceinline__ void pr_partials(C rho, C T, const Phys<C>& ph, C& dp_drho, C& dpdT,
                                                     C& dpdT_drho, C& dpdT_dT) {
  const C sq = fsqrt(T * ph.Tc);
  const C s = C(1) + ph.kpr * (C(1) - fsqrt(T / ph.Tc));  // xi = s^2
  const C xi = s * s;
  const C sp = -ph.kpr / (C(2) * sq);                      // ds/dT
  const C spp = ph.kpr / (C(4) * T * sq);                  // d2s/dT2
  const C dxi = C(2) * s * sp;
  const C d2xi = C(2) * (sp * sp + s * spp);
  const C br = ph.b * rho;
  const C om = C(1) - br;
  const C D = C(1) + C(2) * br - br * br;
  const C dD = C(2) * ph.b - C(2) * ph.b * br;
  const C q = (C(2) * rho * D - rho * rho * dD) / (D * D);  // d(rho^2/D)/drho
  dp_drho = ph.R * T / (om * om) - ph.a * xi * q;
  dpdT = rho * ph.R / om - ph.a * dxi * rho * rho / D;
  dpdT_drho = ph.R / (om * om) - ph.a * dxi * q;
  dpdT_dT = -ph.a * d2xi * rho * rho / D;
}

// Adjoint of the outlet fill of Sec. 3.3 at a node of face k (outlet_fill):
// fb holds the adjoint of the completed populations; on return the adjoint
// of the unknown slots is moved to the known populations and to the force
// (Fb), and the unknown slots (never read by the forward step) are zero.
template <typename C>
__host__ __device__ __forceinline__ void outlet_fill_adj(C* fb, int k, C* Fb) {
  const int a = k >> 1;
  const int s = (k & 1) ? 1 : -1;
  const int ta = a == 0 ? 1 : 0;
  const int tb = a == 2 ? 1 : 2;
  C rub = C(0), dab = C(0), dbb = C(0), dnb = C(0);
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const int c3[3] = {CX[i], CY[i], CZ[i]};
    if (c3[a] * s != -1) continue;
    const C v = fb[i];
    fb[opp19(i)] += v;
    if (c3[ta] == 0 && c3[tb] == 0) {
      rub -= cdiv<3>(v);
    } else {
      rub -= cdiv<6>(v);
      dab += C(c3[ta]) * v;
      dbb += C(c3[tb]) * v;
      dnb -= v;
    }
    fb[i] = C(0);
  }
  // ru = sig0 + 2 sig1 + rho_ref + Fn/2 - rho_out; da = -t0/2 - F_ta/4;
  // db = -t1/2 - F_tb/4; dn = -Fn/8; Fn = s F_a
  const C Fnb = C(0.5) * rub - cdiv<8>(dnb);
  Fb[a] += C(s) * Fnb;
  Fb[ta] -= C(0.25) * dab;
  Fb[tb] -= C(0.25) * dbb;
  const C t0b = -C(0.5) * dab, t1b = -C(0.5) * dbb;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const int c3[3] = {CX[i], CY[i], CZ[i]};
    const int cn = c3[a] * s;
    if (cn == 0) fb[i] += rub + C(c3[ta]) * t0b + C(c3[tb]) * t1b;
    else if (cn == 1) fb[i] += C(2) * rub;
  }
}

}  // namespace lbm

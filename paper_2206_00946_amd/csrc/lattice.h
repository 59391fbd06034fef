// Per-cell lattice arithmetic of the coupled D3Q19 / D3Q7 step, shared by
// every kernel of the library.  Method: Huang, Wang, He & Huang, arXiv
// 2206.00946 (Sec. 2, Appendix A).  All populations handled here are
// deviations from the rest equilibrium: ft_i = f_i - w_i rho_ref and
// gt_i = g_i - w_i T_ref (rho_ref = T_ref = 0 gives the plain populations).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

namespace lbm {

enum { FACE_PERIODIC = 0, FACE_WALL = 1, FACE_PRESSURE = 2 };

// D3Q19 velocities in the order fixed by rows 1-3 of the transform (A.1):
// rest, +x, -x, +y, -y, +z, -z, then the xy, xz and yz face diagonals.
constexpr int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
// opposite velocity: pairs (1,2), (3,4), ..., (17,18)
__host__ __device__ constexpr int opp19(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
// D3Q7: rest, +x, -x, +y, -y, +z, -z (rows 1-3 of (A.2)); the first seven D3Q19 ones.

template <typename C>
__host__ __device__ constexpr C w19(int i) {
  return i == 0 ? C(1) / C(3) : (i < 7 ? C(1) / C(18) : C(1) / C(36));
}

// Physical and lattice parameters in the compute precision C.
template <typename C>
struct Phys {
  C a, b, R, G, Tc, kpr;      // Peng-Robinson, eqs. (54)-(55); kpr = 0.37464 + 1.54226 w - 0.26992 w^2
  C s_e, s_nu, s_q, s_pi;     // eq. (11)
  C w0, w1, wbar, cs2T;       // D3Q7 weights and c_s^2 = wbar/3
  C vflux, vother;            // varsigma_{1,2,3} and the remaining rates
  C cv;
  C kappa_w;                  // eq. (37)
  C rho_ref, T_ref;           // deviation references
  C inv_b;
  int var_lambda;             // 1: conductivity linear in rho between the two phases
  C lam_v, lam_l, lam_rv, lam_inv_drho;
};

// varsigma_{1,2,3} of the D3Q7 collision at density rho: 1 / (1/2 + lambda / c_s^2),
// lambda uniform or linear in rho between the vapour and liquid values
template <typename C>
__host__ __device__ __forceinline__ C vflux_at(C rho, const Phys<C>& ph) {
  if (!ph.var_lambda) return ph.vflux;
  C fr = (rho - ph.lam_rv) * ph.lam_inv_drho;
  fr = fr < C(0) ? C(0) : (fr > C(1) ? C(1) : fr);
  const C lam = ph.lam_v + (ph.lam_l - ph.lam_v) * fr;
  return C(1) / (C(0.5) + lam / ph.cs2T);
}

// ---------------------------------------------------------------- arithmetic
// FP32 uses the hardware reciprocal and square root (about 1 ulp); FP64 keeps
// correctly rounded division and square root.  The host versions exist for
// the CPU unit checks of the per-cell arithmetic.
#if defined(__HIP_DEVICE_COMPILE__)
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
#else
inline float rcp(float x) { return 1.0f / x; }
inline float div(float a, float b) { return a / b; }
inline float fsqrt(float x) { return std::sqrt(x); }
#endif
__host__ __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__host__ __device__ __forceinline__ double div(double a, double b) { return a / b; }
__host__ __device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }
// division by a small integer constant: a multiplication for FP32
template <int K>
__host__ __device__ __forceinline__ float cdiv(float x) { return x * (1.0f / K); }
template <int K>
__host__ __device__ __forceinline__ double cdiv(double x) { return x / K; }

// ---------------------------------------------------------------- EOS
template <typename C>
__host__ __device__ __forceinline__ C pr_xi_sq_root(C T, const Phys<C>& ph) {
  // 1 + kappa (1 - sqrt(T/Tc)), whose square is xi(T)
  return C(1) + ph.kpr * (C(1) - fsqrt(div(T, ph.Tc)));
}

template <typename C>
__host__ __device__ __forceinline__ C pr_pressure(C rho, C T, const Phys<C>& ph) {
  const C s = pr_xi_sq_root(T, ph);
  const C br = ph.b * rho;
  return div(rho * ph.R * T, C(1) - br) - div(ph.a * (s * s) * rho * rho, C(1) + C(2) * br - br * br);
}

// (d p / d T) at constant rho
template <typename C>
__host__ __device__ __forceinline__ C pr_dpdT(C rho, C T, const Phys<C>& ph) {
  const C s = pr_xi_sq_root(T, ph);
  const C dxi = div(-ph.kpr * s, fsqrt(T * ph.Tc));
  const C br = ph.b * rho;
  return div(rho * ph.R, C(1) - br) - div(ph.a * dxi * rho * rho, C(1) + C(2) * br - br * br);
}

// radicand of eq. (7): 2 (p - rho c_s^2) / G with c_s^2 = 1/3
template <typename C>
__host__ __device__ __forceinline__ C psi_radicand(C rho, C T, const Phys<C>& ph) {
  return div(C(2) * (pr_pressure(rho, T, ph) - cdiv<3>(rho)), ph.G);
}

template <typename C>
__host__ __device__ __forceinline__ bool nonphysical(C rho, C T, C rad, const Phys<C>& ph) {
  // written so that NaN in any input also trips the flag
  return !(rho > C(0)) || !(rho * ph.b < C(1)) || !(T > C(0)) || !(rad >= C(0));
}

// ---------------------------------------------------------------- D3Q19
// Deviation moments m = M ft of the transform (A.1), written out row by row
// (monomials 1, x, y, z, |c|^2, 2x^2-y^2-z^2, y^2-z^2, xy, xz, yz, x^2y, xy^2,
// x^2z, xz^2, y^2z, yz^2, x^2y^2, x^2z^2, y^2z^2).
template <typename C>
__host__ __device__ __forceinline__ void moments19(const C* f, C* m) {
  const C ax = f[1] + f[2], ay = f[3] + f[4], az = f[5] + f[6];
  const C dxy = f[7] + f[8] + f[9] + f[10];
  const C dxz = f[11] + f[12] + f[13] + f[14];
  const C dyz = f[15] + f[16] + f[17] + f[18];
  m[0] = f[0] + ax + ay + az + dxy + dxz + dyz;
  const C a78 = f[7] - f[8], a910 = f[9] - f[10];
  const C a1112 = f[11] - f[12], a1314 = f[13] - f[14];
  const C a1516 = f[15] - f[16], a1718 = f[17] - f[18];
  m[1] = (f[1] - f[2]) + a78 + a910 + a1112 + a1314;
  m[2] = (f[3] - f[4]) + a78 - a910 + a1516 + a1718;
  m[3] = (f[5] - f[6]) + a1112 - a1314 + a1516 - a1718;
  m[4] = ax + ay + az + C(2) * (dxy + dxz + dyz);
  m[5] = C(2) * ax - ay - az + dxy + dxz - C(2) * dyz;
  m[6] = ay - az + dxy - dxz;
  m[7] = (f[7] + f[8]) - (f[9] + f[10]);
  m[8] = (f[11] + f[12]) - (f[13] + f[14]);
  m[9] = (f[15] + f[16]) - (f[17] + f[18]);
  m[10] = a78 - a910;
  m[11] = a78 + a910;
  m[12] = a1112 - a1314;
  m[13] = a1112 + a1314;
  m[14] = a1516 - a1718;
  m[15] = a1516 + a1718;
  m[16] = dxy;
  m[17] = dxz;
  m[18] = dyz;
}

// Inverse transform f = M^-1 m, solved group by group: each face-diagonal
// quadruple from its four moments, the axis pairs from the second-order
// moments, the rest population from m0 and m4.
template <typename C>
__host__ __device__ __forceinline__ void populations19(const C* m, C* f) {
  const C q = C(0.25);
  f[7] = q * (m[16] + m[10] + m[11] + m[7]);
  f[8] = q * (m[16] - m[10] - m[11] + m[7]);
  f[9] = q * (m[16] - m[10] + m[11] - m[7]);
  f[10] = q * (m[16] + m[10] - m[11] - m[7]);
  f[11] = q * (m[17] + m[12] + m[13] + m[8]);
  f[12] = q * (m[17] - m[12] - m[13] + m[8]);
  f[13] = q * (m[17] - m[12] + m[13] - m[8]);
  f[14] = q * (m[17] + m[12] - m[13] - m[8]);
  f[15] = q * (m[18] + m[14] + m[15] + m[9]);
  f[16] = q * (m[18] - m[14] - m[15] + m[9]);
  f[17] = q * (m[18] - m[14] + m[15] - m[9]);
  f[18] = q * (m[18] + m[14] - m[15] - m[9]);
  const C S = m[4] - C(2) * (m[16] + m[17] + m[18]);      // sum of the six axis populations
  const C P = m[5] - m[16] - m[17] + C(2) * m[18];         // 2A - B - C
  const C Q = m[6] - m[16] + m[17];                         // B - C
  const C A = cdiv<3>(S + P);
  const C B = C(0.5) * (S - A + Q);
  const C Cz = C(0.5) * (S - A - Q);
  const C dx = m[1] - m[11] - m[13];
  const C dy = m[2] - m[10] - m[15];
  const C dz = m[3] - m[12] - m[14];
  f[0] = m[0] - m[4] + m[16] + m[17] + m[18];
  f[1] = C(0.5) * (A + dx);
  f[2] = C(0.5) * (A - dx);
  f[3] = C(0.5) * (B + dy);
  f[4] = C(0.5) * (B - dy);
  f[5] = C(0.5) * (Cz + dz);
  f[6] = C(0.5) * (Cz - dz);
}

// eq. (8): m* = m - L (m - meq(u_eq)) + [meq(u_eq + du) - meq(u_eq)], applied
// to deviations: mt*_k = (1 - s_k)(mt_k - rt e_k - q_k(u_eq)) + rt e_k + q_k(u_eq + du),
// rt = rho - rho_ref, where rho e + q(rho, u) are the equilibrium moments of
// eq. (10) (e: moments of the rest weights, 1 at rows 0 and 4, 1/9 at rows
// 16-18).  f is overwritten by the post-collision deviations.
template <typename C>
__host__ __device__ __forceinline__ void collide19(C* f, C rho, C rt, C ux, C uy, C uz, C dux, C duy,
                                          C duz, const Phys<C>& ph) {
  C m[19];
  moments19(f, m);
  const C vx = ux + dux, vy = uy + duy, vz = uz + duz;
  const C third = C(1) / C(3);
  const C xx0 = ux * ux, yy0 = uy * uy, zz0 = uz * uz, s0 = xx0 + yy0 + zz0;
  const C xx1 = vx * vx, yy1 = vy * vy, zz1 = vz * vz, s1 = xx1 + yy1 + zz1;
  const C oe = C(1) - ph.s_e, on = C(1) - ph.s_nu, oq = C(1) - ph.s_q, op = C(1) - ph.s_pi;
  // rows 0-3 relax with rate 1: density and momentum after forcing
  m[0] = rt;
  m[1] = rho * vx;
  m[2] = rho * vy;
  m[3] = rho * vz;
  m[4] = oe * (m[4] - rt - rho * s0) + rt + rho * s1;
  m[5] = on * (m[5] - rho * (C(2) * xx0 - yy0 - zz0)) + rho * (C(2) * xx1 - yy1 - zz1);
  m[6] = on * (m[6] - rho * (yy0 - zz0)) + rho * (yy1 - zz1);
  m[7] = on * (m[7] - rho * ux * uy) + rho * vx * vy;
  m[8] = on * (m[8] - rho * ux * uz) + rho * vx * vz;
  m[9] = on * (m[9] - rho * uy * uz) + rho * vy * vz;
  const C r3 = rho * third;
  m[10] = oq * (m[10] - r3 * uy) + r3 * vy;
  m[11] = oq * (m[11] - r3 * ux) + r3 * vx;
  m[12] = oq * (m[12] - r3 * uz) + r3 * vz;
  m[13] = oq * (m[13] - r3 * ux) + r3 * vx;
  m[14] = oq * (m[14] - r3 * uz) + r3 * vz;
  m[15] = oq * (m[15] - r3 * uy) + r3 * vy;
  const C e9 = cdiv<9>(rt);
  const C rest0 = cdiv<6>(-rho * s0), rest1 = cdiv<6>(-rho * s1);
  m[16] = op * (m[16] - e9 - rest0 - r3 * (xx0 + yy0)) + e9 + rest1 + r3 * (xx1 + yy1);
  m[17] = op * (m[17] - e9 - rest0 - r3 * (xx0 + zz0)) + e9 + rest1 + r3 * (xx1 + zz1);
  m[18] = op * (m[18] - e9 - rest0 - r3 * (yy0 + zz0)) + e9 + rest1 + r3 * (yy1 + zz1);
  populations19(m, f);
}

// ---------------------------------------------------------------- D3Q7
// Collision of eq. (13) with the D3Q7 transform (A.2) and theta = 0, on
// deviations: n = M gt, n* = n - L (n - (Tt, 0, 0, 0, wbar Tt, 0, 0)),
// varsigma_{1,2,3} = vflux (the node's conductivity),
// gt* = M^-1 n* - w_i Fbar (source of eq. (15)).  Tt = T - T_ref = n0.
template <typename C>
__host__ __device__ __forceinline__ void collide7(C* g, C Fbar, C vflux, const Phys<C>& ph) {
  const C n0 = g[0] + g[1] + g[2] + g[3] + g[4] + g[5] + g[6];
  C n1 = g[1] - g[2], n2 = g[3] - g[4], n3 = g[5] - g[6];
  C n4 = g[1] + g[2] + g[3] + g[4] + g[5] + g[6];
  C n5 = g[1] + g[2] - g[3] - g[4];
  C n6 = g[1] + g[2] - g[5] - g[6];
  const C om = C(1) - ph.vother;
  const C of = C(1) - vflux;
  n1 *= of;
  n2 *= of;
  n3 *= of;
  n4 = n4 - ph.vother * (n4 - ph.wbar * n0);
  n5 *= om;
  n6 *= om;
  const C s6 = cdiv<6>(n4);
  const C a = cdiv<6>(n5 + n6);
  g[0] = n0 - n4 - ph.w0 * Fbar;
  g[1] = C(0.5) * n1 + s6 + a - ph.w1 * Fbar;
  g[2] = -C(0.5) * n1 + s6 + a - ph.w1 * Fbar;
  const C n5_3 = cdiv<3>(n5), n5_6 = cdiv<6>(n5), n6_3 = cdiv<3>(n6), n6_6 = cdiv<6>(n6);
  g[3] = C(0.5) * n2 + s6 - n5_3 + n6_6 - ph.w1 * Fbar;
  g[4] = -C(0.5) * n2 + s6 - n5_3 + n6_6 - ph.w1 * Fbar;
  g[5] = C(0.5) * n3 + s6 + n5_6 - n6_3 - ph.w1 * Fbar;
  g[6] = -C(0.5) * n3 + s6 + n5_6 - n6_3 - ph.w1 * Fbar;
}

// eqs. (27)-(29): c_s^2 dT/dx_a = -varsigma_a m_a (dt = 1) with the
// pre-collision first moments of g (their equilibrium part is zero).
template <typename C>
__host__ __device__ __forceinline__ void local_gradT(const C* g, C vflux, const Phys<C>& ph, C& gx, C& gy,
                                                     C& gz) {
  const C k = div(-vflux, ph.cs2T);
  gx = k * (g[1] - g[2]);
  gy = k * (g[3] - g[4]);
  gz = k * (g[5] - g[6]);
}

// eq. (2) deviation: f^eq_i(rho, u) - w_i rho_ref
template <typename C>
__host__ __device__ __forceinline__ C feq19_dev(int i, C rho, C rho_ref, C ux, C uy, C uz) {
  const C cu = C(CX[i]) * ux + C(CY[i]) * uy + C(CZ[i]) * uz;
  const C usq = ux * ux + uy * uy + uz * uz;
  return w19<C>(i) * (rho * (C(1) + C(3) * cu + C(4.5) * cu * cu - C(1.5) * usq) - rho_ref);
}

}  // namespace lbm

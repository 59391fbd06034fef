// Unfused kernels of the coupled step, one pass per stage of the update
// (Huang, Wang, He & Huang, arXiv 2206.00946, Sec. 2-3):
//   k_macro              -- eqs. (35)-(36) at the nodes of bounded faces (g in
//                           place), rho, T (eq. (3), T = sum g), psi (eq. (7)),
//                           flag
//   k_force              -- interaction force (eq. (6)) with ghost rules,
//                           outlet fill (Sec. 3.3), u_eq and du (eqs. (3)-(5))
//   k_collide_push       -- div u, local grad T, Fbar (eq. (15)), D3Q19 and
//                           D3Q7 collisions, push streaming with bounce-back
//                           (eq. (34)) and the rho c_v blend (eq. (13))
// They serve every storage precision and every boundary kind; the fused
// single-pass kernel is the fast path for the supported subset.
#pragma once

#include "lattice.h"
#include "storage.h"

namespace lbm {

struct Geom {
  int nx, ny, nz;
  int face[6];
  long long N;
  long long pitch;  // elements from one direction plane to the next
};

// Device layout of the populations: plane-major structure of arrays.
// Population i of cell (x, y, z) of a Q-velocity lattice is element
// (z*Q + i)*pitch + x + nx*y, so one plane of one direction is contiguous.
// The pitch is nx*ny plus kPlanePad elements: with an unpadded power-of-two
// plane the 26 direction planes of a z level start at the same offset modulo
// large powers of two and their streams crowd the same memory channels.
constexpr long long kPlanePad = 64;
__host__ __device__ inline long long plane_pitch(int nx, int ny) { return (long long)nx * ny + kPlanePad; }

__device__ __forceinline__ long long pidx(const Geom& g, int Q, int i, int x, int y, int z) {
  return ((long long)z * Q + i) * g.pitch + x + (long long)g.nx * y;
}

template <typename C>
struct Faces {
  C face_T[6];
  C face_rho[6];
  const double* Tw[2];  // optional wall fields of faces 4 (-z) and 5 (+z), nx*ny
};

__device__ __forceinline__ long long cell_index(const Geom& g, int x, int y, int z) {
  return (long long)x + (long long)g.nx * ((long long)y + (long long)g.ny * (long long)z);
}

// Node classification: the bounded faces a node lies on, its inward
// (diagonal at edges) neighbour offset and the face that sets its boundary
// values, by priority -z, +z, -y, +y, -x, +x.
struct Node {
  int count;     // number of bounded faces through the node
  int prio;      // face setting T_b / rho_out, or -1
  int ix, iy, iz;
  bool pressure; // on at least one pressure face
  bool wall;     // on a wall face
  int pface;     // the pressure face when count == 1
};

__device__ __forceinline__ Node classify(const Geom& g, int x, int y, int z) {
  Node n;
  n.count = 0;
  n.prio = -1;
  n.ix = n.iy = n.iz = 0;
  n.pressure = false;
  n.wall = false;
  n.pface = -1;
  const int c[3] = {x, y, z};
  const int ext[3] = {g.nx, g.ny, g.nz};
  bool on[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int a = k >> 1;
    const bool hi = k & 1;
    on[k] = g.face[k] != FACE_PERIODIC && c[a] == (hi ? ext[a] - 1 : 0);
    if (on[k]) {
      n.count++;
      const int inw = hi ? -1 : 1;
      if (a == 0) n.ix += inw;
      if (a == 1) n.iy += inw;
      if (a == 2) n.iz += inw;
      if (g.face[k] == FACE_PRESSURE) {
        n.pressure = true;
        n.pface = k;
      }
      if (g.face[k] == FACE_WALL) n.wall = true;
    }
  }
  const int order[6] = {4, 5, 2, 3, 0, 1};
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    if (n.prio < 0 && on[order[q]]) n.prio = order[q];
  }
  return n;
}

template <typename C>
__device__ __forceinline__ C boundary_T(const Geom& g, const Faces<C>& fc, int prio, int x, int y) {
  if (prio == 4 && fc.Tw[0]) return C(fc.Tw[0][x + g.nx * y]);
  if (prio == 5 && fc.Tw[1]) return C(fc.Tw[1][x + g.nx * y]);
  return fc.face_T[prio];
}

// Resolve a coordinate one step outside [0, n) on an axis whose faces are
// periodic or pressure (wrap, or copy of the face node).
__device__ __forceinline__ int resolve_open(int c, int n, int kind) {
  if (c < 0) return kind == FACE_PERIODIC ? c + n : 0;
  if (c >= n) return kind == FACE_PERIODIC ? c - n : n - 1;
  return c;
}

__device__ __forceinline__ int wrapp(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

// psi at (x, y, z) within one cell of the domain, with the ghost rules:
// periodic wrap, copy of the face node beyond pressure faces, eq. (37)
// beyond wall faces (tangential differences periodic).
template <typename C>
__device__ __forceinline__ C psi_at(const C* __restrict__ psi, const Geom& g, C kappa_w, int x, int y,
                                    int z) {
  x = resolve_open(x, g.nx, g.face[0]);
  y = resolve_open(y, g.ny, g.face[2]);
  if (z >= 0 && z < g.nz) return psi[cell_index(g, x, y, z)];
  const int k = z < 0 ? 4 : 5;
  if (g.face[k] == FACE_PERIODIC) return psi[cell_index(g, x, y, wrapp(z, g.nz))];
  if (g.face[k] == FACE_PRESSURE) return psi[cell_index(g, x, y, z < 0 ? 0 : g.nz - 1)];
  const int zw = z < 0 ? 0 : g.nz - 1;
  const int zi = z < 0 ? 1 : g.nz - 2;
  const C dx = psi[cell_index(g, wrapp(x + 1, g.nx), y, zw)] - psi[cell_index(g, wrapp(x - 1, g.nx), y, zw)];
  const C dy = psi[cell_index(g, x, wrapp(y + 1, g.ny), zw)] - psi[cell_index(g, x, wrapp(y - 1, g.ny), zw)];
  return psi[cell_index(g, x, y, zi)] + sqrt(dx * dx + dy * dy) * kappa_w;
}

// Real velocity of eq. (5) at (x, y, z) within one cell of the domain, from
// the field k_force stores: 0 beyond walls, copy beyond pressure faces, wrap
// if periodic.
template <typename C>
__device__ __forceinline__ void u_real_at(const C* __restrict__ ureal, const Geom& g, int x, int y, int z, C& ux,
                                          C& uy, C& uz) {
  x = resolve_open(x, g.nx, g.face[0]);
  y = resolve_open(y, g.ny, g.face[2]);
  if (z < 0 || z >= g.nz) {
    const int k = z < 0 ? 4 : 5;
    if (g.face[k] == FACE_WALL) {
      ux = uy = uz = C(0);
      return;
    }
    z = resolve_open(z, g.nz, g.face[4]);
  }
  const long long c = cell_index(g, x, y, z);
  ux = ureal[c];
  uy = ureal[c + g.N];
  uz = ureal[c + 2 * g.N];
}

// ---------------------------------------------------------------- kernels

// S0-S2 per node.  At a node of a bounded face, g is first completed in
// place by eqs. (35)-(36): g_i(x_b) = w_i T_b + g_i(x_f) - w_i T(x_f) from
// the inward (diagonal at edges) neighbour x_f, which lies on no bounded
// face (bounded axes have >= 3 cells), so no thread reads a g another
// thread writes.  T is the sum of the stored (rounded) g.
template <typename S>
__global__ void __launch_bounds__(256) k_macro(const S* __restrict__ fpop, S* __restrict__ gpop,
                                               typename Storage<S>::C* __restrict__ rho_out,
                                               typename Storage<S>::C* __restrict__ T_out,
                                               typename Storage<S>::C* __restrict__ psi_out,
                                               int* __restrict__ flag, Geom g,
                                               Faces<typename Storage<S>::C> fc,
                                               Phys<typename Storage<S>::C> ph) {
  using C = typename Storage<S>::C;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  const int x = (int)(c % g.nx);
  const int y = (int)((c / g.nx) % g.ny);
  const int z = (int)(c / ((long long)g.nx * g.ny));
  const Node n = classify(g, x, y, z);
  C sf = C(0), sg = C(0);
#pragma unroll
  for (int i = 0; i < 19; ++i) sf += Storage<S>::load(fpop + pidx(g, 19, i, x, y, z));
  if (n.count > 0) {
    C gf[7];
    C sum = C(0);
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      gf[i] = Storage<S>::load(gpop + pidx(g, 7, i, x + n.ix, y + n.iy, z + n.iz));
      sum += gf[i];
    }
    const C Tb = boundary_T(g, fc, n.prio, x, y);
    const C d = Tb - ph.T_ref - sum;  // T_b - T(x_f), both relative to T_ref
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      const C w = i == 0 ? ph.w0 : ph.w1;
      S v;
      Storage<S>::store(&v, gf[i] + w * d);
      Storage<S>::store(gpop + pidx(g, 7, i, x, y, z), Storage<S>::load(&v));
      sg += Storage<S>::load(&v);
    }
  } else {
#pragma unroll
    for (int i = 0; i < 7; ++i) sg += Storage<S>::load(gpop + pidx(g, 7, i, x, y, z));
  }
  C rho = ph.rho_ref + sf;
  if (n.pressure) rho = fc.face_rho[n.prio];
  const C T = ph.T_ref + sg;
  const C rad = psi_radicand(rho, T, ph);
  if (nonphysical(rho, T, rad, ph)) flag[0] = 1;
  rho_out[c] = rho;
  T_out[c] = T;
  psi_out[c] = sqrt(rad);
}

// Constant-pressure outlet (Sec. 3.3) at a node of exactly one pressure face
// k: the +z derivation mapped to face k by the lattice symmetry taking its
// outward normal to +z.  f holds deviations; unknowns (c.n = -1) are filled.
template <typename C>
__host__ __device__ __forceinline__ void outlet_fill(C* f, int k, C rho_out, const C* F, const Phys<C>& ph) {
  const int a = k >> 1;
  const int s = (k & 1) ? 1 : -1;
  C sig0 = C(0), sig1 = C(0), t0 = C(0), t1 = C(0);
  const int ta = a == 0 ? 1 : 0;   // first tangent axis
  const int tb = a == 2 ? 1 : 2;   // second tangent axis
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const int c3[3] = {CX[i], CY[i], CZ[i]};
    const int cn = c3[a] * s;
    if (cn == 0) {
      sig0 += f[i];
      t0 += C(c3[ta]) * f[i];
      t1 += C(c3[tb]) * f[i];
    } else if (cn == 1) {
      sig1 += f[i];
    }
  }
  const C Fn = C(s) * F[a];
  // full-population sums: sig0 + 2 sig1 + rho_ref (rest weights of those links sum to 1)
  const C un = (sig0 + C(2) * sig1 + ph.rho_ref + C(0.5) * Fn - rho_out) / rho_out;
  const C da = -C(0.5) * t0 - C(0.25) * F[ta];
  const C db = -C(0.5) * t1 - C(0.25) * F[tb];
  const C dn = -Fn / C(8);
  const C ru = rho_out * un;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const int c3[3] = {CX[i], CY[i], CZ[i]};
    if (c3[a] * s != -1) continue;
    const int j = opp19(i);
    if (c3[ta] == 0 && c3[tb] == 0) {
      f[i] = f[j] - ru / C(3);
    } else {
      f[i] = f[j] - ru / C(6) + C(c3[ta]) * da + C(c3[tb]) * db - dn;
    }
  }
}

template <typename S>
__global__ void __launch_bounds__(256) k_force(S* __restrict__ fpop, const typename Storage<S>::C* __restrict__ rho_f,
                                               const typename Storage<S>::C* __restrict__ psi,
                                               typename Storage<S>::C* __restrict__ ueq,
                                               typename Storage<S>::C* __restrict__ du,
                                               typename Storage<S>::C* __restrict__ ureal, Geom g,
                                               Faces<typename Storage<S>::C> fc,
                                               Phys<typename Storage<S>::C> ph) {
  using C = typename Storage<S>::C;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  const int x = (int)(c % g.nx);
  const int y = (int)((c / g.nx) % g.ny);
  const int z = (int)(c / ((long long)g.nx * g.ny));
  // eq. (6): F = -G psi(x) sum_i varpi(|c_i|^2) psi(x + c_i) c_i
  C ax = C(0), ay = C(0), az = C(0);
#pragma unroll
  for (int i = 1; i < 19; ++i) {
    const C wgt = i < 7 ? C(1) / C(6) : C(1) / C(12);
    const C pn = psi_at(psi, g, ph.kappa_w, x + CX[i], y + CY[i], z + CZ[i]);
    if (CX[i]) ax += wgt * C(CX[i]) * pn;
    if (CY[i]) ay += wgt * C(CY[i]) * pn;
    if (CZ[i]) az += wgt * C(CZ[i]) * pn;
  }
  const C pc = -ph.G * psi[c];
  C F[3] = {pc * ax, pc * ay, pc * az};
  const C rho = rho_f[c];
  C f[19];
#pragma unroll
  for (int i = 0; i < 19; ++i) f[i] = Storage<S>::load(fpop + pidx(g, 19, i, x, y, z));
  const Node n = classify(g, x, y, z);
  if (n.pressure) {
    const C rout = fc.face_rho[n.prio];
    if (n.count == 1) {
      outlet_fill(f, n.pface, rout, F, ph);
    } else {
      // edge / corner of pressure faces: non-equilibrium extrapolation of
      // every population from the inward diagonal neighbour x_f
      C ff[19];
      C sfr = C(0), jx = C(0), jy = C(0), jz = C(0);
#pragma unroll
      for (int i = 0; i < 19; ++i) {
        ff[i] = Storage<S>::load(fpop + pidx(g, 19, i, x + n.ix, y + n.iy, z + n.iz));
        sfr += ff[i];
        jx += C(CX[i]) * ff[i];
        jy += C(CY[i]) * ff[i];
        jz += C(CZ[i]) * ff[i];
      }
      const C rf = ph.rho_ref + sfr;
      const C vx = jx / rf, vy = jy / rf, vz = jz / rf;
      const C dr = rout - rf;
      const C usq = vx * vx + vy * vy + vz * vz;
#pragma unroll
      for (int i = 0; i < 19; ++i) {
        const C cu = C(CX[i]) * vx + C(CY[i]) * vy + C(CZ[i]) * vz;
        f[i] = ff[i] + dr * w19<C>(i) * (C(1) + C(3) * cu + C(4.5) * cu * cu - C(1.5) * usq);
      }
    }
#pragma unroll
    for (int i = 0; i < 19; ++i) Storage<S>::store(fpop + pidx(g, 19, i, x, y, z), f[i]);
  }
  C jx = C(0), jy = C(0), jz = C(0);
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    if (CX[i]) jx += C(CX[i]) * f[i];
    if (CY[i]) jy += C(CY[i]) * f[i];
    if (CZ[i]) jz += C(CZ[i]) * f[i];
  }
  const C dux = F[0] / rho, duy = F[1] / rho, duz = F[2] / rho;
  C ux = jx / rho, uy = jy / rho, uz = jz / rho;
  if (n.wall) {  // Sec. 3.1: the real velocity at a wall node is set to 0
    ux = -C(0.5) * dux;
    uy = -C(0.5) * duy;
    uz = -C(0.5) * duz;
  }
  ueq[c] = ux;
  ueq[c + g.N] = uy;
  ueq[c + 2 * g.N] = uz;
  du[c] = dux;
  du[c + g.N] = duy;
  du[c + 2 * g.N] = duz;
  {  // the real velocity of eq. (5), in the operation order of u_at
    ureal[c] = ux + C(0.5) * dux;
    ureal[c + g.N] = uy + C(0.5) * duy;
    ureal[c + 2 * g.N] = uz + C(0.5) * duz;
  }
}

// Isotropic divergence of the real velocity at (x, y, z):
// (1/c_s^2) sum_i w_i c_i . u(x + c_i), with the ghost rules of u_real_at.
// The one definition serves the step and the adjoint's stored fields.
template <typename C>
__device__ __forceinline__ C div_u_at(const C* __restrict__ ureal, const Geom& g, int x, int y, int z) {
  C div = C(0);
#pragma unroll
  for (int i = 1; i < 19; ++i) {
    C vx, vy, vz;
    u_real_at(ureal, g, x + CX[i], y + CY[i], z + CZ[i], vx, vy, vz);
    div += C(3) * w19<C>(i) * (C(CX[i]) * vx + C(CY[i]) * vy + C(CZ[i]) * vz);
  }
  return div;
}

template <typename S>
__global__ void __launch_bounds__(256) k_collide_push(const S* __restrict__ fA, const S* __restrict__ gA,
                                                      S* __restrict__ fB, S* __restrict__ gB,
                                                      const typename Storage<S>::C* __restrict__ rho_f,
                                                      const typename Storage<S>::C* __restrict__ T_f,
                                                      const typename Storage<S>::C* __restrict__ ueq,
                                                      const typename Storage<S>::C* __restrict__ du,
                                                      const typename Storage<S>::C* __restrict__ ureal,
                                                      const typename Storage<S>::C* __restrict__ Th1,
                                                      typename Storage<S>::C* __restrict__ Th2, int corr,
                                                      typename Storage<S>::C* __restrict__ div_out, Geom g,
                                                      Phys<typename Storage<S>::C> ph) {
  using C = typename Storage<S>::C;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  const int x = (int)(c % g.nx);
  const int y = (int)((c / g.nx) % g.ny);
  const int z = (int)(c / ((long long)g.nx * g.ny));
  const long long N = g.N;
  const C rho = rho_f[c];
  const C T = T_f[c];
  const C ux = ueq[c], uy = ueq[c + N], uz = ueq[c + 2 * N];
  const C dux = du[c], duy = du[c + N], duz = du[c + 2 * N];
  // div u, kept for the adjoint when div_out is given
  const C div = div_u_at(ureal, g, x, y, z);
  if (div_out) div_out[c] = div;
  C gp[7];
#pragma unroll
  for (int i = 0; i < 7; ++i) gp[i] = Storage<S>::load(gA + pidx(g, 7, i, x, y, z));
  const C vf = vflux_at(rho, ph);
  C gx, gy, gz;
  local_gradT(gp, vf, ph, gx, gy, gz);
  const C rux = ux + C(0.5) * dux, ruy = uy + C(0.5) * duy, ruz = uz + C(0.5) * duz;
  C Fbar = rho * ph.cv * (rux * gx + ruy * gy + ruz * gz) + T * pr_dpdT(rho, T, ph) * div;
  if (corr) {
    // eq. (16), vartheta = 1: S_i = w_i rho c_v (dt/2) d2T/dt2 with the
    // backward difference T(t) - 2 T(t-1) + T(t-2); Th1 holds T(t-1), Th2
    // holds T(t-2) and receives T(t)
    if (corr == 2) Fbar -= C(0.5) * rho * ph.cv * (T - C(2) * Th1[c] + Th2[c]);
    Th2[c] = T;
  }
  C f[19];
#pragma unroll
  for (int i = 0; i < 19; ++i) f[i] = Storage<S>::load(fA + pidx(g, 19, i, x, y, z));
  collide19(f, rho, rho - ph.rho_ref, ux, uy, uz, dux, duy, duz, ph);
  collide7(gp, Fbar, vf, ph);
  // push streaming, eq. (9); links leaving through a wall bounce back (eq. (34))
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    int xd = x + CX[i], yd = y + CY[i], zd = z + CZ[i];
    bool ok = true, bounce = false;
    if (xd < 0 || xd >= g.nx) {
      if (g.face[0] == FACE_PERIODIC) xd = wrapp(xd, g.nx); else ok = false;
    }
    if (yd < 0 || yd >= g.ny) {
      if (g.face[2] == FACE_PERIODIC) yd = wrapp(yd, g.ny); else ok = false;
    }
    if (zd < 0 || zd >= g.nz) {
      const int k = zd < 0 ? 4 : 5;
      if (g.face[k] == FACE_PERIODIC) zd = wrapp(zd, g.nz);
      else {
        ok = false;
        bounce = g.face[k] == FACE_WALL;
      }
    }
    if (ok) Storage<S>::store(fB + pidx(g, 19, i, xd, yd, zd), f[i]);
    else if (bounce) Storage<S>::store(fB + pidx(g, 19, opp19(i), x, y, z), f[i]);
  }
  // D3Q7 push with the rho c_v blend of eq. (13), rho at the destination, time t
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    int xd = x + CX[i], yd = y + CY[i], zd = z + CZ[i];
    bool ok = true;
    if (xd < 0 || xd >= g.nx) {
      if (g.face[0] == FACE_PERIODIC) xd = wrapp(xd, g.nx); else ok = false;
    }
    if (yd < 0 || yd >= g.ny) {
      if (g.face[2] == FACE_PERIODIC) yd = wrapp(yd, g.ny); else ok = false;
    }
    if (zd < 0 || zd >= g.nz) {
      if (g.face[4] == FACE_PERIODIC) zd = wrapp(zd, g.nz); else ok = false;
    }
    if (!ok) continue;
    const long long cd = cell_index(g, xd, yd, zd);
    const C gold = Storage<S>::load(gA + pidx(g, 7, i, xd, yd, zd));
    const C inv = C(1) / (rho_f[cd] * ph.cv);
    Storage<S>::store(gB + pidx(g, 7, i, xd, yd, zd), gold + (gp[i] - gold) * inv);
  }
}

// ---------------------------------------------------------------- init / output

template <typename S>
__global__ void __launch_bounds__(256) k_init(S* __restrict__ fpop, S* __restrict__ gpop,
                                              const double* __restrict__ rho, const double* __restrict__ u,
                                              const double* __restrict__ T, long long c0, long long len,
                                              long long PS, long long pitch, double rho_ref, double T_ref,
                                              double w0, double w1) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= len) return;
  const long long c = c0 + t;
  const long long zc = c / PS, xy = c - zc * PS;
  const double r = rho[t];
  const double vx = u ? u[t] : 0.0, vy = u ? u[t + len] : 0.0, vz = u ? u[t + 2 * len] : 0.0;
#pragma unroll
  for (int i = 0; i < 19; ++i)
    Storage<S>::store(fpop + (zc * 19 + i) * pitch + xy,
                      (typename Storage<S>::C)feq19_dev<double>(i, r, rho_ref, vx, vy, vz));
  const double dT = T[t] - T_ref;
#pragma unroll
  for (int i = 0; i < 7; ++i)
    Storage<S>::store(gpop + (zc * 7 + i) * pitch + xy, (typename Storage<S>::C)((i == 0 ? w0 : w1) * dT));
}

template <typename C>
__global__ void __launch_bounds__(256) k_fields_out(const C* __restrict__ rho, const C* __restrict__ T,
                                                    const C* __restrict__ ueq, const C* __restrict__ du,
                                                    double* __restrict__ orho, double* __restrict__ ou,
                                                    double* __restrict__ oT, long long c0, long long len,
                                                    long long N, long long ustride) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= len) return;
  const long long c = c0 + t;
  if (orho) orho[t] = (double)rho[c];
  if (oT) oT[t] = (double)T[c];
  if (ou) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
      ou[t + a * ustride] = (double)(ueq[c + a * N] + C(0.5) * du[c + a * N]);
  }
}

template <typename S>
__global__ void __launch_bounds__(256) k_pops_out(const S* __restrict__ fpop, const S* __restrict__ gpop,
                                                  double* __restrict__ of, double* __restrict__ og,
                                                  long long c0, long long len, long long PS, long long pitch,
                                                  double rho_ref, double T_ref, double w0, double w1) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= len) return;
  const long long c = c0 + t;
  const long long zc = c / PS, xy = c - zc * PS;
  if (of) {
#pragma unroll
    for (int i = 0; i < 19; ++i)
      of[t + i * len] = (double)Storage<S>::load(fpop + (zc * 19 + i) * pitch + xy) + w19<double>(i) * rho_ref;
  }
  if (og) {
#pragma unroll
    for (int i = 0; i < 7; ++i)
      og[t + i * len] = (double)Storage<S>::load(gpop + (zc * 7 + i) * pitch + xy) + (i == 0 ? w0 : w1) * T_ref;
  }
}

// ---------------------------------------------------------------- FP64 reductions

constexpr int RED_BLOCKS = 1024;
constexpr int RED_THREADS = 256;
constexpr int RED_VALUES = 4;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Per block partial sums of (rho, rho c_v T, [rho > mid], clip fraction) in a
// fixed order: grid-stride over cells, wavefront shuffles, then LDS.
template <typename C>
__global__ void __launch_bounds__(RED_THREADS) k_diag_partials(const C* __restrict__ rho, const C* __restrict__ T,
                                                               long long N, double cv, double rv, double rl,
                                                               double* __restrict__ partials) {
  double acc[RED_VALUES] = {0.0, 0.0, 0.0, 0.0};
  const double mid = 0.5 * (rv + rl);
  const double inv = 1.0 / (rl - rv);
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N;
       c += (long long)gridDim.x * blockDim.x) {
    const double r = (double)rho[c];
    acc[0] += r;
    acc[1] += r * cv * (double)T[c];
    acc[2] += r > mid ? 1.0 : 0.0;
    acc[3] += fmin(fmax((r - rv) * inv, 0.0), 1.0);
  }
  __shared__ double red[RED_THREADS / 64][RED_VALUES];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < RED_VALUES; ++k) {
    const double s = wave_sum(acc[k]);
    if (lane == 0) red[wave][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < RED_VALUES) {
    double s = 0.0;
    for (int w = 0; w < RED_THREADS / 64; ++w) s += red[w][threadIdx.x];
    partials[blockIdx.x * RED_VALUES + threadIdx.x] = s;
  }
}

__global__ void __launch_bounds__(RED_THREADS) k_diag_final(const double* __restrict__ partials, int nblocks,
                                                            double* __restrict__ out) {
  double acc[RED_VALUES] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
#pragma unroll
    for (int k = 0; k < RED_VALUES; ++k) acc[k] += partials[b * RED_VALUES + k];
  }
  __shared__ double red[RED_THREADS / 64][RED_VALUES];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < RED_VALUES; ++k) {
    const double s = wave_sum(acc[k]);
    if (lane == 0) red[wave][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < RED_VALUES) {
    double s = 0.0;
    for (int w = 0; w < RED_THREADS / 64; ++w) s += red[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

}  // namespace lbm

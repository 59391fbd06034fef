// Discrete adjoint of one coupled time step (reverse mode of the stages of
// Huang, Wang, He & Huang, arXiv 2206.00946, Sec. 2 and 3), for domains
// periodic in x and y with periodic, wall or pressure z faces.
//
// Forward stages of step t (state s_t -> s_{t+1}) and their reverse, in the
// order the kernels below run them:
//   S9/S10 push + blend, S8 D3Q7 collision, S7 D3Q19 collision, S6 source
//                                            -> k_adj_collide (per cell, gathers)
//   S6 divergence stencil, S5 velocities    -> k_adj_velocity
//   S4 outlet fill                           -> k_adj_outlet (pressure planes)
//   eq. (37) wetting ghost layer             -> k_adj_ghost (wall planes)
//   S3 force stencil, S2 psi, S1 moments     -> k_adj_psi
//   S0 thermal Dirichlet (eqs. (35)-(36))    -> k_adj_dirichlet (face planes)
// Each kernel consumes the forward fields of step t (rho, T, psi, u_eq, du
// recomputed from the stored state) and the adjoint of s_{t+1}; together they
// give the adjoint of s_t and add the step's contribution to dJ/dT_w and
// dJ/dkappa_w.  Adjoints are held in the compute type C in the population
// layout of the state; gradients accumulate in FP64.
//
// Deferred moment update.  The reverse of S1 (rho = sum f, T = sum g) adds
// the same rho-adjoint rb and momentum adjoint jb to every f_i (as rb +
// c_i . jb) and the T-adjoint Tb to every g_i of a cell.  k_adj_psi stores
// those five values per cell, d = (rb, jb_x, jb_y, jb_z, Tb), instead of
// reading and rewriting the 26 adjoint populations, and the adjoint of s_t
// is the pair (l~, d): lf_i = l~f_i + rb + c_i . jb, lg_i = l~g_i + Tb.
// k_adj_collide of the next reverse step adds d where it gathers, and
// k_adj_dirichlet where it reads the face planes.
#pragma once

#include "adjoint.h"
#include "kernels_ref.h"

namespace lbm {

// z one step outside the domain: wrap if periodic and report whether the
// node exists.
__device__ __forceinline__ bool z_inside(const Geom& g, int& z) {
  if (z >= 0 && z < g.nz) return true;
  if (g.face[z < 0 ? 4 : 5] == FACE_PERIODIC) {
    z = wrapp(z, g.nz);
    return true;
  }
  return false;
}

// Neighbour addressing of cell (x, y, z) with x and y periodic: in-plane
// offsets of x +- 1 and y +- 1 with wrap, and the levels z - 1, z, z + 1
// (wrapped when z is periodic; zin false beyond a bounded face).  Replaces
// the per-neighbour 64-bit index arithmetic of cell_index / pidx.
struct AdjNbr {
  int col;
  int ox[3], oy[3];
  int zl[3];
  bool zin[3];
  long long PS, pitch;
  __device__ __forceinline__ AdjNbr(const Geom& g, int x, int y, int z) {
    col = x + g.nx * y;
    ox[0] = x == 0 ? g.nx - 1 : -1;
    ox[1] = 0;
    ox[2] = x == g.nx - 1 ? 1 - g.nx : 1;
    oy[0] = y == 0 ? (g.ny - 1) * g.nx : -g.nx;
    oy[1] = 0;
    oy[2] = y == g.ny - 1 ? (1 - g.ny) * g.nx : g.nx;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      zl[d] = z + d - 1;
      zin[d] = z_inside(g, zl[d]);
    }
    PS = (long long)g.nx * g.ny;
    pitch = g.pitch;
  }
  // column of x + s c_i (s = +1 or -1)
  __device__ __forceinline__ int ncol(int i, int s) const { return col + ox[s * CX[i] + 1] + oy[s * CY[i] + 1]; }
  // cell index and population index at column cl, level zz
  __device__ __forceinline__ long long cell(int zz, int cl) const { return (long long)zz * PS + cl; }
  __device__ __forceinline__ long long pop(int Q, int i, int zz, int cl) const {
    return ((long long)zz * Q + i) * pitch + cl;
  }
};

template <typename C>
__device__ __forceinline__ C varpi(int i) {
  return i < 7 ? C(1) / C(6) : C(1) / C(12);
}

// adjoint state at t = N of J = M(0) - M(N): dJ/df_i = -1 where rho = sum f
template <typename C>
__global__ void __launch_bounds__(256) k_adj_seed(C* __restrict__ lf, C* __restrict__ lg, C* __restrict__ d,
                                                  Geom g) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  const int x = (int)(c % g.nx);
  const int y = (int)((c / g.nx) % g.ny);
  const int z = (int)(c / ((long long)g.nx * g.ny));
  const Node n = classify(g, x, y, z);
  const C v = n.pressure ? C(0) : C(-1);
#pragma unroll
  for (int i = 0; i < 19; ++i) lf[pidx(g, 19, i, x, y, z)] = v;
#pragma unroll
  for (int i = 0; i < 7; ++i) lg[pidx(g, 7, i, x, y, z)] = C(0);
#pragma unroll
  for (int k = 0; k < 5; ++k) d[c + k * g.N] = C(0);
}

// div u of a state from its stored real velocity, with the step's own
// definition (div_u_at), for states whose fields no recomputed step wrote.
template <typename C>
__global__ void __launch_bounds__(256) k_div(const C* __restrict__ ureal, C* __restrict__ div_out, Geom g) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  const int x = (int)(c % g.nx);
  const int y = (int)((c / g.nx) % g.ny);
  const int z = (int)(c / ((long long)g.nx * g.ny));
  div_out[c] = div_u_at(ureal, g, x, y, z);
}

// Reverse of S10, S9, S8, S7 and the local part of S6 at every cell x.
//   lfi, lgi: adjoint of s_{t+1}; gA: post-Dirichlet g of s_t; gnext: g of s_{t+1}
//   lfo, lgo: partial adjoint of the completed f, g of s_t
//   a_rho, a_T: partial adjoints of rho and T; a_ueq, a_du: of u_eq and du
//   (the wall override of S5 already applied); a_div: of div u at x
template <typename S>
__global__ void __launch_bounds__(256)
    k_adj_collide(const typename Storage<S>::C* __restrict__ lfi, const typename Storage<S>::C* __restrict__ lgi,
                  const typename Storage<S>::C* __restrict__ di, const S* __restrict__ gA, const S* __restrict__ gnext,
                  const typename Storage<S>::C* __restrict__ rho_f, const typename Storage<S>::C* __restrict__ T_f,
                  const typename Storage<S>::C* __restrict__ ueq, const typename Storage<S>::C* __restrict__ du,
                  const typename Storage<S>::C* __restrict__ divf,
                  typename Storage<S>::C* __restrict__ lfo, typename Storage<S>::C* __restrict__ lgo,
                  typename Storage<S>::C* __restrict__ a_rho, typename Storage<S>::C* __restrict__ a_T,
                  typename Storage<S>::C* __restrict__ a_ueq, typename Storage<S>::C* __restrict__ a_du,
                  typename Storage<S>::C* __restrict__ a_div, Geom g, Phys<typename Storage<S>::C> ph) {
  using C = typename Storage<S>::C;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  const int x = (int)(c % g.nx);
  const int y = (int)((c / g.nx) % g.ny);
  const int z = (int)(c / ((long long)g.nx * g.ny));
  const long long N = g.N;
  const Node n = classify(g, x, y, z);
  const C rho = rho_f[c], T = T_f[c];
  const C ux = ueq[c], uy = ueq[c + N], uz = ueq[c + 2 * N];
  const C dux = du[c], duy = du[c + N], duz = du[c + 2 * N];
  const AdjNbr nb(g, x, y, z);
  const int col = nb.col;
  auto ncol = [&](int i) { return nb.ncol(i, 1); };
  auto pop = [&](int Q, int i, int zz, int cl) { return nb.pop(Q, i, zz, cl); };
  const bool* zin = nb.zin;
  const int* zl = nb.zl;

  // adjoint of f_i, g_i of s_{t+1} at column cl, level zz: the stored part
  // plus the deferred moment update of that cell
  // (only the momentum components along c_i are read)
  auto lf_at = [&](int i, int zz, int cl) -> C {
    const long long cc = nb.cell(zz, cl);
    C v = lfi[pop(19, i, zz, cl)] + di[cc];
    if (CX[i]) v += C(CX[i]) * di[cc + N];
    if (CY[i]) v += C(CY[i]) * di[cc + 2 * N];
    if (CZ[i]) v += C(CZ[i]) * di[cc + 3 * N];
    return v;
  };
  // S9: f*_i(x) went to slot i at x + c_i, to slot opp(i) at x (wall), or
  // left the domain (outlet)
  C fsb[19];
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const int d = CZ[i] + 1;
    if (zin[d]) fsb[i] = lf_at(i, zl[d], ncol(i));
    else if (g.face[CZ[i] < 0 ? 4 : 5] == FACE_WALL) fsb[i] = lf_at(opp19(i), z, col);
    else fsb[i] = C(0);
  }
  // S10: g*_i(x) enters the blend at y = x + c_i with weight 1/(rho(y) c_v)
  C gsb[7];
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    const int d = CZ[i] + 1;
    gsb[i] = C(0);
    if (zin[d]) {
      const long long cd = nb.cell(zl[d], ncol(i));
      gsb[i] = (lgi[pop(7, i, zl[d], ncol(i))] + di[cd + 4 * N]) / (rho_f[cd] * ph.cv);
    }
  }
  C fb[19], gb[7];
  C rb = C(0);
  C ub[3] = {C(0), C(0), C(0)}, dub[3] = {C(0), C(0), C(0)};
  collide19_adj(fsb, rho, ux, uy, uz, dux, duy, duz, ph, fb, rb, ub, dub);  // S7
  C Fbarb;
  collide7_adj(gsb, ph, gb, Fbarb);  // S8

  // S6 (local part): Fbar = rho c_v u . grad T + T (dp/dT) div u
  C gp[7];
#pragma unroll
  for (int i = 0; i < 7; ++i) gp[i] = Storage<S>::load(gA + pop(7, i, z, col));
  C gx, gy, gz;
  local_gradT(gp, ph.vflux, ph, gx, gy, gz);
  const C rux = ux + C(0.5) * dux, ruy = uy + C(0.5) * duy, ruz = uz + C(0.5) * duz;
  // div u of the forward step (stored with the fields)
  const C div = divf[c];
  C dp_dr, dpdT, dpdT_dr, dpdT_dT;
  pr_partials(rho, T, ph, dp_dr, dpdT, dpdT_dr, dpdT_dT);
  rb += Fbarb * (ph.cv * (rux * gx + ruy * gy + ruz * gz) + T * dpdT_dr * div);
  C Tb = Fbarb * (dpdT + T * dpdT_dT) * div;
  const C divb = Fbarb * T * dpdT;
  const C rcv = Fbarb * rho * ph.cv;
  const C urb[3] = {rcv * gx, rcv * gy, rcv * gz};
  const C kq = -ph.vflux / ph.cs2T;  // grad T = kq * (first moments of g)
  gb[1] += kq * rcv * rux;
  gb[2] -= kq * rcv * rux;
  gb[3] += kq * rcv * ruy;
  gb[4] -= kq * rcv * ruy;
  gb[5] += kq * rcv * ruz;
  gb[6] -= kq * rcv * ruz;

  // S10 with x as the destination: g_i(x, t+1) = g_i + (g*_i(src) - g_i) / (rho c_v)
  const C inv = C(1) / (rho * ph.cv);
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    const C l = lgi[pop(7, i, z, col)] + di[c + 4 * N];
    if (zin[1 - CZ[i]]) {
      gb[i] += l * (C(1) - inv);
      if (n.count == 0) {
        // the adjoint of s_{t+1} vanishes on bounded-face nodes, where the
        // next step's Dirichlet condition overwrites g
        const C gn = Storage<S>::load(gnext + pop(7, i, z, col));
        rb -= l * (gn - gp[i]) / rho;
      }
    } else {
      gb[i] += l;
    }
  }
  // S5: u = u_eq + du/2, except at wall nodes where u = 0 and u_eq = -du/2
  if (n.wall) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      dub[a] -= C(0.5) * ub[a];
      ub[a] = C(0);
    }
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      ub[a] += urb[a];
      dub[a] += C(0.5) * urb[a];
    }
  }
#pragma unroll
  for (int i = 0; i < 19; ++i) lfo[pop(19, i, z, col)] = fb[i];
#pragma unroll
  for (int i = 0; i < 7; ++i) lgo[pop(7, i, z, col)] = gb[i];
  a_rho[c] = rb;
  a_T[c] = Tb;
  a_div[c] = divb;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    a_ueq[c + a * N] = ub[a];
    a_du[c + a * N] = dub[a];
  }
}

// Reverse of the divergence stencil (every reader of u at y) and of S5.  On
// return a_ueq holds the adjoint of the momentum j, a_du the adjoint of the
// force F, a_rho the partial adjoint of rho; k_adj_outlet then completes the
// outlet nodes (kept apart so that this kernel's registers stay few).
template <typename C>
__global__ void __launch_bounds__(256)
    k_adj_velocity(const C* __restrict__ a_div, C* __restrict__ a_ueq, C* __restrict__ a_du,
                   C* __restrict__ a_rho, const C* __restrict__ rho_f, const C* __restrict__ ueq,
                   const C* __restrict__ du, Geom g) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  const int x = (int)(c % g.nx);
  const int y = (int)((c / g.nx) % g.ny);
  const int z = (int)(c / ((long long)g.nx * g.ny));
  const long long N = g.N;
  // x and y are periodic: the bounded faces are the z planes
  const bool wall = (z == 0 && g.face[4] == FACE_WALL) || (z == g.nz - 1 && g.face[5] == FACE_WALL);
  C ueb[3], dub[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ueb[a] = a_ueq[c + a * N];
    dub[a] = a_du[c + a * N];
  }
  if (!wall) {
    // readers of u(y): x = y - c_i directly, and on an outlet plane the
    // same-plane readers whose ghost neighbour is a copy of y
    const AdjNbr nb(g, x, y, z);
    C vb[3] = {C(0), C(0), C(0)};
#pragma unroll
    for (int i = 1; i < 19; ++i) {
      const int cr = nb.ncol(i, -1);
      C d = C(0);
      if (nb.zin[1 - CZ[i]]) d += a_div[nb.cell(nb.zl[1 - CZ[i]], cr)];
      if (!nb.zin[1 + CZ[i]] && g.face[CZ[i] < 0 ? 4 : 5] == FACE_PRESSURE) d += a_div[nb.cell(z, cr)];
      d *= C(3) * w19<C>(i);
      vb[0] += C(CX[i]) * d;
      vb[1] += C(CY[i]) * d;
      vb[2] += C(CZ[i]) * d;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      ueb[a] += vb[a];
      dub[a] += C(0.5) * vb[a];
    }
  }
  const C irho = C(1) / rho_f[c];
  C rb = a_rho[c];
  C jb[3], Fb[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    // u_eq = j / rho (the wall value was moved to du in k_adj_collide), du = F / rho
    jb[a] = ueb[a] * irho;
    Fb[a] = dub[a] * irho;
    rb -= (ueb[a] * ueq[c + a * N] + dub[a] * du[c + a * N]) * irho;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    a_ueq[c + a * N] = jb[a];
    a_du[c + a * N] = Fb[a];
  }
  a_rho[c] = rb;
}

// Reverse of the outlet fill (S4) at the nodes of pressure z faces, one
// thread per (x, y), after k_adj_velocity: f_i(x_b) entered the fill and the
// momentum j, whose adjoint a_ueq carries; the fill's F part goes to a_du.
// The adjoint of f becomes final there, and a_ueq, a_rho vanish (rho =
// rho_out is fixed on outlet nodes).
template <typename C>
__global__ void __launch_bounds__(256) k_adj_outlet(C* __restrict__ lfo, C* __restrict__ a_ueq,
                                                    C* __restrict__ a_du, C* __restrict__ a_rho, Geom g) {
  const long long P = (long long)g.nx * g.ny;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P) return;
  const int x = (int)(t % g.nx), y = (int)(t / g.nx);
  const long long N = g.N;
  for (int s = 0; s < 2; ++s) {
    const int k = 4 + s;
    if (g.face[k] != FACE_PRESSURE) continue;
    const int z = s ? g.nz - 1 : 0;
    const long long c = cell_index(g, x, y, z);
    C jb[3], Fb[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      jb[a] = a_ueq[c + a * N];
      Fb[a] = a_du[c + a * N];
    }
    C fb[19];
#pragma unroll
    for (int i = 0; i < 19; ++i)
      fb[i] = lfo[pidx(g, 19, i, x, y, z)] + C(CX[i]) * jb[0] + C(CY[i]) * jb[1] + C(CZ[i]) * jb[2];
    outlet_fill_adj(fb, k, Fb);
#pragma unroll
    for (int i = 0; i < 19; ++i) lfo[pidx(g, 19, i, x, y, z)] = fb[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      a_ueq[c + a * N] = C(0);
      a_du[c + a * N] = Fb[a];
    }
    a_rho[c] = C(0);
  }
}

// Reverse of the wetting ghost layer of eq. (37) on each wall face, one
// thread per (x, y): psi_ghost = psi(x, y, z_in) + kappa_w |grad_t psi(x, y, z_w)|.
// gadj = adjoint of psi_ghost (from the force of the wall-plane readers);
// ax, ay route it to the tangential differences; kap accumulates its kappa_w
// part over the reverse sweep (FP64, one entry per wall node, summed once at
// the end).
// Planes are indexed face * nx*ny + x + nx*y, face 0 = -z, 1 = +z.
template <typename C>
__global__ void __launch_bounds__(256) k_adj_ghost(const C* __restrict__ Fb, const C* __restrict__ psi,
                                                   C* __restrict__ gadj, C* __restrict__ ax, C* __restrict__ ay,
                                                   double* __restrict__ kap, Geom g, Phys<C> ph) {
  const long long P = (long long)g.nx * g.ny;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P) return;
  const int x = (int)(t % g.nx), y = (int)(t / g.nx);
  const long long N = g.N;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (g.face[4 + s] != FACE_WALL) continue;
    const int zw = s ? g.nz - 1 : 0;
    const int out = s ? 1 : -1;
    C G = C(0);
#pragma unroll
    for (int i = 1; i < 19; ++i) {
      if (CZ[i] != out) continue;
      const long long cr = cell_index(g, wrapp(x - CX[i], g.nx), wrapp(y - CY[i], g.ny), zw);
      G += -ph.G * psi[cr] * varpi<C>(i) *
           (C(CX[i]) * Fb[cr] + C(CY[i]) * Fb[cr + N] + C(CZ[i]) * Fb[cr + 2 * N]);
    }
    const C dx = psi[cell_index(g, wrapp(x + 1, g.nx), y, zw)] - psi[cell_index(g, wrapp(x - 1, g.nx), y, zw)];
    const C dy = psi[cell_index(g, x, wrapp(y + 1, g.ny), zw)] - psi[cell_index(g, x, wrapp(y - 1, g.ny), zw)];
    const C sq = sqrt(dx * dx + dy * dy);
    gadj[s * P + t] = G;
    kap[s * P + t] += (double)(G * sq);
    // d sqrt(s) at s = 0 is taken as 0
    ax[s * P + t] = sq > C(0) ? G * ph.kappa_w * dx / sq : C(0);
    ay[s * P + t] = sq > C(0) ? G * ph.kappa_w * dy / sq : C(0);
  }
}

// Reverse of S3 (force stencil, with every ghost rule), S2 (psi) and S1
// (rho = sum f, T = sum g).  Completes the adjoint of the completed f and g
// of s_t by its deferred moment update d (rb, jb, Tb per cell).
template <typename C>
__global__ void __launch_bounds__(256)
    k_adj_psi(C* __restrict__ dO, const C* __restrict__ a_rho, const C* __restrict__ a_T,
              const C* __restrict__ jb_f, const C* __restrict__ Fb, const C* __restrict__ psi,
              const C* __restrict__ rho_f, const C* __restrict__ T_f, const C* __restrict__ gadj,
              const C* __restrict__ ax, const C* __restrict__ ay, Geom g, Phys<C> ph) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.N) return;
  const int x = (int)(c % g.nx);
  const int y = (int)((c / g.nx) % g.ny);
  const int z = (int)(c / ((long long)g.nx * g.ny));
  const long long N = g.N;
  const long long P = (long long)g.nx * g.ny;
  const Node n = classify(g, x, y, z);
  const AdjNbr nb(g, x, y, z);
  // F(y) = -G psi(y) sum_i varpi_i c_i psi(y + c_i)
  C acx = C(0), acy = C(0), acz = C(0);
  C pb = C(0);
#pragma unroll
  for (int i = 1; i < 19; ++i) {
    const int d = CZ[i] + 1;
    // psi(y + c_i): a node, or the ghost beyond a bounded z face
    const C pn = nb.zin[d] ? psi[nb.cell(nb.zl[d], nb.ncol(i, 1))]
                           : psi_at(psi, g, ph.kappa_w, x + CX[i], y + CY[i], z + CZ[i]);
    acx += varpi<C>(i) * C(CX[i]) * pn;
    acy += varpi<C>(i) * C(CY[i]) * pn;
    acz += varpi<C>(i) * C(CZ[i]) * pn;
    // y as the neighbour x + c_i of the readers x = y - c_i, and of the
    // same-plane readers beyond an outlet (ghost = copy of y)
    const int cl = nb.ncol(i, -1);
    const C wc = -ph.G * varpi<C>(i);
    if (nb.zin[1 - CZ[i]]) {
      const long long cr = nb.cell(nb.zl[1 - CZ[i]], cl);
      pb += wc * psi[cr] * (C(CX[i]) * Fb[cr] + C(CY[i]) * Fb[cr + N] + C(CZ[i]) * Fb[cr + 2 * N]);
    }
    if (!nb.zin[d] && g.face[CZ[i] < 0 ? 4 : 5] == FACE_PRESSURE) {
      const long long cr = nb.cell(z, cl);
      pb += wc * psi[cr] * (C(CX[i]) * Fb[cr] + C(CY[i]) * Fb[cr + N] + C(CZ[i]) * Fb[cr + 2 * N]);
    }
  }
  pb += -ph.G * (acx * Fb[c] + acy * Fb[c + N] + acz * Fb[c + 2 * N]);
  // wetting ghost layers: psi(x, y, z_in) enters directly, the wall plane
  // through the tangential differences
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (g.face[4 + s] != FACE_WALL) continue;
    const int zw = s ? g.nz - 1 : 0;
    const int zi = s ? g.nz - 2 : 1;
    const long long o = s * P;
    if (z == zi) pb += gadj[o + nb.col];
    if (z == zw) {
      pb += ax[o + nb.col + nb.ox[0]] - ax[o + nb.col + nb.ox[2]] + ay[o + nb.col + nb.oy[0]] -
            ay[o + nb.col + nb.oy[2]];
    }
  }
  // eq. (7): psi = sqrt(2 (p - rho/3) / G)
  const C rho = rho_f[c], T = T_f[c], ps = psi[c];
  C dp_dr, dpdT, dpdT_dr, dpdT_dT;
  pr_partials(rho, T, ph, dp_dr, dpdT, dpdT_dr, dpdT_dT);
  const C q = ps > C(0) ? pb / (ph.G * ps) : C(0);
  const C Tb = a_T[c] + q * dpdT;
  // on outlet nodes rho is fixed and the known populations took their
  // adjoint in k_adj_outlet
  const bool inner = !n.pressure;
  dO[c] = inner ? a_rho[c] + q * (dp_dr - C(1) / C(3)) : C(0);
  dO[c + N] = inner ? jb_f[c] : C(0);
  dO[c + 2 * N] = inner ? jb_f[c + N] : C(0);
  dO[c + 3 * N] = inner ? jb_f[c + 2 * N] : C(0);
  dO[c + 4 * N] = Tb;
}

// Reverse of S0 on the z faces, one thread per (x, y): g_i(x_b) = w_i T_b +
// g_i(x_f) - w_i sum_j g_j(x_f).  Adds sum_i w_i gb_i(x_b) to dJ/dT_b of the
// selected face and clears the adjoint of the overwritten g(x_b) (its
// stored part and its deferred Tb).
template <typename C>
__global__ void __launch_bounds__(256) k_adj_dirichlet(C* __restrict__ lgo, C* __restrict__ dO,
                                                       double* __restrict__ grad_Tw, int grad_face, Geom g,
                                                       Phys<C> ph) {
  const long long P = (long long)g.nx * g.ny;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P) return;
  const int x = (int)(t % g.nx), y = (int)(t / g.nx);
  for (int s = 0; s < 2; ++s) {
    const int k = 4 + s;
    if (g.face[k] == FACE_PERIODIC) continue;
    const int zb = s ? g.nz - 1 : 0;
    const int zf = s ? g.nz - 2 : 1;
    C l[7];
    C S = C(0);
    const long long cb = cell_index(g, x, y, zb);
    const C Tbd = dO[cb + 4 * g.N];
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      l[i] = lgo[pidx(g, 7, i, x, y, zb)] + Tbd;
      S += (i == 0 ? ph.w0 : ph.w1) * l[i];
    }
    dO[cb + 4 * g.N] = C(0);
    if (k == grad_face) grad_Tw[t] += (double)S;
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      lgo[pidx(g, 7, i, x, y, zf)] += l[i] - S;
      lgo[pidx(g, 7, i, x, y, zb)] = C(0);
    }
  }
}

// v[0 .. n) = 0 (accumulators of the reverse sweep; a kernel rather than a
// memset, so that the sweep enqueues only kernels and copies)
__global__ void __launch_bounds__(256) k_zero_f64(double* __restrict__ v, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = 0.0;
}

// Fixed-order sum of n values into *acc (one workgroup).
template <typename C>
__global__ void __launch_bounds__(RED_THREADS) k_accumulate(const C* __restrict__ v, long long n,
                                                            double* __restrict__ acc) {
  double s = 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) s += (double)v[i];
  __shared__ double red[RED_THREADS / 64];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < RED_THREADS / 64; ++w) t += red[w];
    acc[0] += t;
  }
}

}  // namespace lbm

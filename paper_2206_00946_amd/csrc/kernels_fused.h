// Fused single-pass step: one kernel launch per time step reads every
// population once and writes it once (Huang, Wang, He & Huang, arXiv
// 2206.00946, Sec. 2 and 3.1).
//
// Domain: periodic in x and y; z periodic, or bounded by two faces each a
// no-slip wall (ghost psi of eq. (37): the first interior layer plus kappa_w
// times the tangential difference magnitude on the wall layer) or a
// constant-pressure outlet (Sec. 3.3: rho = rho_out on the face, unknown
// populations filled, ghost psi and u copies of the face node).  ny must be
// a multiple of the tile height; nx is any size >= 8 (the last tile column of
// a ragged nx is partly idle, see below).  Other set-ups use the unfused
// kernels.
//
// A workgroup owns a 64 x TY column tile (one wavefront per row, one thread
// per column) and marches through z.  For every plane p it loads the
// populations of the tile plus a two-cell halo in x and y and keeps
//   psi (eq. (7))           -> LDS ring of 3 planes, 2-cell halo
//   rho, u_eq = j/rho       -> LDS rings, 1-cell halo
// The interaction force of plane p-1 (eq. (6)) then gives the real velocity
// u (eq. (5)) on a 1-cell halo, the D3Q19 MRT-EDM collision of plane p-1
// (eq. (8)) and its push (eq. (9), bounce-back eq. (34)).  The divergence of
// u is accumulated plane by plane, so the D3Q7 collision (eqs. (13)-(15))
// runs on plane p-2.  The rho*c_v blend of eq. (13) needs the old g_i at the
// destination: in-tile in-plane transfers are finished by the destination
// one plane later (its own old value, the source's g* through LDS); transfers
// leaving the tile use the halo's old values kept in a small LDS ring; z
// transfers stay in the thread's column registers.
// Dirichlet temperatures on bounded-face nodes (eqs. (35)-(36)) are applied
// to the values loaded for a face plane, from the next plane inward; a time
// step is exactly one launch of this kernel.
//
// Ragged nx: tiles start every 64 columns and the last one holds
// W = nx - x0 < 64 cells.  Its lanes tx >= W take the cells that follow
// periodically (x0 + tx mod nx), so the stencils of the W active cells read
// the right neighbours from LDS; those lanes compute but store nothing, except
// that lane W finishes the +x D3Q7 link coming from the active cell W-1 (its
// destination, cell x0 + W mod nx, gets that link from no other tile).
#pragma once

#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "lbm3d.h"
#include "kernels_ref.h"

namespace lbm {

constexpr int FTX = 64;
// D3Q19 directions pushed before the second barrier of a steady plane step
constexpr int kEarlyF = 10;
// cache policy of the population stores: non-temporal (2) for FP64, where
// it shortens the step by about 3 %; the default policy for the narrower
// formats, where non-temporal stores are slower (FP32 +11 %)
template <typename S>
constexpr int store_cache_policy() { return sizeof(S) == 8 ? 2 : 0; }

// Optional per-cell outputs of a step (the adjoint's recomputation keeps
// them for the reverse sweep): rho, T, psi (S1-S2), u_eq, du = F/rho and the
// real velocity (S5, 3 components each, component planes of N cells), div u
// (S6), all of the state the step starts from, flat index x + nx (y + ny z).
template <typename C>
struct FusedFields {
  C *rho, *T, *psi, *ueq, *du, *ureal, *div;
};

template <typename C>
struct FusedArgs {
  Phys<C> ph;
  int nx, ny, nz;
  long long pitch;  // elements from one direction plane to the next
  int zbound;      // 1: z bounded by the faces at z = 0 and z = nz - 1; 0: periodic z
  int zpres[2];    // bounded face is a pressure outlet (1) or a no-slip wall (0)
  C face_rho[2];   // rho_out of a pressure face
  int tiles_x, ntiles, chunk;
  int xcd_blocks;  // 1: each XCD owns a 2 x 4 block of the tile grid
  C wall_T[2];            // Dirichlet temperatures of the z = 0 and z = nz - 1 faces
  const double* wall_Tw[2];  // optional per-cell face temperature fields (nx*ny)
  int* flag;
  FusedFields<C> fo;  // written by the FLD instantiation only
  void* g_face;       // FLD: the start state's g, whose bounded-face planes get the Dirichlet completion
};

template <int TY>
struct Tile {
  static constexpr int TX = FTX;
  static constexpr int NT = TX * TY;
  static constexpr int EX = TX + 4;
  static constexpr int EY = TY + 4;
  static constexpr int E2 = EX * EY;                  // tile + 2-cell halo
  static constexpr int NH = E2 - NT;                  // halo cells
  static constexpr int NR1 = (TX + 2) * (TY + 2) - NT;  // first halo ring
  static constexpr int NGR = 2 * TX + 2 * TY;         // ring cells fed by in-plane D3Q7 links
  static_assert(NT >= NH && NT >= NR1, "tile too small for one helper cell per thread");

  __device__ static int interior_e(int tx, int ty) { return (ty + 2) * EX + tx + 2; }

  // k-th cell of the 2-cell halo: two full rows below, 4 side cells per
  // interior row, two full rows above
  __device__ static void halo_cell(int k, int& ex, int& ey) {
    if (k < 2 * EX) {
      ey = k / EX;
      ex = k % EX;
    } else if (k < 2 * EX + 4 * TY) {
      const int m = k - 2 * EX;
      ey = 2 + m / 4;
      const int c = m % 4;
      ex = c < 2 ? c : EX - 4 + c;
    } else {
      const int m = k - 2 * EX - 4 * TY;
      ey = TY + 2 + m / EX;
      ex = m % EX;
    }
  }

  // k-th cell of the first halo ring
  __device__ static void ring1_cell(int k, int& ex, int& ey) {
    if (k < TX + 2) {
      ey = 1;
      ex = 1 + k;
    } else if (k < TX + 2 + 2 * TY) {
      const int m = k - (TX + 2);
      ey = 2 + m / 2;
      ex = (m & 1) ? EX - 2 : 1;
    } else {
      ey = TY + 2;
      ex = 1 + (k - (TX + 2) - 2 * TY);
    }
  }

  // ring cell fed by an in-plane D3Q7 link leaving the tile: its slot in the
  // ring of old values and the direction (1 +x, 2 -x, 3 +y, 4 -y), or -1
  __device__ static int receiver(int ex, int ey, int& dir) {
    if (ex == EX - 2 && ey >= 2 && ey < TY + 2) { dir = 1; return ey - 2; }
    if (ex == 1 && ey >= 2 && ey < TY + 2) { dir = 2; return TY + ey - 2; }
    if (ey == TY + 2 && ex >= 2 && ex < TX + 2) { dir = 3; return 2 * TY + ex - 2; }
    if (ey == 1 && ex >= 2 && ex < TX + 2) { dir = 4; return 2 * TY + TX + ex - 2; }
    dir = 0;
    return -1;
  }
};

__device__ __forceinline__ int wrapn(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Node of a z pressure face (hi: the face at z = nz - 1, else z = 0), Sec.
// 3.3.  After streaming the node knows the populations with c_z = 0 or c_z
// pointing out of the domain; the outlet condition uses their combination
// rho_ref + sum_{c_z = 0} f + 2 sum_{c_z outward} f (deviations).
template <typename C>
__device__ __forceinline__ C outlet_known(const C* f, int hi, C rho_ref) {
  C s0 = C(0), s1 = C(0);
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    if (CZ[i] == 0) s0 += f[i];
    else if (CZ[i] == (hi ? 1 : -1)) s1 += f[i];
  }
  return s0 + C(2) * s1 + rho_ref;
}
// u_eq = j / rho_out at such a node from the known sum kn and the force F:
// the filled populations carry the tangential momenta -F_x/2, -F_y/2 (the
// real tangential velocity is zero) and the outward momentum
// rho_out u_n - F_n/2 with u_n = (kn + F_n/2 - rho_out) / rho_out.  Equal to
// filling the unknowns and summing c_i f_i, up to rounding, and the same on
// whichever thread evaluates it.
template <typename C>
__device__ __forceinline__ void outlet_ueq(C kn, int hi, C rho_out, C Fx, C Fy, C Fz, C& ux, C& uy, C& uz) {
  const C sn = hi ? C(1) : C(-1);
  const C Fn = sn * Fz;
  const C ir = rcp(rho_out);
  const C un = (kn + C(0.5) * Fn - rho_out) * ir;
  ux = (-C(0.5) * Fx) * ir;
  uy = (-C(0.5) * Fy) * ir;
  uz = sn * (rho_out * un - C(0.5) * Fn) * ir;
}

// Population access with the plane-major layout: one buffer descriptor over
// all directions of one plane (uniform, scalar registers), the direction as a
// scalar byte offset (i * plane bytes) and the cell as a per-lane byte offset.
template <typename S>
__device__ __forceinline__ typename Storage<S>::C ld_at(const S* plane, unsigned bytes, unsigned voff,
                                                        unsigned soff) {
  return Buf<S>::load(buffer_range(plane, bytes), voff, soff);
}
template <typename S>
__device__ __forceinline__ void st_at(S* plane, unsigned bytes, unsigned voff, unsigned soff,
                                      typename Storage<S>::C v) {
  Buf<S>::template store<store_cache_policy<S>()>(buffer_range(plane, bytes), voff, soff, v);
}

// OUT: the set-up has a pressure z face.  Closed and periodic set-ups run
// the instantiation without the outlet code, which keeps that code's scalar
// registers out of the march.  RAG: nx is not a multiple of 64 (a last tile
// column with idle lanes); with whole tiles every lane stores, and the
// instantiation carries no lane predicate around its stores (the predicate
// costs the 16-bit steps 8 %).  FLD: also write the fields of the start
// state (FusedFields) and its Dirichlet-completed face-plane g, as the
// general kernels' prepass leaves them (adjoint recomputation, 8-row
// tiles).  A face-plane g may be rewritten while a neighbouring tile loads
// it as halo: that tile replaces the loaded value by the same completion,
// which reads only the plane inside.
// XP: x-deferred streaming between the steps of one multi-step call (whole
// 8-row tiles).  A D3Q19 population f*_i(x, y, z) may be stored at
// (x, y + c_iy, z + c_iz), streamed in y and z only; the step that reads
// such a state takes direction i of cell x from column x - c_ix, which
// finishes the streaming (eq. (9)) at load time.  Every wave then stores
// whole rows in place of rows shifted by one cell, which touch one more
// cache line each, and the shifted loads fall in the lines the side halo
// brings in anyway.  Bit 0: the input is such a state; bit 1: the output is
// (the first step of a call reads, and its last step writes, the ordinary
// post-streaming state).  The D3Q7 populations are streamed as always.
// Used for FP64 storage, whose non-temporal stores of shifted rows write
// partial lines (512 x 512 x 384: 10.6 -> 9.8 ms per step); with 4- and
// 2-byte storage the shifted loads add as many line requests as the stores
// save (FP32 4.94 -> 5.04 ms, FP16 3.96 -> 4.29 ms), and those steps store
// shifted rows.
template <typename S, int TY, bool OUT, bool RAG, bool FLD = false, int XP = 0>
__global__ void __launch_bounds__(FTX * TY) k_fused(const S* __restrict__ fA, const S* __restrict__ gA,
                                                   S* __restrict__ fB, S* __restrict__ gB,
                                                   FusedArgs<typename Storage<S>::C> a) {
  using C = typename Storage<S>::C;
  using TL = Tile<TY>;
  constexpr int TX = TL::TX, NT = TL::NT, EX = TL::EX, E2 = TL::E2;
  __shared__ C s_psi[3][E2];
  __shared__ C s_rho[4][E2];
  __shared__ C s_ueq[2][3][E2];
  __shared__ C s_u[3][E2];
  __shared__ C s_gr[4][TL::NGR];
  __shared__ C s_gs[4][NT];

  const Phys<C> ph = a.ph;
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  int b = blockIdx.x;
  const int nb = gridDim.x;
  // Blocks are dealt to the 8 XCDs round-robin and run in rounds of 256, one
  // workgroup per compute unit.  Each XCD gets runs of consecutive tiles; with
  // several rounds, the runs of one round are adjacent bands (XCD k takes
  // tiles 32k .. 32k + 31 of the round's 256), so the halo rows at a band's
  // edge are loaded at the same time by the neighbouring XCD and come from
  // the shared last-level cache rather than from HBM (FP32 step 5.04 -> 4.97
  // ms, FP64 11.45 -> 10.99 ms at 512 x 512 x 384 against one run of 64
  // tiles per XCD spanning both rounds)
  if (nb % 256 == 0 && nb > 256) b = (b >> 8) * 256 + (b & 7) * 32 + ((b & 255) >> 3);
  else if ((nb & 7) == 0) b = (b & 7) * (nb >> 3) + (b >> 3);
  const int tile = b % a.ntiles, chunk = b / a.ntiles;
  int x0 = (tile % a.tiles_x) * TX, y0 = (tile / a.tiles_x) * TY;
  if (a.xcd_blocks) {
    // XCD k (block index mod 8) owns tile block (k % 2, k / 2) of a 2 x 4
    // split; its blocks are dealt row by row within that block
    const int bxw = a.tiles_x / 2, byh = (a.ntiles / a.tiles_x) / 4;
    const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3;
    x0 = ((xcd & 1) * bxw + local % bxw) * TX;
    y0 = ((xcd >> 1) * byh + local / bxw) * TY;
  }
  const int z0 = chunk * a.chunk, z1 = min(a.nz, z0 + a.chunk);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  // active columns of this tile (all 64 unless nx is ragged); lanes from W on
  // are idle duplicates of the cells that follow
  const int W = RAG ? min(TX, nx - x0) : TX;
  const bool act = !RAG || tx < W;
  const long long PS = a.pitch;  // population planes: direction i of level z starts at (z*Q + i)*PS
  // 16-bit storage: tiles start 2 columns past a 64-column boundary, so that
  // the side halo columns lie in 128-byte lines the tile loads itself (a row
  // of 64 cells then spans two lines instead of one): FP16 / BF16 steps 3 %
  // shorter.  With 4- and 8-byte storage the extra line per row costs more
  // than it saves (FP32 +4 %, FP64 +9 %), so those tiles stay aligned, and so
  // do the tiles of x-deferred steps, whose rows are stored in place.
  constexpr bool INP = (XP & 1) != 0, OUTP = (XP & 2) != 0;
  static_assert(XP == 0 || (TY == 8 && !RAG && !FLD), "x-deferred streaming: whole 8-row tiles only");
  constexpr int XS = sizeof(S) == 2 && XP == 0 ? 2 : 0;
  x0 += XS;
  const int x = RAG ? (x0 + tx) % nx : (XS ? wrapn(x0 + tx, nx) : x0 + tx), y = y0 + ty;
  constexpr unsigned ES = sizeof(S);
  const unsigned col = (unsigned)(x + nx * y);
  const unsigned colb = col * ES;
  const unsigned PB = (unsigned)a.pitch * ES;  // bytes from one direction plane to the next
  const unsigned F19 = 19 * PB, G7 = 7 * PB;       // bytes of all directions of one plane
  // byte offsets from this column to its periodic x / y neighbours in a plane
  const int dxm = (wrapn(x - 1, nx) - x) * (int)ES, dxp = (wrapn(x + 1, nx) - x) * (int)ES;
  const int dym = (wrapn(y - 1, ny) - y) * nx * (int)ES, dyp = (wrapn(y + 1, ny) - y) * nx * (int)ES;
  auto nb_off = [&](int cx, int cy) -> unsigned {
    return colb + (unsigned)((cx < 0 ? dxm : (cx > 0 ? dxp : 0)) + (cy < 0 ? dym : (cy > 0 ? dyp : 0)));
  };
  const int e_own = TL::interior_e(tx, ty);
  const C inv_cv = rcp(ph.cv);

  // helper cells of this thread
  int hex, hey;
  TL::halo_cell(tid < TL::NH ? tid : 0, hex, hey);
  const bool has_halo = tid < TL::NH;
  const int hxc = (x0 + hex - 2 + nx) % nx, hyc = wrapn(y0 + hey - 2, ny);
  const unsigned hcol = (unsigned)(hxc + nx * hyc);
  const unsigned hcolb = hcol * ES;
  // a cell's byte offset and those of its x - 1 and x + 1 columns: an
  // x-deferred input holds direction i of the cell at column x - c_ix
  const unsigned colb3[3] = {colb + (unsigned)dxm, colb, colb + (unsigned)dxp};
  const unsigned hcolb3[3] = {(unsigned)(wrapn(hxc - 1, nx) + nx * hyc) * ES, hcolb,
                              (unsigned)(wrapn(hxc + 1, nx) + nx * hyc) * ES};
  const int he = hey * EX + hex;
  int rdir;
  const int ridx = TL::receiver(hex, hey, rdir);
  int rex, rey;
  TL::ring1_cell(tid < TL::NR1 ? tid : 0, rex, rey);
  const bool has_ring = tid < TL::NR1;
  const int re = rey * EX + rex;

  C fa[19], fb[19], ga[7], gb[7], gc[7];
#pragma unroll
  for (int i = 0; i < 19; ++i) fa[i] = fb[i] = C(0);
#pragma unroll
  for (int i = 0; i < 7; ++i) ga[i] = gb[i] = gc[i] = C(0);
  C rho_a = C(1), rho_b = C(1), rho_c = C(1);
  C ua[3] = {C(0), C(0), C(0)}, ub[3] = {C(0), C(0), C(0)};
  C d0 = C(0), d1 = C(0), d2 = C(0);
  C g6_old = C(0), pend_rho = C(1);
  C pend_g[4] = {C(0), C(0), C(0), C(0)};
  bool pend_valid = false;
  int pend_z = 0;

  auto plane_of = [&](int p, int& zp) -> bool {
    if (a.zbound) {
      zp = p;
      return p >= 0 && p < nz;
    }
    zp = ((p % nz) + nz) % nz;
    return true;
  };

  // in-tile in-plane D3Q7 transfers into the plane collided one iteration ago
  auto finish_pulls = [&]() {
    if (!pend_valid) return;
    S* gz = gB + PS * 7 * pend_z;
#pragma unroll
    for (int i = 1; i <= 4; ++i) {
      const int sx = tx - CX[i], sy = ty - CY[i];
      // the source must be an active cell of this tile
      if (sx < 0 || sx >= W || sy < 0 || sy >= TY) continue;
      const C gs = s_gs[i - 1][sy * TX + sx];
      st_at(gz, G7, colb, i * PB, pend_g[i - 1] + (gs - pend_g[i - 1]) * (inv_cv * rcp(pend_rho)));
    }
  };

  // register prefetch of the next plane's populations (tile and halo cell);
  // with 16 rows or FP64 the registers are not there and planes load in place
  constexpr bool PF = TY <= 8 && sizeof(C) == 4;
  C pfi[26], pfh[26];
  auto load_f = [&](int zn, const unsigned* o3, C* l) {
    const S* fz = fA + PS * 19 * zn;
#pragma unroll
    for (int i = 0; i < 19; ++i) l[i] = ld_at(fz, F19, o3[INP ? 1 - CX[i] : 1], i * PB);
  };
  auto load_g = [&](int zn, unsigned off, C* l) {
    const S* gz = gA + PS * 7 * zn;
#pragma unroll
    for (int i = 0; i < 7; ++i) l[19 + i] = ld_at(gz, G7, off, i * PB);
  };
  auto load_cell = [&](int zn, const unsigned* o3, C* l) {
    load_f(zn, o3, l);
    load_g(zn, o3[1], l);
  };
  // lanes without a halo cell load from beyond the descriptor range: the
  // hardware returns 0 without a memory access, and the load count stays
  // the same on every path (the compiler then waits only for these loads)
  const unsigned hcolb_pf[3] = {has_halo ? hcolb3[0] : 0xFFFFFF00u, has_halo ? hcolb : 0xFFFFFF00u,
                                has_halo ? hcolb3[2] : 0xFFFFFF00u};
  auto prefetch = [&](int zn) {
    load_cell(zn, colb3, pfi);
    load_cell(zn, hcolb_pf, pfh);
  };
#pragma unroll
  for (int i = 0; i < 26; ++i) pfi[i] = pfh[i] = C(0);

  const int p_begin = z0 - 2, p_end = z1 + 1;
  // values of the plane being taken in: tile cell (fb, gc) and halo cell (hv, gv)
  C hv[19], gv[7];
#pragma unroll
  for (int i = 0; i < 19; ++i) hv[i] = C(0);
#pragma unroll
  for (int i = 0; i < 7; ++i) gv[i] = C(0);
  auto take_prefetched = [&]() {
#pragma unroll
    for (int i = 0; i < 19; ++i) fb[i] = pfi[i];
#pragma unroll
    for (int i = 0; i < 7; ++i) gc[i] = pfi[19 + i];
#pragma unroll
    for (int i = 0; i < 19; ++i) hv[i] = pfh[i];
#pragma unroll
    for (int i = 0; i < 7; ++i) gv[i] = pfh[19 + i];
  };
  if constexpr (PF) {
    int zf;
    if (plane_of(p_begin, zf)) {
      prefetch(zf);
      take_prefetched();
    }
  }
  // One plane step of the march.  In the steady part of the march (ST) the
  // planes p, p-1 and p-2 are interior planes of this chunk: no wrap, no wall
  // and every stage runs, so each step issues the same memory operations.
  auto step = [&](int p, auto steady) __attribute__((always_inline)) {
    constexpr bool ST = decltype(steady)::value;
    const int k = p - p_begin;
    const int s3 = k % 3, s4 = k & 3, s2 = k & 1;
    int zp;
    const bool exists = ST ? (zp = p, true) : plane_of(p, zp);
    // ---------------------------------------------------------------- plane p: take the prefetched values
    if constexpr (!PF) {
      if (exists) {
        C li[26];
        load_cell(zp, colb3, li);
#pragma unroll
        for (int i = 0; i < 19; ++i) fb[i] = li[i];
#pragma unroll
        for (int i = 0; i < 7; ++i) gc[i] = li[19 + i];
      }
    }
    // with prefetch, fb/gc/hv/gv already hold plane p (taken in at the end of
    // the previous step); issue the loads of plane p+1, which complete while
    // planes p-1 and p-2 are updated.  In the steady march only the tile's
    // f loads are issued here; the halo loads follow once plane p is in LDS
    // and the tile's g loads after the second barrier, which spreads the
    // step's memory traffic over its three stages
    bool next_loaded = false;
    if constexpr (PF) {
      int zn;
      if (ST) {
        // memory instructions of the steady march are issued at wave
        // priority 1, so that they reach the memory path ahead of arithmetic
        // of the other wave on the SIMD
        __builtin_amdgcn_s_setprio(1);
        load_f(p + 1, colb3, pfi);
        __builtin_amdgcn_s_setprio(0);
        next_loaded = true;
      } else if (p < p_end && plane_of(p + 1, zn)) {
        prefetch(zn);
        next_loaded = true;
      }
    }
    if (exists) {
      const bool face_plane = !ST && a.zbound && (zp == 0 || zp == nz - 1);
      const int zin = zp == 0 ? 1 : nz - 2;
      const int wk = zp == 0 ? 0 : 1;
      const bool pres_plane = OUT && face_plane && a.zpres[wk];
      // eqs. (35)-(36) on a face plane: g_b = w T_b + g(x_f) - w T(x_f), on deviations
      auto dirichlet = [&](C* g7, unsigned off, unsigned fcol) {
        const S* gin = gA + PS * 7 * zin;
        C gf[7], sfg = C(0);
#pragma unroll
        for (int i = 0; i < 7; ++i) {
          gf[i] = ld_at(gin, G7, off, i * PB);
          sfg += gf[i];
        }
        const C Tb = a.wall_Tw[wk] ? C(a.wall_Tw[wk][fcol]) : a.wall_T[wk];
        const C d = Tb - ph.T_ref - sfg;
#pragma unroll
        for (int i = 0; i < 7; ++i) g7[i] = gf[i] + (i == 0 ? ph.w0 : ph.w1) * d;
      };
      if (face_plane) dirichlet(gc, colb, col);
      C sf = C(0), jx = C(0), jy = C(0), jz = C(0), sg = C(0);
#pragma unroll
      for (int i = 0; i < 19; ++i) {
        sf += fb[i];
        if (CX[i]) jx += C(CX[i]) * fb[i];
        if (CY[i]) jy += C(CY[i]) * fb[i];
        if (CZ[i]) jz += C(CZ[i]) * fb[i];
      }
#pragma unroll
      for (int i = 0; i < 7; ++i) sg += gc[i];
      // rho = rho_out on a pressure face; u_eq there needs the force, so the
      // plane keeps the outlet sum of the known populations instead
      rho_c = pres_plane ? a.face_rho[wk] : ph.rho_ref + sf;
      const C T = ph.T_ref + sg;
      const C rad = psi_radicand(rho_c, T, ph);
      if (nonphysical(rho_c, T, rad, ph)) a.flag[0] = 1;
      s_psi[s3][e_own] = fsqrt(rad);
      if constexpr (FLD) {
        if (act && p >= z0 && p < z1) {
          const long long cidx = (long long)zp * nx * ny + col;
          a.fo.rho[cidx] = rho_c;
          a.fo.T[cidx] = T;
          a.fo.psi[cidx] = fsqrt(rad);
          if (face_plane) {
            S* gw = (S*)a.g_face + PS * 7 * zp;
#pragma unroll
            for (int i = 0; i < 7; ++i) st_at(gw, G7, colb, i * PB, gc[i]);
          }
        }
      }
      s_rho[s4][e_own] = rho_c;
      if (pres_plane) {
        s_ueq[s2][0][e_own] = C(0);
        s_ueq[s2][1][e_own] = C(0);
        s_ueq[s2][2][e_own] = outlet_known(fb, wk, ph.rho_ref);
      } else {
        const C ir = rcp(rho_c);
        s_ueq[s2][0][e_own] = jx * ir;
        s_ueq[s2][1][e_own] = jy * ir;
        s_ueq[s2][2][e_own] = jz * ir;
      }
      if (has_halo) {
        if constexpr (!PF) {
          C lh[26];
          load_cell(zp, hcolb3, lh);
#pragma unroll
          for (int i = 0; i < 19; ++i) hv[i] = lh[i];
#pragma unroll
          for (int i = 0; i < 7; ++i) gv[i] = lh[19 + i];
        }
        if (face_plane) dirichlet(gv, hcolb, hcol);
        C hs = C(0), hx = C(0), hy = C(0), hz = C(0), hg = C(0);
#pragma unroll
        for (int i = 0; i < 19; ++i) {
          hs += hv[i];
          if (CX[i]) hx += C(CX[i]) * hv[i];
          if (CY[i]) hy += C(CY[i]) * hv[i];
          if (CZ[i]) hz += C(CZ[i]) * hv[i];
        }
#pragma unroll
        for (int i = 0; i < 7; ++i) hg += gv[i];
        const C hr = pres_plane ? a.face_rho[wk] : ph.rho_ref + hs;
        const C hT = ph.T_ref + hg;
        s_psi[s3][he] = fsqrt(psi_radicand(hr, hT, ph));
        s_rho[s4][he] = hr;
        if (pres_plane) {
          s_ueq[s2][0][he] = C(0);
          s_ueq[s2][1][he] = C(0);
          s_ueq[s2][2][he] = outlet_known(hv, wk, ph.rho_ref);
        } else {
          const C ihr = rcp(hr);
          s_ueq[s2][0][he] = hx * ihr;
          s_ueq[s2][1][he] = hy * ihr;
          s_ueq[s2][2][he] = hz * ihr;
        }
        if (ridx >= 0) s_gr[s4][ridx] = gv[rdir];
      }
    }
    __syncthreads();
    // ---------------------------------------------------------------- plane p-1: force, u, D3Q19
    if constexpr (ST && PF) {
      __builtin_amdgcn_s_setprio(1);
      load_cell(p + 1, hcolb_pf, pfh);
      __builtin_amdgcn_s_setprio(0);
    }
    finish_pulls();
    const int q = p - 1;
    int zq = q;
    const bool do_u = ST ? true : (q >= z0 - 1 && plane_of(q, zq));
    // plane q on a bounded face: wall or pressure; ghost_cz = the c_z whose
    // neighbours lie beyond a pressure face (their u is a copy of plane q)
    const bool face_q = !ST && do_u && a.zbound && (zq == 0 || zq == nz - 1);
    const int qk = zq == 0 ? 0 : 1;
    const bool pres_q = OUT && face_q && a.zpres[qk];
    const int ghost_cz = pres_q ? (qk ? 1 : -1) : 0;
    if (do_u) {
      // psi slots of planes q-1, q, q+1 (walls: the ghost layer mirrors the
      // first interior layer, eq. (37) with theta = 90 degrees; pressure
      // faces: it copies the face plane)
      int sm = (k + 1) % 3, s0 = (k + 2) % 3, sp = s3;
      if (face_q && zq == 0) sm = pres_q ? s0 : sp;
      if (face_q && zq == nz - 1) sp = pres_q ? s0 : sm;
      const bool wall_plane = face_q && !pres_q;
      const int sq = (k + 1) & 1;  // ueq slot of plane q
      const int rq = (k + 3) & 3;  // rho slot of plane q
      // eq. (37): the ghost layer adds kappa_w |grad_t psi| of the wall layer
      // (periodic tangential differences, all within the 2-cell halo for the
      // tile's own cells)
      const int gdir = !wall_plane || ph.kappa_w == C(0) ? 0 : (zq == 0 ? -1 : 1);
      auto force_at = [&](int e, C& Fx, C& Fy, C& Fz) {
        C ax = C(0), ay = C(0), az = C(0);
#pragma unroll
        for (int i = 1; i < 19; ++i) {
          const C wgt = i < 7 ? C(1) / C(6) : C(1) / C(12);
          const int slot = CZ[i] < 0 ? sm : (CZ[i] > 0 ? sp : s0);
          const int en = e + CX[i] + CY[i] * EX;
          C pn = s_psi[slot][en];
          if (gdir != 0 && CZ[i] == gdir) {
            const C tx = s_psi[s0][en + 1] - s_psi[s0][en - 1];
            const C ty = s_psi[s0][en + EX] - s_psi[s0][en - EX];
            pn += ph.kappa_w * fsqrt(tx * tx + ty * ty);
          }
          if (CX[i]) ax += wgt * C(CX[i]) * pn;
          if (CY[i]) ay += wgt * C(CY[i]) * pn;
          if (CZ[i]) az += wgt * C(CZ[i]) * pn;
        }
        const C pc = -ph.G * s_psi[s0][e];
        Fx = pc * ax;
        Fy = pc * ay;
        Fz = pc * az;
      };
      {
        C Fx, Fy, Fz;
        force_at(e_own, Fx, Fy, Fz);
        const C rho = rho_b;
        const C irho = rcp(rho);
        const C dux = Fx * irho, duy = Fy * irho, duz = Fz * irho;
        C uex = s_ueq[sq][0][e_own], uey = s_ueq[sq][1][e_own], uez = s_ueq[sq][2][e_own];
        if (wall_plane) {
          uex = -C(0.5) * dux;
          uey = -C(0.5) * duy;
          uez = -C(0.5) * duz;
        } else if (pres_q) {
          outlet_ueq(uez, qk, rho, Fx, Fy, Fz, uex, uey, uez);
        }
        ub[0] = uex + C(0.5) * dux;
        ub[1] = uey + C(0.5) * duy;
        ub[2] = uez + C(0.5) * duz;
        if constexpr (FLD) {
          if (act && q >= z0 && q < z1) {
            const long long NC = (long long)nx * ny * nz;
            const long long cidx = (long long)zq * nx * ny + col;
            const C ue[3] = {uex, uey, uez}, dd[3] = {dux, duy, duz};
#pragma unroll
            for (int c3 = 0; c3 < 3; ++c3) {
              a.fo.ueq[cidx + c3 * NC] = ue[c3];
              a.fo.du[cidx + c3 * NC] = dd[c3];
              a.fo.ureal[cidx + c3 * NC] = ub[c3];
            }
          }
        }
        s_u[0][e_own] = ub[0];
        s_u[1][e_own] = ub[1];
        s_u[2][e_own] = ub[2];
        if (act && (ST || (q >= z0 && q < z1))) {
          if (pres_q) {
            // Sec. 3.3: the unknown populations of the outlet node
            const C F3[3] = {Fx, Fy, Fz};
            outlet_fill(fa, 4 + qk, rho, F3, ph);
          }
          collide19(fa, rho, rho - ph.rho_ref, uex, uey, uez, dux, duy, duz, ph);
          // destination planes q-1, q, q+1 (periodic wrap); at a wall the
          // links leaving the domain bounce back onto the opposite slot, at
          // a pressure face they leave
          const bool lo_out = !ST && zq == 0, hi_out = !ST && zq == nz - 1;
          S* pm = fB + PS * 19 * (lo_out ? nz - 1 : zq - 1);
          S* p0 = fB + PS * 19 * zq;
          S* pp = fB + PS * 19 * (hi_out ? 0 : zq + 1);
          if (ST) {
            // steady march: the first kEarlyF directions here, the rest after
            // the next barrier, so that the plane's stores reach memory in two
            // smaller bursts
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int i = 0; i < kEarlyF; ++i)
              st_at(CZ[i] < 0 ? pm : (CZ[i] > 0 ? pp : p0), F19, nb_off(OUTP ? 0 : CX[i], CY[i]), i * PB, fa[i]);
            __builtin_amdgcn_s_setprio(0);
          } else if (!(a.zbound && (lo_out || hi_out))) {
#pragma unroll
            for (int i = 0; i < 19; ++i)
              st_at(CZ[i] < 0 ? pm : (CZ[i] > 0 ? pp : p0), F19, nb_off(OUTP ? 0 : CX[i], CY[i]), i * PB, fa[i]);
          } else {
#pragma unroll
            for (int i = 0; i < 19; ++i) {
              const bool out = (CZ[i] < 0 && lo_out) || (CZ[i] > 0 && hi_out);
              if (out) {
                // bounce-back: f_opp(i)(x) = f*_i(x), x-deferred at column x + c_ix
                if (!pres_q) st_at(p0, F19, OUTP ? nb_off(CX[i], 0) : colb, opp19(i) * PB, fa[i]);
              } else
                st_at(CZ[i] < 0 ? pm : (CZ[i] > 0 ? pp : p0), F19, nb_off(OUTP ? 0 : CX[i], CY[i]), i * PB, fa[i]);
            }
          }
        }
      }
      if (has_ring) {
        // u vanishes on wall nodes; elsewhere the same operation order as the
        // tile's own u, so that u does not depend on which thread evaluates it
        C vx = C(0), vy = C(0), vz = C(0);
        if (!wall_plane) {
          C Fx, Fy, Fz;
          force_at(re, Fx, Fy, Fz);
          const C rr = s_rho[rq][re];
          const C ir = rcp(rr);
          C ex = s_ueq[sq][0][re], ey = s_ueq[sq][1][re], ez = s_ueq[sq][2][re];
          if (pres_q) outlet_ueq(ez, qk, rr, Fx, Fy, Fz, ex, ey, ez);
          vx = ex + C(0.5) * (Fx * ir);
          vy = ey + C(0.5) * (Fy * ir);
          vz = ez + C(0.5) * (Fz * ir);
        }
        s_u[0][re] = vx;
        s_u[1][re] = vy;
        s_u[2][re] = vz;
      }
    }
    __syncthreads();
    if constexpr (ST) __builtin_amdgcn_s_setprio(1);
    if constexpr (ST && PF) load_g(p + 1, colb, pfi);
    if constexpr (ST) {
      // the remaining D3Q19 pushes of plane q = p-1 (interior planes: no wrap)
      S* pm = fB + PS * 19 * (p - 2);
      S* p0 = fB + PS * 19 * (p - 1);
      S* pp = fB + PS * 19 * p;
      if (act) {
#pragma unroll
        for (int i = kEarlyF; i < 19; ++i)
          st_at(CZ[i] < 0 ? pm : (CZ[i] > 0 ? pp : p0), F19, nb_off(OUTP ? 0 : CX[i], CY[i]), i * PB, fa[i]);
      }
      __builtin_amdgcn_s_setprio(0);
    }
    // ---------------------------------------------------------------- divergence contributions of u(q)
    if (do_u) {
#pragma unroll
      for (int i = 1; i < 19; ++i) {
        const int e = e_own + CX[i] + CY[i] * EX;
        const C c = C(3) * w19<C>(i) * (C(CX[i]) * s_u[0][e] + C(CY[i]) * s_u[1][e] + C(CZ[i]) * s_u[2][e]);
        if (CZ[i] > 0) d0 += c;        // u(q) is the +z neighbour of plane q-1 = p-2
        else if (CZ[i] == 0) d1 += c;  // in-plane neighbour of plane q
        else d2 += c;                  // -z neighbour of plane q+1 = p
        // beyond a pressure face the ghost u copies plane q
        if (!ST && CZ[i] != 0 && CZ[i] == ghost_cz) d1 += c;
      }
    }
    // ---------------------------------------------------------------- plane p-2: D3Q7
    const int r = p - 2;
    int zr;
    const bool r_exists = ST ? (zr = r, true) : plane_of(r, zr);
    const C og1 = ga[1], og2 = ga[2], og3 = ga[3], og4 = ga[4], og6 = ga[6];
    const bool do_g = ST || (r_exists && r >= z0 && r < z1);
    if (do_g) {
      const C T = ph.T_ref + (ga[0] + ga[1] + ga[2] + ga[3] + ga[4] + ga[5] + ga[6]);
      const C rho = rho_a;
      const C vf = vflux_at(rho, ph);
      C gx, gy, gz;
      local_gradT(ga, vf, ph, gx, gy, gz);
      const C Fbar = rho * ph.cv * (ua[0] * gx + ua[1] * gy + ua[2] * gz) + T * pr_dpdT(rho, T, ph) * d0;
      if constexpr (FLD) {
        if (act) a.fo.div[(long long)zr * nx * ny + col] = d0;
      }
      const C og0 = ga[0];
      collide7(ga, Fbar, vf, ph);
      if (act) st_at(gB + PS * 7 * zr, G7, colb, 0u, og0 + (ga[0] - og0) * (inv_cv * rcp(rho)));
      // +z: destination is plane r+1 of this column (old value in gb)
      {
        int zd = zr + 1;
        bool ok = true;
        if (!ST && zd >= nz) {
          if (a.zbound) ok = false; else zd = 0;
        }
        if (ok && act)
          st_at(gB + PS * 7 * zd, G7, colb, 5 * PB, gb[5] + (ga[5] - gb[5]) * (inv_cv * rcp(rho_b)));
      }
      // -z: destination is plane r-1 of this column (old value kept from last iteration)
      {
        int zd = zr - 1;
        bool ok = true;
        if (!ST && zd < 0) {
          if (a.zbound) ok = false; else zd = nz - 1;
        }
        if (ok && act)
          st_at(gB + PS * 7 * zd, G7, colb, 6 * PB, g6_old + (ga[6] - g6_old) * (inv_cv * rcp(pend_rho)));
      }
      const int rs = (k + 2) & 3;  // rho / ring slot of plane r
#pragma unroll
      for (int i = 1; i <= 4; ++i) {
        const int dx = tx + CX[i], dy = ty + CY[i];
        if (dx >= 0 && dx < TX && dy >= 0 && dy < TY) {
          s_gs[i - 1][tid] = ga[i];
        } else if (act) {
          const int slot = i == 1 ? ty : (i == 2 ? TY + ty : (i == 3 ? 2 * TY + tx : 2 * TY + TX + tx));
          const C gold = s_gr[rs][slot];
          const C rd = s_rho[rs][e_own + CX[i] + CY[i] * EX];
          const unsigned db = nb_off(CX[i], CY[i]);
          st_at(gB + PS * 7 * zr, G7, db, i * PB, gold + (ga[i] - gold) * (inv_cv * rcp(rd)));
        }
      }
    }
    pend_valid = do_g;
    pend_z = zr;
    pend_g[0] = og1;
    pend_g[1] = og2;
    pend_g[2] = og3;
    pend_g[3] = og4;
    pend_rho = rho_a;
    g6_old = og6;
    // ---------------------------------------------------------------- rotate
    d0 = d1;
    d1 = d2;
    d2 = C(0);
#pragma unroll
    for (int i = 0; i < 19; ++i) fa[i] = fb[i];
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      ga[i] = gb[i];
      gb[i] = gc[i];
    }
    rho_a = rho_b;
    rho_b = rho_c;
    ua[0] = ub[0];
    ua[1] = ub[1];
    ua[2] = ub[2];
    if constexpr (PF) {
      if (next_loaded) take_prefetched();
    }
  };
  // warm-up, steady march, drain (also without the register prefetch: the
  // steady step's staged pushes and missing boundary checks take the FP64
  // step on the 256^3 heated wall from 2.05 to 1.75 ms)
  const int s_lo = z0 + 3, s_hi = z1 - 2;
  int p = p_begin;
  for (; p <= p_end && p < s_lo; ++p) step(p, std::false_type{});
  if (p <= s_hi) {
    // nothing in flight on entry: inside the steady loop the wait for the
    // prefetched plane then leaves the previous plane's stores outstanding
    if constexpr (PF) __builtin_amdgcn_s_waitcnt(0);
    for (; p <= s_hi; ++p) step(p, std::true_type{});
  }
  for (; p <= p_end; ++p) step(p, std::false_type{});
  __syncthreads();
  finish_pulls();
}

// Tile height: 8 rows (512 threads, one workgroup of 8 waves per compute
// unit with room for the prefetch registers).  LBM_FUSED_TY=16 selects
// 16-row tiles (fewer halo reads, 128-register limit) for 32- and 16-bit
// storage; FP64 always uses 8 rows (its LDS rings need twice the space).
// Read once, when a context is created.
inline int fused_tile_height(int precision) {
  if (precision == LBM_FP64) return 8;
  if (const char* ev = std::getenv("LBM_FUSED_TY")) {
    if (std::atoi(ev) == 16) return 16;
  }
  return 8;
}

// z planes per workgroup.  One workgroup runs on a compute unit at a time,
// so a launch takes ceil(workgroups / 256) rounds of one chunk's march: the
// chunk count (chunks of >= 8 planes) with the least rounds x (planes per
// chunk + 8) is taken, the 8 standing for a march's halo planes, start and
// end.
inline int fused_chunk_planes(int nx, int ny, int nz, int ty) {
  const long long ntiles = (long long)((nx + FTX - 1) / FTX) * (ny / ty);
  long long nchunks = 1, best = -1;
  for (long long n = 1; n <= std::max(1, nz / 8); ++n) {
    const long long cost = (ntiles * n + 255) / 256 * ((nz + n - 1) / n + 8);
    if (best < 0 || cost < best) {
      best = cost;
      nchunks = n;
    }
  }
  return (int)((nz + nchunks - 1) / nchunks);
}

inline bool fused_supported(const lbm_params& p, int ty) {
  for (int k = 0; k < 4; ++k)
    if (p.face[k] != LBM_FACE_PERIODIC) return false;
  const bool zper = p.face[4] == LBM_FACE_PERIODIC && p.face[5] == LBM_FACE_PERIODIC;
  const bool zbound = p.face[4] != LBM_FACE_PERIODIC && p.face[5] != LBM_FACE_PERIODIC;
  if (!zper && !zbound) return false;
  if (ty != 8 && (ty != 16 || p.precision == LBM_FP64)) return false;
  if (p.nx < 8 || p.ny % ty != 0) return false;
  if (p.nx % FTX != 0 && ty != 8) return false;  // ragged nx: 8-row tiles only
  if (p.nz < 4) return false;
  // buffer offsets are 32-bit: the 19 direction planes of one level must span
  // less than the offset that marks a halo lane without a cell (0xFFFFFF00)
  const long long es = p.precision == LBM_FP64 ? 8 : (p.precision == LBM_FP32_DEV ? 4 : 2);
  if (19 * plane_pitch(p.nx, p.ny) * es >= 0xF0000000ll) return false;
  return true;
}

template <typename S>
struct FusedImpl {
  using C = typename Storage<S>::C;
  // ty: tile height (8, or 16 for 32/16-bit storage); chunk_planes: z planes
  // per workgroup (0: all); xcd_map: give each XCD a 2 x 4 block of tiles
  // fo: NULL for a plain step; otherwise the step also writes the fields of
  // its start state there and completes the start state's face-plane g in
  // place (8-row tiles).  xmode: x-deferred streaming of the input (bit 0)
  // and of the output (bit 1), for plain steps on whole 8-row tiles
  static hipError_t step(const lbm_params& p, const Phys<C>& ph, hipStream_t stream, const S* fA, const S* gA, S* fB,
                         S* gB, const double* Tw0, const double* Tw1, int* flag, int ty, int chunk_planes,
                         bool xcd_map, const FusedFields<C>* fo = nullptr, int xmode = 0) {
    FusedArgs<C> a;
    a.ph = ph;
    a.nx = p.nx;
    a.ny = p.ny;
    a.nz = p.nz;
    a.pitch = plane_pitch(p.nx, p.ny);
    a.zbound = p.face[4] != LBM_FACE_PERIODIC;
    a.zpres[0] = p.face[4] == LBM_FACE_PRESSURE;
    a.zpres[1] = p.face[5] == LBM_FACE_PRESSURE;
    a.face_rho[0] = (C)p.face_rho[4];
    a.face_rho[1] = (C)p.face_rho[5];
    const int TY = ty;
    a.tiles_x = (p.nx + FTX - 1) / FTX;
    a.ntiles = a.tiles_x * (p.ny / TY);
    a.chunk = chunk_planes > 0 ? chunk_planes : p.nz;
    const int nchunks = (p.nz + a.chunk - 1) / a.chunk;
    a.xcd_blocks = xcd_map && nchunks == 1 && a.tiles_x % 2 == 0 && (p.ny / TY) % 4 == 0 && a.ntiles % 8 == 0;
    a.wall_T[0] = (C)p.face_T[4];
    a.wall_T[1] = (C)p.face_T[5];
    a.wall_Tw[0] = Tw0;
    a.wall_Tw[1] = Tw1;
    a.flag = flag;
    a.fo = fo ? *fo : FusedFields<C>{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    a.g_face = const_cast<S*>(gA);
    const bool out = a.zpres[0] || a.zpres[1];
    if (xmode != 0 && (fo || TY != 8 || p.nx % FTX != 0 || xmode < 0 || xmode > 3)) return hipErrorInvalidValue;
    if (fo) {
      // the same instantiation as the plain step of this grid, plus the
      // field stores (the stores only read values the step computes anyway,
      // so the state it produces is the plain step's)
      if (TY != 8) return hipErrorInvalidValue;
      const dim3 grid(a.ntiles * nchunks), block(FTX * 8);
      if (p.nx % FTX != 0) {
        if (out) hipLaunchKernelGGL((k_fused<S, 8, true, true, true>), grid, block, 0, stream, fA, gA, fB, gB, a);
        else hipLaunchKernelGGL((k_fused<S, 8, false, true, true>), grid, block, 0, stream, fA, gA, fB, gB, a);
      } else {
        if (out) hipLaunchKernelGGL((k_fused<S, 8, true, false, true>), grid, block, 0, stream, fA, gA, fB, gB, a);
        else hipLaunchKernelGGL((k_fused<S, 8, false, false, true>), grid, block, 0, stream, fA, gA, fB, gB, a);
      }
      return hipGetLastError();
    }
    if (p.nx % FTX != 0) {
      // ragged nx: 8-row tiles (the context asks for no other height then)
      if (out) return launch_rag<true>(a, nchunks, stream, fA, gA, fB, gB);
      return launch_rag<false>(a, nchunks, stream, fA, gA, fB, gB);
    }
    if (out) return launch<true>(a, TY, nchunks, stream, fA, gA, fB, gB, xmode);
    return launch<false>(a, TY, nchunks, stream, fA, gA, fB, gB, xmode);
  }
  template <bool OUT>
  static hipError_t launch(const FusedArgs<C>& a, int TY, int nchunks, hipStream_t stream, const S* fA, const S* gA,
                           S* fB, S* gB, int xmode) {
    if constexpr (sizeof(S) <= 4) {
      if (TY == 16) {
        hipLaunchKernelGGL((k_fused<S, 16, OUT, false>), dim3(a.ntiles * nchunks), dim3(FTX * 16), 0, stream, fA,
                           gA, fB, gB, a);
        return hipGetLastError();
      }
    }
    const dim3 grid(a.ntiles * nchunks), block(FTX * 8);
    if constexpr (sizeof(S) == 8) {
      switch (xmode) {
        case 1:
          hipLaunchKernelGGL((k_fused<S, 8, OUT, false, false, 1>), grid, block, 0, stream, fA, gA, fB, gB, a);
          return hipGetLastError();
        case 2:
          hipLaunchKernelGGL((k_fused<S, 8, OUT, false, false, 2>), grid, block, 0, stream, fA, gA, fB, gB, a);
          return hipGetLastError();
        case 3:
          hipLaunchKernelGGL((k_fused<S, 8, OUT, false, false, 3>), grid, block, 0, stream, fA, gA, fB, gB, a);
          return hipGetLastError();
        default:
          break;
      }
    } else if (xmode != 0) {
      return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL((k_fused<S, 8, OUT, false>), grid, block, 0, stream, fA, gA, fB, gB, a);
    return hipGetLastError();
  }
  template <bool OUT>
  static hipError_t launch_rag(const FusedArgs<C>& a, int nchunks, hipStream_t stream, const S* fA, const S* gA,
                               S* fB, S* gB) {
    hipLaunchKernelGGL((k_fused<S, 8, OUT, true>), dim3(a.ntiles * nchunks), dim3(FTX * 8), 0, stream, fA, gA, fB,
                       gB, a);
    return hipGetLastError();
  }
};

}  // namespace lbm

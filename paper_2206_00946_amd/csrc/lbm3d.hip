// C ABI of the coupled D3Q19 / D3Q7 thermal pseudopotential LBM library for
// MI355X (gfx950).  See include/lbm3d.h for the contract of every entry point.
#include "lbm3d.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "kernels_ref.h"
#include "kernels_fused.h"
#include "kernels_adjoint.h"

using namespace lbm;

namespace {

std::string g_create_error;

// Workspace of lbm_adjoint_noalloc: one fixed array in device memory, which
// every GPU the library runs on holds (its own copy) until the process ends.
// Host code never passes the array's name to a kernel (on the host it only
// stands for the symbol); the device address of each GPU's copy is looked up
// once per device with hipGetSymbolAddress and used instead.
constexpr size_t kNoAllocBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

constexpr size_t kAlign = 256;
constexpr long long kSlab = 1ll << 22;  // cells per host<->device staging slab

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

size_t elem_size(int prec) {
  switch (prec) {
    case LBM_FP64: return 8;
    case LBM_FP32_DEV: return 4;
    default: return 2;
  }
}
size_t compute_size(int prec) { return prec == LBM_FP64 ? 8 : 4; }

}  // namespace

struct lbm_ctx {
  lbm_params p;
  hipStream_t stream = nullptr;
  char* base = nullptr;
  size_t bytes = 0;
  bool owns = false;
  // populations (A = current state, B = next)
  void* fA = nullptr;
  void* gA = nullptr;
  void* fB = nullptr;
  void* gB = nullptr;
  // fields in the compute precision
  void* rho = nullptr;
  void* T = nullptr;
  void* psi = nullptr;
  void* ueq = nullptr;
  void* du = nullptr;
  void* ureal = nullptr;             // real velocity of eq. (5), written by the prepass
  void* Th[2] = {nullptr, nullptr};  // S1 temperatures of the last two steps (vartheta = 1)
  int hist = 0;                      // how many of them are valid
  double* Tw[2] = {nullptr, nullptr};
  bool has_Tw[2] = {false, false};
  double* partials = nullptr;
  double* sums = nullptr;
  int* flag = nullptr;
  double* staging = nullptr;  // kSlab * 26 doubles
  bool initialised = false;
  int64_t step = 0;
  double mass0 = 0.0;
  bool fused_ok = false;
  int fused_chunk = 0;  // z planes per workgroup of the fused kernel (0: all)
  int fused_ty = 8;     // tile height of the fused kernel
  bool fused_map = false;  // fused kernel: each XCD a 2 x 4 block of tiles
  // the steps of one lbm_step call pass x-deferred states to each other
  // (FP64 storage, whole 8-row tiles of the fused kernel)
  bool fused_xdefer = false;
  int device = 0;  // HIP device current at lbm_create
  std::string err;
};

namespace {

long long ncells(const lbm_params& p) { return (long long)p.nx * p.ny * p.nz; }

// The per-cell fields of one state in the compute precision: rho, T, psi,
// u_eq = j/rho, Delta u = F/rho, the real velocity of eq. (5) and, where a
// buffer is given (the adjoint's stored fields), div u
struct FieldSet {
  void *rho, *T, *psi, *ueq, *du, *ureal, *div;
};

FieldSet ctx_fields(const lbm_ctx* ctx) {
  return {ctx->rho, ctx->T, ctx->psi, ctx->ueq, ctx->du, ctx->ureal, nullptr};
}

struct Layout {
  size_t state = 0, scratch = 0;
  size_t off_fA, off_gA, off_fB, off_gB, off_rho, off_T, off_psi, off_ueq, off_du, off_ureal, off_Th0, off_Th1,
      off_Tw0, off_Tw1, off_part, off_sums, off_flag, off_stage;
};

Layout layout_of(const lbm_params& p) {
  Layout L;
  const size_t N = (size_t)ncells(p);
  const size_t es = elem_size(p.precision), cs = compute_size(p.precision);
  size_t o = 0;
  const size_t NP = (size_t)p.nz * plane_pitch(p.nx, p.ny);  // population slots per direction
  L.off_fA = o; o = align_up(o + 19 * NP * es);
  L.off_gA = o; o = align_up(o + 7 * NP * es);
  L.off_fB = o; o = align_up(o + 19 * NP * es);
  L.off_gB = o; o = align_up(o + 7 * NP * es);
  L.state = o;
  L.off_rho = o; o = align_up(o + N * cs);
  L.off_T = o; o = align_up(o + N * cs);
  L.off_psi = o; o = align_up(o + N * cs);
  L.off_ueq = o; o = align_up(o + 3 * N * cs);
  L.off_du = o; o = align_up(o + 3 * N * cs);
  L.off_ureal = o; o = align_up(o + 3 * N * cs);
  const size_t nh = p.theta_corr ? N : 0;  // temperature history for vartheta = 1
  L.off_Th0 = o; o = align_up(o + nh * cs);
  L.off_Th1 = o; o = align_up(o + nh * cs);
  L.off_Tw0 = o; o = align_up(o + (size_t)p.nx * p.ny * 8);
  L.off_Tw1 = o; o = align_up(o + (size_t)p.nx * p.ny * 8);
  L.off_part = o; o = align_up(o + RED_BLOCKS * RED_VALUES * 8);
  L.off_sums = o; o = align_up(o + RED_VALUES * 8);
  L.off_flag = o; o = align_up(o + 64);
  L.off_stage = o; o = align_up(o + (size_t)std::min<long long>(kSlab, (long long)N) * 26 * 8);
  L.scratch = o - L.state;
  return L;
}

bool in_open01(double v) { return v > 0.0 && v < 1.0; }
bool in_rate(double v) { return v > 0.0 && v < 2.0; }

lbm_status validate(const lbm_params* p, std::string& msg) {
  if (!p) { msg = "params is NULL"; return LBM_EINVAL; }
  if (p->nx <= 0 || p->ny <= 0 || p->nz <= 0) { msg = "grid sizes must be positive"; return LBM_EINVAL; }
  if ((double)p->nx * p->ny * p->nz > 4.0e9) { msg = "grid too large"; return LBM_EINVAL; }
  if (p->precision < LBM_FP64 || p->precision > LBM_BF16_DEV) { msg = "unknown precision"; return LBM_EINVAL; }
  for (int k = 0; k < 6; ++k)
    if (p->face[k] < LBM_FACE_PERIODIC || p->face[k] > LBM_FACE_PRESSURE) { msg = "unknown face kind"; return LBM_EINVAL; }
  const int ext[3] = {p->nx, p->ny, p->nz};
  for (int a = 0; a < 3; ++a) {
    const bool lo = p->face[2 * a] == LBM_FACE_PERIODIC, hi = p->face[2 * a + 1] == LBM_FACE_PERIODIC;
    if (lo != hi) { msg = "periodic faces must come in pairs"; return LBM_EINVAL; }
    if (!lo && ext[a] < 3) { msg = "a bounded axis needs at least 3 cells"; return LBM_EINVAL; }
  }
  if (!(p->a > 0 && p->b > 0 && p->R > 0 && p->omega > -1 && std::isfinite(p->G) && p->G != 0.0)) {
    msg = "invalid equation-of-state parameters"; return LBM_EINVAL;
  }
  if (!(in_rate(p->s_e) && in_rate(p->s_nu) && in_rate(p->s_q) && in_rate(p->s_pi) && in_rate(p->s_T_other))) {
    msg = "relaxation rates must lie in (0, 2)"; return LBM_EINVAL;
  }
  if (!in_open01(p->wbar)) { msg = "wbar must lie in (0, 1)"; return LBM_EINVAL; }
  if (!(p->lambda > 0 && p->cv > 0)) { msg = "lambda and cv must be positive"; return LBM_EINVAL; }
  if (!(std::isfinite(p->kappa_w) && std::isfinite(p->rho_ref) && std::isfinite(p->T_ref))) {
    msg = "kappa_w, rho_ref and T_ref must be finite"; return LBM_EINVAL;
  }
  for (int k = 0; k < 6; ++k) {
    if (p->face[k] != LBM_FACE_PERIODIC && !(p->face_T[k] > 0)) { msg = "bounded faces need face_T > 0"; return LBM_EINVAL; }
    if (p->face[k] == LBM_FACE_PRESSURE && !(p->face_rho[k] > 0 && p->face_rho[k] * p->b < 1)) {
      msg = "pressure faces need 0 < face_rho < 1/b"; return LBM_EINVAL;
    }
  }
  if (p->lambda_vapour != 0.0 || p->lambda_liquid != 0.0) {
    if (!(p->lambda_vapour > 0 && p->lambda_liquid > 0 && p->lambda_rho_l > p->lambda_rho_v)) {
      msg = "density-dependent conductivity needs lambda_vapour, lambda_liquid > 0 and lambda_rho_l > lambda_rho_v";
      return LBM_EINVAL;
    }
  }
  if (p->theta_corr != 0 && p->theta_corr != 1) { msg = "theta_corr must be 0 or 1"; return LBM_EINVAL; }
  for (int k = 0; k < 4; ++k)
    if (p->face[k] == LBM_FACE_WALL) { msg = "walls are supported on the z faces only"; return LBM_EUNSUPPORTED; }
  if ((p->face[4] == LBM_FACE_WALL || p->face[5] == LBM_FACE_WALL))
    for (int k = 0; k < 4; ++k)
      if (p->face[k] != LBM_FACE_PERIODIC) { msg = "a z wall requires periodic x and y"; return LBM_EUNSUPPORTED; }
  return LBM_OK;
}

template <typename C>
Phys<C> phys_of(const lbm_params& p) {
  Phys<C> ph;
  const double Tc = 0.0778 * p.a / (0.45724 * p.b * p.R);  // eq. (55) solved for Tc
  const double kpr = 0.37464 + 1.54226 * p.omega - 0.26992 * p.omega * p.omega;
  const double cs2T = p.wbar / 3.0;
  ph.a = (C)p.a; ph.b = (C)p.b; ph.R = (C)p.R; ph.G = (C)p.G; ph.Tc = (C)Tc; ph.kpr = (C)kpr;
  ph.s_e = (C)p.s_e; ph.s_nu = (C)p.s_nu; ph.s_q = (C)p.s_q; ph.s_pi = (C)p.s_pi;
  ph.w0 = (C)(1.0 - p.wbar); ph.w1 = (C)(p.wbar / 6.0); ph.wbar = (C)p.wbar; ph.cs2T = (C)cs2T;
  ph.vflux = (C)(1.0 / (0.5 + p.lambda / cs2T));  // lambda = (1/varsigma - 1/2) c_s^2
  ph.vother = (C)p.s_T_other;
  ph.cv = (C)p.cv;
  ph.kappa_w = (C)p.kappa_w;
  ph.rho_ref = (C)p.rho_ref;
  ph.T_ref = (C)p.T_ref;
  ph.inv_b = (C)(1.0 / p.b);
  ph.var_lambda = p.lambda_vapour > 0.0 && p.lambda_liquid > 0.0;
  ph.lam_v = (C)p.lambda_vapour;
  ph.lam_l = (C)p.lambda_liquid;
  ph.lam_rv = (C)p.lambda_rho_v;
  ph.lam_inv_drho = ph.var_lambda ? (C)(1.0 / (p.lambda_rho_l - p.lambda_rho_v)) : (C)0;
  return ph;
}

Geom geom_of(const lbm_params& p) {
  Geom g;
  g.nx = p.nx; g.ny = p.ny; g.nz = p.nz;
  for (int k = 0; k < 6; ++k) g.face[k] = p.face[k];
  g.N = ncells(p);
  g.pitch = plane_pitch(p.nx, p.ny);
  return g;
}

template <typename C>
Faces<C> faces_of(const lbm_ctx* ctx) {
  Faces<C> fc;
  for (int k = 0; k < 6; ++k) {
    fc.face_T[k] = (C)ctx->p.face_T[k];
    fc.face_rho[k] = (C)ctx->p.face_rho[k];
  }
  fc.Tw[0] = ctx->has_Tw[0] ? ctx->Tw[0] : nullptr;
  fc.Tw[1] = ctx->has_Tw[1] ? ctx->Tw[1] : nullptr;
  return fc;
}

lbm_status hip_fail(lbm_ctx* ctx, hipError_t e, const char* where) {
  ctx->err = std::string(where) + ": " + hipGetErrorString(e);
  return LBM_EHIP;
}

#define HIPCHK(ctx, call)                                   \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call);  \
  } while (0)

unsigned blocks_for(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// ------------------------------------------------------------- dispatch by storage type

template <typename S>
struct Impl {
  using C = typename Storage<S>::C;

  // S0-S5 of the state (f, g) into the field set F: Dirichlet completion of g
  // and rho, T, psi (k_macro), then the outlet fill of f and the velocities
  // (k_force), both in place on the state
  static hipError_t prepass_to(lbm_ctx* ctx, S* f, S* g, const FieldSet& F) {
    const lbm_params& p = ctx->p;
    const Geom geo = geom_of(p);
    const Phys<C> ph = phys_of<C>(p);
    const Faces<C> fc = faces_of<C>(ctx);
    const unsigned nb = blocks_for(geo.N);
    hipLaunchKernelGGL(k_macro<S>, dim3(nb), dim3(256), 0, ctx->stream, f, g, (C*)F.rho, (C*)F.T, (C*)F.psi,
                       ctx->flag, geo, fc, ph);
    hipLaunchKernelGGL(k_force<S>, dim3(nb), dim3(256), 0, ctx->stream, f, (const C*)F.rho, (const C*)F.psi,
                       (C*)F.ueq, (C*)F.du, (C*)F.ureal, geo, fc, ph);
    return hipGetLastError();
  }

  static hipError_t prepass_on(lbm_ctx* ctx, S* f, S* g) { return prepass_to(ctx, f, g, ctx_fields(ctx)); }

  static hipError_t prepass(lbm_ctx* ctx) { return prepass_on(ctx, (S*)ctx->fA, (S*)ctx->gA); }

  // One step from the state (fs, gs) into (fd, gd).  The unfused kernels
  // complete the boundary nodes of (fs, gs) in place; the fused kernel only
  // reads it.
  static hipError_t step_ref_to(lbm_ctx* ctx, S* fs, S* gs, S* fd, S* gd, const FieldSet& F) {
    hipError_t e = prepass_to(ctx, fs, gs, F);
    if (e != hipSuccess) return e;
    const Geom geo = geom_of(ctx->p);
    // vartheta = 1: record T, and apply the correction once two past values exist
    const int corr = ctx->p.theta_corr ? (ctx->hist >= 2 ? 2 : 1) : 0;
    hipLaunchKernelGGL(k_collide_push<S>, dim3(blocks_for(geo.N)), dim3(256), 0, ctx->stream, (const S*)fs,
                       (const S*)gs, fd, gd, (const C*)F.rho, (const C*)F.T, (const C*)F.ueq, (const C*)F.du,
                       (const C*)F.ureal, (const C*)ctx->Th[0], (C*)ctx->Th[1], corr, (C*)F.div, geo,
                       phys_of<C>(ctx->p));
    if (corr) {
      std::swap(ctx->Th[0], ctx->Th[1]);
      ctx->hist = std::min(ctx->hist + 1, 2);
    }
    return hipGetLastError();
  }

  static hipError_t step_ref(lbm_ctx* ctx, S* fs, S* gs, S* fd, S* gd) {
    return step_ref_to(ctx, fs, gs, fd, gd, ctx_fields(ctx));
  }

  static hipError_t step_fused(lbm_ctx* ctx, const S* fs, const S* gs, S* fd, S* gd, int xmode = 0) {
    const lbm_params& p = ctx->p;
    return FusedImpl<S>::step(p, phys_of<C>(p), ctx->stream, fs, gs, fd, gd, ctx->has_Tw[0] ? ctx->Tw[0] : nullptr,
                              ctx->has_Tw[1] ? ctx->Tw[1] : nullptr, ctx->flag, ctx->fused_ty, ctx->fused_chunk,
                              ctx->fused_map, nullptr, xmode);
  }

  // A single-pass step that also writes the fields of its start state into F
  // and completes the start state's face-plane g in place (what the prepass
  // leaves); the adjoint's recomputation on set-ups the single-pass kernel
  // takes.
  static hipError_t step_fused_fields(lbm_ctx* ctx, const S* fs, S* gs, S* fd, S* gd, const FieldSet& F) {
    const lbm_params& p = ctx->p;
    const FusedFields<C> fo{(C*)F.rho, (C*)F.T, (C*)F.psi, (C*)F.ueq, (C*)F.du, (C*)F.ureal, (C*)F.div};
    return FusedImpl<S>::step(p, phys_of<C>(p), ctx->stream, fs, gs, fd, gd, ctx->has_Tw[0] ? ctx->Tw[0] : nullptr,
                              ctx->has_Tw[1] ? ctx->Tw[1] : nullptr, ctx->flag, 8, ctx->fused_chunk, false, &fo);
  }

  static hipError_t step_from(lbm_ctx* ctx, S* fs, S* gs, S* fd, S* gd) {
    return ctx->fused_ok ? step_fused(ctx, fs, gs, fd, gd) : step_ref(ctx, fs, gs, fd, gd);
  }

  // xmode (fused kernel, whole 8-row tiles): bit 0, the current state is
  // x-deferred; bit 1, leave the next state x-deferred
  static hipError_t step(lbm_ctx* ctx, int xmode = 0) {
    hipError_t e = xmode ? step_fused(ctx, (S*)ctx->fA, (S*)ctx->gA, (S*)ctx->fB, (S*)ctx->gB, xmode)
                         : step_from(ctx, (S*)ctx->fA, (S*)ctx->gA, (S*)ctx->fB, (S*)ctx->gB);
    if (e != hipSuccess) return e;
    std::swap(ctx->fA, ctx->fB);
    std::swap(ctx->gA, ctx->gB);
    return hipSuccess;
  }

  static hipError_t init_slab(lbm_ctx* ctx, const double* drho, const double* du, const double* dT, long long c0,
                              long long len) {
    const lbm_params& p = ctx->p;
    hipLaunchKernelGGL(k_init<S>, dim3(blocks_for(len)), dim3(256), 0, ctx->stream, (S*)ctx->fA, (S*)ctx->gA, drho,
                       du, dT, c0, len, (long long)p.nx * p.ny, plane_pitch(p.nx, p.ny), p.rho_ref, p.T_ref,
                       1.0 - p.wbar, p.wbar / 6.0);
    return hipGetLastError();
  }

  static hipError_t fields_slab(lbm_ctx* ctx, double* orho, double* ou, double* oT, long long c0, long long len,
                                long long ustride) {
    hipLaunchKernelGGL(k_fields_out<C>, dim3(blocks_for(len)), dim3(256), 0, ctx->stream, (const C*)ctx->rho,
                       (const C*)ctx->T, (const C*)ctx->ueq, (const C*)ctx->du, orho, ou, oT, c0, len,
                       ncells(ctx->p), ustride);
    return hipGetLastError();
  }

  static hipError_t pops_slab(lbm_ctx* ctx, double* of, double* og, long long c0, long long len) {
    const lbm_params& p = ctx->p;
    hipLaunchKernelGGL(k_pops_out<S>, dim3(blocks_for(len)), dim3(256), 0, ctx->stream, (const S*)ctx->fA,
                       (const S*)ctx->gA, of, og, c0, len, (long long)p.nx * p.ny, plane_pitch(p.nx, p.ny),
                       p.rho_ref, p.T_ref, 1.0 - p.wbar, p.wbar / 6.0);
    return hipGetLastError();
  }

  static hipError_t diag(lbm_ctx* ctx) {
    const lbm_params& p = ctx->p;
    hipLaunchKernelGGL(k_diag_partials<C>, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, ctx->stream, (const C*)ctx->rho,
                       (const C*)ctx->T, ncells(p), p.cv, p.diag_rho_v, p.diag_rho_l, ctx->partials);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(RED_THREADS), 0, ctx->stream, (const double*)ctx->partials,
                       RED_BLOCKS, ctx->sums);
    return hipGetLastError();
  }
};

template <typename F>
hipError_t dispatch(lbm_ctx* ctx, F&& fn) {
  switch (ctx->p.precision) {
    case LBM_FP64: return fn(Impl<double>());
    case LBM_FP32_DEV: return fn(Impl<float>());
    case LBM_FP16_DEV: return fn(Impl<_Float16>());
    default: return fn(Impl<bf16>());
  }
}

lbm_status reduce_now(lbm_ctx* ctx, double out[RED_VALUES]) {
  HIPCHK(ctx, dispatch(ctx, [&](auto impl) { return decltype(impl)::prepass(ctx); }));
  HIPCHK(ctx, dispatch(ctx, [&](auto impl) { return decltype(impl)::diag(ctx); }));
  HIPCHK(ctx, hipMemcpyAsync(out, ctx->sums, RED_VALUES * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return LBM_OK;
}


// ------------------------------------------------------------- adjoint

// Memory plan of lbm_adjoint: checkpoints of the state every L steps, one
// segment of L recomputed states, two copies of the adjoint populations,
// the adjoint fields and wall planes, the FP64 gradient accumulators.
struct AdjPlan {
  int nsteps = 0, nseg = 0, L = 0;
  size_t fbytes = 0, gbytes = 0;
  size_t off_ck = 0, off_seg = 0, off_lf[2] = {0, 0}, off_lg[2] = {0, 0}, off_d[2] = {0, 0}, off_rho = 0, off_T = 0,
         off_div = 0,
         off_ueq = 0, off_du = 0, off_gadj = 0, off_ax = 0, off_ay = 0, off_kap = 0, off_grad = 0, off_acc = 0,
         off_fdiv = 0;
  // fields of every state of a segment, kept from its recomputation; with
  // the single-pass kernel (fused) the step from a segment's last state is
  // taken once more into a spare state (off_spare) to write that state's
  // fields, so that every state's fields come from the same kernel
  bool cache = false, fused = false;
  size_t off_fields = 0, fslot = 0, fN = 0, off_spare = 0;
  size_t total = 0;
  size_t state() const { return fbytes + gbytes; }
  FieldSet fields(char* base, int j) const {
    char* q = base + off_fields + (size_t)j * fslot;
    return {q, q + fN, q + 2 * fN, q + 3 * fN, q + 6 * fN, q + 9 * fN, q + 12 * fN};
  }
};

AdjPlan adjoint_plan(const lbm_params& p, const lbm_adjoint_spec& sp, bool fused) {
  AdjPlan a;
  a.nsteps = sp.nsteps;
  int K = sp.n_checkpoints > 0 ? sp.n_checkpoints : (int)std::ceil(std::sqrt((double)sp.nsteps));
  K = std::max(1, std::min(K, sp.nsteps));
  a.L = (sp.nsteps + K - 1) / K;
  a.nseg = (sp.nsteps + a.L - 1) / a.L;
  const size_t N = (size_t)ncells(p);
  const size_t P = (size_t)p.nx * p.ny;
  const size_t es = elem_size(p.precision), cs = compute_size(p.precision);
  const size_t NP = (size_t)p.nz * plane_pitch(p.nx, p.ny);
  a.fbytes = align_up(19 * NP * es);
  a.gbytes = align_up(7 * NP * es);
  size_t o = 0;
  a.off_ck = o; o += (size_t)a.nseg * a.state();
  a.off_seg = o; o += (size_t)a.L * a.state();
  for (int k = 0; k < 2; ++k) {
    a.off_lf[k] = o; o = align_up(o + 19 * NP * cs);
    a.off_lg[k] = o; o = align_up(o + 7 * NP * cs);
    a.off_d[k] = o; o = align_up(o + 5 * N * cs);  // deferred moment update (rb, jb, Tb) per cell
  }
  a.off_rho = o; o = align_up(o + N * cs);
  a.off_T = o; o = align_up(o + N * cs);
  a.off_div = o; o = align_up(o + N * cs);
  a.off_ueq = o; o = align_up(o + 3 * N * cs);
  a.off_du = o; o = align_up(o + 3 * N * cs);
  a.off_gadj = o; o = align_up(o + 2 * P * cs);
  a.off_ax = o; o = align_up(o + 2 * P * cs);
  a.off_ay = o; o = align_up(o + 2 * P * cs);
  a.off_kap = o; o = align_up(o + 2 * P * 8);
  a.off_grad = o; o = align_up(o + P * 8);
  a.off_acc = o; o = align_up(o + 64);
  a.off_fdiv = o; o = align_up(o + N * cs);  // div u of the state when the fields are not stored
  a.cache = true;
  a.fused = fused;
  a.fN = N * cs;
  a.fslot = align_up(13 * a.fN);
  a.off_fields = o; o += (size_t)a.L * a.fslot;
  if (a.fused) {
    a.off_spare = o; o += a.state();
  }
  a.total = o;
  return a;
}

lbm_status adjoint_check(const lbm_ctx* ctx, const lbm_adjoint_spec* sp, std::string& msg) {
  if (!sp) { msg = "spec is NULL"; return LBM_EINVAL; }
  if (sp->nsteps < 1) { msg = "nsteps must be >= 1"; return LBM_EINVAL; }
  if (sp->n_checkpoints < 0) { msg = "n_checkpoints must be >= 0"; return LBM_EINVAL; }
  if (sp->objective != 0) { msg = "unknown objective"; return LBM_EINVAL; }
  if (sp->wall_face != 4 && sp->wall_face != 5) { msg = "wall_face must be 4 or 5"; return LBM_EINVAL; }
  if (ctx->p.face[sp->wall_face] == LBM_FACE_PERIODIC) { msg = "wall_face is periodic"; return LBM_EINVAL; }
  for (int k = 0; k < 4; ++k)
    if (ctx->p.face[k] != LBM_FACE_PERIODIC) {
      msg = "the adjoint needs periodic x and y faces"; return LBM_EUNSUPPORTED;
    }
  if (ctx->p.lambda_vapour > 0.0) { msg = "the adjoint needs a uniform conductivity"; return LBM_EUNSUPPORTED; }
  if (ctx->p.theta_corr) { msg = "the adjoint is built for vartheta = 0"; return LBM_EUNSUPPORTED; }
  return LBM_OK;
}

struct DeviceBlock {
  void* ptr = nullptr;
  hipStream_t stream = nullptr;
  ~DeviceBlock() {
    if (ptr) {
      (void)hipStreamSynchronize(stream);
      (void)hipFree(ptr);
    }
  }
};

// workspace: NULL allocates the plan's workspace for the call (and frees it
// on return); otherwise ws_bytes of device memory the caller provides.
template <typename S>
lbm_status adjoint_run(lbm_ctx* ctx, const lbm_adjoint_spec& sp, double* J, double* dJ_dTw, double* dJ_dkappa,
                       int32_t on_device, void* workspace = nullptr, size_t ws_bytes = 0) {
  using C = typename Storage<S>::C;
  using I = Impl<S>;
  const lbm_params& p = ctx->p;
  const AdjPlan a = adjoint_plan(p, sp, ctx->fused_ok);
  const Geom geo = geom_of(p);
  const long long N = geo.N;
  const long long P = (long long)p.nx * p.ny;
  DeviceBlock blk;
  blk.stream = ctx->stream;
  char* b = nullptr;
  if (workspace) {
    if (a.total > ws_bytes) {
      ctx->err = std::string("adjoint workspace of ") + std::to_string(a.total) + " bytes exceeds the " +
                 std::to_string(ws_bytes) + " bytes available";
      return LBM_ENOMEM;
    }
    b = (char*)workspace;
  } else {
    const hipError_t e = hipMalloc(&blk.ptr, a.total);
    if (e != hipSuccess) {
      blk.ptr = nullptr;
      ctx->err = std::string("adjoint workspace of ") + std::to_string(a.total) + " bytes: " + hipGetErrorString(e);
      return LBM_ENOMEM;
    }
    b = (char*)blk.ptr;
  }
  auto ck_f = [&](int k) { return (S*)(b + a.off_ck + (size_t)k * a.state()); };
  auto ck_g = [&](int k) { return (S*)(b + a.off_ck + (size_t)k * a.state() + a.fbytes); };
  auto sg_f = [&](int j) { return (S*)(b + a.off_seg + (size_t)j * a.state()); };
  auto sg_g = [&](int j) { return (S*)(b + a.off_seg + (size_t)j * a.state() + a.fbytes); };
  C* lf[2] = {(C*)(b + a.off_lf[0]), (C*)(b + a.off_lf[1])};
  C* lg[2] = {(C*)(b + a.off_lg[0]), (C*)(b + a.off_lg[1])};
  C* ld[2] = {(C*)(b + a.off_d[0]), (C*)(b + a.off_d[1])};
  C* a_rho = (C*)(b + a.off_rho);
  C* a_T = (C*)(b + a.off_T);
  C* a_div = (C*)(b + a.off_div);
  C* a_ueq = (C*)(b + a.off_ueq);
  C* a_du = (C*)(b + a.off_du);
  C* gadj = (C*)(b + a.off_gadj);
  C* ax = (C*)(b + a.off_ax);
  C* ay = (C*)(b + a.off_ay);
  double* kap = (double*)(b + a.off_kap);
  double* grad = (double*)(b + a.off_grad);
  double* acc = (double*)(b + a.off_acc);
  const hipStream_t st = ctx->stream;
  const size_t NP = (size_t)p.nz * plane_pitch(p.nx, p.ny);
  const size_t fsz = 19 * NP * sizeof(S), gsz = 7 * NP * sizeof(S);
  const bool walls = p.face[4] == LBM_FACE_WALL || p.face[5] == LBM_FACE_WALL;
  const bool outlets = p.face[4] == LBM_FACE_PRESSURE || p.face[5] == LBM_FACE_PRESSURE;

  // forward pass with checkpoints; J = M(t0) - M(t0 + N)
  double s0[RED_VALUES], s1[RED_VALUES];
  lbm_status rs = reduce_now(ctx, s0);
  if (rs != LBM_OK) return rs;
  for (int k = 0; k < a.nseg; ++k) {
    HIPCHK(ctx, hipMemcpyAsync(ck_f(k), ctx->fA, fsz, hipMemcpyDeviceToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(ck_g(k), ctx->gA, gsz, hipMemcpyDeviceToDevice, st));
    const int len = std::min(a.L, a.nsteps - k * a.L);
    for (int j = 0; j < len; ++j) {
      HIPCHK(ctx, I::step(ctx));
      ctx->step++;
    }
  }
  rs = reduce_now(ctx, s1);
  if (rs != LBM_OK) return rs;
  {
    int flag = 0;
    HIPCHK(ctx, hipMemcpyAsync(&flag, ctx->flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(ctx, hipStreamSynchronize(st));
    if (flag) { ctx->err = "non-physical state in the forward pass"; return LBM_ENONPHYS; }
  }

  // reverse sweep, one segment at a time
  const Phys<C> ph = phys_of<C>(p);
  const unsigned nb = blocks_for(N), npb = blocks_for(P);
  hipLaunchKernelGGL(k_adj_seed<C>, dim3(nb), dim3(256), 0, st, lf[0], lg[0], ld[0], geo);
  hipLaunchKernelGGL(k_zero_f64, dim3(npb), dim3(256), 0, st, grad, P);
  hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(256), 0, st, acc, 8ll);
  hipLaunchKernelGGL(k_zero_f64, dim3(blocks_for(2 * P)), dim3(256), 0, st, kap, 2 * P);
  HIPCHK(ctx, hipGetLastError());
  int cur = 0;
  for (int k = a.nseg - 1; k >= 0; --k) {
    const int len = std::min(a.L, a.nsteps - k * a.L);
    HIPCHK(ctx, hipMemcpyAsync(sg_f(0), ck_f(k), fsz, hipMemcpyDeviceToDevice, st));
    HIPCHK(ctx, hipMemcpyAsync(sg_g(0), ck_g(k), gsz, hipMemcpyDeviceToDevice, st));
    // recompute the segment, keeping the fields of every state
    for (int j = 1; j < len; ++j) {
      if (a.fused)
        HIPCHK(ctx, I::step_fused_fields(ctx, sg_f(j - 1), sg_g(j - 1), sg_f(j), sg_g(j), a.fields(b, j - 1)));
      else HIPCHK(ctx, I::step_ref_to(ctx, sg_f(j - 1), sg_g(j - 1), sg_f(j), sg_g(j), a.fields(b, j - 1)));
    }
    for (int j = len - 1; j >= 0; --j) {
      const S* gnext = j + 1 < len ? sg_g(j + 1) : (k + 1 < a.nseg ? ck_g(k + 1) : (const S*)ctx->gA);
      FieldSet F = a.cache ? a.fields(b, j) : ctx_fields(ctx);
      if (!F.div) F.div = b + a.off_fdiv;
      if (j == len - 1) {
        // fields of a state no recomputed step has written
        if (a.fused) {
          // its step once more, into the spare state
          HIPCHK(ctx, I::step_fused_fields(ctx, sg_f(j), sg_g(j), (S*)(b + a.off_spare),
                                           (S*)(b + a.off_spare + a.fbytes), F));
        } else {
          // S0-S5, then div u with the step's own definition
          HIPCHK(ctx, I::prepass_to(ctx, sg_f(j), sg_g(j), F));
          hipLaunchKernelGGL(k_div<C>, dim3(nb), dim3(256), 0, st, (const C*)F.ureal, (C*)F.div, geo);
        }
      }
      const C* rho = (const C*)F.rho;
      const C* T = (const C*)F.T;
      const C* psi = (const C*)F.psi;
      const C* ueq = (const C*)F.ueq;
      const C* du = (const C*)F.du;
      const int nx = 1 - cur;
      hipLaunchKernelGGL(k_adj_collide<S>, dim3(nb), dim3(256), 0, st, (const C*)lf[cur], (const C*)lg[cur],
                         (const C*)ld[cur], (const S*)sg_g(j), gnext, rho, T, ueq, du, (const C*)F.div, lf[nx], lg[nx], a_rho, a_T,
                         a_ueq, a_du, a_div, geo, ph);
      hipLaunchKernelGGL(k_adj_velocity<C>, dim3(nb), dim3(256), 0, st, (const C*)a_div, a_ueq, a_du,
                         a_rho, rho, ueq, du, geo);
      if (outlets) hipLaunchKernelGGL(k_adj_outlet<C>, dim3(npb), dim3(256), 0, st, lf[nx], a_ueq, a_du, a_rho, geo);
      if (walls)
        hipLaunchKernelGGL(k_adj_ghost<C>, dim3(npb), dim3(256), 0, st, (const C*)a_du, psi, gadj, ax, ay, kap, geo,
                           ph);
      hipLaunchKernelGGL(k_adj_psi<C>, dim3(nb), dim3(256), 0, st, ld[nx], (const C*)a_rho,
                         (const C*)a_T, (const C*)a_ueq, (const C*)a_du, psi, rho, T, (const C*)gadj, (const C*)ax,
                         (const C*)ay, geo, ph);
      hipLaunchKernelGGL(k_adj_dirichlet<C>, dim3(npb), dim3(256), 0, st, lg[nx], ld[nx], grad, (int)sp.wall_face,
                         geo, ph);
      HIPCHK(ctx, hipGetLastError());
      cur = nx;
    }
  }
  if (walls) hipLaunchKernelGGL(k_accumulate<double>, dim3(1), dim3(RED_THREADS), 0, st, (const double*)kap, 2 * P, acc);
  double kappa_grad = 0.0;
  HIPCHK(ctx, hipMemcpyAsync(&kappa_grad, acc, sizeof(double), hipMemcpyDeviceToHost, st));
  if (dJ_dTw)
    HIPCHK(ctx, hipMemcpyAsync(dJ_dTw, grad, P * 8, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipStreamSynchronize(st));
  if (J) *J = s0[0] - s1[0];
  if (dJ_dkappa) *dJ_dkappa = kappa_grad;
  return LBM_OK;
}

// ---------------------------------------------------------------- checkpoint / resume

// Host image of a context's state: this header, then the raw population
// buffers A (f, then g, in the device layout and storage format), the two
// temperature-history fields when theta_corr = 1, and the two wall
// temperature planes.
struct SaveHeader {
  char magic[8];
  int32_t version, precision, nx, ny, nz, theta_corr, hist;
  int32_t has_Tw[2];
  int64_t step;
  double mass0, kappa_w;
  uint64_t fbytes, gbytes, hbytes, twbytes;
};
constexpr char kSaveMagic[8] = {'L', 'B', 'M', '3', 'D', 'S', 'V', '1'};

struct SaveSizes {
  size_t f, g, h, tw, total;
};

SaveSizes save_sizes(const lbm_params& p) {
  SaveSizes z;
  const size_t NP = (size_t)p.nz * plane_pitch(p.nx, p.ny);
  const size_t es = elem_size(p.precision), cs = compute_size(p.precision);
  z.f = 19 * NP * es;
  z.g = 7 * NP * es;
  z.h = p.theta_corr ? (size_t)ncells(p) * cs : 0;
  z.tw = (size_t)p.nx * p.ny * 8;
  z.total = sizeof(SaveHeader) + z.f + z.g + 2 * z.h + 2 * z.tw;
  return z;
}

}  // namespace

extern "C" {

lbm_status lbm_default_params(lbm_params* p, int32_t nx, int32_t ny, int32_t nz) {
  if (!p) return LBM_EINVAL;
  std::memset(p, 0, sizeof(*p));
  p->nx = nx; p->ny = ny; p->nz = nz;
  p->precision = LBM_FP32_DEV;
  p->a = 3.0 / 49.0; p->b = 2.0 / 21.0; p->R = 1.0; p->omega = 0.344; p->G = -1.0;
  p->s_e = 1.25; p->s_nu = 0.8; p->s_q = 1.0; p->s_pi = 1.0;
  p->wbar = 0.75; p->lambda = 1.0 / 3.0; p->cv = 5.0; p->s_T_other = 1.0;
  p->theta_corr = 0;
  for (int k = 0; k < 6; ++k) { p->face[k] = LBM_FACE_PERIODIC; p->face_T[k] = 0.0; p->face_rho[k] = 0.0; }
  p->kappa_w = 0.0;
  const double Tc = 0.0778 * p->a / (0.45724 * p->b * p->R);
  p->rho_ref = 0.3796789993997207;
  p->T_ref = 0.86 * Tc;
  p->diag_rho_v = 0.3796789993997207;
  p->diag_rho_l = 6.4989457632878835;
  return LBM_OK;
}

lbm_status lbm_required_bytes(const lbm_params* p, size_t* state_bytes, size_t* scratch_bytes) {
  std::string msg;
  const lbm_status s = validate(p, msg);
  if (s != LBM_OK) { g_create_error = msg; return s; }
  if (!state_bytes || !scratch_bytes) return LBM_EINVAL;
  const Layout L = layout_of(*p);
  *state_bytes = L.state;
  *scratch_bytes = L.scratch;
  return LBM_OK;
}

lbm_status lbm_create(const lbm_params* p, void* device_buffer, size_t buffer_bytes, void* hip_stream,
                      lbm_ctx** out) {
  if (!out) { g_create_error = "out is NULL"; return LBM_EINVAL; }
  *out = nullptr;
  std::string msg;
  const lbm_status s = validate(p, msg);
  if (s != LBM_OK) { g_create_error = msg; return s; }
  const Layout L = layout_of(*p);
  const size_t need = L.state + L.scratch;
  lbm_ctx* ctx = new (std::nothrow) lbm_ctx();
  if (!ctx) { g_create_error = "host allocation failed"; return LBM_ENOMEM; }
  ctx->p = *p;
  ctx->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&ctx->device) != hipSuccess) ctx->device = -1;
  if (device_buffer) {
    if (buffer_bytes < need || ((uintptr_t)device_buffer % kAlign) != 0) {
      g_create_error = "device_buffer too small or not 256-byte aligned";
      delete ctx;
      return LBM_ENOMEM;
    }
    ctx->base = (char*)device_buffer;
    ctx->owns = false;
  } else {
    void* ptr = nullptr;
    hipError_t e = hipMalloc(&ptr, need);
    if (e != hipSuccess) {
      g_create_error = std::string("hipMalloc: ") + hipGetErrorString(e);
      delete ctx;
      return LBM_ENOMEM;
    }
    ctx->base = (char*)ptr;
    ctx->owns = true;
  }
  ctx->bytes = need;
  char* b = ctx->base;
  ctx->fA = b + L.off_fA; ctx->gA = b + L.off_gA; ctx->fB = b + L.off_fB; ctx->gB = b + L.off_gB;
  ctx->rho = b + L.off_rho; ctx->T = b + L.off_T; ctx->psi = b + L.off_psi;
  ctx->ueq = b + L.off_ueq; ctx->du = b + L.off_du; ctx->ureal = b + L.off_ureal;
  ctx->Th[0] = b + L.off_Th0; ctx->Th[1] = b + L.off_Th1;
  ctx->Tw[0] = (double*)(b + L.off_Tw0); ctx->Tw[1] = (double*)(b + L.off_Tw1);
  ctx->partials = (double*)(b + L.off_part);
  ctx->sums = (double*)(b + L.off_sums);
  ctx->flag = (int*)(b + L.off_flag);
  ctx->staging = (double*)(b + L.off_stage);
  ctx->fused_ty = fused_tile_height(p->precision);
  ctx->fused_ok = fused_supported(*p, ctx->fused_ty) && p->theta_corr == 0;
  if (const char* ev = std::getenv("LBM_FUSED_MAP")) ctx->fused_map = std::atoi(ev) == 1;
  {
    ctx->fused_chunk = fused_chunk_planes(p->nx, p->ny, p->nz, ctx->fused_ty);
    if (const char* ev = std::getenv("LBM_FUSED")) {
      if (ev[0] == '0') ctx->fused_ok = false;
    }
    if (const char* ev = std::getenv("LBM_FUSED_CHUNK")) ctx->fused_chunk = std::max(1, std::atoi(ev));
    ctx->fused_xdefer = ctx->fused_ok && ctx->fused_ty == 8 && p->nx % FTX == 0 && p->precision == LBM_FP64;
    if (const char* ev = std::getenv("LBM_FUSED_XDEFER")) {
      if (ev[0] == '0') ctx->fused_xdefer = false;
    }
  }
  hipError_t e = hipMemsetAsync(ctx->flag, 0, 64, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    g_create_error = std::string("hipMemsetAsync: ") + hipGetErrorString(e);
    if (ctx->owns) (void)hipFree(ctx->base);
    delete ctx;
    return LBM_EHIP;
  }
  *out = ctx;
  return LBM_OK;
}

lbm_status lbm_init(lbm_ctx* ctx, const double* rho, const double* u, const double* T) {
  if (!ctx) return LBM_EINVAL;
  if (!rho || !T) { ctx->err = "rho and T are required"; return LBM_EINVAL; }
  const long long N = ncells(ctx->p);
  const long long slab = std::min(kSlab, N);
  double* srho = ctx->staging;
  double* su = srho + slab;
  double* sT = su + 3 * slab;
  for (long long c0 = 0; c0 < N; c0 += slab) {
    const long long len = std::min(slab, N - c0);
    HIPCHK(ctx, hipMemcpyAsync(srho, rho + c0, len * 8, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(sT, T + c0, len * 8, hipMemcpyHostToDevice, ctx->stream));
    if (u) {
      for (int a = 0; a < 3; ++a)
        HIPCHK(ctx, hipMemcpyAsync(su + a * len, u + a * N + c0, len * 8, hipMemcpyHostToDevice, ctx->stream));
    }
    HIPCHK(ctx, dispatch(ctx, [&](auto impl) {
      return decltype(impl)::init_slab(ctx, srho, u ? su : nullptr, sT, c0, len);
    }));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  }
  HIPCHK(ctx, hipMemsetAsync(ctx->flag, 0, 64, ctx->stream));
  ctx->initialised = true;
  ctx->step = 0;
  ctx->hist = 0;
  double sums[RED_VALUES];
  const lbm_status s = reduce_now(ctx, sums);
  if (s != LBM_OK) return s;
  ctx->mass0 = sums[0];
  return LBM_OK;
}

lbm_status lbm_set_wall_T(lbm_ctx* ctx, int32_t face, const double* Tw) {
  if (!ctx) return LBM_EINVAL;
  if (face != 4 && face != 5) { ctx->err = "wall temperature fields exist for faces 4 and 5"; return LBM_EINVAL; }
  if (ctx->p.face[face] != LBM_FACE_WALL) { ctx->err = "face is not a wall"; return LBM_EINVAL; }
  const int k = face - 4;
  if (!Tw) { ctx->has_Tw[k] = false; return LBM_OK; }
  const size_t n = (size_t)ctx->p.nx * ctx->p.ny;
  for (size_t i = 0; i < n; ++i)
    if (!(Tw[i] > 0) || !std::isfinite(Tw[i])) { ctx->err = "wall temperatures must be positive"; return LBM_EINVAL; }
  HIPCHK(ctx, hipMemcpyAsync(ctx->Tw[k], Tw, n * 8, hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  ctx->has_Tw[k] = true;
  return LBM_OK;
}

lbm_status lbm_set_kappa(lbm_ctx* ctx, double kappa_w) {
  if (!ctx) return LBM_EINVAL;
  if (!std::isfinite(kappa_w)) { ctx->err = "kappa_w must be finite"; return LBM_EINVAL; }
  ctx->p.kappa_w = kappa_w;
  return LBM_OK;
}

lbm_status lbm_save_bytes(const lbm_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return LBM_EINVAL;
  *bytes = save_sizes(ctx->p).total;
  return LBM_OK;
}

lbm_status lbm_save(lbm_ctx* ctx, void* host_dst, size_t bytes) {
  if (!ctx || !host_dst) return LBM_EINVAL;
  if (!ctx->initialised) { ctx->err = "lbm_save before lbm_init"; return LBM_ESTATE; }
  const SaveSizes z = save_sizes(ctx->p);
  if (bytes < z.total) { ctx->err = "lbm_save: buffer smaller than lbm_save_bytes"; return LBM_EINVAL; }
  SaveHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, kSaveMagic, 8);
  h.version = 1;
  h.precision = ctx->p.precision;
  h.nx = ctx->p.nx; h.ny = ctx->p.ny; h.nz = ctx->p.nz;
  h.theta_corr = ctx->p.theta_corr;
  h.hist = ctx->hist;
  h.has_Tw[0] = ctx->has_Tw[0]; h.has_Tw[1] = ctx->has_Tw[1];
  h.step = ctx->step;
  h.mass0 = ctx->mass0;
  h.kappa_w = ctx->p.kappa_w;
  h.fbytes = z.f; h.gbytes = z.g; h.hbytes = z.h; h.twbytes = z.tw;
  char* o = (char*)host_dst;
  std::memcpy(o, &h, sizeof(h));
  o += sizeof(h);
  const hipStream_t st = ctx->stream;
  HIPCHK(ctx, hipMemcpyAsync(o, ctx->fA, z.f, hipMemcpyDeviceToHost, st)); o += z.f;
  HIPCHK(ctx, hipMemcpyAsync(o, ctx->gA, z.g, hipMemcpyDeviceToHost, st)); o += z.g;
  for (int k = 0; k < 2 && z.h; ++k) { HIPCHK(ctx, hipMemcpyAsync(o, ctx->Th[k], z.h, hipMemcpyDeviceToHost, st)); o += z.h; }
  for (int k = 0; k < 2; ++k) { HIPCHK(ctx, hipMemcpyAsync(o, ctx->Tw[k], z.tw, hipMemcpyDeviceToHost, st)); o += z.tw; }
  HIPCHK(ctx, hipStreamSynchronize(st));
  return LBM_OK;
}

lbm_status lbm_load(lbm_ctx* ctx, const void* host_src, size_t bytes) {
  if (!ctx || !host_src) return LBM_EINVAL;
  const SaveSizes z = save_sizes(ctx->p);
  SaveHeader h;
  if (bytes < sizeof(h)) { ctx->err = "lbm_load: image too short"; return LBM_EINVAL; }
  std::memcpy(&h, host_src, sizeof(h));
  if (std::memcmp(h.magic, kSaveMagic, 8) != 0 || h.version != 1) {
    ctx->err = "lbm_load: not an image written by lbm_save"; return LBM_EINVAL;
  }
  if (h.precision != ctx->p.precision || h.nx != ctx->p.nx || h.ny != ctx->p.ny || h.nz != ctx->p.nz ||
      h.theta_corr != ctx->p.theta_corr) {
    ctx->err = "lbm_load: grid, precision or theta_corr differ from this context"; return LBM_EINVAL;
  }
  if (h.fbytes != z.f || h.gbytes != z.g || h.hbytes != z.h || h.twbytes != z.tw || bytes < z.total) {
    ctx->err = "lbm_load: image size does not match this context"; return LBM_EINVAL;
  }
  if (h.hist < 0 || h.hist > 2) { ctx->err = "lbm_load: corrupt history count"; return LBM_EINVAL; }
  const char* o = (const char*)host_src + sizeof(h);
  const hipStream_t st = ctx->stream;
  HIPCHK(ctx, hipMemcpyAsync(ctx->fA, o, z.f, hipMemcpyHostToDevice, st)); o += z.f;
  HIPCHK(ctx, hipMemcpyAsync(ctx->gA, o, z.g, hipMemcpyHostToDevice, st)); o += z.g;
  for (int k = 0; k < 2 && z.h; ++k) { HIPCHK(ctx, hipMemcpyAsync(ctx->Th[k], o, z.h, hipMemcpyHostToDevice, st)); o += z.h; }
  for (int k = 0; k < 2; ++k) { HIPCHK(ctx, hipMemcpyAsync(ctx->Tw[k], o, z.tw, hipMemcpyHostToDevice, st)); o += z.tw; }
  HIPCHK(ctx, hipMemsetAsync(ctx->flag, 0, 64, st));
  HIPCHK(ctx, hipStreamSynchronize(st));
  ctx->step = h.step;
  ctx->mass0 = h.mass0;
  ctx->hist = h.hist;
  ctx->has_Tw[0] = h.has_Tw[0] != 0;
  ctx->has_Tw[1] = h.has_Tw[1] != 0;
  ctx->p.kappa_w = h.kappa_w;
  ctx->initialised = true;
  return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* ctx, int32_t nsteps) {
  if (!ctx) return LBM_EINVAL;
  if (nsteps < 0) { ctx->err = "nsteps must be >= 0"; return LBM_EINVAL; }
  if (!ctx->initialised) { ctx->err = "lbm_step before lbm_init"; return LBM_ESTATE; }
  // between the steps of one call the D3Q19 populations may stay x-deferred
  // (streamed in y and z; the next step reads them shifted in x); the state
  // the call leaves is the ordinary one
  for (int s = 0; s < nsteps; ++s) {
    const int xmode = ctx->fused_xdefer ? (s > 0 ? 1 : 0) | (s + 1 < nsteps ? 2 : 0) : 0;
    HIPCHK(ctx, dispatch(ctx, [&](auto impl) { return decltype(impl)::step(ctx, xmode); }));
    ctx->step++;
  }
  int flag = 0;
  HIPCHK(ctx, hipMemcpyAsync(&flag, ctx->flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if (flag) { ctx->err = "non-physical state (rho, T or psi out of range, or NaN)"; return LBM_ENONPHYS; }
  return LBM_OK;
}

lbm_status lbm_fields(lbm_ctx* ctx, double* rho, double* u, double* T, int32_t dst_on_device) {
  if (!ctx) return LBM_EINVAL;
  if (!ctx->initialised) { ctx->err = "lbm_fields before lbm_init"; return LBM_ESTATE; }
  HIPCHK(ctx, dispatch(ctx, [&](auto impl) { return decltype(impl)::prepass(ctx); }));
  const long long N = ncells(ctx->p);
  if (dst_on_device) {
    HIPCHK(ctx, dispatch(ctx, [&](auto impl) { return decltype(impl)::fields_slab(ctx, rho, u, T, 0, N, N); }));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return LBM_OK;
  }
  const long long slab = std::min(kSlab, N);
  double* srho = ctx->staging;
  double* su = srho + slab;
  double* sT = su + 3 * slab;
  for (long long c0 = 0; c0 < N; c0 += slab) {
    const long long len = std::min(slab, N - c0);
    HIPCHK(ctx, dispatch(ctx, [&](auto impl) {
      return decltype(impl)::fields_slab(ctx, rho ? srho : nullptr, u ? su : nullptr, T ? sT : nullptr, c0, len, len);
    }));
    if (rho) HIPCHK(ctx, hipMemcpyAsync(rho + c0, srho, len * 8, hipMemcpyDeviceToHost, ctx->stream));
    if (T) HIPCHK(ctx, hipMemcpyAsync(T + c0, sT, len * 8, hipMemcpyDeviceToHost, ctx->stream));
    if (u)
      for (int a = 0; a < 3; ++a)
        HIPCHK(ctx, hipMemcpyAsync(u + a * N + c0, su + a * len, len * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  }
  return LBM_OK;
}

lbm_status lbm_populations(lbm_ctx* ctx, double* f, double* g) {
  if (!ctx) return LBM_EINVAL;
  if (!ctx->initialised) { ctx->err = "lbm_populations before lbm_init"; return LBM_ESTATE; }
  const long long N = ncells(ctx->p);
  const long long slab = std::min(kSlab, N);
  double* sf = ctx->staging;
  double* sg = sf + 19 * slab;
  for (long long c0 = 0; c0 < N; c0 += slab) {
    const long long len = std::min(slab, N - c0);
    HIPCHK(ctx, dispatch(ctx, [&](auto impl) {
      return decltype(impl)::pops_slab(ctx, f ? sf : nullptr, g ? sg : nullptr, c0, len);
    }));
    if (f)
      for (int i = 0; i < 19; ++i)
        HIPCHK(ctx, hipMemcpyAsync(f + i * N + c0, sf + i * len, len * 8, hipMemcpyDeviceToHost, ctx->stream));
    if (g)
      for (int i = 0; i < 7; ++i)
        HIPCHK(ctx, hipMemcpyAsync(g + i * N + c0, sg + i * len, len * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  }
  return LBM_OK;
}

lbm_status lbm_reduce(lbm_ctx* ctx, lbm_diag* out) {
  if (!ctx || !out) return LBM_EINVAL;
  if (!ctx->initialised) { ctx->err = "lbm_reduce before lbm_init"; return LBM_ESTATE; }
  double sums[RED_VALUES];
  const lbm_status s = reduce_now(ctx, sums);
  if (s != LBM_OK) return s;
  out->mass = sums[0];
  out->energy = sums[1];
  out->vol_hard = sums[2];
  out->vol_smooth = sums[3];
  out->evap_mass = ctx->mass0 - sums[0];
  out->step = ctx->step;
  return LBM_OK;
}

lbm_status lbm_adjoint_bytes(const lbm_ctx* ctx, const lbm_adjoint_spec* spec, size_t* bytes) {
  if (!ctx || !bytes) return LBM_EINVAL;
  std::string msg;
  const lbm_status s = adjoint_check(ctx, spec, msg);
  if (s != LBM_OK) return s;
  *bytes = adjoint_plan(ctx->p, *spec, ctx->fused_ok).total;
  return LBM_OK;
}

lbm_status lbm_adjoint(lbm_ctx* ctx, const lbm_adjoint_spec* spec, double* J, double* dJ_dTw, double* dJ_dkappa,
                       int32_t dst_on_device) {
  if (!ctx) return LBM_EINVAL;
  const lbm_status s = adjoint_check(ctx, spec, ctx->err);
  if (s != LBM_OK) return s;
  if (!ctx->initialised) { ctx->err = "lbm_adjoint before lbm_init"; return LBM_ESTATE; }
  switch (ctx->p.precision) {
    case LBM_FP64: return adjoint_run<double>(ctx, *spec, J, dJ_dTw, dJ_dkappa, dst_on_device);
    case LBM_FP32_DEV: return adjoint_run<float>(ctx, *spec, J, dJ_dTw, dJ_dkappa, dst_on_device);
    case LBM_FP16_DEV: return adjoint_run<_Float16>(ctx, *spec, J, dJ_dTw, dJ_dkappa, dst_on_device);
    default: return adjoint_run<bf16>(ctx, *spec, J, dJ_dTw, dJ_dkappa, dst_on_device);
  }
}

lbm_status lbm_adjoint_noalloc(lbm_ctx* ctx, const lbm_adjoint_spec* spec, double* J, double* dJ_dTw,
                               double* dJ_dkappa, int32_t dst_on_device) {
  if (!ctx) return LBM_EINVAL;
  const lbm_status s = adjoint_check(ctx, spec, ctx->err);
  if (s != LBM_OK) return s;
  if (!ctx->initialised) { ctx->err = "lbm_adjoint_noalloc before lbm_init"; return LBM_ESTATE; }
  int dev = -1;
  HIPCHK(ctx, hipGetDevice(&dev));
  if (dev != ctx->device || dev < 0 || dev >= kMaxDevices) {
    ctx->err = "lbm_adjoint_noalloc: the context's device is not the current device";
    return LBM_EINVAL;
  }
  void* ws = nullptr;
  {
    // the device address of this GPU's copy of the workspace array, looked up
    // once per device with that device current
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr) return hip_fail(ctx, e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                   "hipGetSymbolAddress(scratch)");
      g_scratch_ptr[dev] = ptr;
    }
    ws = g_scratch_ptr[dev];
  }
  switch (ctx->p.precision) {
    case LBM_FP64: return adjoint_run<double>(ctx, *spec, J, dJ_dTw, dJ_dkappa, dst_on_device, ws, kNoAllocBytes);
    case LBM_FP32_DEV: return adjoint_run<float>(ctx, *spec, J, dJ_dTw, dJ_dkappa, dst_on_device, ws, kNoAllocBytes);
    case LBM_FP16_DEV:
      return adjoint_run<_Float16>(ctx, *spec, J, dJ_dTw, dJ_dkappa, dst_on_device, ws, kNoAllocBytes);
    default: return adjoint_run<bf16>(ctx, *spec, J, dJ_dTw, dJ_dkappa, dst_on_device, ws, kNoAllocBytes);
  }
}

const char* lbm_last_error(const lbm_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

void lbm_destroy(lbm_ctx* ctx) {
  if (!ctx) return;
  if (ctx->owns && ctx->base) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(ctx->base);
  }
  delete ctx;
}

}  // extern "C"

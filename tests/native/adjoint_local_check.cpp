// Host-side check of the per-cell adjoint arithmetic of the library against
// the forward per-cell functions it transposes: dot-product identities for
// the linear maps, central differences for the nonlinear ones.  Prints one
// line "name max_relative_error" per check.
#include <cmath>
#include <cstdio>
#include <random>

#include "adjoint.h"
#include "kernels_ref.h"

using namespace lbm;

static std::mt19937_64 rng(12345);
static double uni(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }

static Phys<double> phys() {
  Phys<double> ph{};
  ph.a = 3.0 / 49.0; ph.b = 2.0 / 21.0; ph.R = 1.0; ph.G = -1.0;
  ph.Tc = 0.0778 * ph.a / (0.45724 * ph.b * ph.R);
  const double om = 0.344;
  ph.kpr = 0.37464 + 1.54226 * om - 0.26992 * om * om;
  ph.s_e = 1.25; ph.s_nu = 0.8; ph.s_q = 1.1; ph.s_pi = 0.9;
  ph.wbar = 0.75; ph.w0 = 0.25; ph.w1 = 0.125; ph.cs2T = 0.25;
  ph.vflux = 1.0 / (0.5 + (1.0 / 3.0) / 0.25); ph.vother = 1.2;
  ph.cv = 5.0; ph.kappa_w = 0.3; ph.rho_ref = 0.38; ph.T_ref = 0.094; ph.inv_b = 10.5;
  return ph;
}

// Central difference with one Richardson step: exact for cubic polynomials,
// O(h^4) otherwise.
template <typename F>
static double deriv(F&& J, double h) {
  const double d1 = (J(h) - J(-h)) / (2 * h);
  const double d2 = (J(h / 2) - J(-h / 2)) / h;
  return (4 * d2 - d1) / 3;
}

static double rel(double a, double b) { return std::fabs(a - b) / std::fmax(1e-300, std::fmax(std::fabs(a), std::fabs(b))); }

int main() {
  const Phys<double> ph = phys();
  double worst_lin = 0, worst_c19 = 0, worst_c7 = 0, worst_eos = 0, worst_zh = 0;
  for (int trial = 0; trial < 200; ++trial) {
    // linear maps: <a, P b> = <P^T a, b>
    double m[19], f[19], a[19], Pt[19], Mf[19], Mt[19];
    for (int k = 0; k < 19; ++k) { m[k] = uni(-1, 1); a[k] = uni(-1, 1); f[k] = uni(-1, 1); }
    double Pm[19];
    populations19(m, Pm);
    populations19_T(a, Pt);
    double l = 0, r = 0;
    for (int k = 0; k < 19; ++k) { l += a[k] * Pm[k]; r += Pt[k] * m[k]; }
    worst_lin = std::fmax(worst_lin, rel(l, r));
    moments19(f, Mf);
    moments19_T(a, Mt);
    l = r = 0;
    for (int k = 0; k < 19; ++k) { l += a[k] * Mf[k]; r += Mt[k] * f[k]; }
    worst_lin = std::fmax(worst_lin, rel(l, r));

    // collide19: J = <fsb, f*(f, rho, u, du)>
    const double rho = uni(0.3, 6.0);
    double u[3], du[3], fsb[19], df[19], dr = uni(-1, 1), duu[3], ddu[3];
    for (int c = 0; c < 3; ++c) { u[c] = uni(-0.1, 0.1); du[c] = uni(-0.05, 0.05); duu[c] = uni(-1, 1); ddu[c] = uni(-1, 1); }
    for (int k = 0; k < 19; ++k) { fsb[k] = uni(-1, 1); df[k] = uni(-1, 1); f[k] = uni(-0.1, 0.1); }
    auto J19 = [&](double h) {
      double ff[19];
      for (int k = 0; k < 19; ++k) ff[k] = f[k] + h * df[k];
      const double rr = rho + h * dr;
      collide19(ff, rr, rr - ph.rho_ref, u[0] + h * duu[0], u[1] + h * duu[1], u[2] + h * duu[2], du[0] + h * ddu[0],
                du[1] + h * ddu[1], du[2] + h * ddu[2], ph);
      double s = 0;
      for (int k = 0; k < 19; ++k) s += fsb[k] * ff[k];
      return s;
    };
    const double h = 1e-2;
    const double fd = deriv(J19, h);
    double fb[19], rb = 0, ub[3] = {0, 0, 0}, dub[3] = {0, 0, 0};
    collide19_adj(fsb, rho, u[0], u[1], u[2], du[0], du[1], du[2], ph, fb, rb, ub, dub);
    double ad = rb * dr;
    for (int k = 0; k < 19; ++k) ad += fb[k] * df[k];
    for (int c = 0; c < 3; ++c) ad += ub[c] * duu[c] + dub[c] * ddu[c];
    worst_c19 = std::fmax(worst_c19, rel(fd, ad));

    // collide7: J = <gsb, g*(g, Fbar)>
    double g[7], dg[7], gsb[7];
    const double Fbar = uni(-0.01, 0.01), dF = uni(-1, 1);
    for (int k = 0; k < 7; ++k) { g[k] = uni(-0.01, 0.01); dg[k] = uni(-1, 1); gsb[k] = uni(-1, 1); }
    auto J7 = [&](double hh) {
      double gg[7];
      for (int k = 0; k < 7; ++k) gg[k] = g[k] + hh * dg[k];
      collide7(gg, Fbar + hh * dF, ph.vflux, ph);
      double s = 0;
      for (int k = 0; k < 7; ++k) s += gsb[k] * gg[k];
      return s;
    };
    const double fd7 = deriv(J7, h);
    double gb[7], Fb;
    collide7_adj(gsb, ph, gb, Fb);
    double ad7 = Fb * dF;
    for (int k = 0; k < 7; ++k) ad7 += gb[k] * dg[k];
    worst_c7 = std::fmax(worst_c7, rel(fd7, ad7));

    // Peng-Robinson partials
    const double T = uni(0.8, 1.1) * ph.Tc;
    double dp_dr, dpdT, dpdT_dr, dpdT_dT;
    pr_partials(rho, T, ph, dp_dr, dpdT, dpdT_dr, dpdT_dT);
    const double e = 1e-3;
    // scale of each derivative: the size of its two terms, so that a
    // derivative that happens to cancel near zero is judged fairly
    const double sp = std::fabs(ph.R * T / ((1 - ph.b * rho) * (1 - ph.b * rho))) + 1.0;
    auto chk = [&](double ad, double fdv, double scale) {
      worst_eos = std::fmax(worst_eos, std::fabs(ad - fdv) / scale);
    };
    chk(dp_dr, deriv([&](double hh) { return pr_pressure(rho + hh * rho, T, ph); }, e) / rho, sp);
    chk(dpdT, deriv([&](double hh) { return pr_pressure(rho, T + hh * T, ph); }, e) / T, std::fabs(dpdT) + sp);
    chk(dpdT, pr_dpdT(rho, T, ph), std::fabs(dpdT));
    chk(dpdT_dr, deriv([&](double hh) { return pr_dpdT(rho + hh * rho, T, ph); }, e) / rho, sp / T);
    chk(dpdT_dT, deriv([&](double hh) { return pr_dpdT(rho, T + hh * T, ph); }, e) / T, std::fabs(dpdT) / T);

    // outlet fill on every face: linear in (f, F)
    for (int k = 0; k < 6; ++k) {
      double F[3], dFv[3], ob[19], dff[19];
      for (int c = 0; c < 3; ++c) { F[c] = uni(-0.01, 0.01); dFv[c] = uni(-1, 1); }
      for (int i = 0; i < 19; ++i) { f[i] = uni(-0.1, 0.1); dff[i] = uni(-1, 1); ob[i] = uni(-1, 1); }
      const double rout = uni(0.3, 1.0);
      auto JZ = [&](double hh) {
        double ff[19], FF[3];
        for (int i = 0; i < 19; ++i) ff[i] = f[i] + hh * dff[i];
        for (int c = 0; c < 3; ++c) FF[c] = F[c] + hh * dFv[c];
        outlet_fill(ff, k, rout, FF, ph);
        double s = 0;
        for (int i = 0; i < 19; ++i) s += ob[i] * ff[i];
        return s;
      };
      const double fdz = (JZ(1.0) - JZ(-1.0)) / 2.0;  // exact: the fill is affine
      double fbz[19], Fbz[3] = {0, 0, 0};
      for (int i = 0; i < 19; ++i) fbz[i] = ob[i];
      outlet_fill_adj(fbz, k, Fbz);
      double adz = 0;
      for (int i = 0; i < 19; ++i) adz += fbz[i] * dff[i];
      for (int c = 0; c < 3; ++c) adz += Fbz[c] * dFv[c];
      worst_zh = std::fmax(worst_zh, rel(fdz, adz));
    }
  }
  std::printf("linear_transposes %.3e\n", worst_lin);
  std::printf("collide19 %.3e\n", worst_c19);
  std::printf("collide7 %.3e\n", worst_c7);
  std::printf("peng_robinson %.3e\n", worst_eos);
  std::printf("outlet_fill %.3e\n", worst_zh);
  return 0;
}

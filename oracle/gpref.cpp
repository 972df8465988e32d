/*
 * gpref.cpp -- CPU FP64 ORACLE (test infrastructure only; see gpref.h).
 *
 * A plain, slow, step-by-step implementation of the split-step Crank-Nicolson method
 * for the 3D Gross-Pitaevskii equation (paper: program summary, "Solution method";
 * program summaries (i) and (ii)).  Everything is std::complex<double>; the only
 * parallelism is an OpenMP loop over independent lines or points.  It is written to be
 * checked by eye against the definitions below, not to be fast.
 *
 * Conventions where the paper prints no formula (each is a stated reading):
 *   grid      x_i = (i - (N-1)/2) dx, i = 0..N-1, ghosts psi_{-1} = psi_N = 0 (Dirichlet)
 *   potential V = 1/2 (nux^2 x^2 + nuy^2 y^2 + nuz^2 z^2)
 *   N-step    psi <- exp(-tau (V + g|psi|^2)) psi    (imaginary time, calcnu)
 *             psi <- exp(-i tau (V + g|psi|^2)) psi  (real time), |psi|^2 taken at the
 *             start of the sub-step
 *   sweep     Crank-Nicolson for dpsi/dt = (1/2) d2psi/da2 (imaginary) or
 *             (i/2) d2psi/da2 (real) with the 3-point second difference:
 *             -c u_{i-1} + (1+2c) u_i - c u_{i+1} = c p_{i-1} + (1-2c) p_i + c p_{i+1},
 *             c = tau/(4 da^2) (imaginary) or i tau/(4 da^2) (real)  (calclux/y/z)
 *             solved by the Thomas algorithm, forward elimination from i = 0.
 *   step      Lie: N(dt), x, y, z.  Strang: N(dt/2), x, y, z, N(dt/2).
 *   imaginary psi <- psi / sqrt(dV sum|psi|^2) after every step (renormalisation)
 *   sums      Riemann sums times dV = dx dy dz
 */
#include "gpref.h"

#include <cmath>
#include <complex>
#include <cstdlib>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef std::complex<double> cd;

struct gpref_ctx {
  gpref_params p;
  cd* psi;           /* caller-owned, [nx][ny][nz] */
  double npre;       /* last pre-renormalisation norm */
  std::vector<double> x, y, z;
};

static bool bad_params(const gpref_params* p) {
  if (!p) return true;
  if (p->nx < 3 || p->ny < 3 || p->nz < 3) return true;
  if (!(p->dx > 0) || !(p->dy > 0) || !(p->dz > 0) || !(p->dt > 0)) return true;
  if (!(p->nux >= 0) || !(p->nuy >= 0) || !(p->nuz >= 0)) return true;
  if (!std::isfinite(p->g) || !std::isfinite(p->dt)) return true;
  if (p->split != 0 && p->split != 1) return true;
  return false;
}

static inline int64_t idx(const gpref_params& p, int64_t i, int64_t j, int64_t k) {
  return (i * p.ny + j) * p.nz + k;   /* z stride 1, y stride nz, x stride ny*nz */
}

static void make_axis(std::vector<double>& a, int n, double d) {
  a.resize(n);
  for (int i = 0; i < n; ++i) a[i] = (i - 0.5 * (n - 1)) * d;
}

extern "C" int gpref_set_threads(int32_t nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  return 0;
}

extern "C" int gpref_init(const gpref_params* p, double* psi, gpref_ctx** out) {
  if (bad_params(p) || !psi || !out) return -1;
  gpref_ctx* c = new gpref_ctx;
  c->p = *p;
  c->psi = reinterpret_cast<cd*>(psi);
  c->npre = 1.0;
  make_axis(c->x, p->nx, p->dx);
  make_axis(c->y, p->ny, p->dy);
  make_axis(c->z, p->nz, p->dz);
  *out = c;
  return 0;
}

extern "C" int gpref_destroy(gpref_ctx* c) {
  delete c;
  return 0;
}

extern "C" int gpref_set_g(gpref_ctx* c, double g) {
  if (!c || !std::isfinite(g)) return -1;
  c->p.g = g;
  return 0;
}

/* Thomas solve of the constant-coefficient CN system on one line, in place. */
static void cn_solve(int n, cd cc, cd* line, cd* r, cd* cp, cd* dp) {
  /* right-hand side (I + (c) delta^2) p with zero ghosts */
  for (int i = 0; i < n; ++i) {
    cd left = (i > 0) ? line[i - 1] : cd(0.0, 0.0);
    cd right = (i < n - 1) ? line[i + 1] : cd(0.0, 0.0);
    r[i] = cc * left + (1.0 - 2.0 * cc) * line[i] + cc * right;
  }
  /* forward elimination on -c u_{i-1} + (1+2c) u_i - c u_{i+1} = r_i */
  cd diag = 1.0 + 2.0 * cc;
  cd gam = 1.0 / diag;
  cp[0] = -cc * gam;
  dp[0] = r[0] * gam;
  for (int i = 1; i < n; ++i) {
    gam = 1.0 / (diag + cc * cp[i - 1]);
    cp[i] = -cc * gam;
    dp[i] = (r[i] + cc * dp[i - 1]) * gam;
  }
  /* back substitution */
  line[n - 1] = dp[n - 1];
  for (int i = n - 2; i >= 0; --i) line[i] = dp[i] - cp[i] * line[i + 1];
}

extern "C" int gpref_cn_line(int32_t n, double c_re, double c_im, double* line) {
  if (n < 1 || !line) return -1;
  std::vector<cd> r(n), cp(n), dp(n);
  cn_solve(n, cd(c_re, c_im), reinterpret_cast<cd*>(line), r.data(), cp.data(), dp.data());
  return 0;
}

/* potential + nonlinear sub-step over time tau (calcnu) */
static void nstep(gpref_ctx* c, bool imag, double tau) {
  const gpref_params& p = c->p;
  const double hx = 0.5 * p.nux * p.nux, hy = 0.5 * p.nuy * p.nuy, hz = 0.5 * p.nuz * p.nuz;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < p.nx; ++i)
    for (int64_t j = 0; j < p.ny; ++j)
      for (int64_t k = 0; k < p.nz; ++k) {
        const double V = hx * c->x[i] * c->x[i] + hy * c->y[j] * c->y[j] + hz * c->z[k] * c->z[k];
        cd& v = c->psi[idx(p, i, j, k)];
        const double w = V + p.g * std::norm(v);
        if (imag)
          v *= std::exp(-tau * w);
        else
          v *= std::exp(cd(0.0, -tau * w));
      }
}

/* Crank-Nicolson sweep along one axis (calclux / calcluy / calcluz) */
static void sweep(gpref_ctx* c, int axis, bool imag, double tau) {
  const gpref_params& p = c->p;
  const int n = axis == 0 ? p.nx : axis == 1 ? p.ny : p.nz;
  const double d = axis == 0 ? p.dx : axis == 1 ? p.dy : p.dz;
  const cd cc = imag ? cd(tau / (4.0 * d * d), 0.0) : cd(0.0, tau / (4.0 * d * d));
  const int64_t stride = axis == 0 ? (int64_t)p.ny * p.nz : axis == 1 ? p.nz : 1;
  /* the two indices that label a line */
  const int64_t na = axis == 0 ? p.ny : p.nx;
  const int64_t nb = axis == 2 ? p.ny : p.nz;
#pragma omp parallel
  {
    std::vector<cd> line(n), r(n), cp(n), dp(n);
#pragma omp for schedule(static)
    for (int64_t ab = 0; ab < na * nb; ++ab) {
      const int64_t a = ab / nb, b = ab % nb;
      int64_t base;
      if (axis == 0) base = idx(p, 0, a, b);
      else if (axis == 1) base = idx(p, a, 0, b);
      else base = idx(p, a, b, 0);
      for (int i = 0; i < n; ++i) line[i] = c->psi[base + i * stride];
      cn_solve(n, cc, line.data(), r.data(), cp.data(), dp.data());
      for (int i = 0; i < n; ++i) c->psi[base + i * stride] = line[i];
    }
  }
}

extern "C" int gpref_substep(gpref_ctx* c, int32_t which, int32_t imag, double tau) {
  if (!c || which < 0 || which > 3 || !(tau > 0)) return -1;
  if (which == 0) nstep(c, imag != 0, tau);
  else sweep(c, which - 1, imag != 0, tau);
  return 0;
}

static double sum_norm(gpref_ctx* c) {
  const gpref_params& p = c->p;
  const int64_t n = (int64_t)p.nx * p.ny * p.nz;
  double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
  for (int64_t q = 0; q < n; ++q) s += std::norm(c->psi[q]);
  return s * p.dx * p.dy * p.dz;
}

static void one_step(gpref_ctx* c, bool imag) {
  const double dt = c->p.dt;
  if (c->p.split == 0) {
    nstep(c, imag, dt);
    for (int a = 0; a < 3; ++a) sweep(c, a, imag, dt);
  } else {
    nstep(c, imag, 0.5 * dt);
    for (int a = 0; a < 3; ++a) sweep(c, a, imag, dt);
    nstep(c, imag, 0.5 * dt);
  }
  if (imag) {
    const double nrm = sum_norm(c);
    c->npre = nrm;
    const double s = 1.0 / std::sqrt(nrm);
    const int64_t n = (int64_t)c->p.nx * c->p.ny * c->p.nz;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) c->psi[q] *= s;
  }
}

extern "C" int gpref_step_imag(gpref_ctx* c, int32_t n) {
  if (!c || n < 0) return -1;
  for (int32_t s = 0; s < n; ++s) one_step(c, true);
  return 0;
}

extern "C" int gpref_step_real(gpref_ctx* c, int32_t n) {
  if (!c || n < 0) return -1;
  for (int32_t s = 0; s < n; ++s) one_step(c, false);
  return 0;
}

extern "C" int gpref_last_npre(gpref_ctx* c, double* npre) {
  if (!c || !npre) return -1;
  *npre = c->npre;
  return 0;
}

extern "C" int gpref_norm(gpref_ctx* c, double* norm) {
  if (!c || !norm) return -1;
  *norm = sum_norm(c);
  return 0;
}

extern "C" int gpref_raw_sums(gpref_ctx* c, double raw[9]) {
  if (!c || !raw) return -1;
  const gpref_params& p = c->p;
  const double hx = 0.5 * p.nux * p.nux, hy = 0.5 * p.nuy * p.nuy, hz = 0.5 * p.nuz * p.nuz;
  double s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0, s6 = 0, s7 = 0, s8 = 0;
#pragma omp parallel for reduction(+ : s0, s1, s2, s3, s4, s5, s6, s7, s8) schedule(static)
  for (int64_t i = 0; i < p.nx; ++i)
    for (int64_t j = 0; j < p.ny; ++j)
      for (int64_t k = 0; k < p.nz; ++k) {
        const cd v = c->psi[idx(p, i, j, k)];
        const double n2 = std::norm(v);
        /* +1 link along each axis; the neighbour past the last point is the zero ghost */
        const cd vx = (i + 1 < p.nx) ? c->psi[idx(p, i + 1, j, k)] : cd(0, 0);
        const cd vy = (j + 1 < p.ny) ? c->psi[idx(p, i, j + 1, k)] : cd(0, 0);
        const cd vz = (k + 1 < p.nz) ? c->psi[idx(p, i, j, k + 1)] : cd(0, 0);
        double lx = std::norm(vx - v), ly = std::norm(vy - v), lz = std::norm(vz - v);
        /* the link from the zero ghost at index -1 to the first point */
        if (i == 0) lx += n2;
        if (j == 0) ly += n2;
        if (k == 0) lz += n2;
        const double V = hx * c->x[i] * c->x[i] + hy * c->y[j] * c->y[j] + hz * c->z[k] * c->z[k];
        s0 += n2;
        s1 += lx;
        s2 += ly;
        s3 += lz;
        s4 += V * n2;
        s5 += n2 * n2;
        s6 += c->x[i] * c->x[i] * n2;
        s7 += c->y[j] * c->y[j] * n2;
        s8 += c->z[k] * c->z[k] * n2;
      }
  const double dV = p.dx * p.dy * p.dz;
  s[0] = s0 * dV;
  s[1] = 0.5 * s1 * dV / (p.dx * p.dx);
  s[2] = 0.5 * s2 * dV / (p.dy * p.dy);
  s[3] = 0.5 * s3 * dV / (p.dz * p.dz);
  s[4] = s4 * dV;
  s[5] = s5 * dV;
  s[6] = s6 * dV;
  s[7] = s7 * dV;
  s[8] = s8 * dV;
  for (int q = 0; q < 9; ++q) raw[q] = s[q];
  return 0;
}

/* Energy and chemical potential of the normalised state phi = psi / sqrt(N):
 *   E  = (T + U)/N + (g/2) I/N^2,   mu = (T + U)/N + g I/N^2   (calcmuen) */
extern "C" int gpref_energy_mu(gpref_ctx* c, double* energy, double* mu) {
  if (!c || !energy || !mu) return -1;
  double r[9];
  gpref_raw_sums(c, r);
  const double N = r[0];
  const double T = r[1] + r[2] + r[3];
  const double lin = (T + r[4]) / N;
  const double nl = c->p.g * r[5] / (N * N);
  *energy = lin + 0.5 * nl;
  *mu = lin + nl;
  return 0;
}

/* root-mean-square sizes <a^2>^(1/2) of the normalised state (calcrms) */
extern "C" int gpref_rms(gpref_ctx* c, double rms[4]) {
  if (!c || !rms) return -1;
  double r[9];
  gpref_raw_sums(c, r);
  const double N = r[0];
  rms[0] = std::sqrt(r[6] / N);
  rms[1] = std::sqrt(r[7] / N);
  rms[2] = std::sqrt(r[8] / N);
  rms[3] = std::sqrt((r[6] + r[7] + r[8]) / N);
  return 0;
}

// Oracle: a plain, slow, FP64 CPU implementation of one projection time step
// of incompressible two-phase VOF flow with temperature-dependent surface
// tension (Zimbrod, Schreter, Schilp 2022, arXiv 2209.09671).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
// or calls this file; only the tests, the smoke check and the CPU baseline of
// the benchmark do.  It shares no code with the GPU path: the only common
// inputs are the parameter sheet and the seeded initial fields.
//
// Every function states the passage of the paper it follows.  Where the paper
// is silent the reading is stated in a comment marked "reading:"; the same
// readings are listed in the design notes of the repository.
//
// Build: g++ -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
// Loops are plain; OpenMP only splits independent cell/face loops, and every
// sum is taken in a fixed order, so results do not depend on thread count.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

// Plain parameter block; field order mirrored by oracle/pyoracle.py.
struct OrcConfig {
  int dim, nx, ny, nz;
  double h;
  int flags;  // 1: transport only; 2: periodic (with 1); 4: sigma*kappa := sigkap_const
  double rho1, rho2, mu1, mu2, rhocp1, rhocp2, lam1, lam2;  // phase 1: alpha=0, phase 2: alpha=1
  double sigma0, dsigma_dT, T0;
  int T_bc[6];        // -x,+x,-y,+y,-z,+z : 0 Neumann, 1 Dirichlet
  double T_wall[6];
  double q_power, q_radius, q_x0, q_y0, q_vx, q_vy;
  double weno_eps, normal_eps;
  double p_rtol;
  int p_maxit;
  int mg_nu;
  double mg_omega_c;
  int mg_coarse_sweeps;
  double sigkap_const;
  // solutal Marangoni (in-situ alloying, eq. 5): a species field c carried
  // like alpha, sigma = sigma0 + dsigma_dT (T - T0) + dsigma_dc (c - c0)
  int species;
  double dsigma_dc, c0;
  // time integrator: 0 = transport SSP-RK3 with frozen u^n, then one
  // forward-Euler predictor and one projection; 1 = SSP-RK3 over the whole
  // state with a projection in every stage
  int integrator;
  // N-phase VOF (eq. 1 for each phase j; several phases in one domain):
  // nphases 0 or 2 = the two-phase model above; 3 or 4 add phases 3 and 4
  // (fractions carried like alpha) with the material values below, and
  // surface tension per pair of phases, pairs ordered (1,2), (1,3), (1,4),
  // (2,3), (2,4), (3,4): sigma_ij = sig0_pair + dsig_pair (T - T0)
  int nphases;
  double rho34[2], mu34[2], rhocp34[2], lam34[2];
  double sig0_pair[6], dsig_pair[6];
};

struct OrcInfo {
  int cg_iters;
  int status;  // 0 ok, 3 not converged, 4 non-finite
  double p_relres, div_rel, sum_alpha, alpha_min, alpha_max, cfl_max;
};

}  // extern "C"

namespace {

constexpr int F_TRANSPORT_ONLY = 1, F_PERIODIC = 2, F_CONST_SIGKAP = 4;

// ---------------------------------------------------------------------------
// Grid and index maps.  Cell (i,j,k) has centre ((i+1/2)h, (j+1/2)h, (k+1/2)h).
// x-face i lies between cells i-1 and i (i = 0..nx; 0 and nx are walls).
struct Grid {
  const OrcConfig& c;
  int nx, ny, nz, dim;
  double h;
  bool per;
  const double* cf = nullptr;  // species field (read by the geometry when c.species)
  int nph;                                  // number of phases (2: the two-phase model)
  const double* ph3 = nullptr;              // fractions of phases 3 and 4 (N-phase model)
  const double* ph4 = nullptr;
  explicit Grid(const OrcConfig& cc)
      : c(cc), nx(cc.nx), ny(cc.ny), nz(cc.dim == 2 ? 1 : cc.nz), dim(cc.dim), h(cc.h),
        per((cc.flags & F_PERIODIC) != 0), nph(cc.nphases > 2 ? cc.nphases : 2) {}
  long N() const { return (long)nx * ny * nz; }
  long Nu() const { return (long)(nx + 1) * ny * nz; }
  long Nv() const { return (long)nx * (ny + 1) * nz; }
  long Nw() const { return dim == 3 ? (long)nx * ny * (nz + 1) : 0; }
  long cell(int i, int j, int k) const { return i + (long)nx * (j + (long)ny * k); }
  long fx(int i, int j, int k) const { return i + (long)(nx + 1) * (j + (long)ny * k); }
  long fy(int i, int j, int k) const { return i + (long)nx * (j + (long)(ny + 1) * k); }
  long fz(int i, int j, int k) const { return i + (long)nx * (j + (long)ny * k); }
  int n_of(int d) const { return d == 0 ? nx : (d == 1 ? ny : nz); }
};

// Even reflection of a cell index about the wall (ghost m outside = interior m).
inline int refl(int i, int n) {
  if (i < 0) return -1 - i;
  if (i >= n) return 2 * n - 1 - i;
  return i;
}
inline int wrapi(int i, int n) { return ((i % n) + n) % n; }

// ---------------------------------------------------------------------------
// Ghost-extended accessors (3 layers).
// reading: alpha is reflected evenly at walls (zero normal gradient).
double A(const Grid& g, const double* a, int i, int j, int k) {
  if (g.per) return a[g.cell(wrapi(i, g.nx), wrapi(j, g.ny), wrapi(k, g.nz))];
  return a[g.cell(refl(i, g.nx), refl(j, g.ny), g.dim == 3 ? refl(k, g.nz) : 0)];
}

// Temperature ghost: even reflection (Neumann) or T_ghost = 2 T_wall - T_mirror
// (Dirichlet).  Only ghosts outside a single wall are ever requested.
double Tg(const Grid& g, const double* t, int i, int j, int k) {
  if (g.per) return t[g.cell(wrapi(i, g.nx), wrapi(j, g.ny), wrapi(k, g.nz))];
  double v = t[g.cell(refl(i, g.nx), refl(j, g.ny), g.dim == 3 ? refl(k, g.nz) : 0)];
  const int idx[3] = {i, j, k};
  for (int d = 0; d < g.dim; ++d) {
    int n = g.n_of(d);
    int wall = -1;
    if (idx[d] < 0) wall = 2 * d;
    else if (idx[d] >= n) wall = 2 * d + 1;
    if (wall >= 0 && g.c.T_bc[wall] == 1) v = 2.0 * g.c.T_wall[wall] - v;
  }
  return v;
}

// Face velocity with ghosts.  Component d lives on d-faces; its face index
// along d runs 0..n_d (walls carry zero).  Beyond a wall it is odd-reflected
// about the wall face (normal direction) and odd-reflected about the wall for
// the tangential directions (no slip).
double Ucomp(const Grid& g, const double* u, int d, int i, int j, int k) {
  int id[3] = {i, j, k};
  double sgn = 1.0;
  for (int e = 0; e < g.dim; ++e) {
    int n = g.n_of(e);
    if (e == d) {
      if (g.per) {
        id[e] = wrapi(id[e], n);
      } else {
        if (id[e] < 0) { id[e] = -id[e]; sgn = -sgn; }
        else if (id[e] > n) { id[e] = 2 * n - id[e]; sgn = -sgn; }
      }
    } else {
      if (g.per) {
        id[e] = wrapi(id[e], n);
      } else {
        if (id[e] < 0) { id[e] = -1 - id[e]; sgn = -sgn; }
        else if (id[e] >= n) { id[e] = 2 * n - 1 - id[e]; sgn = -sgn; }
      }
    }
  }
  if (g.dim == 2) id[2] = 0;
  long ix;
  if (d == 0) ix = g.fx(id[0], id[1], id[2]);
  else if (d == 1) ix = g.fy(id[0], id[1], id[2]);
  else ix = g.fz(id[0], id[1], id[2]);
  return sgn * u[ix];
}

// ---------------------------------------------------------------------------
// Material laws (Table I / Table II give the phase values).
// reading: linear mixing in the clamped volume fraction.
inline double clamp01(double a) { return a < 0.0 ? 0.0 : (a > 1.0 ? 1.0 : a); }
inline double mix(double a, double p1, double p2) { return p1 + clamp01(a) * (p2 - p1); }

// N-phase model (reading: eq. 1 holds for every phase; the paper gives no
// mixture laws or pairwise surface tension for several phases).  Phase 1 is
// the background, alpha_1 = 1 - sum_{j>=2} alpha_j; phase 2 is alpha, phases
// 3 and 4 are carried like it.  A material law stays linear in each clamped
// fraction relative to phase 1, P = P_1 + sum_{j>=2} clamp(alpha_j) (P_j -
// P_1), which is mix() for two phases.
enum MatKind { MAT_RHO = 0, MAT_MU, MAT_RHOCP, MAT_LAM };
double A(const Grid& g, const double* a, int i, int j, int k);
double matp(const Grid& g, const double* a, int i, int j, int k, int which) {
  const OrcConfig& c = g.c;
  const double p1[4] = {c.rho1, c.mu1, c.rhocp1, c.lam1}, p2[4] = {c.rho2, c.mu2, c.rhocp2, c.lam2};
  const double* p34[4] = {c.rho34, c.mu34, c.rhocp34, c.lam34};
  double v = p1[which] + clamp01(A(g, a, i, j, k)) * (p2[which] - p1[which]);
  v += clamp01(A(g, g.ph3, i, j, k)) * (p34[which][0] - p1[which]);
  if (g.nph == 4) v += clamp01(A(g, g.ph4, i, j, k)) * (p34[which][1] - p1[which]);
  return v;
}
// fraction of phase q (1..4) at a cell, ghosts by even reflection
double phase(const Grid& g, const double* a, int q, int i, int j, int k) {
  if (q == 2) return A(g, a, i, j, k);
  if (q == 3) return A(g, g.ph3, i, j, k);
  if (q == 4) return A(g, g.ph4, i, j, k);
  double s = A(g, a, i, j, k) + A(g, g.ph3, i, j, k);
  if (g.nph == 4) s += A(g, g.ph4, i, j, k);
  return 1.0 - s;
}
// pairs (i, j), i < j, of an N-phase grid and their slots in the pair tables
int phase_pairs(int nph, int pi[6], int pj[6], int slot[6]) {
  const int I[6] = {1, 1, 1, 2, 2, 3}, J[6] = {2, 3, 4, 3, 4, 4};
  int n = 0;
  for (int q = 0; q < 6; ++q)
    if (J[q] <= nph) {
      pi[n] = I[q];
      pj[n] = J[q];
      slot[n] = q;
      ++n;
    }
  return n;
}

// ---------------------------------------------------------------------------
// WENO5-JS (Jiang & Shu 1996): value at the right edge of cell c from cell
// averages (a,b,c,d,e) = q_{c-2..c+2}.  The paper uses WENO reconstruction of
// the convective terms (Section "Implementation", Gaertner et al. library).
double weno5(double a, double b, double c, double d, double e, double eps) {
  double q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
  double q1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
  double q2 = (2.0 * c + 5.0 * d - e) / 6.0;
  double s0 = (13.0 / 12.0) * (a - 2.0 * b + c) * (a - 2.0 * b + c) +
              0.25 * (a - 4.0 * b + 3.0 * c) * (a - 4.0 * b + 3.0 * c);
  double s1 = (13.0 / 12.0) * (b - 2.0 * c + d) * (b - 2.0 * c + d) + 0.25 * (b - d) * (b - d);
  double s2 = (13.0 / 12.0) * (c - 2.0 * d + e) * (c - 2.0 * d + e) +
              0.25 * (3.0 * c - 4.0 * d + e) * (3.0 * c - 4.0 * d + e);
  double a0 = 0.1 / ((eps + s0) * (eps + s0));
  double a1 = 0.6 / ((eps + s1) * (eps + s1));
  double a2 = 0.3 / ((eps + s2) * (eps + s2));
  return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

// Upwind WENO5 value at the point between samples m-1 and m of a 1-D
// sequence q(.) (cell averages or staggered values).
// reading: a zero advecting velocity takes the left-biased branch.
template <class Q>
double upwind_weno(const Q& q, int m, double vel, double eps) {
  if (vel >= 0.0) return weno5(q(m - 3), q(m - 2), q(m - 1), q(m), q(m + 1), eps);
  return weno5(q(m + 2), q(m + 1), q(m), q(m - 1), q(m - 2), eps);
}

// ---------------------------------------------------------------------------
// Heat source.
// reading: Gaussian surface flux 2P/(pi r^2) exp(-2 rho^2/r^2) centred on a
// beam moving at (q_vx, q_vy), applied volumetrically as Q * delta_s.
double heat_flux(const OrcConfig& c, double x, double y, double t) {
  if (c.q_power == 0.0) return 0.0;
  double xl = c.q_x0 + c.q_vx * t, yl = c.q_y0 + c.q_vy * t;
  double r2 = (x - xl) * (x - xl) + (y - yl) * (y - yl);
  double R2 = c.q_radius * c.q_radius;
  return 2.0 * c.q_power / (M_PI * R2) * std::exp(-2.0 * r2 / R2);
}

// Regularised gradient norm (eqs. 6-7).
// reading: |g|_eps = sqrt(|g|^2 + eps_n^2), n = g/|g|_eps,
// delta_s = |g|_eps - eps_n written as |g|^2/(|g|_eps + eps_n).
void grad_alpha(const Grid& g, const double* a, int i, int j, int k, double gr[3]) {
  double ih2 = 1.0 / (2.0 * g.h);
  gr[0] = (A(g, a, i + 1, j, k) - A(g, a, i - 1, j, k)) * ih2;
  gr[1] = (A(g, a, i, j + 1, k) - A(g, a, i, j - 1, k)) * ih2;
  gr[2] = g.dim == 3 ? (A(g, a, i, j, k + 1) - A(g, a, i, j, k - 1)) * ih2 : 0.0;
}
double delta_s_of(const double gr[3], double eps_n) {
  double g2 = gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2];
  double ge = std::sqrt(g2 + eps_n * eps_n);
  return g2 / (ge + eps_n);
}

// ---------------------------------------------------------------------------
// S1 right-hand sides: La = -div(u alpha) (eq. 1) and
// LT = -div(u T) + [div(lambda grad T) + Q delta_s] / (rho c_p).
// reading: the energy equation is not written out in the paper; this is its
// standard conservative form with an explicit conduction term.
void transport_rhs(const Grid& g, double t, const double* a, const double* T, const double* u,
                   const double* v, const double* w, double* La, double* LT) {
  const OrcConfig& c = g.c;
  const double h = g.h, eps = c.weno_eps;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  std::vector<double> Fa[3], Ft[3];
  const double* vel[3] = {u, v, w};
  for (int d = 0; d < g.dim; ++d) {
    long nf = d == 0 ? g.Nu() : (d == 1 ? g.Nv() : g.Nw());
    Fa[d].assign(nf, 0.0);
    Ft[d].assign(nf, 0.0);
    int fnx = nx + (d == 0), fny = ny + (d == 1), fnz = nz + (d == 2);
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < fnz; ++k)
      for (int j = 0; j < fny; ++j)
        for (int i = 0; i < fnx; ++i) {
          long fi = (long)i + (long)fnx * (j + (long)fny * k);
          int m = d == 0 ? i : (d == 1 ? j : k);
          int n = g.n_of(d);
          if (!g.per && (m == 0 || m == n)) continue;  // wall: zero flux
          if (g.per && m == n) continue;               // duplicate of face 0
          double uf = vel[d][fi];
          auto qa = [&](int mm) {
            return d == 0 ? A(g, a, mm, j, k) : (d == 1 ? A(g, a, i, mm, k) : A(g, a, i, j, mm));
          };
          auto qt = [&](int mm) {
            return d == 0 ? Tg(g, T, mm, j, k) : (d == 1 ? Tg(g, T, i, mm, k) : Tg(g, T, i, j, mm));
          };
          Fa[d][fi] = uf * upwind_weno(qa, m, uf, eps);
          Ft[d][fi] = uf * upwind_weno(qt, m, uf, eps);
        }
    if (g.per) {  // face n carries the same flux as face 0
      for (int k = 0; k < fnz; ++k)
        for (int j = 0; j < fny; ++j)
          for (int i = 0; i < fnx; ++i) {
            int m = d == 0 ? i : (d == 1 ? j : k);
            if (m != g.n_of(d)) continue;
            long fi = (long)i + (long)fnx * (j + (long)fny * k);
            int i0 = d == 0 ? 0 : i, j0 = d == 1 ? 0 : j, k0 = d == 2 ? 0 : k;
            long f0 = (long)i0 + (long)fnx * (j0 + (long)fny * k0);
            Fa[d][fi] = Fa[d][f0];
            Ft[d][fi] = Ft[d][f0];
          }
    }
  }
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        long ci = g.cell(i, j, k);
        double diva = (Fa[0][g.fx(i + 1, j, k)] - Fa[0][g.fx(i, j, k)]) +
                      (Fa[1][g.fy(i, j + 1, k)] - Fa[1][g.fy(i, j, k)]);
        double divt = (Ft[0][g.fx(i + 1, j, k)] - Ft[0][g.fx(i, j, k)]) +
                      (Ft[1][g.fy(i, j + 1, k)] - Ft[1][g.fy(i, j, k)]);
        if (g.dim == 3) {
          diva += Fa[2][g.fz(i, j, k + 1)] - Fa[2][g.fz(i, j, k)];
          divt += Ft[2][g.fz(i, j, k + 1)] - Ft[2][g.fz(i, j, k)];
        }
        La[ci] = -diva / h;
        // conduction: sum over the cell's faces of lambda_f (T_nb - T_c) / h^2,
        // lambda_f the arithmetic mean of the two cells' conductivities.
        double Tc = T[ci];
        const bool np = g.nph > 2;
        double lc = np ? matp(g, a, i, j, k, MAT_LAM) : mix(a[ci], c.lam1, c.lam2);
        double cond = 0.0;
        const int off[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        for (int d = 0; d < g.dim; ++d)
          for (int sgn = -1; sgn <= 1; sgn += 2) {
            int ii = i + sgn * off[d][0], jj = j + sgn * off[d][1], kk = k + sgn * off[d][2];
            double lf = 0.5 * (lc + (np ? matp(g, a, ii, jj, kk, MAT_LAM) : mix(A(g, a, ii, jj, kk), c.lam1, c.lam2)));
            cond += lf * (Tg(g, T, ii, jj, kk) - Tc);
          }
        cond /= h * h;
        double src = 0.0;
        if (c.q_power != 0.0) {
          double gr[3];
          if (np) {
            // N phases: the flux heats the boundary of the condensed phases,
            // the gradient of alpha_c = 1 - alpha_1 (alpha for two phases)
            auto ac = [&](int ii, int jj, int kk) { return 1.0 - phase(g, a, 1, ii, jj, kk); };
            const double ih2 = 1.0 / (2.0 * g.h);
            gr[0] = (ac(i + 1, j, k) - ac(i - 1, j, k)) * ih2;
            gr[1] = (ac(i, j + 1, k) - ac(i, j - 1, k)) * ih2;
            gr[2] = g.dim == 3 ? (ac(i, j, k + 1) - ac(i, j, k - 1)) * ih2 : 0.0;
          } else {
            grad_alpha(g, a, i, j, k, gr);
          }
          src = heat_flux(c, (i + 0.5) * h, (j + 0.5) * h, t) * delta_s_of(gr, c.normal_eps);
        }
        LT[ci] = -divt / h + (cond + src) / (np ? matp(g, a, i, j, k, MAT_RHOCP) : mix(a[ci], c.rhocp1, c.rhocp2));
      }
}

// Species right-hand side Lc = -div(u c): the same WENO5 upwind flux as alpha
// (eq. 1 with c in place of alpha), with even ghosts (no flux through walls).
// reading: the species is carried without diffusion.
void advect_rhs(const Grid& g, const double* q, const double* u, const double* v, const double* w, double* Lq) {
  const double h = g.h, eps = g.c.weno_eps;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  std::vector<double> F[3];
  const double* vel[3] = {u, v, w};
  for (int d = 0; d < g.dim; ++d) {
    long nf = d == 0 ? g.Nu() : (d == 1 ? g.Nv() : g.Nw());
    F[d].assign(nf, 0.0);
    int fnx = nx + (d == 0), fny = ny + (d == 1), fnz = nz + (d == 2);
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < fnz; ++k)
      for (int j = 0; j < fny; ++j)
        for (int i = 0; i < fnx; ++i) {
          long fi = (long)i + (long)fnx * (j + (long)fny * k);
          int m = d == 0 ? i : (d == 1 ? j : k);
          if (m == 0 || m == g.n_of(d)) continue;  // wall: zero flux
          double uf = vel[d][fi];
          auto qq = [&](int mm) {
            return d == 0 ? A(g, q, mm, j, k) : (d == 1 ? A(g, q, i, mm, k) : A(g, q, i, j, mm));
          };
          F[d][fi] = uf * upwind_weno(qq, m, uf, eps);
        }
  }
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double div = (F[0][g.fx(i + 1, j, k)] - F[0][g.fx(i, j, k)]) + (F[1][g.fy(i, j + 1, k)] - F[1][g.fy(i, j, k)]);
        if (g.dim == 3) div += F[2][g.fz(i, j, k + 1)] - F[2][g.fz(i, j, k)];
        Lq[g.cell(i, j, k)] = -div / h;
      }
}

// S1: SSP-RK3 (Shu-Osher) for alpha and T (and the species c, when given)
// with the face velocity frozen.
// reading: the paper does not state its time integrator.
// Shu-Osher SSP-RK3 combination of stage s (0, 1, 2) from the base value q^n
// and the forward-Euler update x = q^(s) + dt L(q^(s)), written exactly as
// the two-phase stages below so that the variants agree where they must.
inline double rk_stage(int s, double base, double x) {
  return s == 0 ? x : (s == 1 ? 0.75 * base + 0.25 * x : base / 3.0 + 2.0 / 3.0 * x);
}

// N-phase transport: the same three stages for alpha, T and the fractions of
// phases 3 (and 4); each stage's T right-hand side takes its materials from
// that stage's fractions.
void transport_rk3_nphase(const Grid& g, double t, double dt, std::vector<double>& a, std::vector<double>& T,
                          std::vector<double>& p3, std::vector<double>* p4, const double* u, const double* v,
                          const double* w) {
  const long N = g.N();
  const std::vector<double> an(a), Tn(T), p3n(p3), p4n = p4 ? *p4 : std::vector<double>();
  std::vector<double> as(a), Ts(T), q3(p3), q4 = p4n, La(N), LT(N), L3(N), L4(p4 ? N : 0);
  Grid gs = g;
  for (int s = 0; s < 3; ++s) {
    gs.ph3 = q3.data();
    gs.ph4 = p4 ? q4.data() : nullptr;
    transport_rhs(gs, t, as.data(), Ts.data(), u, v, w, La.data(), LT.data());
    advect_rhs(g, q3.data(), u, v, w, L3.data());
    if (p4) advect_rhs(g, q4.data(), u, v, w, L4.data());
    for (long q = 0; q < N; ++q) {
      as[q] = rk_stage(s, an[q], as[q] + dt * La[q]);
      Ts[q] = rk_stage(s, Tn[q], Ts[q] + dt * LT[q]);
      q3[q] = rk_stage(s, p3n[q], q3[q] + dt * L3[q]);
      if (p4) q4[q] = rk_stage(s, p4n[q], q4[q] + dt * L4[q]);
    }
  }
  a = as;
  T = Ts;
  p3 = q3;
  if (p4) *p4 = q4;
}

void transport_rk3(const Grid& g, double t, double dt, std::vector<double>& a, std::vector<double>& T,
                   const double* u, const double* v, const double* w, std::vector<double>* cs = nullptr) {
  long N = g.N();
  if (cs) {  // the species: the same three stages with its own right-hand side
    std::vector<double>& c = *cs;
    std::vector<double> Lc(N), c1(N), c2(N);
    advect_rhs(g, c.data(), u, v, w, Lc.data());
    for (long q = 0; q < N; ++q) c1[q] = c[q] + dt * Lc[q];
    advect_rhs(g, c1.data(), u, v, w, Lc.data());
    for (long q = 0; q < N; ++q) c2[q] = 0.75 * c[q] + 0.25 * (c1[q] + dt * Lc[q]);
    advect_rhs(g, c2.data(), u, v, w, Lc.data());
    for (long q = 0; q < N; ++q) c[q] = c[q] / 3.0 + 2.0 / 3.0 * (c2[q] + dt * Lc[q]);
  }
  std::vector<double> La(N), LT(N), a1(N), T1(N), a2(N), T2(N);
  transport_rhs(g, t, a.data(), T.data(), u, v, w, La.data(), LT.data());
  for (long c = 0; c < N; ++c) {
    a1[c] = a[c] + dt * La[c];
    T1[c] = T[c] + dt * LT[c];
  }
  transport_rhs(g, t, a1.data(), T1.data(), u, v, w, La.data(), LT.data());
  for (long c = 0; c < N; ++c) {
    a2[c] = 0.75 * a[c] + 0.25 * (a1[c] + dt * La[c]);
    T2[c] = 0.75 * T[c] + 0.25 * (T1[c] + dt * LT[c]);
  }
  transport_rhs(g, t, a2.data(), T2.data(), u, v, w, La.data(), LT.data());
  for (long c = 0; c < N; ++c) {
    a[c] = a[c] / 3.0 + 2.0 / 3.0 * (a2[c] + dt * La[c]);
    T[c] = T[c] / 3.0 + 2.0 / 3.0 * (T2[c] + dt * LT[c]);
  }
}

// ---------------------------------------------------------------------------
// S2-S3: interface geometry on interior cells (eqs. 4, 6, 7 and the
// surface-tension field of Section "Implementation").
// Outputs: n (3N), kappa, delta_s, sigma*kappa, Marangoni vector M (3N).
// reading: kappa = -div(n) by central differences of cell-centre normals;
// M = delta_s (grad sigma - n (n . grad sigma)), the tangential part of the
// surface-tension gradient; sigma = sigma0 + dsigma_dT (T - T0), plus
// dsigma_dc (c - c0) with a species field, whose gradient enters grad sigma
// by the chain rule of eq. 5 (central differences, even ghosts).
void geometry(const Grid& g, const double* a, const double* T, double* nout, double* kap,
              double* ds, double* sk, double* M) {
  const OrcConfig& c = g.c;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int ex = nx + 2, ey = ny + 2, ez = g.dim == 3 ? nz + 2 : 1;
  const int oz = g.dim == 3 ? 1 : 0;
  std::vector<double> nn(3L * ex * ey * ez);
  auto eidx = [&](int i, int j, int k) { return (long)(i + 1) + (long)ex * ((j + 1) + (long)ey * (k + oz)); };
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = -oz; k < nz + oz; ++k)
    for (int j = -1; j < ny + 1; ++j)
      for (int i = -1; i < nx + 1; ++i) {
        double gr[3];
        grad_alpha(g, a, i, j, k, gr);
        double ge = std::sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2] + c.normal_eps * c.normal_eps);
        long e = eidx(i, j, k);
        for (int d = 0; d < 3; ++d) nn[3 * e + d] = gr[d] / ge;
      }
  const double ih2 = 1.0 / (2.0 * g.h);
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        long ci = g.cell(i, j, k);
        double divn = (nn[3 * eidx(i + 1, j, k) + 0] - nn[3 * eidx(i - 1, j, k) + 0]) * ih2 +
                      (nn[3 * eidx(i, j + 1, k) + 1] - nn[3 * eidx(i, j - 1, k) + 1]) * ih2;
        if (g.dim == 3) divn += (nn[3 * eidx(i, j, k + 1) + 2] - nn[3 * eidx(i, j, k - 1) + 2]) * ih2;
        double kappa = -divn;
        double gr[3];
        grad_alpha(g, a, i, j, k, gr);
        double dls = delta_s_of(gr, c.normal_eps);
        double sigma = c.sigma0 + c.dsigma_dT * (T[ci] - c.T0);
        double gs[3];
        gs[0] = c.dsigma_dT * (Tg(g, T, i + 1, j, k) - Tg(g, T, i - 1, j, k)) * ih2;
        gs[1] = c.dsigma_dT * (Tg(g, T, i, j + 1, k) - Tg(g, T, i, j - 1, k)) * ih2;
        gs[2] = g.dim == 3 ? c.dsigma_dT * (Tg(g, T, i, j, k + 1) - Tg(g, T, i, j, k - 1)) * ih2 : 0.0;
        if (c.species && g.cf) {
          const double* q = g.cf;
          sigma += c.dsigma_dc * (q[ci] - c.c0);
          gs[0] += c.dsigma_dc * (A(g, q, i + 1, j, k) - A(g, q, i - 1, j, k)) * ih2;
          gs[1] += c.dsigma_dc * (A(g, q, i, j + 1, k) - A(g, q, i, j - 1, k)) * ih2;
          if (g.dim == 3) gs[2] += c.dsigma_dc * (A(g, q, i, j, k + 1) - A(g, q, i, j, k - 1)) * ih2;
        }
        const double* n = &nn[3 * eidx(i, j, k)];
        double ndg = n[0] * gs[0] + n[1] * gs[1] + n[2] * gs[2];
        for (int d = 0; d < 3; ++d) {
          if (nout) nout[3 * ci + d] = n[d];
          M[3 * ci + d] = dls * (gs[d] - n[d] * ndg);
        }
        kap[ci] = kappa;
        ds[ci] = dls;
        sk[ci] = (c.flags & F_CONST_SIGKAP) ? c.sigkap_const : sigma * kappa;
      }
}

// N-phase interface geometry (reading; eqs. 4-7 applied to each pair of
// phases).  For a pair i < j the pair gradient g_ij = alpha_i grad alpha_j -
// alpha_j grad alpha_i points into phase j (for two phases g_12 = grad
// alpha); n_ij = g_ij / |g_ij|_eps, delta_ij and kappa_ij = -div n_ij as in
// geometry(); sigma_ij = sig0_pair + dsig_pair (T - T0) and M_ij = delta_ij
// (grad sigma_ij - n_ij (n_ij . grad sigma_ij)).  Outputs per pair p (in the
// order of phase_pairs): sigma_ij kappa_ij (skp[p N + c]) and delta_ij
// (dsp[p N + c]), and the Marangoni vector summed over the pairs (M, 3N).
void geometry_n(const Grid& g, const double* a, const double* T, double* skp, double* dsp, double* M) {
  const OrcConfig& c = g.c;
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const long N = g.N();
  const int ex = nx + 2, ey = ny + 2, ez = g.dim == 3 ? nz + 2 : 1;
  const int oz = g.dim == 3 ? 1 : 0;
  const double ih2 = 1.0 / (2.0 * g.h);
  int pi[6], pj[6], slot[6];
  const int np = phase_pairs(g.nph, pi, pj, slot);
  auto eidx = [&](int i, int j, int k) { return (long)(i + 1) + (long)ex * ((j + 1) + (long)ey * (k + oz)); };
  for (long q = 0; q < 3 * N; ++q) M[q] = 0.0;
  std::vector<double> nn(3L * ex * ey * ez);
  for (int p = 0; p < np; ++p) {
    const int I = pi[p], J = pj[p];
    auto pg = [&](int i, int j, int k, double gr[3]) {  // g_IJ at a cell of the ghost ring or inside
      const double ai = phase(g, a, I, i, j, k), aj = phase(g, a, J, i, j, k);
      auto d = [&](int q, int di, int dj, int dk) {
        return (phase(g, a, q, i + di, j + dj, k + dk) - phase(g, a, q, i - di, j - dj, k - dk)) * ih2;
      };
      gr[0] = ai * d(J, 1, 0, 0) - aj * d(I, 1, 0, 0);
      gr[1] = ai * d(J, 0, 1, 0) - aj * d(I, 0, 1, 0);
      gr[2] = g.dim == 3 ? ai * d(J, 0, 0, 1) - aj * d(I, 0, 0, 1) : 0.0;
    };
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = -oz; k < nz + oz; ++k)
      for (int j = -1; j < ny + 1; ++j)
        for (int i = -1; i < nx + 1; ++i) {
          double gr[3];
          pg(i, j, k, gr);
          double ge = std::sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2] + c.normal_eps * c.normal_eps);
          long e = eidx(i, j, k);
          for (int d = 0; d < 3; ++d) nn[3 * e + d] = gr[d] / ge;
        }
    const double s0 = c.sig0_pair[slot[p]], sT = c.dsig_pair[slot[p]];
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          long ci = g.cell(i, j, k);
          double divn = (nn[3 * eidx(i + 1, j, k) + 0] - nn[3 * eidx(i - 1, j, k) + 0]) * ih2 +
                        (nn[3 * eidx(i, j + 1, k) + 1] - nn[3 * eidx(i, j - 1, k) + 1]) * ih2;
          if (g.dim == 3) divn += (nn[3 * eidx(i, j, k + 1) + 2] - nn[3 * eidx(i, j, k - 1) + 2]) * ih2;
          double gr[3];
          pg(i, j, k, gr);
          double dls = delta_s_of(gr, c.normal_eps);
          double sigma = s0 + sT * (T[ci] - c.T0);
          double gs[3];
          gs[0] = sT * (Tg(g, T, i + 1, j, k) - Tg(g, T, i - 1, j, k)) * ih2;
          gs[1] = sT * (Tg(g, T, i, j + 1, k) - Tg(g, T, i, j - 1, k)) * ih2;
          gs[2] = g.dim == 3 ? sT * (Tg(g, T, i, j, k + 1) - Tg(g, T, i, j, k - 1)) * ih2 : 0.0;
          const double* n = &nn[3 * eidx(i, j, k)];
          double ndg = n[0] * gs[0] + n[1] * gs[1] + n[2] * gs[2];
          for (int d = 0; d < 3; ++d) M[3 * ci + d] += dls * (gs[d] - n[d] * ndg);
          skp[p * N + ci] = sigma * -divn;
          if (dsp) dsp[p * N + ci] = dls;
        }
  }
}

// N-phase face force along d between cells L and R (reading): the pair
// forces sigma_ij kappa_ij g_ij with the face form of the pair gradient,
// G_ij = avg(alpha_i) (alpha_j,R - alpha_j,L)/h - avg(alpha_j) (alpha_i,R -
// alpha_i,L)/h (which is (alpha_R - alpha_L)/h for two phases, the
// balanced-force face gradient), plus the face average of the Marangoni
// vector.
double face_force_n(const Grid& g, const double* a, const double* skp, const double* M, int d, int i, int j,
                    int k) {
  int L[3] = {i, j, k};
  L[d] -= 1;
  const long cL = g.cell(L[0], L[1], L[2]), cR = g.cell(i, j, k);
  const long N = g.N();
  int pi[6], pj[6], slot[6];
  const int np = phase_pairs(g.nph, pi, pj, slot);
  double f = 0.5 * (M[3 * cL + d] + M[3 * cR + d]);
  for (int p = 0; p < np; ++p) {
    const double iL = phase(g, a, pi[p], L[0], L[1], L[2]), iR = phase(g, a, pi[p], i, j, k);
    const double jL = phase(g, a, pj[p], L[0], L[1], L[2]), jR = phase(g, a, pj[p], i, j, k);
    const double G = (0.5 * (iL + iR) * (jR - jL) - 0.5 * (jL + jR) * (iR - iL)) / g.h;
    f += 0.5 * (skp[p * N + cL] + skp[p * N + cR]) * G;
  }
  return f;
}

// ---------------------------------------------------------------------------
// S4-S5: momentum predictor on interior faces.
//   u* = u + dt [ -C(u) + (V(u) + f_st) / rho_f ]
// C: conservative convection with WENO5-reconstructed advected velocity and
// averaged advecting velocity; V: divergence of mu (grad u + grad u^T);
// f_st: face CSF force (eq. 4).
// reading: balanced-force face force
//   f = 1/2 (sk_L + sk_R) (alpha_R - alpha_L)/h + 1/2 (M_L + M_R),
// mu on edges = mean of the four surrounding cells, rho_f = mean of two cells.
void predictor(const Grid& g, double dt, const double* a, const double* T, const double* u,
               const double* v, const double* w, double* us, double* vs, double* ws) {
  const OrcConfig& c = g.c;
  const int nx = g.nx, ny = g.ny, nz = g.nz, dim = g.dim;
  const double h = g.h, eps = c.weno_eps;
  long N = g.N();
  const bool nphase = g.nph > 2;
  std::vector<double> kap(N), ds(N), sk(N), M(3 * N), skp;
  if (nphase) {
    skp.assign(6 * N, 0.0);
    geometry_n(g, a, T, skp.data(), nullptr, M.data());
  } else {
    geometry(g, a, T, nullptr, kap.data(), ds.data(), sk.data(), M.data());
  }
  const double* vel[3] = {u, v, w};
  double* out[3] = {us, vs, ws};
  auto mu = [&](int i, int j, int k) {
    return nphase ? matp(g, a, i, j, k, MAT_MU) : mix(A(g, a, i, j, k), c.mu1, c.mu2);
  };
  auto rho = [&](int i, int j, int k) {
    return nphase ? matp(g, a, i, j, k, MAT_RHO) : mix(a[g.cell(i, j, k)], c.rho1, c.rho2);
  };
  for (int d = 0; d < dim; ++d) {
    int fnx = nx + (d == 0), fny = ny + (d == 1), fnz = nz + (d == 2);
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < fnz; ++k)
      for (int j = 0; j < fny; ++j)
        for (int i = 0; i < fnx; ++i) {
          long fi = (long)i + (long)fnx * (j + (long)fny * k);
          int id[3] = {i, j, k};
          int m = id[d];
          if (m == 0 || m == g.n_of(d)) { out[d][fi] = 0.0; continue; }
          // cells on the low (L) and high (R) side of this face
          int L[3] = {i, j, k};
          L[d] -= 1;
          long cL = g.cell(L[0], L[1], L[2]), cR = g.cell(i, j, k);
          // ud(o): this velocity component at the face offset by o (face index units)
          auto ud = [&](int oi, int oj, int ok) { return Ucomp(g, vel[d], d, i + oi, j + oj, k + ok); };
          double conv = 0.0, visc = 0.0;
          for (int e = 0; e < dim; ++e) {
            int oe[3] = {0, 0, 0};
            oe[e] = 1;
            if (e == d) {
              // flux at the two cell centres adjacent to the face along d
              double Fhi, Flo, Thi, Tlo;
              for (int side = 0; side < 2; ++side) {
                // cell centre between faces (m-1+side) and (m+side)
                int s0 = side - 1;  // offset of the lower face of that cell
                double Ub = 0.5 * (ud(s0 * oe[0], s0 * oe[1], s0 * oe[2]) +
                                   ud((s0 + 1) * oe[0], (s0 + 1) * oe[1], (s0 + 1) * oe[2]));
                auto q = [&](int mm) {  // mm: face index relative to this face
                  return ud(mm * oe[0], mm * oe[1], mm * oe[2]);
                };
                // point between faces s0 and s0+1 -> sample index "m" = s0+1
                double Uh = upwind_weno(q, s0 + 1, Ub, eps);
                int cc[3] = {i, j, k};
                cc[d] += s0;  // cell index of that centre
                double tau = 2.0 * mu(cc[0], cc[1], cc[2]) *
                             (ud((s0 + 1) * oe[0], (s0 + 1) * oe[1], (s0 + 1) * oe[2]) -
                              ud(s0 * oe[0], s0 * oe[1], s0 * oe[2])) / h;
                if (side == 1) { Fhi = Ub * Uh; Thi = tau; }
                else { Flo = Ub * Uh; Tlo = tau; }
              }
              conv += (Fhi - Flo) / h;
              visc += (Thi - Tlo) / h;
            } else {
              // edges at e-face positions (id[e]) and (id[e]+1) of this face's column
              double Fhi, Flo, Thi, Tlo;
              for (int side = 0; side < 2; ++side) {
                int ef = id[e] + side;  // e-face index of the edge
                // advecting velocity: component e at e-face ef, averaged over the
                // two cells L and R of this d-face
                int pL[3] = {L[0], L[1], L[2]}, pR[3] = {i, j, k};
                pL[e] = ef;
                pR[e] = ef;
                double Vb = 0.5 * (Ucomp(g, vel[e], e, pL[0], pL[1], pL[2]) +
                                   Ucomp(g, vel[e], e, pR[0], pR[1], pR[2]));
                // advected: component d along e, samples at cell index id[e]+mm
                auto q = [&](int mm) {
                  int o[3] = {0, 0, 0};
                  o[e] = mm - id[e];
                  return ud(o[0], o[1], o[2]);
                };
                double Uh = upwind_weno(q, ef, Vb, eps);
                // shear stress on the edge
                int o0[3] = {0, 0, 0}, o1[3] = {0, 0, 0};
                o0[e] = ef - 1 - id[e];
                o1[e] = ef - id[e];
                double dud = (ud(o1[0], o1[1], o1[2]) - ud(o0[0], o0[1], o0[2])) / h;
                double dve = (Ucomp(g, vel[e], e, pR[0], pR[1], pR[2]) -
                              Ucomp(g, vel[e], e, pL[0], pL[1], pL[2])) / h;
                // four cells around the edge: {L,R} x {ef-1, ef} along e
                int c1[3] = {L[0], L[1], L[2]}, c2[3] = {i, j, k};
                c1[e] = ef - 1;
                c2[e] = ef - 1;
                int c3[3] = {L[0], L[1], L[2]}, c4[3] = {i, j, k};
                c3[e] = ef;
                c4[e] = ef;
                double me = 0.25 * (mu(c1[0], c1[1], c1[2]) + mu(c2[0], c2[1], c2[2]) +
                                    mu(c3[0], c3[1], c3[2]) + mu(c4[0], c4[1], c4[2]));
                double tau = me * (dud + dve);
                if (side == 1) { Fhi = Vb * Uh; Thi = tau; }
                else { Flo = Vb * Uh; Tlo = tau; }
              }
              conv += (Fhi - Flo) / h;
              visc += (Thi - Tlo) / h;
            }
          }
          double fst = nphase ? face_force_n(g, a, skp.data(), M.data(), d, i, j, k)
                              : 0.5 * (sk[cL] + sk[cR]) * (a[cR] - a[cL]) / h + 0.5 * (M[3 * cL + d] + M[3 * cR + d]);
          double rhof = 0.5 * (rho(L[0], L[1], L[2]) + rho(i, j, k));
          out[d][fi] = vel[d][fi] + dt * (-conv + (visc + fst) / rhof);
        }
  }
}

// (D u)_c = (1/h) sum_d (u_{d,+} - u_{d,-})
void divergence(const Grid& g, const double* u, const double* v, const double* w, double* out) {
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < g.nz; ++k)
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i) {
        double s = (u[g.fx(i + 1, j, k)] - u[g.fx(i, j, k)]) + (v[g.fy(i, j + 1, k)] - v[g.fy(i, j, k)]);
        if (g.dim == 3) s += w[g.fz(i, j, k + 1)] - w[g.fz(i, j, k)];
        out[g.cell(i, j, k)] = s / g.h;
      }
}

// ---------------------------------------------------------------------------
// Fixed-order FP64 reductions (chunked, deterministic).
double dot(const double* x, const double* y, long n) {
  const long CH = 4096;
  long nch = (n + CH - 1) / CH;
  std::vector<double> part(nch, 0.0);
#pragma omp parallel for schedule(static)
  for (long b = 0; b < nch; ++b) {
    double s = 0.0;
    for (long i = b * CH; i < std::min(n, (b + 1) * CH); ++i) s += x[i] * y[i];
    part[b] = s;
  }
  double s = 0.0;
  for (long b = 0; b < nch; ++b) s += part[b];
  return s;
}
double sum(const double* x, long n) {
  const long CH = 4096;
  long nch = (n + CH - 1) / CH;
  std::vector<double> part(nch, 0.0);
#pragma omp parallel for schedule(static)
  for (long b = 0; b < nch; ++b) {
    double s = 0.0;
    for (long i = b * CH; i < std::min(n, (b + 1) * CH); ++i) s += x[i];
    part[b] = s;
  }
  double s = 0.0;
  for (long b = 0; b < nch; ++b) s += part[b];
  return s;
}

// ---------------------------------------------------------------------------
// Pressure operator.  (A p)_c = (1/h^2) sum_{interior faces f of c} beta_f (p_nb - p_c),
// beta_f = 1 / rho_f.  A is the discrete div(beta grad) with zero flux through
// walls; the solver works with K = -A (symmetric positive semi-definite).
// Levels store face weights a_f (beta_f/h^2 on the finest level); wall faces 0.
struct Level {
  int nx, ny, nz, dim;
  std::vector<double> ax, ay, az, diag;
  long N() const { return (long)nx * ny * nz; }
};

void apply_K(const Level& L, const double* x, double* y) {
  const int nx = L.nx, ny = L.ny, nz = L.nz;
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        long c = i + (long)nx * (j + (long)ny * k);
        double xc = x[c], s = 0.0;
        long fxl = i + (long)(nx + 1) * (j + (long)ny * k);
        long fyl = i + (long)nx * (j + (long)(ny + 1) * k);
        if (i > 0) s += L.ax[fxl] * (xc - x[c - 1]);
        if (i < nx - 1) s += L.ax[fxl + 1] * (xc - x[c + 1]);
        if (j > 0) s += L.ay[fyl] * (xc - x[c - nx]);
        if (j < ny - 1) s += L.ay[fyl + nx] * (xc - x[c + nx]);
        if (L.dim == 3) {
          long fzl = c;
          if (k > 0) s += L.az[fzl] * (xc - x[c - (long)nx * ny]);
          if (k < nz - 1) s += L.az[fzl + (long)nx * ny] * (xc - x[c + (long)nx * ny]);
        }
        y[c] = s;
      }
}

void make_diag(Level& L) {
  L.diag.assign(L.N(), 0.0);
  const int nx = L.nx, ny = L.ny, nz = L.nz;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        long c = i + (long)nx * (j + (long)ny * k);
        long fxl = i + (long)(nx + 1) * (j + (long)ny * k);
        long fyl = i + (long)nx * (j + (long)(ny + 1) * k);
        double d = L.ax[fxl] + L.ax[fxl + 1] + L.ay[fyl] + L.ay[fyl + nx];
        if (L.dim == 3) d += L.az[c] + L.az[c + (long)nx * ny];
        L.diag[c] = d;
      }
}

Level finest_level(const Grid& g, const double* a) {
  const OrcConfig& c = g.c;
  Level L;
  L.nx = g.nx; L.ny = g.ny; L.nz = g.nz; L.dim = g.dim;
  L.ax.assign(g.Nu(), 0.0);
  L.ay.assign(g.Nv(), 0.0);
  if (g.dim == 3) L.az.assign(g.Nw(), 0.0);
  const double ih2 = 1.0 / (g.h * g.h);
  for (int k = 0; k < g.nz; ++k)
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i) {
        auto rho = [&](int ii, int jj, int kk) {
          return g.nph > 2 ? matp(g, a, ii, jj, kk, MAT_RHO) : mix(a[g.cell(ii, jj, kk)], c.rho1, c.rho2);
        };
        double rc = rho(i, j, k);
        if (i > 0) L.ax[g.fx(i, j, k)] = ih2 / (0.5 * (rho(i - 1, j, k) + rc));
        if (j > 0) L.ay[g.fy(i, j, k)] = ih2 / (0.5 * (rho(i, j - 1, k) + rc));
        if (g.dim == 3 && k > 0) L.az[g.fz(i, j, k)] = ih2 / (0.5 * (rho(i, j, k - 1) + rc));
      }
  make_diag(L);
  return L;
}

// Galerkin coarse level for piecewise-constant prolongation P and R = P^T:
// a coarse face weight is the sum of the fine face weights it covers.
Level coarsen(const Level& F) {
  Level C;
  C.dim = F.dim;
  C.nx = F.nx / 2; C.ny = F.ny / 2; C.nz = F.dim == 3 ? F.nz / 2 : 1;
  C.ax.assign((long)(C.nx + 1) * C.ny * C.nz, 0.0);
  C.ay.assign((long)C.nx * (C.ny + 1) * C.nz, 0.0);
  if (C.dim == 3) C.az.assign((long)C.nx * C.ny * (C.nz + 1), 0.0);
  int kz = C.dim == 3 ? 2 : 1;
  for (int K = 0; K < C.nz; ++K)
    for (int J = 0; J < C.ny; ++J)
      for (int I = 0; I <= C.nx; ++I) {
        double s = 0.0;
        for (int dk = 0; dk < kz; ++dk)
          for (int dj = 0; dj < 2; ++dj)
            s += F.ax[2 * I + (long)(F.nx + 1) * ((2 * J + dj) + (long)F.ny * (kz * K + dk))];
        C.ax[I + (long)(C.nx + 1) * (J + (long)C.ny * K)] = s;
      }
  for (int K = 0; K < C.nz; ++K)
    for (int J = 0; J <= C.ny; ++J)
      for (int I = 0; I < C.nx; ++I) {
        double s = 0.0;
        for (int dk = 0; dk < kz; ++dk)
          for (int di = 0; di < 2; ++di)
            s += F.ay[(2 * I + di) + (long)F.nx * (2 * J + (long)(F.ny + 1) * (kz * K + dk))];
        C.ay[I + (long)C.nx * (J + (long)(C.ny + 1) * K)] = s;
      }
  if (C.dim == 3)
    for (int K = 0; K <= C.nz; ++K)
      for (int J = 0; J < C.ny; ++J)
        for (int I = 0; I < C.nx; ++I) {
          double s = 0.0;
          for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di)
              s += F.az[(2 * I + di) + (long)F.nx * ((2 * J + dj) + (long)F.ny * (2 * K))];
          C.az[I + (long)C.nx * (J + (long)C.ny * K)] = s;
        }
  make_diag(C);
  return C;
}

std::vector<Level> hierarchy(const Grid& g, const double* a) {
  std::vector<Level> Ls;
  Ls.push_back(finest_level(g, a));
  for (;;) {
    const Level& L = Ls.back();
    bool can = L.nx % 2 == 0 && L.ny % 2 == 0 && L.nx >= 4 && L.ny >= 4 &&
               (L.dim == 2 || (L.nz % 2 == 0 && L.nz >= 4)) && L.N() > 64;
    if (!can) break;
    Ls.push_back(coarsen(L));
  }
  return Ls;
}

// Damped Jacobi sweep x <- x + w (b - K x) / diag.
void jacobi(const Level& L, double wj, const double* b, std::vector<double>& x, std::vector<double>& t) {
  apply_K(L, x.data(), t.data());
  long N = L.N();
  for (long c = 0; c < N; ++c) x[c] += wj * (b[c] - t[c]) / L.diag[c];
}

// Symmetric V-cycle z = M r (zero initial guess on every level): nu damped
// Jacobi sweeps before and after the coarse correction, coarse correction
// scaled by omega_c, fixed Jacobi sweeps on the coarsest level.
void vcycle(const std::vector<Level>& Ls, size_t l, const OrcConfig& c, const double* b, std::vector<double>& x) {
  const Level& L = Ls[l];
  long N = L.N();
  double wj = L.dim == 2 ? 0.8 : 6.0 / 7.0;
  x.assign(N, 0.0);
  std::vector<double> t(N);
  if (l + 1 == Ls.size()) {
    for (int s = 0; s < c.mg_coarse_sweeps; ++s) jacobi(L, wj, b, x, t);
    return;
  }
  for (int s = 0; s < c.mg_nu; ++s) jacobi(L, wj, b, x, t);
  apply_K(L, x.data(), t.data());
  const Level& C = Ls[l + 1];
  std::vector<double> rc(C.N(), 0.0), ec;
  int kz = L.dim == 3 ? 2 : 1;
  for (int k = 0; k < L.nz; ++k)
    for (int j = 0; j < L.ny; ++j)
      for (int i = 0; i < L.nx; ++i) {
        long f = i + (long)L.nx * (j + (long)L.ny * k);
        rc[(i / 2) + (long)C.nx * ((j / 2) + (long)C.ny * (k / kz))] += b[f] - t[f];
      }
  vcycle(Ls, l + 1, c, rc.data(), ec);
  for (int k = 0; k < L.nz; ++k)
    for (int j = 0; j < L.ny; ++j)
      for (int i = 0; i < L.nx; ++i)
        x[i + (long)L.nx * (j + (long)L.ny * k)] += c.mg_omega_c * ec[(i / 2) + (long)C.nx * ((j / 2) + (long)C.ny * (k / kz))];
  for (int s = 0; s < c.mg_nu; ++s) jacobi(L, wj, b, x, t);
}

// S7: solve A p = b by preconditioned CG on K p = -b, warm start from p,
// stop when ||r|| <= rtol ||b||; the gauge is fixed by mean(p) = 0.
// reading: rhs is first made mean-free (the all-Neumann problem is solvable
// only for mean-free data); a zero rhs gives p = 0.
int solve_pressure(const Grid& g, const double* a, const double* b_in, double* p, OrcInfo* info) {
  const OrcConfig& c = g.c;
  long N = g.N();
  std::vector<double> rhs(N);
  double mb = sum(b_in, N) / (double)N;
  for (long i = 0; i < N; ++i) rhs[i] = -(b_in[i] - mb);
  double bn = std::sqrt(dot(rhs.data(), rhs.data(), N));
  int st = 0, it = 0;
  double rel = 0.0;
  if (bn == 0.0) {
    for (long i = 0; i < N; ++i) p[i] = 0.0;
  } else {
    std::vector<Level> Ls = hierarchy(g, a);
    std::vector<double> x(p, p + N), r(N), z, d(N), q(N);
    apply_K(Ls[0], x.data(), q.data());
    for (long i = 0; i < N; ++i) r[i] = rhs[i] - q[i];
    double rn = std::sqrt(dot(r.data(), r.data(), N));
    if (rn > c.p_rtol * bn) {
      vcycle(Ls, 0, c, r.data(), z);
      d = z;
      double rz = dot(r.data(), z.data(), N);
      st = 3;
      for (it = 1; it <= c.p_maxit; ++it) {
        apply_K(Ls[0], d.data(), q.data());
        double al = rz / dot(d.data(), q.data(), N);
        for (long i = 0; i < N; ++i) {
          x[i] += al * d[i];
          r[i] -= al * q[i];
        }
        rn = std::sqrt(dot(r.data(), r.data(), N));
        if (rn <= c.p_rtol * bn) { st = 0; break; }
        vcycle(Ls, 0, c, r.data(), z);
        double rz2 = dot(r.data(), z.data(), N);
        double be = rz2 / rz;
        rz = rz2;
        for (long i = 0; i < N; ++i) d[i] = z[i] + be * d[i];
      }
      if (it > c.p_maxit) it = c.p_maxit;
    }
    rel = rn / bn;
    double mx = sum(x.data(), N) / (double)N;
    for (long i = 0; i < N; ++i) p[i] = x[i] - mx;
  }
  if (info) {
    info->cg_iters = it;
    info->p_relres = rel;
  }
  return st;
}

// S8: u^{n+1}_f = u*_f - dt beta_f (p_R - p_L)/h on interior faces; 0 on walls.
void project(const Grid& g, double dt, const double* a, const double* p, const double* us,
             const double* vs, const double* ws, double* u, double* v, double* w) {
  const OrcConfig& c = g.c;
  const double* src[3] = {us, vs, ws};
  double* dst[3] = {u, v, w};
  for (int d = 0; d < g.dim; ++d) {
    int fnx = g.nx + (d == 0), fny = g.ny + (d == 1), fnz = g.nz + (d == 2);
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < fnz; ++k)
      for (int j = 0; j < fny; ++j)
        for (int i = 0; i < fnx; ++i) {
          long fi = (long)i + (long)fnx * (j + (long)fny * k);
          int id[3] = {i, j, k};
          if (id[d] == 0 || id[d] == g.n_of(d)) { dst[d][fi] = 0.0; continue; }
          int L[3] = {i, j, k};
          L[d] -= 1;
          long cL = g.cell(L[0], L[1], L[2]), cR = g.cell(i, j, k);
          double rhof = g.nph > 2 ? 0.5 * (matp(g, a, L[0], L[1], L[2], MAT_RHO) + matp(g, a, i, j, k, MAT_RHO))
                                  : 0.5 * (mix(a[cL], c.rho1, c.rho2) + mix(a[cR], c.rho1, c.rho2));
          dst[d][fi] = src[d][fi] - dt * (1.0 / rhof) * (p[cR] - p[cL]) / g.h;
        }
  }
}

// One step of the per-stage projected SSP-RK3 (integrator 1).
// reading: the paper does not state its time integrator.  This variant
// applies the three Shu-Osher stages to the whole state (alpha, T, c, u):
// every right-hand side of a stage (transport with the stage's own velocity,
// the heat source at the stage time t, t + dt, t + dt/2, and the momentum
// predictor with its geometry and CSF force) is taken at the stage state;
// the stage's velocity is the same convex combination as the scalars and is
// then projected with the density of the stage state, the alpha at which
// the stage's momentum right-hand side was taken (so that the velocity moves
// along P_alpha F of one state; projecting with the stage's new alpha instead
// costs an O(dt^2) error per step wherever the density varies).  The
// projection uses the stage's weight on dt (1, 1/4, 2/3) as its step (any
// positive factor gives the same velocity; it only scales p).  Returns the
// worst solver status; info gets the last stage's solve and divergence ratio.
int step_rk3p(Grid& g, double t, double dt, std::vector<double>& av, std::vector<double>& tv,
              std::vector<double>* cv, double* u, double* v, double* w, double* p, OrcInfo& inf) {
  const OrcConfig& c = g.c;
  const long N = g.N();
  const bool mom = !(c.flags & F_TRANSPORT_ONLY);
  double* vel[3] = {u, v, w};
  const long nf[3] = {g.Nu(), g.Nv(), g.Nw()};
  const std::vector<double> an(av), Tn(tv), cn = cv ? *cv : std::vector<double>();
  std::vector<double> un[3];
  for (int d = 0; d < g.dim; ++d) un[d].assign(vel[d], vel[d] + nf[d]);
  std::vector<double> La(N), LT(N), Lc(cv ? N : 0), b(N), dv(N), as(N);
  std::vector<double> us[3] = {std::vector<double>(g.Nu()), std::vector<double>(g.Nv()),
                               std::vector<double>(g.Nw() ? g.Nw() : 1)};
  const double tc[3] = {0.0, 1.0, 0.5}, wdt[3] = {1.0, 0.25, 2.0 / 3.0};
  int status = 0;
  for (int s = 0; s < 3; ++s) {
    // right-hand sides at the stage state (av, tv, cv, u)
    transport_rhs(g, t + tc[s] * dt, av.data(), tv.data(), u, v, w, La.data(), LT.data());
    if (cv) advect_rhs(g, cv->data(), u, v, w, Lc.data());
    if (mom) {
      g.cf = cv ? cv->data() : nullptr;
      predictor(g, dt, av.data(), tv.data(), u, v, w, us[0].data(), us[1].data(), us[2].data());
    }
    as = av;  // the stage state's alpha, for the projection
    for (long q = 0; q < N; ++q) {
      av[q] = rk_stage(s, an[q], av[q] + dt * La[q]);
      tv[q] = rk_stage(s, Tn[q], tv[q] + dt * LT[q]);
    }
    if (cv)
      for (long q = 0; q < N; ++q) (*cv)[q] = rk_stage(s, cn[q], (*cv)[q] + dt * Lc[q]);
    if (!mom) continue;
    for (int d = 0; d < g.dim; ++d)
      for (long f = 0; f < nf[d]; ++f) us[d][f] = rk_stage(s, un[d][f], us[d][f]);
    const double dts = wdt[s] * dt;
    divergence(g, us[0].data(), us[1].data(), g.dim == 3 ? us[2].data() : nullptr, b.data());
    const double nstar = std::sqrt(dot(b.data(), b.data(), N));
    for (long q = 0; q < N; ++q) b[q] /= dts;
    const int st = solve_pressure(g, as.data(), b.data(), p, &inf);
    if (st) status = st;
    project(g, dts, as.data(), p, us[0].data(), us[1].data(), us[2].data(), u, v, w);
    divergence(g, u, v, g.dim == 3 ? w : nullptr, dv.data());
    const double nnew = std::sqrt(dot(dv.data(), dv.data(), N));
    inf.div_rel = nstar > 0.0 ? nnew / nstar : 0.0;
  }
  g.cf = cv ? cv->data() : nullptr;
  return status;
}

bool finite_all(const double* x, long n) {
  for (long i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

}  // namespace

// ===========================================================================
// C entry points (called from the tests through ctypes).
extern "C" {

double orc_weno5(double a, double b, double c, double d, double e, double eps) {
  return weno5(a, b, c, d, e, eps);
}

double orc_heat_flux(const OrcConfig* c, double x, double y, double t) { return heat_flux(*c, x, y, t); }

void orc_transport_rhs(const OrcConfig* c, double t, const double* a, const double* T, const double* u,
                       const double* v, const double* w, double* La, double* LT) {
  Grid g(*c);
  transport_rhs(g, t, a, T, u, v, w, La, LT);
}

// cf: species field (NULL without one)
void orc_geometry(const OrcConfig* c, const double* a, const double* T, double* n, double* kap,
                  double* ds, double* sk, double* M, const double* cf) {
  Grid g(*c);
  g.cf = cf;
  geometry(g, a, T, n, kap, ds, sk, M);
}

// a3, a4: fractions of phases 3 and 4 (N-phase configs; NULL otherwise)
void orc_predictor(const OrcConfig* c, double dt, const double* a, const double* T, const double* u,
                   const double* v, const double* w, double* us, double* vs, double* ws, const double* cf,
                   const double* a3, const double* a4) {
  Grid g(*c);
  g.cf = cf;
  g.ph3 = a3;
  g.ph4 = a4;
  predictor(g, dt, a, T, u, v, w, us, vs, ws);
}

// N-phase geometry: per pair sigma_ij kappa_ij and delta_ij (npairs x N, in
// the order (1,2), (1,3), (1,4), (2,3), (2,4), (3,4) restricted to the
// phases present) and the summed Marangoni vector (3N).
void orc_geometry_n(const OrcConfig* c, const double* a, const double* a3, const double* a4, const double* T,
                    double* skp, double* dsp, double* M) {
  Grid g(*c);
  g.ph3 = a3;
  g.ph4 = a4;
  geometry_n(g, a, T, skp, dsp, M);
}

void orc_divergence(const OrcConfig* c, const double* u, const double* v, const double* w, double* out) {
  Grid g(*c);
  divergence(g, u, v, w, out);
}

// out = A p (the negative semi-definite operator of the Poisson equation)
void orc_apply_A(const OrcConfig* c, const double* a, const double* p, double* out) {
  Grid g(*c);
  Level L = finest_level(g, a);
  apply_K(L, p, out);
  for (long i = 0; i < g.N(); ++i) out[i] = -out[i];
}

// z = M r, the V-cycle preconditioner of K = -A
void orc_apply_mg(const OrcConfig* c, const double* a, const double* r, double* z) {
  Grid g(*c);
  std::vector<Level> Ls = hierarchy(g, a);
  std::vector<double> x;
  vcycle(Ls, 0, *c, r, x);
  std::memcpy(z, x.data(), sizeof(double) * g.N());
}

int orc_mg_levels(const OrcConfig* c) {
  Grid g(*c);
  std::vector<double> a(g.N(), 0.0);
  return (int)hierarchy(g, a.data()).size();
}

int orc_solve_pressure(const OrcConfig* c, const double* a, const double* b, double* p, OrcInfo* info,
                       const double* a3, const double* a4) {
  Grid g(*c);
  g.ph3 = a3;
  g.ph4 = a4;
  return solve_pressure(g, a, b, p, info);
}

void orc_project(const OrcConfig* c, double dt, const double* a, const double* p, const double* us,
                 const double* vs, const double* ws, double* u, double* v, double* w, const double* a3,
                 const double* a4) {
  Grid g(*c);
  g.ph3 = a3;
  g.ph4 = a4;
  project(g, dt, a, p, us, vs, ws, u, v, w);
}

void orc_transport_step(const OrcConfig* c, double t, double dt, double* a, double* T, const double* u,
                        const double* v, const double* w, double* cf, double* a3, double* a4) {
  Grid g(*c);
  if (g.nph > 2) {  // N phases: alpha, T and the fractions of phases 3 (and 4)
    const long N = g.N();
    std::vector<double> av(a, a + N), tv(T, T + N), p3(a3, a3 + N), p4;
    if (g.nph == 4) p4.assign(a4, a4 + N);
    transport_rk3_nphase(g, t, dt, av, tv, p3, g.nph == 4 ? &p4 : nullptr, u, v, w);
    std::memcpy(a, av.data(), sizeof(double) * N);
    std::memcpy(T, tv.data(), sizeof(double) * N);
    std::memcpy(a3, p3.data(), sizeof(double) * N);
    if (g.nph == 4) std::memcpy(a4, p4.data(), sizeof(double) * N);
    return;
  }
  std::vector<double> av(a, a + g.N()), tv(T, T + g.N());
  std::vector<double> cv;
  if (cf) cv.assign(cf, cf + g.N());
  transport_rk3(g, t, dt, av, tv, u, v, w, cf ? &cv : nullptr);
  std::memcpy(a, av.data(), sizeof(double) * g.N());
  std::memcpy(T, tv.data(), sizeof(double) * g.N());
  if (cf) std::memcpy(cf, cv.data(), sizeof(double) * g.N());
}

// nsteps full steps S1..S8, state updated in place; t advances by dt per step.
// cf: species field (NULL without one), advanced in place with the state.
// a3, a4: fractions of phases 3 and 4 of an N-phase config (advanced in
// place; NULL otherwise).  Returns 5 for a combination the oracle does not
// define (N phases with a species or with integrator 1, missing fractions).
int orc_step(const OrcConfig* c, double t0, double dt, int nsteps, double* a, double* T, double* u,
             double* v, double* w, double* p, OrcInfo* info, double* cf, double* a3, double* a4) {
  Grid g(*c);
  long N = g.N();
  if (g.nph > 2 && (!a3 || (g.nph == 4 && !a4) || c->species || c->integrator == 1 || g.nph > 4)) return 5;
  std::vector<double> av(a, a + N), tv(T, T + N);
  std::vector<double> cv, p3, p4;
  if (cf) cv.assign(cf, cf + N);
  g.cf = cf ? cv.data() : nullptr;
  if (g.nph > 2) {
    p3.assign(a3, a3 + N);
    if (g.nph == 4) p4.assign(a4, a4 + N);
    g.ph3 = p3.data();
    g.ph4 = g.nph == 4 ? p4.data() : nullptr;
  }
  std::vector<double> us(g.Nu()), vs(g.Nv()), ws(g.Nw() ? g.Nw() : 1), b(N), dv(N);
  int status = 0;
  OrcInfo inf{};
  for (int s = 0; s < nsteps; ++s) {
    double t = t0 + s * dt;
    if (c->integrator == 1) {
      const int st = step_rk3p(g, t, dt, av, tv, cf ? &cv : nullptr, u, v, w, p, inf);
      if (st) status = st;
    } else if (g.nph > 2) {
      transport_rk3_nphase(g, t, dt, av, tv, p3, g.nph == 4 ? &p4 : nullptr, u, v, w);
      g.ph3 = p3.data();
      g.ph4 = g.nph == 4 ? p4.data() : nullptr;
    } else {
      transport_rk3(g, t, dt, av, tv, u, v, w, cf ? &cv : nullptr);
    }
    if (c->integrator != 1 && !(c->flags & F_TRANSPORT_ONLY)) {
      predictor(g, dt, av.data(), tv.data(), u, v, w, us.data(), vs.data(), ws.data());
      divergence(g, us.data(), vs.data(), g.dim == 3 ? ws.data() : nullptr, b.data());
      double nstar = std::sqrt(dot(b.data(), b.data(), N));
      for (long i = 0; i < N; ++i) b[i] /= dt;
      int st = solve_pressure(g, av.data(), b.data(), p, &inf);
      if (st) status = st;
      project(g, dt, av.data(), p, us.data(), vs.data(), ws.data(), u, v, w);
      divergence(g, u, v, g.dim == 3 ? w : nullptr, dv.data());
      double nnew = std::sqrt(dot(dv.data(), dv.data(), N));
      inf.div_rel = nstar > 0.0 ? nnew / nstar : 0.0;
    }
    bool fin = finite_all(av.data(), N) && finite_all(tv.data(), N) && finite_all(u, g.Nu()) &&
               finite_all(v, g.Nv()) && (g.dim == 2 || finite_all(w, g.Nw())) && finite_all(p, N);
    if (!fin) { status = 4; break; }
  }
  std::memcpy(a, av.data(), sizeof(double) * N);
  std::memcpy(T, tv.data(), sizeof(double) * N);
  if (cf) std::memcpy(cf, cv.data(), sizeof(double) * N);
  if (g.nph > 2) std::memcpy(a3, p3.data(), sizeof(double) * N);
  if (g.nph == 4) std::memcpy(a4, p4.data(), sizeof(double) * N);
  inf.sum_alpha = sum(a, N);
  inf.alpha_min = *std::min_element(a, a + N);
  inf.alpha_max = *std::max_element(a, a + N);
  double um = 0.0;
  for (long i = 0; i < g.Nu(); ++i) um = std::max(um, std::fabs(u[i]));
  for (long i = 0; i < g.Nv(); ++i) um = std::max(um, std::fabs(v[i]));
  for (long i = 0; i < g.Nw(); ++i) um = std::max(um, std::fabs(w[i]));
  inf.cfl_max = dt * um / g.h;
  inf.status = status;
  if (info) *info = inf;
  return status;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"

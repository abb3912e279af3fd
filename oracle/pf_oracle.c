/*
 * Plain FP64 CPU oracle of the pore-scale freezing/thawing phase-field model
 * (P. Strachota, "Three-dimensional phase-field simulations of water freezing
 * and thawing at pore-scale", arXiv 2401.01672).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline of the benchmark load this library.  It shares no code, header or
 * constant with the GPU path; its only common ground with it is the seeded
 * input generator.
 *
 * What is computed, and where it comes from:
 *   - material blending                     Sec. 2.1, eq. (material-properties-blending-formula)
 *   - heat equation                          Sec. 2.2, eq. (heat-equation)
 *   - Allen-Cahn equation                    Sec. 2.2, eq. (Allen-Cahn-equation)
 *   - water indicator I_W(G)                 Sec. 2.2, eq. (water-indicator)
 *   - SigmaP1-P reaction term                Sec. 2.2, eq. (reaction-term-SigmaP1-P)
 *   - GradP reaction term                    Sec. 2.2, eq. (reaction-term-GradP)
 *   - Sigma limiter                          Sec. 2.2, eq. (Sigma-limiter)
 *   - boundary conditions                    Sec. 2.2, eqs. (BC-temperature-cap)-(BC-PF)
 *   - Temp model                             Sec. 2.3, eqs. (explicit-p-dependence-on-T),
 *                                            (combined-heat-xfer-phase-transition)
 *   - micro-scale reduction (lambda = L = 0) Sec. 2.4
 *   - method of lines, finite volumes on a uniform grid, Runge-Kutta-Merson
 *     with adaptive steps                    Sec. 2.5
 *   - ice / water sets and ice fraction      Sec. 3.1 eqs. (water-occupied-subdomain),
 *                                            (frozen-subdomain); Sec. 3.3 eq. (UWC-formula)
 *
 * The paper does not print the discrete scheme.  Readings taken here:
 *   - finite volumes with two-point fluxes on the 6 faces of each cubic cell;
 *     face conductivity = arithmetic mean of the two cell values;
 *   - phase-field flux through a face only when both cells are water
 *     (G < 1/2) and inside the domain (zero-flux phase condition at glass and
 *     at the domain boundary);
 *   - a Dirichlet temperature face uses a ghost value 2 T_D - T_c at the
 *     mirror point and the cell's own conductivity;
 *   - Merson's tableau with the error estimate dt/30 (2k1 - 9k3 + 8k4 - k5),
 *     the max-norm of that estimate over all unknowns, acceptance when it is
 *     at most tol, and the new step safety * dt * (tol/eps)^(1/5), capped at
 *     dt_max; the last step is clipped to land on t_end.
 *
 * Arrays are C-ordered (n3, n2, n1): cell (i1, i2, i3) sits at
 * n = i1 + n1*(i2 + n2*i3).  Temperatures are in kelvin.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_MODEL_AC = 0, OR_MODEL_COUPLED = 1, OR_MODEL_TEMP = 2 };
enum { OR_REACT_SIGMA = 0, OR_REACT_GRADP = 1 };
enum { OR_BC_CONST = 0, OR_BC_RAMP = 1, OR_BC_STEP = 2 };
enum {
  OR_OK = 0,
  OR_EQUILIBRIUM = 1,
  OR_MAXSTEPS = 2,
  OR_NONFINITE = -4,
  OR_DTMIN = -5
};

typedef struct {
  int32_t n1, n2, n3;
  int32_t model;     /* OR_MODEL_*                                          */
  int32_t reaction;  /* OR_REACT_*                                          */
  int32_t phi_face_mask;   /* 1: no phi flux through faces touching glass   */
  int32_t dirichlet_faces; /* bit k: face k of (x1-,x1+,x2-,x2+,x3-,x3+)    */
  int32_t bc_kind;
  double h;
  double xi, alpha, mu, b, eps0, eps1, zeta, t_star, dT, gamma;
  double lam[3];  /* liquid, ice, glass */
  double rhoc[3]; /* volumetric heat capacity: liquid, ice, glass */
  double Lv;      /* volumetric latent heat */
  double bc_T0, bc_T1, bc_t0, bc_t1;
  /* the paper's own material model (Sec. 2.2): density and specific heat
   * blended separately, rho c = blend(rho) blend(c), latent term
   * blend(rho) L; otherwise rhoc and Lv above */
  int32_t rho_c_separate;
  int32_t pad_;
  double rho[3];  /* density: liquid, ice, glass [kg m^-3] */
  double cs[3];   /* specific heat: liquid, ice, glass [J kg^-1 K^-1] */
  double L;       /* specific latent heat [J kg^-1] */
} or_params;

typedef struct {
  double tol, safety, dt_min, dt_max;
} or_ctl;

typedef struct {
  int32_t accepted, status;
  double eps, dt_used, dt_next, maxk1;
} or_step_info;

typedef struct {
  int64_t steps_accepted, steps_rejected;
  double t, dt;
  int32_t status, pad;
} or_run_stats;

/* ------------------------------------------------------------------------ */
/* Pointwise model pieces                                                     */

/* Sigma limiter, eq. (Sigma-limiter): 0 below eps0, 1 above eps1, cubic in
 * between. */
double or_sigma(double w, double e0, double e1) {
  if (w <= e0) return 0.0;
  if (w >= e1) return 1.0;
  double s = (w - e0) / (e1 - e0);
  return 3.0 * s * s - 2.0 * s * s * s;
}

/* Water indicator, eq. (water-indicator). */
double or_water_indicator(double G, double zeta) {
  double v = 1.0 - zeta * G;
  return v > 0.0 ? v : 0.0;
}

/* Blending, eq. (material-properties-blending-formula); w = (L, I, G). */
double or_blend(double G, double phi, const double w[3]) {
  return G * w[2] + (1.0 - G) * (phi * w[1] + (1.0 - phi) * w[0]);
}

/* Heat capacity per volume and latent heat per volume of a cell: the
 * product of the blended density and specific heat, and the blended density
 * times L (eq. heat-equation with rho and c blended by eq.
 * material-properties-blending-formula), or the blended volumetric heat
 * capacity and a constant volumetric latent heat. */
static double or_rhoc(const or_params* p, double G, double phi) {
  if (p->rho_c_separate) return or_blend(G, phi, p->rho) * or_blend(G, phi, p->cs);
  return or_blend(G, phi, p->rhoc);
}
static double or_latent(const or_params* p, double G, double phi) {
  if (p->rho_c_separate) return or_blend(G, phi, p->rho) * p->L;
  return p->Lv;
}

/* Prescribed temperature of the Dirichlet faces, eq. (BC-temperature-cap):
 * constant, a linear ramp from T0 (at t0) to T1 (at t1), or the
 * freeze-then-thaw step (T0 before t0, T1 from t0 on). */
double or_dirichlet_T(const or_params* p, double t) {
  if (p->bc_kind == OR_BC_RAMP) {
    double s = (t - p->bc_t0) / (p->bc_t1 - p->bc_t0);
    if (s < 0.0) s = 0.0;
    if (s > 1.0) s = 1.0;
    return p->bc_T0 + (p->bc_T1 - p->bc_T0) * s;
  }
  if (p->bc_kind == OR_BC_STEP) return t < p->bc_t0 ? p->bc_T0 : p->bc_T1;
  return p->bc_T0;
}

/* Temp model phase field, eq. (explicit-p-dependence-on-T), and its
 * derivative with respect to T. */
static double temp_phi(double G, double T, const or_params* p) {
  return 0.5 * or_water_indicator(G, p->zeta) *
         (1.0 - tanh(p->gamma * (T - p->t_star)));
}
static double temp_dphi_dT(double G, double T, const or_params* p) {
  double th = tanh(p->gamma * (T - p->t_star));
  return -0.5 * or_water_indicator(G, p->zeta) * p->gamma * (1.0 - th * th);
}

/* Neighbour of cell (i1,i2,i3) through face f (0..5 = x1-,x1+,x2-,x2+,x3-,
 * x3+); returns -1 when the face lies on the domain boundary. */
static int64_t neighbour(const or_params* p, int i1, int i2, int i3, int f) {
  int j1 = i1, j2 = i2, j3 = i3;
  switch (f) {
    case 0: j1--; break;
    case 1: j1++; break;
    case 2: j2--; break;
    case 3: j2++; break;
    case 4: j3--; break;
    default: j3++; break;
  }
  if (j1 < 0 || j1 >= p->n1 || j2 < 0 || j2 >= p->n2 || j3 < 0 || j3 >= p->n3)
    return -1;
  return (int64_t)j1 + (int64_t)p->n1 * ((int64_t)j2 + (int64_t)p->n2 * j3);
}

/* |grad phi| at a cell centre for the GradP reaction term: central
 * differences, one-sided where a neighbour is missing or not water (the
 * zero-flux condition makes the normal derivative vanish at the domain
 * boundary and at glass).  With the binary mask a face is open when both
 * cells are water; with the smooth glass field when the neighbour is water
 * (G < 1/2): the phase field inside the glass never evolves (I_W = 0 there)
 * and carries no interface. */
static double grad_phi_norm(const or_params* p, const double* G, const double* phi,
                            int i1, int i2, int i3, int64_t n) {
  double g2 = 0.0;
  for (int ax = 0; ax < 3; ++ax) {
    int64_t m = neighbour(p, i1, i2, i3, 2 * ax);
    int64_t q = neighbour(p, i1, i2, i3, 2 * ax + 1);
    int open_m = m >= 0 && G[m] < 0.5 && (!p->phi_face_mask || G[n] < 0.5);
    int open_q = q >= 0 && G[q] < 0.5 && (!p->phi_face_mask || G[n] < 0.5);
    double d = 0.0;
    if (open_m && open_q) d = (phi[q] - phi[m]) / (2.0 * p->h);
    else if (open_q) d = (phi[q] - phi[n]) / p->h;
    else if (open_m) d = (phi[n] - phi[m]) / p->h;
    g2 += d * d;
  }
  return sqrt(g2);
}

/* ------------------------------------------------------------------------ */
/* Right-hand side of the semi-discrete system (method of lines, Sec. 2.5).   */
/*
 * model AC      : unknown phi; T = T* - dT everywhere (Sec. 2.4).
 * model COUPLED : unknowns phi, T (eqs. heat-equation, Allen-Cahn-equation).
 * model TEMP    : unknown T; phi = varphi(T) (Sec. 2.3).  kphi receives
 *                 varphi'(T) kT so that callers see d phi/dt.
 */
void or_rhs(const or_params* p, const double* G, double t, const double* phi,
            const double* T, double* kphi, double* kT) {
  const int64_t ncell = (int64_t)p->n1 * p->n2 * p->n3;
  const double h2 = p->h * p->h;
  const double TD = or_dirichlet_T(p, t);
  (void)ncell;
#pragma omp parallel for schedule(static)
  for (int i3 = 0; i3 < p->n3; ++i3) {
    for (int i2 = 0; i2 < p->n2; ++i2) {
      for (int i1 = 0; i1 < p->n1; ++i1) {
        const int64_t n = (int64_t)i1 + (int64_t)p->n1 * ((int64_t)i2 + (int64_t)p->n2 * i3);
        const double Gc = G[n];
        double Tc = (p->model == OR_MODEL_AC) ? p->t_star - p->dT : T[n];
        double phic = (p->model == OR_MODEL_TEMP) ? temp_phi(Gc, Tc, p) : phi[n];

        /* Allen-Cahn, eq. (Allen-Cahn-equation) with the Laplacian as the sum
         * of face fluxes over h^2. */
        double kp = 0.0;
        if (p->model != OR_MODEL_TEMP) {
          double lap = 0.0;
          for (int f = 0; f < 6; ++f) {
            int64_t m = neighbour(p, i1, i2, i3, f);
            if (m < 0) continue; /* eq. (BC-PF): no flux through the boundary */
            if (p->phi_face_mask && !(Gc < 0.5 && G[m] < 0.5)) continue;
            lap += phi[m] - phic;
          }
          lap /= h2;
          double react;
          if (p->reaction == OR_REACT_GRADP) {
            double gn = grad_phi_norm(p, G, phi, i1, i2, i3, n);
            react = 2.0 * phic * (1.0 - phic) * (phic - 0.5) +
                    p->xi * p->xi * p->mu * p->alpha * gn * (p->t_star - Tc);
          } else {
            react = 2.0 * phic * (1.0 - phic) *
                    (phic - 0.5 + 0.5 * p->xi * p->b * p->mu * p->alpha *
                                      or_sigma(phic, p->eps0, p->eps1) *
                                      or_sigma(1.0 - phic, p->eps0, p->eps1) *
                                      (p->t_star - Tc));
          }
          kp = or_water_indicator(Gc, p->zeta) * (p->xi * p->xi * lap + react) /
               (p->alpha * p->xi * p->xi);
        }

        if (p->model == OR_MODEL_AC) {
          kphi[n] = kp;
          continue;
        }

        /* Heat conduction, div(lambda grad T), as face fluxes. */
        const double lam_c = or_blend(Gc, phic, p->lam);
        double q = 0.0;
        for (int f = 0; f < 6; ++f) {
          int64_t m = neighbour(p, i1, i2, i3, f);
          if (m >= 0) {
            double phim = (p->model == OR_MODEL_TEMP) ? temp_phi(G[m], T[m], p) : phi[m];
            double lam_m = or_blend(G[m], phim, p->lam);
            q += 0.5 * (lam_c + lam_m) * (T[m] - Tc);
          } else if (p->dirichlet_faces & (1 << f)) {
            /* eq. (BC-temperature-cap): ghost value 2 T_D - T_c */
            q += lam_c * ((2.0 * TD - Tc) - Tc);
          } /* else eq. (BC-temperature-wall): insulated */
        }
        q /= h2;
        const double rc = or_rhoc(p, Gc, phic);
        const double lat = or_latent(p, Gc, phic);
        if (p->model == OR_MODEL_COUPLED) {
          /* eq. (heat-equation): rho c dT/dt = div(lambda grad T) + rho L dphi/dt */
          kT[n] = (q + lat * kp) / rc;
          kphi[n] = kp;
        } else {
          /* eq. (combined-heat-xfer-phase-transition):
           * rho [c - L varphi'(T)] dT/dt = div(lambda grad T) */
          double dp = temp_dphi_dT(Gc, Tc, p);
          double kt = q / (rc - lat * dp);
          kT[n] = kt;
          if (kphi) kphi[n] = dp * kt;
        }
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* One Runge-Kutta-Merson attempt (Sec. 2.5).                                 */

static int nvars(const or_params* p) { return p->model == OR_MODEL_COUPLED ? 2 : 1; }

/* Y = y + dt * sum_j a_j k_j over every unknown; k has 5 slots. */
static void combine(int64_t nd, double* Y, const double* y, double dt, double* const* k,
                    const double a[5]) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nd; ++i) {
    double s = 0.0;
    for (int j = 0; j < 5; ++j)
      if (a[j] != 0.0) s += a[j] * k[j][i];
    Y[i] = y[i] + dt * s;
  }
}

/* Evaluate F on a packed state vector: AC -> [phi], COUPLED -> [phi, T],
 * TEMP -> [T]. */
static void rhs_packed(const or_params* p, const double* G, double t, const double* Y,
                       double* K) {
  const int64_t nc = (int64_t)p->n1 * p->n2 * p->n3;
  if (p->model == OR_MODEL_AC) or_rhs(p, G, t, Y, NULL, K, NULL);
  else if (p->model == OR_MODEL_COUPLED) or_rhs(p, G, t, Y, Y + nc, K, K + nc);
  else or_rhs(p, G, t, NULL, Y, NULL, K);
}

/*
 * One attempt from (t, y) with proposed step *dt.  y is the packed state
 * (see rhs_packed) and is replaced by the new state when the attempt is
 * accepted; *t and *dt are updated.  If eq_tol > 0 and the largest |k1| of
 * the phase field over water cells (G < 1/2) is below it, the state is at
 * equilibrium: nothing else is computed and status = OR_EQUILIBRIUM.
 */
int or_rkm_step(const or_params* p, const double* G, const or_ctl* c, double t_end,
                double eq_tol, double* t, double* dt, double* y, or_step_info* info) {
  const int64_t nc = (int64_t)p->n1 * p->n2 * p->n3;
  const int64_t nd = nc * nvars(p);
  double* buf = (double*)malloc(sizeof(double) * (size_t)nd * 7);
  if (!buf) return -2;
  double* k[5];
  for (int j = 0; j < 5; ++j) k[j] = buf + j * nd;
  double* Y = buf + 5 * nd;
  double* ynew = buf + 6 * nd;
  memset(info, 0, sizeof(*info));

  double h = *dt;
  int clipped = 0;
  if (t_end - *t < h) {
    h = t_end - *t;
    clipped = 1;
  }
  const double t0 = *t;

  rhs_packed(p, G, t0, y, k[0]);
  double maxk1 = 0.0;
  if (p->model != OR_MODEL_TEMP) {
    for (int64_t i = 0; i < nc; ++i)
      if (G[i] < 0.5 && fabs(k[0][i]) > maxk1) maxk1 = fabs(k[0][i]);
  }
  info->maxk1 = maxk1;
  /* the equilibrium test measures the phase-field equation, which the Temp
   * model does not have */
  if (eq_tol > 0.0 && p->model != OR_MODEL_TEMP && maxk1 < eq_tol) {
    info->status = OR_EQUILIBRIUM;
    info->dt_used = 0.0;
    info->dt_next = *dt;
    free(buf);
    return 0;
  }

  /* Merson's stages (Christiansen's formulation, cited in Sec. 2.5). */
  const double a2[5] = {1.0 / 3.0, 0, 0, 0, 0};
  const double a3[5] = {1.0 / 6.0, 1.0 / 6.0, 0, 0, 0};
  const double a4[5] = {1.0 / 8.0, 0, 3.0 / 8.0, 0, 0};
  const double a5[5] = {1.0 / 2.0, 0, -3.0 / 2.0, 2.0, 0};
  const double bw[5] = {1.0 / 6.0, 0, 0, 4.0 / 6.0, 1.0 / 6.0};
  const double ew[5] = {2.0 / 30.0, 0, -9.0 / 30.0, 8.0 / 30.0, -1.0 / 30.0};

  combine(nd, Y, y, h, k, a2);
  rhs_packed(p, G, t0 + h / 3.0, Y, k[1]);
  combine(nd, Y, y, h, k, a3);
  rhs_packed(p, G, t0 + h / 3.0, Y, k[2]);
  combine(nd, Y, y, h, k, a4);
  rhs_packed(p, G, t0 + h / 2.0, Y, k[3]);
  combine(nd, Y, y, h, k, a5);
  rhs_packed(p, G, t0 + h, Y, k[4]);
  combine(nd, ynew, y, h, k, bw);

  /* error estimate and its max-norm over all unknowns */
  double eps = 0.0;
  int nonfinite = 0;
  for (int64_t i = 0; i < nd; ++i) {
    double e = 0.0;
    for (int j = 0; j < 5; ++j) e += ew[j] * k[j][i];
    e = fabs(h * e);
    if (!(e <= DBL_MAX)) nonfinite = 1;
    else if (e > eps) eps = e;
  }
  info->eps = nonfinite ? NAN : eps;
  info->dt_used = h;

  if (nonfinite) {
    info->accepted = 0;
    info->status = OR_NONFINITE;
    info->dt_next = *dt;
    free(buf);
    return 0;
  }
  int accept;
  double dt_next;
  if (c->tol <= 0.0) { /* fixed-step mode */
    accept = 1;
    dt_next = *dt;
  } else {
    accept = eps <= c->tol;
    if (eps == 0.0) dt_next = c->dt_max;
    else {
      dt_next = c->safety * h * pow(c->tol / eps, 0.2);
      if (dt_next > c->dt_max) dt_next = c->dt_max;
    }
  }
  info->accepted = accept;
  info->dt_next = dt_next;
  if (accept) {
    memcpy(y, ynew, sizeof(double) * (size_t)nd);
    *t = clipped ? t_end : t0 + h;
  }
  *dt = dt_next;
  if (c->tol > 0.0 && dt_next < c->dt_min) info->status = OR_DTMIN;
  free(buf);
  return 0;
}

/* Integrate until t_end, max_steps attempts, equilibrium or an error. */
int or_integrate(const or_params* p, const double* G, const or_ctl* c, double t_end,
                 int64_t max_steps, double eq_tol, double* t, double* dt, double* y,
                 or_run_stats* st) {
  memset(st, 0, sizeof(*st));
  for (;;) {
    if (*t >= t_end) { st->status = OR_OK; break; }
    if (st->steps_accepted + st->steps_rejected >= max_steps) {
      st->status = OR_MAXSTEPS;
      break;
    }
    or_step_info info;
    int rc = or_rkm_step(p, G, c, t_end, eq_tol, t, dt, y, &info);
    if (rc) return rc;
    if (info.status == OR_EQUILIBRIUM) { st->status = OR_EQUILIBRIUM; break; }
    if (info.accepted) st->steps_accepted++;
    else st->steps_rejected++;
    if (info.status != OR_OK) { st->status = info.status; break; }
  }
  st->t = *t;
  st->dt = *dt;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Diagnostics.                                                               */
/*
 * out[0] = #{G < 1/2 and phi > 1/2}  (ice cells, eq. frozen-subdomain)
 * out[1] = #{G < 1/2}                (water-occupied cells, eq. water-occupied-subdomain)
 * out[2] = sum of phi over G < 1/2
 * out[3] = h^3 * sum over all cells of (rho c (T - T*) - rho L phi)  (enthalpy
 *          relative to water at T*; T = T* - dT for the micro-scale model)
 */
void or_diagnostics(const or_params* p, const double* G, const double* phi, const double* T,
                    double out[4]) {
  const int64_t nc = (int64_t)p->n1 * p->n2 * p->n3;
  double ice = 0, pore = 0, sphi = 0, H = 0;
  for (int64_t i = 0; i < nc; ++i) {
    double Tc = (p->model == OR_MODEL_AC) ? p->t_star - p->dT : T[i];
    double ph = (p->model == OR_MODEL_TEMP) ? temp_phi(G[i], Tc, p) : phi[i];
    if (G[i] < 0.5) {
      pore += 1.0;
      sphi += ph;
      if (ph > 0.5) ice += 1.0;
    }
    H += or_rhoc(p, G[i], ph) * (Tc - p->t_star) - or_latent(p, G[i], ph) * ph;
  }
  out[0] = ice;
  out[1] = pore;
  out[2] = sphi;
  out[3] = H * p->h * p->h * p->h;
}

/* Unfrozen water content of the bottom half of the vessel (Sec. 3.3, eq.
 * UWC-formula): the water set (eq. water-occupied-subdomain, G < 1/2) and
 * the ice set (eq. frozen-subdomain, phi > 1/2), both restricted to the
 * cells whose centre lies strictly below half the vessel height,
 * (i3 + 1/2) h < n3 h / 2.  Ice cells are counted among the water cells
 * (cells with G >= 1/2 never evolve: their water indicator is 0).
 * out = {water cells, ice cells, UWC = 1 - ice / water (0 if no water)}. */
void or_uwc_bottom_half(const or_params* p, const double* G, const double* phi,
                        const double* T, double out[3]) {
  const int64_t plane = (int64_t)p->n1 * p->n2;
  double water = 0, ice = 0;
  for (int32_t i3 = 0; i3 < p->n3; ++i3) {
    if (!(2.0 * i3 + 1.0 < (double)p->n3)) break;
    for (int64_t j = 0; j < plane; ++j) {
      const int64_t i = (int64_t)i3 * plane + j;
      if (!(G[i] < 0.5)) continue;
      double Tc = (p->model == OR_MODEL_AC) ? p->t_star - p->dT : T[i];
      double ph = (p->model == OR_MODEL_TEMP) ? temp_phi(G[i], Tc, p) : phi[i];
      water += 1.0;
      if (ph > 0.5) ice += 1.0;
    }
  }
  out[0] = water;
  out[1] = ice;
  out[2] = water > 0 ? 1.0 - ice / water : 0.0;
}

/* Threads the oracle's parallel loops use (1 without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
int or_num_threads(void) { return omp_get_max_threads(); }
#else
int or_num_threads(void) { return 1; }
#endif

int or_abi_version(void) { return 1; }

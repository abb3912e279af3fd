// Stencil kernels of the finite-volume right-hand side and the fused
// Runge-Kutta-Merson stages, for gfx950.
//
// Model (paper Sec. 2.2, 2.4): per cell c with neighbours nb through the six
// faces,
//   k_phi = I_W(G_c) [ (sum_open (phi_nb - phi_c)) / (alpha h^2)
//                      + f(phi_c, T_c) / (alpha xi^2) ]
//   f     = 2 phi (1 - phi) (phi - 1/2 + xi b mu alpha / 2
//                               * Sigma(phi) Sigma(1 - phi) (T* - T))
//   k_T   = [ h^-2 sum_faces lambda_f (T_nb - T_c) + L_v k_phi ] / (rho c)_c
// (eqs. Allen-Cahn-equation, reaction-term-SigmaP1-P, Sigma-limiter,
// water-indicator, heat-equation, material-properties-blending-formula), with
// the face rules listed in pf.h.  Temperatures are carried as theta = T - T*.
//
// Execution layout: a workgroup of 256 threads owns 256 consecutive cells of
// the x1-x2 plane (flattened, so ragged n1 wastes no lanes) and marches
// z_chunk planes along x3.  The x3 neighbours rotate through registers; the
// x1/x2 neighbours are re-read from the L1/L2-resident neighbouring rows.
// Workgroups are renumbered so that each XCD (hardware places workgroup b on
// XCD b mod 8) receives a contiguous range of tiles and its L2 serves the
// shared x2 rows.
//
// Merson stages (Sec. 2.5), fused with their linear combinations so that
// each stage is one pass over the grid (per unknown: 13 reads, 9 writes):
//   S1: k1 = F(t, y);            Y2 = y + dt k1/3
//   S2: k2 = F(t + dt/3, Y2);    Y3 = Y2 + dt (k2 - k1)/6       (= y + dt (k1+k2)/6)
//   S3: k3 = F(t + dt/3, Y3);    Y4 = y + dt (k1 + 3 k3)/8
//   S4: k4 = F(t + dt/2, Y4);    Y5 = y + dt (k1/2 - 3 k3/2 + 2 k4),
//                                P  = y + dt (k1 + 4 k4)/6,  C = dt (2 k1 - 9 k3 + 8 k4)/30
//   S5: k5 = F(t + dt, Y5);      y_new = P + dt k5/6,        E = C - dt k5/30
// S1 also reduces the diagnostics of y; S5 reduces max |E| in FP64.
#include <float.h>
#include <math.h>

#include "pf_internal.h"

namespace pf {

// ---------------------------------------------------------------------------
// Small device helpers

__device__ __forceinline__ double dmax_nf(double a, double v) {
  // max that turns NaN/Inf samples into +Inf so they cannot be dropped
  v = (v <= DBL_MAX) ? v : INFINITY;
  return v > a ? v : a;
}

template <typename R>
__device__ __forceinline__ R limiter(R w, R e0, R inv_de) {
  R s = (w - e0) * inv_de;
  s = s < R(0) ? R(0) : (s > R(1) ? R(1) : s);
  return s * s * (R(3) - R(2) * s);
}

__device__ __forceinline__ double dirichlet_theta(const ModelConst& m, double t) {
  if (m.bc_kind == PF_BC_RAMP) {
    double s = (t - m.bc_t0) / (m.bc_t1 - m.bc_t0);
    s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
    return m.bc_T0 + (m.bc_T1 - m.bc_T0) * s;
  }
  if (m.bc_kind == PF_BC_STEP) return t < m.bc_t0 ? m.bc_T0 : m.bc_T1;
  return m.bc_T0;
}

// Bijective renumbering of workgroups so XCD x gets a contiguous tile range.
__device__ __forceinline__ int xcd_tile(int b, int nblk) {
  const int q = nblk >> 3, r = nblk & 7;
  const int x = b & 7, k = b >> 3;
  return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

template <int OP>  // 0: sum, 1: max
__device__ __forceinline__ double wave_reduce(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    double o = __shfl_xor(v, off, 64);
    v = OP ? (o > v ? o : v) : v + o;
  }
  return v;
}

// Block-level reduction of NV values; every lane passes its values, thread 0
// receives the result (fixed order: lanes by xor tree, then waves 0..3).
template <int NV>
__device__ __forceinline__ void block_reduce(double (&v)[NV], const int (&ops)[NV],
                                             double* smem) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    v[j] = ops[j] ? wave_reduce<1>(v[j]) : wave_reduce<0>(v[j]);
    if (lane == 0) smem[j * kWaves + wave] = v[j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      double a = smem[j * kWaves];
      for (int w = 1; w < kWaves; ++w) {
        double o = smem[j * kWaves + w];
        a = ops[j] ? (o > a ? o : a) : a + o;
      }
      v[j] = a;
    }
  }
}

// ---------------------------------------------------------------------------
// Right-hand side of one cell.

template <typename R, int MODEL>
struct CellRHS {
  // phn/thn: neighbour values through faces 0..5 (clamped to the cell itself
  // when the face is on the boundary).  inb: bit f = face f has a neighbour.
  __device__ __forceinline__ static void eval(const ModelConst& m, R phic, R thc,
                                              const R (&phn)[6], const R (&thn)[6],
                                              unsigned code, unsigned inb, unsigned dirf,
                                              R thD, R& kphi, R& kth) {
    const bool glass = code & kGlassBit;
    R lap = R(0);
#pragma unroll
    for (int f = 0; f < 6; ++f) lap += ((code >> f) & 1u) ? (phn[f] - phic) : R(0);
    if (glass) lap = R(0);
    const R sa = limiter<R>(phic, R(m.e0), R(m.inv_de));
    const R sb = limiter<R>(R(1) - phic, R(m.e0), R(m.inv_de));
    const R drive = (MODEL == PF_MODEL_AC) ? R(m.betaAC) : R(m.beta0) * (-thc);
    const R f = R(2) * phic * (R(1) - phic) * (phic - R(0.5) + drive * sa * sb);
    const R iw = glass ? R(m.iw_glass) : R(1);
    kphi = iw * (R(m.cL) * lap + R(m.cR) * f);
    if (MODEL == PF_MODEL_COUPLED) {
      const R lamc = glass ? R(m.lamG) : R(m.lamL) + phic * R(m.dlam);
      R qq = R(0);
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        const bool in = (inb >> f) & 1u;
        const bool nbw = (code >> f) & 1u;
        const R lamn = nbw ? R(m.lamL) + phn[f] * R(m.dlam) : R(m.lamG);
        const R w = in ? (lamc + lamn) : (((dirf >> f) & 1u) ? R(4) * lamc : R(0));
        const R tgt = in ? thn[f] : thD;
        qq += w * (tgt - thc);
      }
      const R rc = glass ? R(m.rcG) : R(m.rcL) + phic * R(m.drc);
      kth = (R(0.5) * R(m.cH) * qq + R(m.Lv) * kphi) / rc;
    } else {
      kth = R(0);
    }
  }
};

// ---------------------------------------------------------------------------
// Stage kernel.  STAGE 0 = standalone RHS (in -> out as k).

template <typename R, int MODEL, int STAGE>
__global__ __launch_bounds__(kBlock) void stage_kernel(StageArgs a) {
  __shared__ double smem[8 * kWaves];
  const ModelConst& m = a.mc;
  double t0 = a.t_fixed, dt = 0.0;
  int cur = 0;
  if (!a.ignore_done) {
    if (a.ctl->done) return;
    t0 = a.ctl->t;
    dt = a.ctl->dt_att;
    cur = a.ctl->cur;
  }
  constexpr double cs = STAGE == 2 ? 1.0 / 3.0 : STAGE == 3 ? 1.0 / 3.0 : STAGE == 4 ? 0.5
                        : STAGE == 5 ? 1.0 : 0.0;
  const double ts = t0 + cs * dt;
  const R thD = R(dirichlet_theta(m, ts) );
  constexpr bool kCoupled = MODEL == PF_MODEL_COUPLED;

  const int nblk = gridDim.x;
  const int tile = xcd_tile(blockIdx.x, nblk);
  const int tp = tile % a.tiles_p, tz = tile / a.tiles_p;
  const int plane = m.n1 * m.n2;
  const int p = tp * kBlock + threadIdx.x;
  const bool active = p < plane;
  const int z0 = tz * a.z_chunk;
  const int z1 = min(z0 + a.z_chunk, m.n3);

  const R* inP = static_cast<const R*>(a.in[0]);
  const R* inT = static_cast<const R*>(a.in[1]);
  const R* yP = static_cast<const R*>(a.y[cur][0]);
  const R* yT = static_cast<const R*>(a.y[cur][1]);
  R* k1P = static_cast<R*>(a.k1[0]);
  R* k1T = static_cast<R*>(a.k1[1]);
  R* k3P = static_cast<R*>(a.k3[0]);
  R* k3T = static_cast<R*>(a.k3[1]);
  R* oP = static_cast<R*>(STAGE == 5 ? a.out_y[1 - cur][0] : a.out[0]);
  R* oT = static_cast<R*>(STAGE == 5 ? a.out_y[1 - cur][1] : a.out[1]);
  if (STAGE == 1) {  // S1's stencil input is the state itself
    inP = yP;
    inT = yT;
  }
  const R rdt = R(dt);

  double red0 = 0.0, red1 = 0.0, red2 = 0.0, red3 = 0.0;
  if (active) {
    const int i1 = p % m.n1;
    const int i2 = p / m.n1;
    unsigned inb_xy = 0;
    inb_xy |= (i1 > 0) ? 1u : 0u;
    inb_xy |= (i1 < m.n1 - 1) ? 2u : 0u;
    inb_xy |= (i2 > 0) ? 4u : 0u;
    inb_xy |= (i2 < m.n2 - 1) ? 8u : 0u;
    const int oxm = (inb_xy & 1u) ? -1 : 0;
    const int oxp = (inb_xy & 2u) ? 1 : 0;
    const int oym = (inb_xy & 4u) ? -m.n1 : 0;
    const int oyp = (inb_xy & 8u) ? m.n1 : 0;
    const unsigned dirf = (unsigned)m.dirichlet_faces;

    int n = p + plane * z0;
    R pc = inP[n], pm = pc;
    R tc = kCoupled ? inT[n] : R(0), tm = tc;
    if (z0 > 0) {
      pm = inP[n - plane];
      if (kCoupled) tm = inT[n - plane];
    }
    for (int z = z0; z < z1; ++z, n += plane) {
      const bool zp_in = z < m.n3 - 1;
      const R pp = zp_in ? inP[n + plane] : pc;
      const R tpv = kCoupled ? (zp_in ? inT[n + plane] : tc) : R(0);
      const unsigned inb = inb_xy | (z > 0 ? 16u : 0u) | (zp_in ? 32u : 0u);
      const unsigned code = a.code[n];
      R phn[6], thn[6];
      phn[0] = inP[n + oxm];
      phn[1] = inP[n + oxp];
      phn[2] = inP[n + oym];
      phn[3] = inP[n + oyp];
      phn[4] = pm;
      phn[5] = pp;
      if (kCoupled) {
        thn[0] = inT[n + oxm];
        thn[1] = inT[n + oxp];
        thn[2] = inT[n + oym];
        thn[3] = inT[n + oyp];
        thn[4] = tm;
        thn[5] = tpv;
      } else {
#pragma unroll
        for (int f = 0; f < 6; ++f) thn[f] = R(0);
      }
      R kp, kt;
      CellRHS<R, MODEL>::eval(m, pc, tc, phn, thn, code, inb, dirf, thD, kp, kt);

      if (STAGE == 0) {
        oP[n] = kp;
        if (kCoupled) oT[n] = kt;
      } else if (STAGE == 1) {
        k1P[n] = kp;
        oP[n] = pc + rdt * (R(1.0 / 3.0) * kp);
        if (kCoupled) {
          k1T[n] = kt;
          oT[n] = tc + rdt * (R(1.0 / 3.0) * kt);
        }
        const bool water = !(code & kGlassBit);
        const double dpc = (double)pc;
        const double thc_d = kCoupled ? (double)tc : -m.dT;
        const double rc = (code & kGlassBit) ? m.rcG : m.rcL + dpc * m.drc;
        if (water) {
          red0 = dmax_nf(red0, fabs((double)kp));
          red1 += dpc;
          red3 += (dpc > 0.5) ? 1.0 : 0.0;
        }
        red2 += rc * thc_d - m.Lv * dpc;
      } else if (STAGE == 2) {
        const R k1p = k1P[n];
        oP[n] = pc + rdt * (R(1.0 / 6.0) * (kp - k1p));
        if (kCoupled) {
          const R k1t = k1T[n];
          oT[n] = tc + rdt * (R(1.0 / 6.0) * (kt - k1t));
        }
      } else if (STAGE == 3) {
        const R k1p = k1P[n], y0p = yP[n];
        k3P[n] = kp;
        oP[n] = y0p + rdt * (R(0.125) * (k1p + R(3) * kp));
        if (kCoupled) {
          const R k1t = k1T[n], y0t = yT[n];
          k3T[n] = kt;
          oT[n] = y0t + rdt * (R(0.125) * (k1t + R(3) * kt));
        }
      } else if (STAGE == 4) {
        {
          const R k1p = k1P[n], k3p = k3P[n], y0p = yP[n];
          oP[n] = y0p + rdt * (R(0.5) * k1p - R(1.5) * k3p + R(2) * kp);
          k1P[n] = y0p + rdt * (R(1.0 / 6.0) * (k1p + R(4) * kp));
          k3P[n] = rdt * (R(1.0 / 30.0) * (R(2) * k1p - R(9) * k3p + R(8) * kp));
        }
        if (kCoupled) {
          const R k1t = k1T[n], k3t = k3T[n], y0t = yT[n];
          oT[n] = y0t + rdt * (R(0.5) * k1t - R(1.5) * k3t + R(2) * kt);
          k1T[n] = y0t + rdt * (R(1.0 / 6.0) * (k1t + R(4) * kt));
          k3T[n] = rdt * (R(1.0 / 30.0) * (R(2) * k1t - R(9) * k3t + R(8) * kt));
        }
      } else if (STAGE == 5) {
        {
          const R P = k1P[n], Cc = k3P[n];
          oP[n] = P + rdt * (R(1.0 / 6.0) * kp);
          const double e = (double)Cc - dt * ((1.0 / 30.0) * (double)kp);
          red0 = dmax_nf(red0, fabs(e));
        }
        if (kCoupled) {
          const R P = k1T[n], Cc = k3T[n];
          oT[n] = P + rdt * (R(1.0 / 6.0) * kt);
          const double e = (double)Cc - dt * ((1.0 / 30.0) * (double)kt);
          red0 = dmax_nf(red0, fabs(e));
        }
      }
      pm = pc;
      pc = pp;
      if (kCoupled) {
        tm = tc;
        tc = tpv;
      }
    }
  }
  if (STAGE == 1) {
    double v[4] = {red0, red1, red2, red3};
    const int ops[4] = {1, 0, 0, 0};
    block_reduce<4>(v, ops, smem);
    if (threadIdx.x == 0) {
      double* o = a.part + (size_t)blockIdx.x * kPartS1;
      o[0] = v[0];
      o[1] = v[1];
      o[2] = v[2];
      o[3] = v[3];
    }
  } else if (STAGE == 5) {
    double v[1] = {red0};
    const int ops[1] = {1};
    block_reduce<1>(v, ops, smem);
    if (threadIdx.x == 0) a.part[blockIdx.x] = v[0];
  }
}

// ---------------------------------------------------------------------------
// Controller: reduces the partials of S1 and S5 in a fixed order and updates
// the device step control (Sec. 2.5; semantics in pf.h).

__global__ __launch_bounds__(256) void controller_kernel(DevCtl* ctl, const double* p1,
                                                         const double* p5, int np,
                                                         double h3) {
  __shared__ double smem[8 * kWaves];
  if (ctl->done) return;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    v[0] = dmax_nf(v[0], p1[(size_t)i * kPartS1 + 0]);
    v[1] += p1[(size_t)i * kPartS1 + 1];
    v[2] += p1[(size_t)i * kPartS1 + 2];
    v[3] += p1[(size_t)i * kPartS1 + 3];
    v[4] = dmax_nf(v[4], p5[i]);
  }
  const int ops[5] = {1, 0, 0, 0, 1};
  block_reduce<5>(v, ops, smem);
  if (threadIdx.x != 0) return;

  DevCtl c = *ctl;
  c.maxk1 = v[0];
  c.sum_phi = v[1];
  c.enthalpy = v[2] * h3;
  c.ice = v[3];
  const double eps = v[4];
  c.eps = eps;
  c.dt_used = c.dt_att;
  c.accepted = 0;
  if (c.eq_tol > 0.0 && c.maxk1 < c.eq_tol) {
    c.status = PF_EQUILIBRIUM;
    c.done = 1;
    c.dt_used = 0.0;
    *ctl = c;
    return;
  }
  if (!(eps <= DBL_MAX)) {
    c.n_rej++;
    c.status = PF_ENONFINITE;
    c.done = 1;
    *ctl = c;
    return;
  }
  int accept;
  double dt_next;
  if (c.tol <= 0.0) {
    accept = 1;
    dt_next = c.dt_nom;
  } else {
    accept = eps <= c.tol;
    if (eps == 0.0) {
      dt_next = c.dt_max;
    } else {
      dt_next = c.safety * c.dt_att * pow(c.tol / eps, 0.2);
      if (dt_next > c.dt_max) dt_next = c.dt_max;
    }
  }
  if (accept) {
    c.t = c.clipped ? c.t_end : c.t + c.dt_att;
    c.cur ^= 1;
    c.n_acc++;
  } else {
    c.n_rej++;
  }
  c.accepted = accept;
  c.dt_nom = dt_next;
  if (c.tol > 0.0 && dt_next < c.dt_min) {
    c.status = PF_EDTMIN;
    c.done = 1;
  } else if (c.t >= c.t_end) {
    c.status = PF_OK;
    c.done = 1;
  } else if (c.n_acc + c.n_rej >= c.max_steps) {
    c.status = PF_MAXSTEPS;
    c.done = 1;
  }
  c.dt_att = c.dt_nom;
  c.clipped = 0;
  if (c.t_end - c.t < c.dt_att) {
    c.dt_att = c.t_end - c.t;
    c.clipped = 1;
  }
  *ctl = c;
}

// ---------------------------------------------------------------------------
// Diagnostics of a state (no stencil): per-workgroup partials of
// (water-cell count, sum phi over water, enthalpy sum, ice count).

template <typename R, int MODEL>
__global__ __launch_bounds__(kBlock) void diag_kernel(const uint8_t* code, const R* phi,
                                                      const R* th, ModelConst m, long long n,
                                                      double* part) {
  __shared__ double smem[8 * kWaves];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock) {
    const bool glass = code[i] & kGlassBit;
    const double ph = (double)phi[i];
    const double thc = MODEL == PF_MODEL_COUPLED ? (double)th[i] : -m.dT;
    const double rc = glass ? m.rcG : m.rcL + ph * m.drc;
    if (!glass) {
      v[0] += 1.0;
      v[1] += ph;
      v[3] += ph > 0.5 ? 1.0 : 0.0;
    }
    v[2] += rc * thc - m.Lv * ph;
  }
  const int ops[4] = {0, 0, 0, 0};
  block_reduce<4>(v, ops, smem);
  if (threadIdx.x == 0)
    for (int j = 0; j < 4; ++j) part[(size_t)blockIdx.x * 4 + j] = v[j];
}

__global__ void diag_final_kernel(const double* part, int np, double h3, double* out) {
  __shared__ double smem[8 * kWaves];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < np; i += blockDim.x)
    for (int j = 0; j < 4; ++j) v[j] += part[(size_t)i * 4 + j];
  const int ops[4] = {0, 0, 0, 0};
  block_reduce<4>(v, ops, smem);
  if (threadIdx.x == 0) {
    out[0] = v[0];
    out[1] = v[1];
    out[2] = v[2] * h3;
    out[3] = v[3];
  }
}

// ---------------------------------------------------------------------------
// Neighbourhood codes from the glass mask.

__global__ void build_code_kernel(const uint8_t* mask, uint8_t* code, int n1, int n2, int n3) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)n1 * n2 * n3;
  if (n >= total) return;
  const int i1 = (int)(n % n1);
  const int i2 = (int)((n / n1) % n2);
  const int i3 = (int)(n / ((long long)n1 * n2));
  const long long pl = (long long)n1 * n2;
  unsigned c = mask[n] ? kGlassBit : 0u;
  if (i1 > 0 && !mask[n - 1]) c |= 1u;
  if (i1 < n1 - 1 && !mask[n + 1]) c |= 2u;
  if (i2 > 0 && !mask[n - n1]) c |= 4u;
  if (i2 < n2 - 1 && !mask[n + n1]) c |= 8u;
  if (i3 > 0 && !mask[n - pl]) c |= 16u;
  if (i3 < n3 - 1 && !mask[n + pl]) c |= 32u;
  code[n] = (uint8_t)c;
}

// ---------------------------------------------------------------------------
// Host launchers

int grid_blocks(const ModelConst& mc, int z_chunk, int* tiles_p, int* tiles_z) {
  const long long plane = (long long)mc.n1 * mc.n2;
  *tiles_p = (int)((plane + kBlock - 1) / kBlock);
  *tiles_z = (mc.n3 + z_chunk - 1) / z_chunk;
  return (*tiles_p) * (*tiles_z);
}

hipError_t launch_build_code(const uint8_t* mask, uint8_t* code, int n1, int n2, int n3,
                             hipStream_t s) {
  const long long total = (long long)n1 * n2 * n3;
  const int threads = 256;
  const long long blocks = (total + threads - 1) / threads;
  hipLaunchKernelGGL(build_code_kernel, dim3((unsigned)blocks), dim3(threads), 0, s, mask, code,
                     n1, n2, n3);
  return hipGetLastError();
}

template <typename R, int MODEL>
static hipError_t launch_stage_t(int stage, const StageArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)(a.tiles_p * a.tiles_z)), block(kBlock);
  switch (stage) {
    case 0: hipLaunchKernelGGL((stage_kernel<R, MODEL, 0>), grid, block, 0, s, a); break;
    case 1: hipLaunchKernelGGL((stage_kernel<R, MODEL, 1>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((stage_kernel<R, MODEL, 2>), grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL((stage_kernel<R, MODEL, 3>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((stage_kernel<R, MODEL, 4>), grid, block, 0, s, a); break;
    case 5: hipLaunchKernelGGL((stage_kernel<R, MODEL, 5>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_stage(int precision, int model, int stage, const StageArgs& a, hipStream_t s) {
  if (precision == PF_FP64) {
    if (model == PF_MODEL_AC) return launch_stage_t<double, PF_MODEL_AC>(stage, a, s);
    if (model == PF_MODEL_COUPLED) return launch_stage_t<double, PF_MODEL_COUPLED>(stage, a, s);
  } else {
    if (model == PF_MODEL_AC) return launch_stage_t<float, PF_MODEL_AC>(stage, a, s);
    if (model == PF_MODEL_COUPLED) return launch_stage_t<float, PF_MODEL_COUPLED>(stage, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_controller(DevCtl* ctl, const double* part1, const double* part5, int nparts,
                             double h3, hipStream_t s) {
  hipLaunchKernelGGL(controller_kernel, dim3(1), dim3(256), 0, s, ctl, part1, part5, nparts, h3);
  return hipGetLastError();
}

hipError_t launch_diag(int precision, int model, const uint8_t* code, const void* phi,
                       const void* th, const ModelConst& m, long long n, double* part, int nparts,
                       double* out4, hipStream_t s) {
  const dim3 grid((unsigned)nparts), block(kBlock);
  if (precision == PF_FP64) {
    if (model == PF_MODEL_COUPLED)
      hipLaunchKernelGGL((diag_kernel<double, PF_MODEL_COUPLED>), grid, block, 0, s, code,
                         (const double*)phi, (const double*)th, m, n, part);
    else
      hipLaunchKernelGGL((diag_kernel<double, PF_MODEL_AC>), grid, block, 0, s, code,
                         (const double*)phi, (const double*)th, m, n, part);
  } else {
    if (model == PF_MODEL_COUPLED)
      hipLaunchKernelGGL((diag_kernel<float, PF_MODEL_COUPLED>), grid, block, 0, s, code,
                         (const float*)phi, (const float*)th, m, n, part);
    else
      hipLaunchKernelGGL((diag_kernel<float, PF_MODEL_AC>), grid, block, 0, s, code,
                         (const float*)phi, (const float*)th, m, n, part);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(256), 0, s, part, nparts, m.h3, out4);
  return hipGetLastError();
}

}  // namespace pf

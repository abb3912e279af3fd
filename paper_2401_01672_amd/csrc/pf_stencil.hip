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
// S1 also reduces max over water cells of |k1_phi| (the equilibrium measure);
// S5 reduces max |E| in FP64.
#include <float.h>
#include <hip/hip_cooperative_groups.h>
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
__device__ __forceinline__ float dmax_nf(float a, float v) {
  v = (v <= FLT_MAX) ? v : INFINITY;
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

// Bit f of code as 0 or 1 in the field precision: a face weight that enters
// the Laplacian through a fused multiply-add (lap + w d is lap + d rounded
// once for w = 1 and exactly lap for w = 0): bit extract, convert and fma
// where a compare and a select would take one more instruction.
template <typename R>
__device__ __forceinline__ R face_weight(unsigned code, int f) {
  return R((code >> f) & 1u);
}

// FP32: bit f of code as an all-ones or all-zeros word, used as an and-mask
// (keep_if: x or +0) and a bitwise select (pick: v_bfi_b32), so that one bit
// extract serves the Laplacian and the conductivity of a face.  The empty asm
// hides that the word is a sign-extended bit: the compiler would otherwise
// turn each use back into a compare and a select.
__device__ __forceinline__ int face_mask(unsigned code, int f) {
  int msk = __builtin_amdgcn_sbfe((int)code, (unsigned)f, 1u);
  asm("" : "+v"(msk));
  return msk;
}
__device__ __forceinline__ float keep_if(int msk, float x) {
  return __int_as_float(__float_as_int(x) & msk);
}
__device__ __forceinline__ float pick(int msk, float a, float b) {
  return __int_as_float((__float_as_int(a) & msk) | (__float_as_int(b) & ~msk));
}

// Sigma limiter with the clamp as one med3 (FP32); s = w inv - e0 inv.
__device__ __forceinline__ float limiter_fast(float w, float inv, float e0inv) {
  const float s = __builtin_amdgcn_fmed3f(fmaf(w, inv, -e0inv), 0.0f, 1.0f);
  return s * s * fmaf(-2.0f, s, 3.0f);
}
__device__ __forceinline__ double limiter_fast(double w, double inv, double e0inv) {
  double s = w * inv - e0inv;
  s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
  return s * s * (3.0 - 2.0 * s);
}

__device__ __forceinline__ float div_fast(float a, float b) {
  return a * __builtin_amdgcn_rcpf(b);  // ~1 ulp: far inside the FP32 error budget
}
__device__ __forceinline__ double div_fast(double a, double b) { return a / b; }  // IEEE

// |grad phi| at the cell centre (GradP): central differences, one-sided where
// a face is closed to the phase field, zero along an axis with both faces
// closed (the zero-flux condition makes the normal derivative vanish there).
template <typename R>
__device__ __forceinline__ R grad_norm(const ModelConst& m, R phic, const R (&phn)[6],
                                       unsigned code) {
  R g2 = R(0);
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const bool om = (code >> (2 * ax)) & 1u, oq = (code >> (2 * ax + 1)) & 1u;
    const R q = oq ? phn[2 * ax + 1] : phic;
    const R mm = om ? phn[2 * ax] : phic;
    const R w = (om && oq) ? R(0.5 * m.inv_h) : R(m.inv_h);
    const R d = (q - mm) * w;
    g2 += d * d;
  }
  return sqrt(g2);
}

// Heat capacity and latent heat per volume of a cell of the voxel mask:
// blended volumetric rho c and a constant rho L, or (the paper's material
// model) the product of the blended density and specific heat and the
// blended density times L (eqs. heat-equation and
// material-properties-blending-formula).
template <typename R>
__device__ __forceinline__ void heat_capacity_mask(const ModelConst& m, bool glass, R phic, R& rc,
                                                   R& lat) {
  if (m.sep) {
    const R rho = glass ? R(m.rhoG) : R(m.rhoL) + phic * R(m.drho);
    rc = rho * (glass ? R(m.csG) : R(m.csL) + phic * R(m.dcs));
    lat = rho * R(m.Lm);
  } else {
    rc = glass ? R(m.rcG) : R(m.rcL) + phic * R(m.drc);
    lat = R(m.Lv);
  }
}

template <typename R, int MODEL, int REACT = PF_REACT_SIGMA>
struct CellRHS {
  // phn/thn: neighbour values through faces 0..5.  Precondition: for a face
  // on the domain boundary thn[f] == thc (the caller passes the cell's own
  // value), so an insulated face contributes exactly zero with no select;
  // the nd Dirichlet faces among the boundary faces add
  // 2 lambda_c (2 theta_D - theta_c - theta_c) each.  Bit f of code: the
  // neighbour through face f exists and is water.
  __device__ __forceinline__ static void eval_nd(const ModelConst& m, R phic, R thc,
                                                 const R (&phn)[6], const R (&thn)[6],
                                                 unsigned code, unsigned nd, R thD, R& kphi,
                                                 R& kth) {
    const bool glass = code & kGlassBit;
    const R lamc = glass ? R(m.lamG) : R(m.lamL) + phic * R(m.dlam);
    R lap = R(0), qq = R(0);
    if constexpr (sizeof(R) == 4) {
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        const int msk = face_mask(code, f);
        lap += keep_if(msk, phn[f] - phic);
        if (MODEL == PF_MODEL_COUPLED) {
          const R lamn = pick(msk, R(m.lamL) + phn[f] * R(m.dlam), R(m.lamG));
          qq += (lamc + lamn) * (thn[f] - thc);
        }
      }
    } else {
#pragma unroll
      for (int f = 0; f < 6; ++f) lap += face_weight<R>(code, f) * (phn[f] - phic);
      if (MODEL == PF_MODEL_COUPLED) {
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          const R lamn = ((code >> f) & 1u) ? R(m.lamL) + phn[f] * R(m.dlam) : R(m.lamG);
          qq += (lamc + lamn) * (thn[f] - thc);
        }
      }
    }
    R f;
    if (REACT == PF_REACT_GRADP) {
      // eq. reaction-term-GradP: 2 phi (1 - phi)(phi - 1/2) + xi^2 mu alpha |grad phi| (T* - T)
      const R gn = glass ? R(0) : grad_norm(m, phic, phn, code);
      const R under = (MODEL == PF_MODEL_AC) ? R(m.dT) : -thc;
      f = R(2) * phic * (R(1) - phic) * (phic - R(0.5)) + R(m.gpc) * gn * under;
    } else {
      const R sa = limiter_fast(phic, R(m.inv_de), R(m.e0 * m.inv_de));
      const R sb = limiter_fast(R(1) - phic, R(m.inv_de), R(m.e0 * m.inv_de));
      const R drive = (MODEL == PF_MODEL_AC) ? R(m.betaAC) : R(m.beta0) * (-thc);
      f = R(2) * phic * (R(1) - phic) * (phic - R(0.5) + drive * sa * sb);
    }
    // glass: no phase-field flux and the water indicator of glass
    kphi = glass ? R(m.iw_glass) * (R(m.cR) * f) : R(m.cL) * lap + R(m.cR) * f;
    if (MODEL == PF_MODEL_COUPLED) {
      // nd = 0: the term is an exact zero
      qq += R(4 * (int)nd) * lamc * (thD - thc);
      R rc, lat;
      heat_capacity_mask(m, glass, phic, rc, lat);
      kth = div_fast(R(0.5) * R(m.cH) * qq + lat * kphi, rc);
    } else {
      kth = R(0);
    }
  }
  // inb: bit f set where face f is inside the domain; dirf: the Dirichlet
  // faces of the domain
  __device__ __forceinline__ static void eval(const ModelConst& m, R phic, R thc,
                                              const R (&phn)[6], const R (&thn)[6],
                                              unsigned code, unsigned inb, unsigned dirf,
                                              R thD, R& kphi, R& kth) {
    eval_nd(m, phic, thc, phn, thn, code, __builtin_popcount(~inb & dirf & 63u), thD, kphi, kth);
  }
};

// Temp model (Sec. 2.3): the unknown is theta alone and the phase field
// follows it, phi = varphi(T) = I_W(G) (1 - tanh(gamma (T - T*)))/2
// (eq. explicit-p-dependence-on-T); the heat equation becomes
// rho [c - L varphi'(T)] dT/dt = div(lambda grad T) (eq.
// combined-heat-xfer-phase-transition).  The caller passes the theta
// neighbours in thn (boundary faces: the cell's own value); kth receives
// d theta/dt and kphi = varphi'(T) d theta/dt.
// With e = exp(2x): (1 - tanh(x))/2 = 1/(1 + e) and (1 - tanh^2(x))/4 =
// e/(1 + e)^2 = 1/(e + 2 + 1/e) -- no cancellation where tanh saturates.
// exp in FP64, the hardware exp2 in FP32.
__device__ __forceinline__ double exp2x(double x) { return exp(2.0 * x); }
__device__ __forceinline__ float exp2x(float x) { return __expf(2.0f * x); }
template <typename R>
__device__ __forceinline__ R logistic_e(R e) { return R(1) / (R(1) + e); }
template <typename R>
__device__ __forceinline__ R bump_e(R e) { return R(1) / (e + R(2) + R(1) / e); }

template <typename R>
__device__ __forceinline__ R temp_phi(const ModelConst& m, R th, R iw) {
  return iw * logistic_e(exp2x(R(m.gamma) * th));
}

template <typename R, int REACT>
struct CellRHS<R, PF_MODEL_TEMP, REACT> {
  __device__ __forceinline__ static void eval(const ModelConst& m, R thc, R /*unused*/,
                                              const R (&thn)[6], const R (&/*unused*/)[6],
                                              unsigned code, unsigned inb, unsigned dirf,
                                              R thD, R& kth, R& kphi) {
    const bool glass = code & kGlassBit;
    const R iw = glass ? R(m.iw_glass) : R(1);
    const R e = exp2x(R(m.gamma) * thc);
    const R phic = iw * logistic_e(e);  // I_W (1 - tanh(gamma theta))/2
    const R lamc = glass ? R(m.lamG) : R(m.lamL) + phic * R(m.dlam);
    R qq = R(0);
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const R lamn =
          ((code >> f) & 1u) ? R(m.lamL) + temp_phi(m, thn[f], R(1)) * R(m.dlam) : R(m.lamG);
      qq += (lamc + lamn) * (thn[f] - thc);
    }
    const unsigned nd = __builtin_popcount(~inb & dirf & 63u);
    if (nd) qq += R(4 * (int)nd) * lamc * (thD - thc);
    R rc, lat;
    heat_capacity_mask(m, glass, phic, rc, lat);
    // varphi'(T) = -gamma I_W (1 - tanh^2)/2
    const R dphi = R(-2) * iw * R(m.gamma) * bump_e(e);
    kth = (R(0.5) * R(m.cH) * qq) / (rc - lat * dphi);
    kphi = dphi * kth;
  }
};

// Paper mode (Sec. 2.1): a smooth glass field G in [0, 1] instead of the
// binary mask.  The phase-field Laplacian acts across every face inside the
// box (no face rule at glass; I_W(G) = max(0, 1 - zeta G) masks the update,
// eq. water-indicator), and lambda, rho c are blended with the cell's own G
// (eq. material-properties-blending-formula).  Gn: G of the six neighbours
// (boundary faces: any value, their differences vanish by the caller's
// precondition thn[f] == thc, phn[f] == phic).  inb: bit f = the neighbour
// through face f exists.
template <typename R>
__device__ __forceinline__ R blend3(R G, R phi, R wL, R dw, R wG) {
  return G * wG + (R(1) - G) * (wL + phi * dw);
}

template <typename R, int MODEL, int REACT>
struct CellRHSSmooth {
  __device__ __forceinline__ static void eval(const ModelConst& m, R phic, R thc,
                                              const R (&phn)[6], const R (&thn)[6], R Gc,
                                              const R (&Gn)[6], unsigned inb, unsigned dirf,
                                              R thD, R& kphi, R& kth) {
    const R iw = fmax(R(0), R(1) - R(m.zeta) * Gc);
    R pc = phic;
    R pn[6];
    R dphi = R(0);
    if (MODEL == PF_MODEL_TEMP) {
      // phi = varphi(T) = I_W(G) (1 - tanh(gamma theta)) / 2
      const R e = exp2x(R(m.gamma) * thc);
      pc = iw * logistic_e(e);
      dphi = R(-2) * iw * R(m.gamma) * bump_e(e);
#pragma unroll
      for (int f = 0; f < 6; ++f)
        pn[f] = temp_phi(m, thn[f], fmax(R(0), R(1) - R(m.zeta) * Gn[f]));
      kphi = R(0);
    } else {
#pragma unroll
      for (int f = 0; f < 6; ++f) pn[f] = phn[f];
      R lap = R(0);
#pragma unroll
      for (int f = 0; f < 6; ++f) lap += pn[f] - pc;
      R fr;
      if (REACT == PF_REACT_GRADP) {
        // |grad phi| over the faces towards water neighbours (G < 1/2): the
        // phase field inside the glass never evolves and carries no interface
        unsigned wnb = 0u;
#pragma unroll
        for (int f = 0; f < 6; ++f) wnb |= (Gn[f] < R(0.5) ? 1u : 0u) << f;
        const R gn = grad_norm(m, pc, pn, inb & wnb);
        const R under = (MODEL == PF_MODEL_AC) ? R(m.dT) : -thc;
        fr = R(2) * pc * (R(1) - pc) * (pc - R(0.5)) + R(m.gpc) * gn * under;
      } else {
        const R sa = limiter_fast(pc, R(m.inv_de), R(m.e0 * m.inv_de));
        const R sb = limiter_fast(R(1) - pc, R(m.inv_de), R(m.e0 * m.inv_de));
        const R drive = (MODEL == PF_MODEL_AC) ? R(m.betaAC) : R(m.beta0) * (-thc);
        fr = R(2) * pc * (R(1) - pc) * (pc - R(0.5) + drive * sa * sb);
      }
      kphi = iw * (R(m.cL) * lap + R(m.cR) * fr);
    }
    if (MODEL == PF_MODEL_AC) {
      kth = R(0);
      return;
    }
    const R lamc = blend3(Gc, pc, R(m.lamL), R(m.dlam), R(m.lamG));
    R qq = R(0);
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const R lamn = blend3(Gn[f], pn[f], R(m.lamL), R(m.dlam), R(m.lamG));
      qq += (lamc + lamn) * (thn[f] - thc);
    }
    const unsigned nd = __builtin_popcount(~inb & dirf & 63u);
    if (nd) qq += R(4 * (int)nd) * lamc * (thD - thc);
    R rc, lat;
    if (m.sep) {
      const R rho = blend3(Gc, pc, R(m.rhoL), R(m.drho), R(m.rhoG));
      rc = rho * blend3(Gc, pc, R(m.csL), R(m.dcs), R(m.csG));
      lat = rho * R(m.Lm);
    } else {
      rc = blend3(Gc, pc, R(m.rcL), R(m.drc), R(m.rcG));
      lat = R(m.Lv);
    }
    if (MODEL == PF_MODEL_TEMP) {
      kth = (R(0.5) * R(m.cH) * qq) / (rc - lat * dphi);
      kphi = dphi * kth;
    } else {
      kth = (R(0.5) * R(m.cH) * qq + lat * kphi) / rc;
    }
  }
};

// ---------------------------------------------------------------------------
// Stage kernel.  STAGE 0 = standalone RHS (in -> out as k).

// the S5 partial of a workgroup, and the folded step controller (below)
__device__ void s5_partial(const StageArgs& a, int slot, double v, double* smem);

template <typename R, int MODEL, int STAGE, int REACT = PF_REACT_SIGMA, int SMOOTH = 0>
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
  if (STAGE == 5 && a.c_from_out) {
    // paired schedule: P lives in K3 and C in the y_new slot, which the pass
    // overwrites in place (each cell reads its C before writing y_new)
    k1P = k3P;
    k1T = k3T;
    k3P = oP;
    k3T = oT;
  }
  const R rdt = R(dt);

  double red0 = 0.0;
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
      R Gc = R(0);
      if (SMOOTH) {
        const R* Gf = static_cast<const R*>(a.G);
        Gc = Gf[n];
        R Gn[6];
        Gn[0] = Gf[n + oxm];
        Gn[1] = Gf[n + oxp];
        Gn[2] = Gf[n + oym];
        Gn[3] = Gf[n + oyp];
        Gn[4] = z > 0 ? Gf[n - plane] : Gc;
        Gn[5] = zp_in ? Gf[n + plane] : Gc;
        // Temp model: the single unknown (theta) travels in the first slot
        if (MODEL == PF_MODEL_TEMP)
          CellRHSSmooth<R, MODEL, REACT>::eval(m, R(0), pc, thn, phn, Gc, Gn, inb, dirf, thD,
                                               kt, kp);
        else
          CellRHSSmooth<R, MODEL, REACT>::eval(m, pc, tc, phn, thn, Gc, Gn, inb, dirf, thD, kp,
                                               kt);
      } else {
        // Temp model: the single unknown (theta) travels in the first slot;
        // kp = d theta/dt, kt = d phi/dt
        CellRHS<R, MODEL, REACT>::eval(m, pc, tc, phn, thn, code, inb, dirf, thD, kp, kt);
      }

      if (STAGE == 0) {
        oP[n] = kp;
        if (kCoupled || (MODEL == PF_MODEL_TEMP && oT)) oT[n] = kt;
      } else if (STAGE == 1) {
        k1P[n] = kp;
        oP[n] = pc + rdt * (R(1.0 / 3.0) * kp);
        if (kCoupled) {
          k1T[n] = kt;
          oT[n] = tc + rdt * (R(1.0 / 3.0) * kt);
        }
        // equilibrium measure: max over water cells of |k1_phi| (the Temp
        // model has no phase-field equation and reports 0)
        const bool water = !(code & kGlassBit);
        if (water && MODEL != PF_MODEL_TEMP) red0 = dmax_nf(red0, fabs((double)kp));
        (void)Gc;
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
    // the sums of the state (phi, enthalpy, ice) are not needed per step:
    // runs report them from a diagnostics pass over the final state
    double v[1] = {red0};
    const int ops[1] = {1};
    block_reduce<1>(v, ops, smem);
    if (threadIdx.x == 0) {
      double* o = a.part + (size_t)blockIdx.x * kPartS1;
      o[0] = v[0];
      o[1] = 0.0;
      o[2] = 0.0;
      o[3] = 0.0;
    }
  } else if (STAGE == 5) {
    double v[1] = {red0};
    const int ops[1] = {1};
    block_reduce<1>(v, ops, smem);
    s5_partial(a, blockIdx.x, v[0], smem);
  }
}

// ---------------------------------------------------------------------------
// Controller: reduces the partials of S1 and S5 in a fixed order and updates
// the device step control (Sec. 2.5; semantics in pf.h).

// One block (256 threads) runs the controller of one control block; smem
// holds 8 * kWaves doubles.  Safe to call repeatedly from a persistent block.
// With FOLDED the maximum of the S5 partials is eps_in (thread 0's value) and
// p5 is not read.
template <bool FOLDED = false>
__device__ void controller_body(DevCtl* ctl, const double* p1, int np1, const double* p5,
                                int np5, double h3, double* smem, double eps_in = 0.0) {
  __syncthreads();  // smem reuse across consecutive calls
  if (ctl->done) return;
  // Only the maxima are reduced per attempt: the stage kernels leave the
  // partial sums of the state (slots 1..3) at zero, and runs report those
  // sums from a diagnostics pass over the final state.
  double v[2] = {0.0, 0.0};
  for (int i = threadIdx.x; i < np1; i += blockDim.x)
    v[0] = dmax_nf(v[0], p1[(size_t)i * kPartS1 + 0]);
  if constexpr (!FOLDED)
    for (int i = threadIdx.x; i < np5; i += blockDim.x) v[1] = dmax_nf(v[1], p5[i]);
  const int ops[2] = {1, 1};
  block_reduce<2>(v, ops, smem);
  if (threadIdx.x != 0) return;
  (void)h3;

  DevCtl c = *ctl;
  c.maxk1 = v[0];
  c.sum_phi = 0.0;
  c.enthalpy = 0.0;
  c.ice = 0.0;
  const double eps = FOLDED ? eps_in : v[1];
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

__global__ __launch_bounds__(256) void controller_kernel(DevCtl* ctl, const double* p1,
                                                         int np1, const double* p5, int np5,
                                                         double h3) {
  __shared__ double smem[8 * kWaves];
  controller_body(ctl, p1, np1, p5, np5, h3, smem);
}

// The S5 partial of slot `slot` (the workgroup's maximum of the error
// estimate), written by thread 0; called by every thread of the workgroup.
// With the controller folded into the pass (a.fold) the partials are instead
// combined by an agent-scope atomic maximum into one word (as unsigned
// integers: the partials are non-negative or +Inf, whose bit patterns order
// like their values), a counter counts them, and the workgroup whose partial
// completes the count reads and clears the word, clears the counter and runs
// the controller: the attempt needs no controller launch.  The S1 partials
// come from an earlier launch and are read plainly.
__device__ void s5_partial(const StageArgs& a, int slot, double v, double* smem) {
  if (!a.fold) {
    if (threadIdx.x == 0) a.part[slot] = v;
    return;
  }
  __shared__ int s_last;
  if (threadIdx.x == 0) {
    const unsigned long long old = __hip_atomic_fetch_max(
        a.fold_acc, (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
        __HIP_MEMORY_SCOPE_AGENT);
    // the count moves only once the maximum has been taken
    asm volatile("" ::"v"(old) : "memory");
    const unsigned prev =
        __hip_atomic_fetch_add(a.fold_ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_last = prev + 1u == (unsigned)a.fold_np5;
  }
  __syncthreads();
  if (!s_last) return;
  double eps = 0.0;
  if (threadIdx.x == 0) {
    eps = __longlong_as_double(
        (long long)__hip_atomic_load(a.fold_acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    __hip_atomic_store(a.fold_acc, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(a.fold_ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  controller_body<true>(a.fold_ctl, a.fold_p1, a.fold_np1, nullptr, 0, 0.0, smem, eps);
}

// ---------------------------------------------------------------------------
// Batched sweep: many independent grids (instances) advanced by one
// persistent cooperative kernel.  Work items are (instance, tile) pairs of
// the vector stage passes (items[i].x = instance, .y = tile); all items of
// one stage are processed (strided over the workgroups), then a grid-wide
// barrier, then the next stage; after S5 one workgroup per instance runs that
// instance's controller on its own control block (own t, dt, status), then a
// barrier.  Instances whose control block says done are skipped, so finished
// instances cost nothing and the remaining ones share the whole GPU.  A launch
// performs at most steps_per_launch attempts and returns; every workgroup
// leaves the loop at the same point (the exit test reads the control blocks
// after a barrier).

template <typename R, int MODEL, int STAGE, bool NT = false, int REACT = PF_REACT_SIGMA,
          int SMOOTH = 0>
__device__ __forceinline__ void stage4_tile(const StageArgs& a, const int tile, const int slot,
                                            double* smem, void* lds);

// Grid-wide barrier: bar[0] counts arrivals, bar[1] is the generation.  The
// last workgroup to arrive resets the count and advances the generation
// (release); the others wait for the generation to change (acquire).  The
// agent-scope fences make every workgroup's global writes before the barrier
// visible to every workgroup after it (L2 write-back / invalidate across
// XCDs).  The wait is bounded: on overrun *err is set and the workgroup
// continues, so the kernel always terminates (the host then reports an
// error).  All workgroups of the launch must be resident (the launch size
// is capped by the occupancy limit and launched cooperatively).
__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned nblocks, unsigned* err) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned gen = __hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned arrived =
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(bar, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(bar + 1, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned spins = 0;
      while (__hip_atomic_load(bar + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > (1u << 24)) {
          __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
    }
    __threadfence();
  }
  __syncthreads();
}

template <typename R, int MODEL>
__global__ __launch_bounds__(kBlock) void batch_kernel(const BatchDesc* desc,
                                                       const int2* items, int nitems,
                                                       int ninst, int steps_per_launch,
                                                       unsigned* bar, unsigned* err) {
  __shared__ double smem[8 * kWaves];
  extern __shared__ __align__(16) unsigned char pf_stage_lds[];
  for (int it = 0; it < steps_per_launch; ++it) {
    // exit when every instance is done (same answer in every workgroup)
    int active = 0;
    for (int i = 0; i < ninst; ++i) active |= desc[i].st[0].ctl->done ? 0 : 1;
    if (!active) break;
#pragma unroll 1
    for (int stage = 1; stage <= 5; ++stage) {
      for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int2 it = items[item];
        const BatchDesc& d = desc[it.x];
        const int tile = it.y;
        switch (stage) {
          case 1: stage4_tile<R, MODEL, 1>(d.st[0], tile, tile, smem, pf_stage_lds); break;
          case 2: stage4_tile<R, MODEL, 2>(d.st[1], tile, tile, smem, pf_stage_lds); break;
          case 3: stage4_tile<R, MODEL, 3>(d.st[2], tile, tile, smem, pf_stage_lds); break;
          case 4: stage4_tile<R, MODEL, 4>(d.st[3], tile, tile, smem, pf_stage_lds); break;
          default: stage4_tile<R, MODEL, 5>(d.st[4], tile, tile, smem, pf_stage_lds); break;
        }
      }
      grid_barrier(bar, gridDim.x, err);
    }
    for (int inst = blockIdx.x; inst < ninst; inst += gridDim.x) {
      const BatchDesc& d = desc[inst];
      controller_body(d.st[0].ctl, d.p1, d.ntiles, d.p5, d.ntiles, d.h3, smem);
    }
    grid_barrier(bar, gridDim.x, err);
  }
}

// Multi-launch form of the batched sweep: one launch per stage over the
// (instance, tile) items of the instances still running (one item per
// workgroup, XCD-aware order), one controller launch with one workgroup per
// listed instance; the host captures a run of attempts into a HIP graph and
// rebuilds the item table (and the graph) when instances finish.  Same
// per-cell arithmetic as batch_kernel.
template <typename R, int MODEL, int STAGE, int SMOOTH = 0>
__global__ __launch_bounds__(kBlock) void batch_stage_kernel(const BatchDesc* desc,
                                                             const int2* items) {
  __shared__ double smem[8 * kWaves];
  extern __shared__ __align__(16) unsigned char pf_stage_lds[];
  const int2 it = items[xcd_tile(blockIdx.x, gridDim.x)];
  stage4_tile<R, MODEL, STAGE, false, PF_REACT_SIGMA, SMOOTH>(desc[it.x].st[STAGE - 1], it.y,
                                                              it.y, smem, pf_stage_lds);
}

// The controllers of the listed instances whose controller is not folded
// into their S5 work items (one workgroup each).
__global__ __launch_bounds__(256) void batch_ctl_kernel(const BatchDesc* desc,
                                                        const int* inst_list) {
  __shared__ double smem[8 * kWaves];
  const BatchDesc& d = desc[inst_list[blockIdx.x]];
  if (d.st[4].fold) return;
  controller_body(d.st[0].ctl, d.p1, d.ntiles, d.p5, d.ntiles, d.h3, smem);
}

// One workgroup of 64 lanes per listed instance copies its control block.
__global__ __launch_bounds__(64) void gather_ctl_kernel(const BatchDesc* desc,
                                                        const int* inst_list, DevCtl* out) {
  static_assert(sizeof(DevCtl) % 8 == 0, "control block of whole doubles");
  constexpr int kWords = (int)(sizeof(DevCtl) / 8);
  const unsigned long long* src =
      reinterpret_cast<const unsigned long long*>(desc[inst_list[blockIdx.x]].st[0].ctl);
  unsigned long long* dst = reinterpret_cast<unsigned long long*>(out + blockIdx.x);
  for (int w = threadIdx.x; w < kWords; w += 64) dst[w] = src[w];
}

hipError_t launch_gather_ctl(const BatchDesc* desc, const int* inst_list, int ninst,
                             DevCtl* out, hipStream_t s) {
  if (ninst < 1) return hipSuccess;
  hipLaunchKernelGGL(gather_ctl_kernel, dim3((unsigned)ninst), dim3(64), 0, s, desc, inst_list,
                     out);
  return hipGetLastError();
}

template <typename R, int MODEL, int SMOOTH>
static hipError_t launch_batch_step_t(const BatchDesc* desc, const int2* items, int nitems,
                                      const int* inst_list, int ninst, bool ctl, size_t lds,
                                      hipStream_t s) {
  const dim3 g((unsigned)nitems), b(kBlock);
  hipLaunchKernelGGL((batch_stage_kernel<R, MODEL, 1, SMOOTH>), g, b, lds, s, desc, items);
  hipLaunchKernelGGL((batch_stage_kernel<R, MODEL, 2, SMOOTH>), g, b, lds, s, desc, items);
  hipLaunchKernelGGL((batch_stage_kernel<R, MODEL, 3, SMOOTH>), g, b, lds, s, desc, items);
  hipLaunchKernelGGL((batch_stage_kernel<R, MODEL, 4, SMOOTH>), g, b, lds, s, desc, items);
  // S5 runs the step controller of the instances with few work items in the
  // last of their items; the others' run in a controller launch
  hipLaunchKernelGGL((batch_stage_kernel<R, MODEL, 5, SMOOTH>), g, b, lds, s, desc, items);
  if (ctl)
    hipLaunchKernelGGL(batch_ctl_kernel, dim3((unsigned)ninst), dim3(256), 0, s, desc, inst_list);
  return hipGetLastError();
}

template <typename R, int SMOOTH>
static hipError_t launch_batch_step_r(int model, const BatchDesc* desc, const int2* items,
                                      int nitems, const int* inst_list, int ninst, bool ctl,
                                      size_t lds, hipStream_t s) {
  return model == PF_MODEL_AC
             ? launch_batch_step_t<R, PF_MODEL_AC, SMOOTH>(desc, items, nitems, inst_list, ninst,
                                                          ctl, lds, s)
             : launch_batch_step_t<R, PF_MODEL_COUPLED, SMOOTH>(desc, items, nitems, inst_list,
                                                               ninst, ctl, lds, s);
}

hipError_t launch_batch_step(int precision, int model, int smooth, const BatchDesc* desc,
                             const int2* items, int nitems, const int* inst_list, int ninst,
                             bool ctl, size_t lds, hipStream_t s) {
  if (precision == PF_FP64)
    return smooth ? launch_batch_step_r<double, 1>(model, desc, items, nitems, inst_list, ninst,
                                                   ctl, lds, s)
                  : launch_batch_step_r<double, 0>(model, desc, items, nitems, inst_list, ninst,
                                                   ctl, lds, s);
  return smooth ? launch_batch_step_r<float, 1>(model, desc, items, nitems, inst_list, ninst, ctl,
                                                lds, s)
                : launch_batch_step_r<float, 0>(model, desc, items, nitems, inst_list, ninst, ctl,
                                                lds, s);
}

template <typename R, int MODEL>
static hipError_t launch_batch_t(const BatchDesc* desc, const int2* items, int nitems,
                                 int ninst, int steps, int grid_blocks, unsigned* bar,
                                 unsigned* err, size_t lds, hipStream_t s) {
  void* args[] = {(void*)&desc, (void*)&items, (void*)&nitems, (void*)&ninst,
                  (void*)&steps, (void*)&bar, (void*)&err};
  return hipLaunchCooperativeKernel((const void*)batch_kernel<R, MODEL>, dim3(grid_blocks),
                                    dim3(kBlock), args, (unsigned)lds, s);
}

hipError_t launch_batch(int precision, int model, const BatchDesc* desc, const int2* items,
                        int nitems, int ninst, int steps, int grid_blocks, unsigned* bar,
                        unsigned* err, size_t lds, hipStream_t s) {
  if (precision == PF_FP64) {
    if (model == PF_MODEL_AC)
      return launch_batch_t<double, PF_MODEL_AC>(desc, items, nitems, ninst, steps,
                                                 grid_blocks, bar, err, lds, s);
    return launch_batch_t<double, PF_MODEL_COUPLED>(desc, items, nitems, ninst, steps,
                                                    grid_blocks, bar, err, lds, s);
  }
  if (model == PF_MODEL_AC)
    return launch_batch_t<float, PF_MODEL_AC>(desc, items, nitems, ninst, steps,
                                              grid_blocks, bar, err, lds, s);
  return launch_batch_t<float, PF_MODEL_COUPLED>(desc, items, nitems, ninst, steps,
                                                 grid_blocks, bar, err, lds, s);
}

int batch_max_blocks(int precision, int model, size_t lds) {
  int per_cu = 0;
  hipError_t e;
  if (precision == PF_FP64)
    e = model == PF_MODEL_AC
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel<double, PF_MODEL_AC>, kBlock, lds)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel<double, PF_MODEL_COUPLED>, kBlock, lds);
  else
    e = model == PF_MODEL_AC
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel<float, PF_MODEL_AC>, kBlock, lds)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel<float, PF_MODEL_COUPLED>, kBlock, lds);
  if (e != hipSuccess || per_cu < 1) return 0;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return per_cu * cus;
}

// ---------------------------------------------------------------------------
// Diagnostics of a state (no stencil): per-workgroup partials of
// (water-cell count, sum phi over water, enthalpy sum, ice count).

template <typename R, int MODEL>
__global__ __launch_bounds__(kBlock) void diag_kernel(const uint8_t* code, const R* G,
                                                      const R* phi, const R* th, ModelConst m,
                                                      long long n, double* part) {
  __shared__ double smem[8 * kWaves];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock) {
    const bool glass = code[i] & kGlassBit;
    const R Gc = G ? G[i] : R(0);
    const R iw = G ? fmax(R(0), R(1) - R(m.zeta) * Gc) : (glass ? R(m.iw_glass) : R(1));
    // Temp model: the state is theta alone (passed as phi), phi = varphi(T)
    const double ph = MODEL == PF_MODEL_TEMP ? (double)temp_phi(m, phi[i], iw) : (double)phi[i];
    const double thc = MODEL == PF_MODEL_COUPLED ? (double)th[i]
                       : MODEL == PF_MODEL_TEMP  ? (double)phi[i]
                                                 : -m.dT;
    const double Gd = (double)Gc;
    // blend (eq. material-properties-blending-formula) of the cell
    auto bl = [&](double wL, double dw, double wG) {
      return G ? Gd * wG + (1.0 - Gd) * (wL + ph * dw) : glass ? wG : wL + ph * dw;
    };
    double rc, lat;
    if (m.sep) {
      const double rho = bl(m.rhoL, m.drho, m.rhoG);
      rc = rho * bl(m.csL, m.dcs, m.csG);
      lat = rho * m.Lm;
    } else {
      rc = bl(m.rcL, m.drc, m.rcG);
      lat = m.Lv;
    }
    if (!glass) {
      v[0] += 1.0;
      v[1] += ph;
      v[3] += ph > 0.5 ? 1.0 : 0.0;
    }
    v[2] += rc * thc - lat * ph;
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
// Vector stage kernel: each thread owns one 16-byte vector of consecutive
// x1-cells (four FP32 or two FP64 cells: one load per field and plane), so
// address arithmetic and load issue are shared by its cells.  The x1
// neighbours come from the thread's own registers and from the adjacent lanes
// (shuffles), the x2 neighbours from LDS.  Needs n1 divisible by the vector
// width (each vector lies in one x1 row).  Same arithmetic per cell as
// stage_kernel.

template <typename R>
struct Quad {  // one 16-byte vector: four FP32 or two FP64 cells
  static constexpr int N = 16 / (int)sizeof(R);
  R v[N];
};

template <typename R>
__device__ __forceinline__ Quad<R> ldq(const R* base, uint32_t idx) {
  Quad<R> q;
  if constexpr (sizeof(R) == 4) {
    const float4 t = *reinterpret_cast<const float4*>(base + idx);
    q.v[0] = t.x;
    q.v[1] = t.y;
    q.v[2] = t.z;
    q.v[3] = t.w;
  } else {
    const double2 t = *reinterpret_cast<const double2*>(base + idx);
    q.v[0] = t.x;
    q.v[1] = t.y;
  }
  return q;
}

// Streaming forms: every output of a pass, and every input read only at the
// cell itself (not a stencil neighbour), is touched once per pass; on grids
// far larger than the caches they are loaded and stored non-temporally and
// leave the L2 to the stencil rows that neighbouring workgroups re-read (on
// cache-resident grids the plain forms are faster).
template <typename R>
__device__ __forceinline__ Quad<R> ldq_nt(const R* base, uint32_t idx) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  typedef double d2 __attribute__((ext_vector_type(2)));
  Quad<R> q;
  if constexpr (sizeof(R) == 4) {
    const f4 t = __builtin_nontemporal_load(reinterpret_cast<const f4*>(base + idx));
    q.v[0] = t.x;
    q.v[1] = t.y;
    q.v[2] = t.z;
    q.v[3] = t.w;
  } else {
    const d2 t = __builtin_nontemporal_load(reinterpret_cast<const d2*>(base + idx));
    q.v[0] = t.x;
    q.v[1] = t.y;
  }
  return q;
}

template <typename R>
__device__ __forceinline__ void stq_plain(R* base, uint32_t idx, const Quad<R>& q) {
  if constexpr (sizeof(R) == 4) {
    *reinterpret_cast<float4*>(base + idx) = make_float4(q.v[0], q.v[1], q.v[2], q.v[3]);
  } else {
    *reinterpret_cast<double2*>(base + idx) = make_double2(q.v[0], q.v[1]);
  }
}

template <typename R>
__device__ __forceinline__ void stq_nt(R* base, uint32_t idx, const Quad<R>& q) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  typedef double d2 __attribute__((ext_vector_type(2)));
  if constexpr (sizeof(R) == 4) {
    const f4 t = {q.v[0], q.v[1], q.v[2], q.v[3]};
    __builtin_nontemporal_store(t, reinterpret_cast<f4*>(base + idx));
  } else {
    const d2 t = {q.v[0], q.v[1]};
    __builtin_nontemporal_store(t, reinterpret_cast<d2*>(base + idx));
  }
}

template <bool NT, typename R>
__device__ __forceinline__ Quad<R> ldq_s(const R* base, uint32_t idx) {
  if constexpr (NT) return ldq_nt(base, idx);
  else return ldq(base, idx);
}

template <bool NT, typename R>
__device__ __forceinline__ void stq_s(R* base, uint32_t idx, const Quad<R>& q) {
  if constexpr (NT) stq_nt(base, idx, q);
  else stq_plain(base, idx, q);
}

// Non-temporal load of quad p of one x1-x2 plane (pb: the plane's first cell,
// plane bytes < 2^32) through a buffer resource.  Its cache policy is part of
// the intrinsic, so a pass that loads a field non-temporally in some waves
// and plainly in others keeps two distinct loads (two plain loads that differ
// only in a non-temporal hint are merged into one plain load).
template <typename R>
__device__ __forceinline__ Quad<R> ldq_plane_nt(const R* pb, uint32_t p, uint32_t plane_bytes) {
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc((void*)pb, 0, (int)plane_bytes, 0x00020000);
  // cache policy 2: nt
  const auto w = __builtin_amdgcn_raw_buffer_load_b128(r, p * (uint32_t)sizeof(R), 0, 2);
  Quad<R> q;
  if constexpr (sizeof(R) == 4) {
    const float4 t = __builtin_bit_cast(float4, w);
    q.v[0] = t.x;
    q.v[1] = t.y;
    q.v[2] = t.z;
    q.v[3] = t.w;
  } else {
    const double2 t = __builtin_bit_cast(double2, w);
    q.v[0] = t.x;
    q.v[1] = t.y;
  }
  return q;
}

template <typename R>
__device__ __forceinline__ R shfl_up1(R v) {
  return __shfl_up(v, 1, 64);
}
template <typename R>
__device__ __forceinline__ R shfl_down1(R v) {
  return __shfl_down(v, 1, 64);
}

template <typename R, int MODEL, int STAGE, bool NT, int REACT, int SMOOTH>
__device__ __forceinline__ void stage4_tile(const StageArgs& a, const int tile,
                                            const int slot, double* smem, void* lds_raw) {
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
  const R thD = R(dirichlet_theta(m, t0 + cs * dt));
  constexpr bool kCoupled = MODEL == PF_MODEL_COUPLED;
  constexpr int NV = kCoupled ? 2 : 1;
  // staged fields: the unknowns' stage values, and (paper mode) the glass
  // field G in slot NV
  constexpr int NL = NV + (SMOOTH ? 1 : 0);
  const R* Gf = static_cast<const R*>(a.G);

  const int tp = tile % a.tiles_p, tz = tile / a.tiles_p;
  const uint32_t plane = (uint32_t)m.n1 * (uint32_t)m.n2;
  constexpr int VW = Quad<R>::N;  // cells per thread
  const uint32_t p = ((uint32_t)tp * kBlock + threadIdx.x) * (uint32_t)VW;
  const bool active = p < plane;
  const int z0 = tz * a.z_chunk;
  const int z1 = min(z0 + a.z_chunk, m.n3);
  const int lane = threadIdx.x & 63;

  const R* in[2] = {static_cast<const R*>(a.in[0]), static_cast<const R*>(a.in[1])};
  const R* yv[2] = {static_cast<const R*>(a.y[cur][0]), static_cast<const R*>(a.y[cur][1])};
  R* k1[2] = {static_cast<R*>(a.k1[0]), static_cast<R*>(a.k1[1])};
  R* k3[2] = {static_cast<R*>(a.k3[0]), static_cast<R*>(a.k3[1])};
  R* out[2] = {static_cast<R*>(STAGE == 5 ? a.out_y[1 - cur][0] : a.out[0]),
               static_cast<R*>(STAGE == 5 ? a.out_y[1 - cur][1] : a.out[1])};
  R* ynew[2] = {static_cast<R*>(a.out_y[1 - cur][0]), static_cast<R*>(a.out_y[1 - cur][1])};
  R* cb[2] = {static_cast<R*>(a.cbuf[0]), static_cast<R*>(a.cbuf[1])};
  if (STAGE == 1) {
    in[0] = yv[0];
    in[1] = yv[1];
  }
  if (STAGE == 5) {  // where S4 left P and C
    if (a.c_from_out) {  // paired schedule: P in K3, C in the y_new slot
      k1[0] = k3[0];
      k1[1] = k3[1];
      k3[0] = out[0];
      k3[1] = out[1];
    } else {  // P in the y_new slot (overwritten in place), C in cbuf
      k1[0] = out[0];
      k1[1] = out[1];
      k3[0] = cb[0];
      k3[1] = cb[1];
    }
  }
  const R rdt = R(dt);
  // Stencil input vector at cell index i of variable v.  S2 and S4 form their
  // stage value from the state and the stored derivatives (Y2 = y + dt k1/3,
  // Y4 = y + dt (k1 + 3 k3)/8; the same expressions as the one-cell kernel);
  // raw (when given) receives the loaded k1 (S2) or y, k1, k3 (S4), which the
  // pass needs again at the cell one plane later (kept in registers: a reload
  // misses the L2 on large grids).
  // LD(field) loads the quad in question of a field.
  auto ldin_g = [&](int v, auto&& LD, Quad<R>* raw) -> Quad<R> {
    if (SMOOTH && v == NV) return LD(Gf);
    if constexpr (STAGE == 2 || STAGE == 4) {
      const Quad<R> y0 = LD(yv[v]), q1 = LD(k1[v]);
      Quad<R> q3, o;
      if constexpr (STAGE == 4) q3 = LD(k3[v]);
#pragma unroll
      for (int k = 0; k < VW; ++k) {
        if constexpr (STAGE == 2) o.v[k] = y0.v[k] + rdt * (R(1.0 / 3.0) * q1.v[k]);
        else o.v[k] = y0.v[k] + rdt * (R(0.125) * (q1.v[k] + R(3) * q3.v[k]));
      }
      if (raw) {
        raw[1] = q1;
        if constexpr (STAGE == 4) {
          raw[0] = y0;
          raw[2] = q3;
        }
      }
      return o;
    } else {
      return LD(in[v]);
    }
  };
  auto ldin = [&](int v, uint32_t i, Quad<R>* raw) -> Quad<R> {
    return ldin_g(v, [&](const R* f) { return ldq(f, i); }, raw);
  };

  double red0 = 0.0;
  // S1's maximum of |k1_phi| in the field precision (max is exact in any
  // precision; widened to FP64 once per tile)
  R red1 = R(0);
  // The workgroup's quads are the run [q0, q0 + kBlock) of the plane's quads
  // (Q per x1-row).  Per plane, the stencil input of the run and of the Q
  // quads on either side (the rows below and above) is staged in LDS, double
  // buffered: [v][W] quads with W = kBlock + 2 Q, run at slot Q + t.  The x3
  // neighbours come from a register window, x1 neighbours inside a wavefront
  // from lane shuffles.
  const uint32_t Q = (uint32_t)m.n1 / VW, nq = plane / VW, W = kBlock + 2u * Q;
  const uint32_t t = threadIdx.x, q0 = (uint32_t)tp * kBlock;
  Quad<R>* lds = static_cast<Quad<R>*>(lds_raw);
  // the vector's position (n1 % VW == 0: its cells share i2)
  const uint32_t i1 = active ? p % (uint32_t)m.n1 : 0u;
  const uint32_t i2 = active ? p / (uint32_t)m.n1 : 0u;
  const bool xm_in = i1 > 0, xp_in = i1 + VW < (uint32_t)m.n1;
  const bool ym_in = i2 > 0, yp_in = i2 + 1 < (uint32_t)m.n2;
  // The first and last Q quads of the run are the x2 halo rows of the
  // neighbouring runs, read by them too; the quads between are read by this
  // workgroup alone, once per pass.  On large grids (NT) the waves that hold
  // only such quads load them non-temporally, which leaves the L2 to the
  // shared rows.  (Not in S1: the extra registers of the second load path
  // would cost that ALU-bound pass a wavefront per SIMD.)
  const uint32_t plane_b = plane * (uint32_t)sizeof(R);
  const uint32_t w0 = threadIdx.x & ~63u;
  const bool wave_nt =
      NT && STAGE != 1 && (uint64_t)plane * sizeof(R) < (1ull << 32) &&
      __builtin_amdgcn_readfirstlane((int)(w0 >= Q && w0 + 64u + Q <= (uint32_t)kBlock)) != 0;
  // the stencil input of the thread's own quad in plane zz, at index i (the
  // x3 window)
  auto ldc = [&](int v, int zz, uint32_t i, Quad<R>* raw) -> Quad<R> {
    if (!wave_nt) return ldin(v, i, raw);
    return ldin_g(v, [&](const R* f) { return ldq_plane_nt(f + plane * (uint32_t)zz, p, plane_b); },
                  raw);
  };
  // lanes whose x-neighbour quad lives in another wavefront (read from LDS)
  const bool xm_remote = xm_in && (lane == 0);
  const bool xp_remote = xp_in && (lane == 63 || p + VW >= plane);
  const unsigned dirf = (unsigned)m.dirichlet_faces;
  // LDS slots of the x2 neighbours; on a boundary face the cell's own slot
  // (the face then carries the cell's own value)
  const uint32_t sym = ym_in ? t : Q + t, syp = yp_in ? 2u * Q + t : Q + t;

  // z window of the stencil input, and the cell's own k1 (S2) or y, k1, k3 (S4)
  Quad<R> cm[3], cc[3], cp[3];
  Quad<R> rc[3][3], rp[3][3];
  uint32_t n = p + plane * (uint32_t)z0;
  // Loads whose values a plane needs right after its barrier (the halo rows,
  // the cell codes) are issued one plane ahead, so that their latency
  // overlaps the previous plane's arithmetic.  The halo prefetch holds one
  // quad per thread: it applies when both rows together have at most kBlock
  // quads, and to passes whose stencil input is a single load (in S2 and S4
  // it is a combination of two or three loads, whose extra registers would
  // cost occupancy).
  constexpr bool kHaloPf = !(STAGE == 2 || STAGE == 4);
  const bool hpf = kHaloPf && 2u * Q <= (uint32_t)kBlock;
  const long long hq = t < Q ? (long long)q0 - (long long)Q + t : (long long)(q0 + kBlock + t - Q);
  const bool hown = hpf && t < 2u * Q && hq >= 0 && hq < (long long)nq;
  const uint32_t hsl = t < Q ? t : t + kBlock;
  Quad<R> hr[3];
  uint32_t codes_nx = 0;
  if (hown) {
#pragma unroll
    for (int v = 0; v < NL; ++v) hr[v] = ldin(v, plane * (uint32_t)z0 + (uint32_t)hq * VW, nullptr);
  }
  auto ld_codes = [&](uint32_t i) -> uint32_t {
    if constexpr (VW == 4) return *reinterpret_cast<const uint32_t*>(a.code + i);
    else return *reinterpret_cast<const uint16_t*>(a.code + i);
  };
  // Passes with a single-load stencil input also keep the x3 window one
  // plane deeper: the plane above is loaded one iteration before its use.
  constexpr bool kDeep = STAGE == 0 || STAGE == 1 || STAGE == 3;
  Quad<R> cn[3];
  if (active) {
    codes_nx = ld_codes(n);
#pragma unroll
    for (int v = 0; v < NL; ++v) {
      cc[v] = ldc(v, z0, n, rc[v]);
      cm[v] = z0 > 0 ? ldc(v, z0 - 1, n - plane, nullptr) : cc[v];
      if constexpr (kDeep) {
        cp[v] = cc[v];
        if (z0 + 1 < m.n3) cp[v] = ldc(v, z0 + 1, n + plane, nullptr);
      }
    }
  }
  for (int z = z0; z < z1; ++z, n += plane) {
    const bool zp_in = z < m.n3 - 1;
    Quad<R>* L = lds + (size_t)((z - z0) & 1) * NL * W;
    Quad<R> ym[3], yp[3];
    R xl[3], xr[3];
    const uint32_t codes = codes_nx;
    if (active) {
      if (z + 1 < z1) codes_nx = ld_codes(n + plane);
#pragma unroll
      for (int v = 0; v < NL; ++v) {
        if constexpr (kDeep) {
          if (z + 2 < m.n3 && z + 1 < z1) cn[v] = ldc(v, z + 2, n + 2u * plane, nullptr);
        } else {
          cp[v] = zp_in ? ldc(v, z + 1, n + plane, rp[v]) : cc[v];
        }
        L[v * W + Q + t] = cc[v];
      }
    }
    // the rows below and above the run, in this plane
    const uint32_t zoff = plane * (uint32_t)z;
    if (hpf) {
      if (hown) {
#pragma unroll
        for (int v = 0; v < NL; ++v) {
          L[v * W + hsl] = hr[v];
          if (z + 1 < z1) hr[v] = ldin(v, zoff + plane + (uint32_t)hq * VW, nullptr);
        }
      }
    } else {
      for (uint32_t h = t; h < 2u * Q; h += kBlock) {
        const long long hh = h < Q ? (long long)q0 - (long long)Q + h : (long long)(q0 + kBlock + h - Q);
        if (hh >= 0 && hh < (long long)nq) {
          const uint32_t sl = h < Q ? h : h + kBlock;
#pragma unroll
          for (int v = 0; v < NL; ++v)
            L[v * W + sl] = ldin(v, zoff + (uint32_t)hh * (uint32_t)VW, nullptr);
        }
      }
    }
    __syncthreads();
    // x neighbours of the end cells: adjacent lanes, or LDS across waves
#pragma unroll
    for (int v = 0; v < NL; ++v) {
      xl[v] = shfl_up1(cc[v].v[VW - 1]);
      xr[v] = shfl_down1(cc[v].v[0]);
      if (active && xm_remote) xl[v] = L[v * W + Q + t - 1].v[VW - 1];
      if (active && xp_remote) xr[v] = L[v * W + Q + t + 1].v[0];
      // a boundary face carries the cell's own value
      if (!xm_in) xl[v] = cc[v].v[0];
      if (!xp_in) xr[v] = cc[v].v[VW - 1];
      ym[v] = L[v * W + sym];
      yp[v] = L[v * W + syp];
    }
    if (active) {
      const unsigned inb_c = (ym_in ? 4u : 0u) | (yp_in ? 8u : 0u) | (z > 0 ? 16u : 0u) |
                             (zp_in ? 32u : 0u);
      // Dirichlet faces on the x2 and x3 sides, shared by the quad's cells
      const unsigned nd_c = __builtin_popcount(~inb_c & dirf & 60u);
      Quad<R> kq[2];
#pragma unroll
      for (int k = 0; k < VW; ++k) {
        const unsigned inb =
            inb_c | ((k > 0 || xm_in) ? 1u : 0u) | ((k < VW - 1 || xp_in) ? 2u : 0u);
        const unsigned code = (codes >> (8 * k)) & 0xffu;
        R phn[6], thn[6];
        phn[0] = k > 0 ? cc[0].v[k - 1] : xl[0];
        phn[1] = k < VW - 1 ? cc[0].v[k + 1] : xr[0];
        phn[2] = ym[0].v[k];
        phn[3] = yp[0].v[k];
        phn[4] = cm[0].v[k];
        phn[5] = cp[0].v[k];
        if (kCoupled) {
          thn[0] = k > 0 ? cc[1].v[k - 1] : xl[1];
          thn[1] = k < VW - 1 ? cc[1].v[k + 1] : xr[1];
          thn[2] = ym[1].v[k];
          thn[3] = yp[1].v[k];
          thn[4] = cm[1].v[k];
          thn[5] = cp[1].v[k];
        } else {
#pragma unroll
          for (int f = 0; f < 6; ++f) thn[f] = R(0);
        }
        R kp, kt;
        if constexpr (SMOOTH) {
          const R Gc = cc[NV].v[k];
          R Gn[6];
          Gn[0] = k > 0 ? cc[NV].v[k - 1] : xl[NV];
          Gn[1] = k < VW - 1 ? cc[NV].v[k + 1] : xr[NV];
          Gn[2] = ym[NV].v[k];
          Gn[3] = yp[NV].v[k];
          Gn[4] = cm[NV].v[k];
          Gn[5] = cp[NV].v[k];
          // Temp model: the single unknown (theta) travels in the first slot
          if (MODEL == PF_MODEL_TEMP)
            CellRHSSmooth<R, MODEL, REACT>::eval(m, R(0), cc[0].v[k], thn, phn, Gc, Gn, inb,
                                                 dirf, thD, kt, kp);
          else
            CellRHSSmooth<R, MODEL, REACT>::eval(m, cc[0].v[k], kCoupled ? cc[1].v[k] : R(0),
                                                 phn, thn, Gc, Gn, inb, dirf, thD, kp, kt);
        } else if constexpr (MODEL == PF_MODEL_TEMP) {
          // Temp model: the single unknown (theta) travels in the first slot
          CellRHS<R, MODEL, REACT>::eval(m, cc[0].v[k], R(0), phn, thn, code, inb, dirf, thD, kp,
                                         kt);
        } else {
          const unsigned nd = nd_c + ((k == 0 && !xm_in) ? (dirf & 1u) : 0u) +
                              ((k == VW - 1 && !xp_in) ? ((dirf >> 1) & 1u) : 0u);
          CellRHS<R, MODEL, REACT>::eval_nd(m, cc[0].v[k], kCoupled ? cc[1].v[k] : R(0), phn,
                                            thn, code, nd, thD, kp, kt);
        }
        // coupled model: pin the cell's results here; otherwise the heat part
        // of the update is sunk towards the stores after the quad, where the
        // face masks of all four cells are live at once (141-146 VGPRs).  The
        // pin is also a scheduling barrier, which costs the latency-bound
        // Allen-Cahn passes of small grids far more than it saves.
        if constexpr (kCoupled) asm volatile("" : "+v"(kp), "+v"(kt));
        kq[0].v[k] = kp;
        kq[1].v[k] = kt;
        // equilibrium measure (no phase-field equation in the Temp model)
        if (STAGE == 1 && MODEL != PF_MODEL_TEMP && !(code & kGlassBit))
          red1 = dmax_nf(red1, fabs(kp));
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const Quad<R>& kk = kq[v];
        Quad<R> o;
        if (STAGE == 0) {
          stq_s<NT>(out[v], n, kk);
        } else if (STAGE == 1) {
          stq_s<NT>(k1[v], n, kk);
        } else if (STAGE == 2) {
          const Quad<R>& q1 = rc[v][1];
#pragma unroll
          for (int k = 0; k < VW; ++k)
            o.v[k] = cc[v].v[k] + rdt * (R(1.0 / 6.0) * (kk.v[k] - q1.v[k]));
          stq_s<NT>(out[v], n, o);
        } else if (STAGE == 3) {
          stq_s<NT>(k3[v], n, kk);
        } else if (STAGE == 4) {
          const Quad<R>&y0 = rc[v][0], &q1 = rc[v][1], &q3 = rc[v][2];
          Quad<R> P, Cc;
#pragma unroll
          for (int k = 0; k < VW; ++k) {
            o.v[k] = y0.v[k] + rdt * (R(0.5) * q1.v[k] - R(1.5) * q3.v[k] + R(2) * kk.v[k]);
            P.v[k] = y0.v[k] + rdt * (R(1.0 / 6.0) * (q1.v[k] + R(4) * kk.v[k]));
            Cc.v[k] = rdt * (R(1.0 / 30.0) * (R(2) * q1.v[k] - R(9) * q3.v[k] + R(8) * kk.v[k]));
          }
          stq_s<NT>(out[v], n, o);
          stq_s<NT>(ynew[v], n, P);
          stq_s<NT>(cb[v], n, Cc);
        } else if (STAGE == 5) {
          const Quad<R> P = ldq_s<NT>(k1[v], n), Cc = ldq_s<NT>(k3[v], n);
#pragma unroll
          for (int k = 0; k < VW; ++k) {
            o.v[k] = P.v[k] + rdt * (R(1.0 / 6.0) * kk.v[k]);
            const double e = (double)Cc.v[k] - dt * ((1.0 / 30.0) * (double)kk.v[k]);
            red0 = dmax_nf(red0, fabs(e));
          }
          stq_s<NT>(out[v], n, o);
        }
      }
#pragma unroll
      for (int v = 0; v < NL; ++v) {
        cm[v] = cc[v];
        cc[v] = cp[v];
        if constexpr (kDeep) {
          if (z + 2 < m.n3) cp[v] = cn[v];  // else cp stays the new cc
        }
        if constexpr (STAGE == 2) rc[v][1] = rp[v][1];
        if constexpr (STAGE == 4) {
#pragma unroll
          for (int r = 0; r < 3; ++r) rc[v][r] = rp[v][r];
        }
      }
    }
  }
  if (STAGE == 1) red0 = (double)red1;
  // the plane buffers are reused by the next tile of a persistent block
  __syncthreads();
  if (STAGE == 1) {
    // the sums of the state (phi, enthalpy, ice) are not needed per step:
    // runs report them from a diagnostics pass over the final state
    double v[1] = {red0};
    const int ops[1] = {1};
    block_reduce<1>(v, ops, smem);
    if (threadIdx.x == 0)
      for (int i = 0; i < 4; ++i) a.part[(size_t)slot * kPartS1 + i] = i == 0 ? v[0] : 0.0;
    __syncthreads();  // smem is reused by the next tile of a persistent block
  } else if (STAGE == 5) {
    double v[1] = {red0};
    const int ops[1] = {1};
    block_reduce<1>(v, ops, smem);
    s5_partial(a, slot, v[0], smem);
    __syncthreads();
  }
}

template <typename R, int MODEL, int STAGE, bool NT = false, int REACT = PF_REACT_SIGMA,
          int SMOOTH = 0>
__global__ __launch_bounds__(kBlock) void stage4_kernel(StageArgs a) {
  __shared__ double smem[8 * kWaves];
  extern __shared__ __align__(16) unsigned char pf_stage_lds[];
  stage4_tile<R, MODEL, STAGE, NT, REACT, SMOOTH>(a, xcd_tile(blockIdx.x, gridDim.x), blockIdx.x,
                                                  smem, pf_stage_lds);
}

// ---------------------------------------------------------------------------
// Paired-stage kernel: two consecutive Merson stages in one pass.
//
//   FIRST = 1: S1 on the tile plus a one-cell ring (y -> k1, Y2), then S2 on
//              the tile (Y2 -> k2, Y3 = Y2 + dt (k2 - k1)/6).  Y2 never leaves
//              LDS; k1 and Y3 go to HBM.
//   FIRST = 3: S3 on tile + ring (Y3 -> k3, Y4), then S4 on the tile
//              (Y4 -> k4; Y5, P, C).  Y4 and k3 never leave the workgroup.
//
// A workgroup owns a TX x TY tile of the x1-x2 plane and marches z_chunk
// planes along x3.  Plane j of the first stage's stencil input is staged in
// LDS over the tile plus a two-cell ring (three planes rotate); the first
// stage is evaluated on the tile plus a one-cell ring of plane j and its
// output (the second stage's input) is kept in LDS (three planes rotate); the
// second stage then runs on plane j-1.  The ring is recomputed by the
// neighbouring tiles: (TX+2)(TY+2)/(TX TY) first-stage evaluations per cell.
// Per unknown and cell the pass moves: first pair r y, w k1, Y3 (3 words);
// second pair r Y3, y, k1, w Y5, P, C (6 words) -- 9 words against 15 for the
// same four stages one pass each.
//
// Buffers that a pass writes are never read by the same pass (neighbouring
// workgroups read rings of the inputs concurrently): Y3 -> B, Y5 -> A,
// P -> K3, C -> the free state slot y[1-cur], which S5 then overwrites in
// place with y_new.

template <int TX, int TY>
__device__ __forceinline__ void ring_cell(int k, int& lx, int& ly) {
  // k-th cell of the one-cell ring around the tile, in ring-local
  // coordinates (0..TX+1, 0..TY+1)
  if (k < TX + 2) {
    lx = k;
    ly = 0;
  } else if (k < 2 * (TX + 2)) {
    lx = k - (TX + 2);
    ly = TY + 1;
  } else {
    const int r = k - 2 * (TX + 2);
    lx = (r < TY) ? 0 : TX + 1;
    ly = 1 + (r < TY ? r : r - TY);
  }
}

template <typename R, int MODEL, int FIRST, int TX, int TY>
__global__ __launch_bounds__(TX* TY) void pair_kernel(PairArgs a) {
  constexpr int NT = TX * TY;
  constexpr bool kCoupled = MODEL == PF_MODEL_COUPLED;
  constexpr int NV = kCoupled ? 2 : 1;
  constexpr int W2 = TX + 4, H2 = TY + 4, N2 = W2 * H2;  // staged input region
  constexpr int W1 = TX + 2, H1 = TY + 2, N1 = W1 * H1;  // first-stage region
  __shared__ R inS[3][NV][N2];
  __shared__ R midS[3][NV][N1];
  __shared__ double smem[8 * (NT / 64)];

  const ModelConst& m = a.mc;
  if (a.ctl->done) return;
  const double t0 = a.ctl->t;
  const double dt = a.ctl->dt_att;
  const int cur = a.ctl->cur;
  const double tA = t0 + (FIRST == 1 ? 0.0 : dt / 3.0);
  const double tB = t0 + (FIRST == 1 ? dt / 3.0 : 0.5 * dt);
  const R thDA = R(dirichlet_theta(m, tA));
  const R thDB = R(dirichlet_theta(m, tB));
  const R rdt = R(dt);

  const int nblk = gridDim.x;
  const int tile = xcd_tile(blockIdx.x, nblk);
  const int tx = tile % a.tiles_x;
  const int rest = tile / a.tiles_x;
  const int ty = rest % a.tiles_y;
  const int tz = rest / a.tiles_y;
  const int x0 = tx * TX, y0 = ty * TY;
  const int z0 = tz * a.z_chunk;
  const int z1 = min(z0 + a.z_chunk, m.n3);
  const int n1 = m.n1, n2 = m.n2, n3 = m.n3;
  const int plane = n1 * n2;
  const unsigned dirf = (unsigned)m.dirichlet_faces;

  const R* src[2];
  if (FIRST == 1) {
    src[0] = static_cast<const R*>(a.y[cur][0]);
    src[1] = static_cast<const R*>(a.y[cur][1]);
  } else {
    src[0] = static_cast<const R*>(a.in[0]);
    src[1] = static_cast<const R*>(a.in[1]);
  }
  const R* yv[2] = {static_cast<const R*>(a.y[cur][0]), static_cast<const R*>(a.y[cur][1])};
  R* k1g[2] = {static_cast<R*>(a.k1[0]), static_cast<R*>(a.k1[1])};
  R* oa[2] = {static_cast<R*>(a.out_a[0]), static_cast<R*>(a.out_a[1])};
  R* op[2] = {static_cast<R*>(a.out_p[0]), static_cast<R*>(a.out_p[1])};
  // C goes to the free state slot (FIRST == 3)
  R* oc[2] = {static_cast<R*>(const_cast<void*>(a.y[1 - cur][0])),
              static_cast<R*>(const_cast<void*>(a.y[1 - cur][1]))};

  // this thread's tile cell
  const int tid = threadIdx.x;
  const int cx = tid % TX, cy = tid / TX;
  const int gx = x0 + cx, gy = y0 + cy;
  const bool own = gx < n1 && gy < n2;
  const int cidx1 = (cy + 1) * W1 + (cx + 1);  // in the first-stage region

  // values of the own cell carried from the first stage (plane j) to the
  // second (plane j, one iteration later)
  R c_k[NV], c_y[NV], c_k1[NV];   // plane being produced
  R p_k[NV], p_y[NV], p_k1[NV];   // plane consumed by the second stage
  unsigned c_code = 0, p_code = 0;
#pragma unroll
  for (int v = 0; v < NV; ++v) c_k[v] = c_y[v] = c_k1[v] = p_k[v] = p_y[v] = p_k1[v] = R(0);

  double red0 = 0.0;

  auto load_plane = [&](int p) {
    const int s = ((p % 3) + 3) % 3;
    for (int i = tid; i < N2; i += NT) {
      const int lx = i % W2, ly = i / W2;
      const int qx = x0 + lx - 2, qy = y0 + ly - 2;
      const bool ok = qx >= 0 && qx < n1 && qy >= 0 && qy < n2;
      const int n = ok ? qx + n1 * qy + plane * p : 0;
#pragma unroll
      for (int v = 0; v < NV; ++v) inS[s][v][i] = ok ? src[v][n] : R(0);
    }
  };

  if (z0 - 2 >= 0) load_plane(z0 - 2);
  if (z0 - 1 >= 0) load_plane(z0 - 1);

  for (int j = z0 - 1; j <= z1; ++j) {
    if (j + 1 < n3 && j + 1 >= 0) load_plane(j + 1);
    __syncthreads();
    // ---- first stage at plane j over tile + ring
    if (j >= 0 && j < n3) {
      const int sm = (((j - 1) % 3) + 3) % 3, s0 = j % 3, sp = (j + 1) % 3;
      const bool zin_m = j > 0, zin_p = j < n3 - 1;
      for (int item = tid; item < N1; item += NT) {
        int lx, ly;
        if (item < NT) {
          lx = 1 + item % TX;
          ly = 1 + item / TX;
        } else {
          ring_cell<TX, TY>(item - NT, lx, ly);
        }
        const int qx = x0 + lx - 1, qy = y0 + ly - 1;
        const int i1 = ly * W1 + lx;
        const bool ok = qx >= 0 && qx < n1 && qy >= 0 && qy < n2;
        if (!ok) {
#pragma unroll
          for (int v = 0; v < NV; ++v) midS[s0][v][i1] = R(0);
          continue;
        }
        const int i2 = (ly + 1) * W2 + (lx + 1);
        const int n = qx + n1 * qy + plane * j;
        const unsigned code = a.code[n];
        const unsigned inb = (qx > 0 ? 1u : 0u) | (qx < n1 - 1 ? 2u : 0u) |
                             (qy > 0 ? 4u : 0u) | (qy < n2 - 1 ? 8u : 0u) |
                             (zin_m ? 16u : 0u) | (zin_p ? 32u : 0u);
        R ctr[2], nb[2][6];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          // a boundary face carries the cell's own value
          ctr[v] = inS[s0][v][i2];
          nb[v][0] = (inb & 1u) ? inS[s0][v][i2 - 1] : ctr[v];
          nb[v][1] = (inb & 2u) ? inS[s0][v][i2 + 1] : ctr[v];
          nb[v][2] = (inb & 4u) ? inS[s0][v][i2 - W2] : ctr[v];
          nb[v][3] = (inb & 8u) ? inS[s0][v][i2 + W2] : ctr[v];
          nb[v][4] = zin_m ? inS[sm][v][i2] : ctr[v];
          nb[v][5] = zin_p ? inS[sp][v][i2] : ctr[v];
        }
        if (!kCoupled) {
          ctr[1] = R(0);
#pragma unroll
          for (int f = 0; f < 6; ++f) nb[1][f] = R(0);
        }
        R kp, kt;
        CellRHS<R, MODEL>::eval(m, ctr[0], ctr[1], nb[0], nb[1], code, inb, dirf, thDA, kp, kt);
        const R kk[2] = {kp, kt};
        const bool mine = item < NT;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          if (FIRST == 1) {
            midS[s0][v][i1] = ctr[v] + rdt * (R(1.0 / 3.0) * kk[v]);
            if (mine) {
              c_k[v] = kk[v];
              c_y[v] = ctr[v];
            }
          } else {
            const R y0v = yv[v][n], k1v = k1g[v][n];
            midS[s0][v][i1] = y0v + rdt * (R(0.125) * (k1v + R(3) * kk[v]));
            if (mine) {
              c_k[v] = kk[v];
              c_y[v] = y0v;
              c_k1[v] = k1v;
            }
          }
        }
        if (mine) {
          c_code = code;
          if (FIRST == 1 && j >= z0 && j < z1) {
            // k1 to HBM and the equilibrium measure (own planes only)
#pragma unroll
            for (int v = 0; v < NV; ++v) k1g[v][n] = kk[v];
            if (!(code & kGlassBit)) red0 = dmax_nf(red0, fabs((double)kp));
          }
        }
      }
    }
    __syncthreads();
    // ---- second stage at plane q = j - 1 over the tile
    const int q = j - 1;
    if (q >= z0 && q < z1 && own) {
      const int sm = (((q - 1) % 3) + 3) % 3, s0 = ((q % 3) + 3) % 3, sp = (q + 1) % 3;
      const bool zin_m = q > 0, zin_p = q < n3 - 1;
      const unsigned inb = (gx > 0 ? 1u : 0u) | (gx < n1 - 1 ? 2u : 0u) |
                           (gy > 0 ? 4u : 0u) | (gy < n2 - 1 ? 8u : 0u) |
                           (zin_m ? 16u : 0u) | (zin_p ? 32u : 0u);
      R ctr[2], nb[2][6];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        ctr[v] = midS[s0][v][cidx1];
        nb[v][0] = (inb & 1u) ? midS[s0][v][cidx1 - 1] : ctr[v];
        nb[v][1] = (inb & 2u) ? midS[s0][v][cidx1 + 1] : ctr[v];
        nb[v][2] = (inb & 4u) ? midS[s0][v][cidx1 - W1] : ctr[v];
        nb[v][3] = (inb & 8u) ? midS[s0][v][cidx1 + W1] : ctr[v];
        nb[v][4] = zin_m ? midS[sm][v][cidx1] : ctr[v];
        nb[v][5] = zin_p ? midS[sp][v][cidx1] : ctr[v];
      }
      if (!kCoupled) {
        ctr[1] = R(0);
#pragma unroll
        for (int f = 0; f < 6; ++f) nb[1][f] = R(0);
      }
      R kp, kt;
      CellRHS<R, MODEL>::eval(m, ctr[0], ctr[1], nb[0], nb[1], p_code, inb, dirf, thDB, kp, kt);
      const R kk[2] = {kp, kt};
      const int n = gx + n1 * gy + plane * q;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (FIRST == 1) {
          oa[v][n] = ctr[v] + rdt * (R(1.0 / 6.0) * (kk[v] - p_k[v]));
        } else {
          const R k1v = p_k1[v], k3v = p_k[v], y0v = p_y[v];
          oa[v][n] = y0v + rdt * (R(0.5) * k1v - R(1.5) * k3v + R(2) * kk[v]);
          op[v][n] = y0v + rdt * (R(1.0 / 6.0) * (k1v + R(4) * kk[v]));
          oc[v][n] = rdt * (R(1.0 / 30.0) * (R(2) * k1v - R(9) * k3v + R(8) * kk[v]));
        }
      }
    }
    // rotate the own-cell carry
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      p_k[v] = c_k[v];
      p_y[v] = c_y[v];
      p_k1[v] = c_k1[v];
    }
    p_code = c_code;
  }

  if (FIRST == 1) {
    // wavefront xor trees, then the waves in order (fixed order: bitwise
    // reproducible)
    constexpr int NW = NT / 64;
    double v[4] = {red0, 0.0, 0.0, 0.0};  // per-step sums of the state are not needed
    const int ops[4] = {1, 0, 0, 0};
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      v[jj] = ops[jj] ? wave_reduce<1>(v[jj]) : wave_reduce<0>(v[jj]);
      if (lane == 0) smem[jj * NW + wave] = v[jj];
    }
    __syncthreads();
    if (tid == 0) {
      for (int jj = 0; jj < 4; ++jj) {
        double acc = smem[jj * NW];
        for (int w = 1; w < NW; ++w) {
          const double o = smem[jj * NW + w];
          acc = ops[jj] ? (o > acc ? o : acc) : acc + o;
        }
        a.part[(size_t)blockIdx.x * kPartS1 + jj] = acc;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Host launchers

int grid_blocks(const ModelConst& mc, int z_chunk, int cells, int* tiles_p, int* tiles_z) {
  const long long plane = (long long)mc.n1 * mc.n2;
  const long long per = (long long)cells * kBlock;
  *tiles_p = (int)((plane + per - 1) / per);
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

template <typename R, int MODEL, int REACT, int SMOOTH>
static hipError_t launch_scalar_t(int stage, const StageArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)(a.tiles_p * a.tiles_z)), block(kBlock);
  switch (stage) {
    case 0: hipLaunchKernelGGL((stage_kernel<R, MODEL, 0, REACT, SMOOTH>), grid, block, 0, s, a); break;
    case 1: hipLaunchKernelGGL((stage_kernel<R, MODEL, 1, REACT, SMOOTH>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((stage_kernel<R, MODEL, 2, REACT, SMOOTH>), grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL((stage_kernel<R, MODEL, 3, REACT, SMOOTH>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((stage_kernel<R, MODEL, 4, REACT, SMOOTH>), grid, block, 0, s, a); break;
    case 5: hipLaunchKernelGGL((stage_kernel<R, MODEL, 5, REACT, SMOOTH>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// GradP or the smooth glass field: one-cell-per-thread kernels only
template <typename R, int MODEL>
static hipError_t launch_simple_t(int stage, const StageArgs& a, hipStream_t s) {
  if (a.vec || (a.mc.smooth && !a.G)) return hipErrorInvalidValue;
  if (a.mc.reaction == PF_REACT_GRADP)
    return a.mc.smooth ? launch_scalar_t<R, MODEL, PF_REACT_GRADP, 1>(stage, a, s)
                       : launch_scalar_t<R, MODEL, PF_REACT_GRADP, 0>(stage, a, s);
  return a.mc.smooth ? launch_scalar_t<R, MODEL, PF_REACT_SIGMA, 1>(stage, a, s)
                     : launch_scalar_t<R, MODEL, PF_REACT_SIGMA, 0>(stage, a, s);
}

template <typename R, int MODEL, int REACT, int SMOOTH>
static hipError_t launch_vector_t(int stage, const StageArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)(a.tiles_p * a.tiles_z)), block(kBlock);
  const size_t lds =
      stage4_lds_bytes(a.mc.n1, (MODEL == PF_MODEL_COUPLED ? 2 : 1) + SMOOTH, sizeof(R));
  if (lds > kStage4MaxLds || (SMOOTH && !a.G)) return hipErrorInvalidValue;
#define PF_S4(S)                                                                        \
  do {                                                                                  \
    if (a.stream_nt)                                                                    \
      hipLaunchKernelGGL((stage4_kernel<R, MODEL, S, true, REACT, SMOOTH>), grid, block,  \
                         lds, s, a);                                                    \
    else                                                                                \
      hipLaunchKernelGGL((stage4_kernel<R, MODEL, S, false, REACT, SMOOTH>), grid, block, \
                         lds, s, a);                                                    \
  } while (0)
  switch (stage) {
    case 0: PF_S4(0); break;
    case 1: PF_S4(1); break;
    case 2: PF_S4(2); break;
    case 3: PF_S4(3); break;
    case 4: PF_S4(4); break;
    case 5: PF_S4(5); break;
    default: return hipErrorInvalidValue;
  }
#undef PF_S4
  return hipGetLastError();
}

template <typename R, int MODEL, int SMOOTH>
static hipError_t launch_vector_m(int stage, const StageArgs& a, hipStream_t s) {
  if constexpr (MODEL == PF_MODEL_TEMP) {
    return launch_vector_t<R, MODEL, PF_REACT_SIGMA, SMOOTH>(stage, a, s);
  } else {
    if (a.mc.reaction != PF_REACT_GRADP)
      return launch_vector_t<R, MODEL, PF_REACT_SIGMA, SMOOTH>(stage, a, s);
    return launch_vector_t<R, MODEL, PF_REACT_GRADP, SMOOTH>(stage, a, s);
  }
}

template <typename R, int MODEL>
static hipError_t launch_stage_t(int stage, const StageArgs& a, hipStream_t s) {
  if (a.vec)
    return a.mc.smooth ? launch_vector_m<R, MODEL, 1>(stage, a, s)
                       : launch_vector_m<R, MODEL, 0>(stage, a, s);
  if (a.mc.smooth || a.mc.reaction == PF_REACT_GRADP || MODEL == PF_MODEL_TEMP)
    return launch_simple_t<R, MODEL>(stage, a, s);
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

int pair_blocks(const ModelConst& mc, int ts, int z_chunk, int* tx, int* ty, int* tz) {
  const int TX = kPairTiles[ts][0], TY = kPairTiles[ts][1];
  *tx = (mc.n1 + TX - 1) / TX;
  *ty = (mc.n2 + TY - 1) / TY;
  *tz = (mc.n3 + z_chunk - 1) / z_chunk;
  return (*tx) * (*ty) * (*tz);
}

template <typename R, int MODEL, int TX, int TY>
static hipError_t launch_pair_t(int first, const PairArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)(a.tiles_x * a.tiles_y * a.tiles_z)), block(TX * TY);
  if (first == 1)
    hipLaunchKernelGGL((pair_kernel<R, MODEL, 1, TX, TY>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((pair_kernel<R, MODEL, 3, TX, TY>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <typename R, int MODEL>
static hipError_t launch_pair_m(int first, int ts, const PairArgs& a, hipStream_t s) {
  switch (ts) {
    case 0: return launch_pair_t<R, MODEL, 64, 4>(first, a, s);
    case 1: return launch_pair_t<R, MODEL, 64, 8>(first, a, s);
    case 2: return launch_pair_t<R, MODEL, 32, 8>(first, a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pair(int precision, int model, int first, int ts, const PairArgs& a,
                       hipStream_t s) {
  if (precision == PF_FP64) {
    if (model == PF_MODEL_AC) return launch_pair_m<double, PF_MODEL_AC>(first, ts, a, s);
    if (model == PF_MODEL_COUPLED) return launch_pair_m<double, PF_MODEL_COUPLED>(first, ts, a, s);
  } else {
    if (model == PF_MODEL_AC) return launch_pair_m<float, PF_MODEL_AC>(first, ts, a, s);
    if (model == PF_MODEL_COUPLED) return launch_pair_m<float, PF_MODEL_COUPLED>(first, ts, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_stage(int precision, int model, int stage, const StageArgs& a, hipStream_t s) {
  if (model == PF_MODEL_TEMP && a.mc.reaction != PF_REACT_SIGMA) return hipErrorInvalidValue;
  if (precision == PF_FP64) {
    if (model == PF_MODEL_AC) return launch_stage_t<double, PF_MODEL_AC>(stage, a, s);
    if (model == PF_MODEL_COUPLED) return launch_stage_t<double, PF_MODEL_COUPLED>(stage, a, s);
    if (model == PF_MODEL_TEMP) return launch_stage_t<double, PF_MODEL_TEMP>(stage, a, s);
  } else {
    if (model == PF_MODEL_AC) return launch_stage_t<float, PF_MODEL_AC>(stage, a, s);
    if (model == PF_MODEL_COUPLED) return launch_stage_t<float, PF_MODEL_COUPLED>(stage, a, s);
    if (model == PF_MODEL_TEMP) return launch_stage_t<float, PF_MODEL_TEMP>(stage, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_controller(DevCtl* ctl, const double* part1, int np1, const double* part5,
                             int np5, double h3, hipStream_t s) {
  hipLaunchKernelGGL(controller_kernel, dim3(1), dim3(256), 0, s, ctl, part1, np1, part5, np5,
                     h3);
  return hipGetLastError();
}

hipError_t launch_diag(int precision, int model, const uint8_t* code, const void* G,
                       const void* phi, const void* th, const ModelConst& m, long long n,
                       double* part, int nparts, double* out4, hipStream_t s) {
  const dim3 grid((unsigned)nparts), block(kBlock);
  if (precision == PF_FP64) {
    if (model == PF_MODEL_COUPLED)
      hipLaunchKernelGGL((diag_kernel<double, PF_MODEL_COUPLED>), grid, block, 0, s, code,
                         (const double*)G, (const double*)phi, (const double*)th, m, n, part);
    else if (model == PF_MODEL_TEMP)
      hipLaunchKernelGGL((diag_kernel<double, PF_MODEL_TEMP>), grid, block, 0, s, code,
                         (const double*)G, (const double*)phi, (const double*)th, m, n, part);
    else
      hipLaunchKernelGGL((diag_kernel<double, PF_MODEL_AC>), grid, block, 0, s, code,
                         (const double*)G, (const double*)phi, (const double*)th, m, n, part);
  } else {
    if (model == PF_MODEL_COUPLED)
      hipLaunchKernelGGL((diag_kernel<float, PF_MODEL_COUPLED>), grid, block, 0, s, code,
                         (const float*)G, (const float*)phi, (const float*)th, m, n, part);
    else if (model == PF_MODEL_TEMP)
      hipLaunchKernelGGL((diag_kernel<float, PF_MODEL_TEMP>), grid, block, 0, s, code,
                         (const float*)G, (const float*)phi, (const float*)th, m, n, part);
    else
      hipLaunchKernelGGL((diag_kernel<float, PF_MODEL_AC>), grid, block, 0, s, code,
                         (const float*)G, (const float*)phi, (const float*)th, m, n, part);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(256), 0, s, part, nparts, m.h3, out4);
  return hipGetLastError();
}

}  // namespace pf

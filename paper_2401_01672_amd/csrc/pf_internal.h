// Internal declarations shared by the HIP translation units of libpf.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "pf.h"

namespace pf {

// Threads per stencil workgroup: one cell of a 256-cell run of the x1-x2
// plane per thread; the workgroup then marches along x3.
constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

// The vector stage kernels give each thread one 16-byte vector of cells.
constexpr int vec_cells(int esize) { return 16 / esize; }
// Their dynamic LDS: two plane buffers of kBlock + 2 n1/vec_cells vectors
// per unknown (the workgroup's run and the rows on either side).
inline size_t stage4_lds_bytes(int n1, int nvar, int esize) {
  return 2u * (size_t)nvar * (size_t)(kBlock + 2 * (n1 / vec_cells(esize))) * 16u;
}
constexpr size_t kStage4MaxLds = 65536;

// Per-cell neighbourhood code (one byte, static): bit f (f = 0..5 for faces
// x1-,x1+,x2-,x2+,x3-,x3+) is set when the neighbour through face f exists
// and is water; bit 6 is set when the cell itself is glass.
constexpr uint8_t kGlassBit = 1u << 6;

// Device-resident step control.  The stage kernels read it; only the
// controller kernel (one thread) writes it, so a run of steps needs no host
// round trip.
struct DevCtl {
  double t;          // current time
  double dt_att;     // step of the pending attempt (clipped to t_end)
  double dt_nom;     // proposed step before clipping
  double t_end;
  double tol, safety, dt_min, dt_max, eq_tol;
  double eps;        // last error norm
  double maxk1;      // last max over water cells of |k1_phi|
  double sum_phi, enthalpy, ice;  // unused (0): runs take them from a diagnostics pass
  double dt_used;    // step of the last attempt
  long long n_acc, n_rej, max_steps;
  int cur;           // which of the two state buffers holds y
  int done;          // nonzero: the run has ended; kernels return at once
  int status;        // PF_* code of the run
  int clipped;       // the pending attempt lands exactly on t_end
  int accepted;      // last attempt accepted
  int pad[3];
};

// Model constants, precomputed on the host in FP64 (cast per kernel).
struct ModelConst {
  int n1, n2, n3;
  int dirichlet_faces;
  int bc_kind;
  int model;
  double cL;        // 1/(alpha h^2): Laplacian weight of the phase equation
  double cR;        // 1/(alpha xi^2): reaction weight
  double beta0;     // xi b mu alpha / 2
  double betaAC;    // beta0 * dT (micro-scale model)
  double e0, inv_de;// Sigma limiter: eps0 and 1/(eps1 - eps0)
  double iw_glass;  // water indicator of a glass cell: max(0, 1 - zeta)
  double cH;        // 1/h^2
  double lamL, dlam, lamG;   // lambda_L, lambda_I - lambda_L, lambda_G
  double rcL, drc, rcG;      // rho c likewise
  double Lv;
  // the paper's material model (pf_params.rho_c_separate): rho and c
  // blended separately, rho c = rho c of the blends, latent term rho L
  int sep;
  double rhoL, drho, rhoG;   // density
  double csL, dcs, csG;      // specific heat
  double Lm;                 // specific latent heat
  double bc_T0, bc_T1, bc_t0, bc_t1;  // Dirichlet schedule (theta units)
  double h3;        // h^3 for the enthalpy
  double gamma;     // Temp model
  double dT;        // supercooling of the micro-scale model (theta = -dT)
  int reaction;     // PF_REACT_SIGMA or PF_REACT_GRADP
  int smooth;       // 1: smooth glass field G (paper mode), 0: binary mask
  double zeta;      // water indicator I_W(G) = max(0, 1 - zeta G)
  double gpc;       // GradP drive coefficient xi^2 mu alpha
  double inv_h;     // 1/h (GradP gradient)
};

struct Buffers {
  void* y[2][2];     // [buffer][var]: state double buffer
  void* a[2];        // stage inputs Y2 / Y4
  void* b[2];        // stage inputs Y3 / Y5
  void* k1[2];       // k1, then P
  void* k3[2];       // k3, then C
};

// Arguments of a stage kernel (passed by value).
struct StageArgs {
  const uint8_t* code;
  const void* G;      // smooth glass field (paper mode), in the field precision; else null
  DevCtl* ctl;
  double* part;       // per-workgroup partial reductions
  const void* in[2];  // stage input (stencil), per variable
  const void* y[2][2];// both state buffers
  void* k1[2];
  void* k3[2];
  void* out[2];       // stored stage value written by the pass
  void* out_y[2][2];  // both state buffers as destinations (S5: y_new)
  void* cbuf[2];      // vector passes: error combination C (S4 -> S5)
  ModelConst mc;
  int z_chunk;
  int tiles_p, tiles_z;  // workgroup grid: plane tiles x z chunks
  int ignore_done;       // standalone RHS: ignore ctl
  int c_from_out;        // S5: C is read from the y_new slot (paired schedule)
  int vec;               // 1: four x1-cells per thread (needs n1 % 4 == 0)
  int stream_nt;         // 1: non-temporal loads/stores of the streamed fields
  double t_fixed;        // standalone RHS time
  // S5 only: the step controller folded into the pass (fold = 1): the
  // fold_np5 workgroup maxima are combined atomically in fold_acc and
  // counted in fold_ctr (both zero between passes), and the workgroup that
  // completes the count runs the controller on fold_ctl, with the S1
  // partials fold_p1 [fold_np1].
  int fold;
  int fold_np1, fold_np5;
  const double* fold_p1;
  unsigned* fold_ctr;
  unsigned long long* fold_acc;
  DevCtl* fold_ctl;
};

// Arguments of a paired-stage kernel (S1+S2 or S3+S4 in one pass; see
// pf_stencil.hip).  Buffers per variable v.
struct PairArgs {
  const uint8_t* code;
  DevCtl* ctl;
  double* part;          // S1 partial reductions (first pair only)
  const void* y[2][2];   // both state buffers
  const void* in[2];     // second pair: Y3 (stencil input of S3)
  void* k1[2];           // first pair writes k1, second pair reads it
  void* out_a[2];        // first pair: Y3; second pair: Y5
  void* out_p[2];        // second pair: P
  ModelConst mc;
  int z_chunk;
  int tiles_x, tiles_y, tiles_z;
};

// One instance of a batched sweep (device-resident table, one per instance).
struct BatchDesc {
  StageArgs st[5];      // per stage; part points at the instance's slots
  const double* p1;     // S1 partials of the instance (ntiles x kPartS1)
  const double* p5;     // S5 partials (ntiles)
  int ntiles;           // work items (stage-pass tiles) of the instance
  double h3;
};

// Stencil schedules of one attempt.
constexpr int kSchedFive = 0;    // S1..S5, one pass each
constexpr int kSchedPaired = 1;  // (S1+S2), (S3+S4), S5

// Partial-reduction slots per workgroup.
constexpr int kPartS1 = 4;  // max |k1_phi| (water); slots 1..3 unused (0)
constexpr int kPartS5 = 1;  // max |E|

}  // namespace pf

// Host-side launchers (pf_stencil.hip).
namespace pf {
hipError_t launch_build_code(const uint8_t* mask, uint8_t* code, int n1, int n2, int n3,
                             hipStream_t s);
hipError_t launch_stage(int precision, int model, int stage, const StageArgs& a,
                        hipStream_t s);
hipError_t launch_controller(DevCtl* ctl, const double* part1, int np1, const double* part5,
                             int np5, double h3, hipStream_t s);
hipError_t launch_diag(int precision, int model, const uint8_t* code, const void* G,
                       const void* phi, const void* th, const ModelConst& m, long long n,
                       double* part, int nparts, double* out4, hipStream_t s);
// workgroups of a stage pass with `cells` x1-cells per thread (1 or vec_cells)
int grid_blocks(const ModelConst& mc, int z_chunk, int cells, int* tiles_p, int* tiles_z);
// paired kernels: tile shape index ts selects (TX, TY) from kPairTiles
constexpr int kPairTiles[3][2] = {{64, 4}, {64, 8}, {32, 8}};
int pair_blocks(const ModelConst& mc, int ts, int z_chunk, int* tx, int* ty, int* tz);
hipError_t launch_pair(int precision, int model, int first, int ts, const PairArgs& a,
                       hipStream_t s);
// batched sweep: cooperative persistent launch; grid_blocks <= batch_max_blocks()
// bar: two zeroed unsigned counters (grid barrier); err: set to 1 when a
// barrier wait overran its bound
// items[i] = (instance, tile); the controllers run for desc[0 .. ninst);
// lds = stage4_lds_bytes of the widest instance
hipError_t launch_batch(int precision, int model, const BatchDesc* desc, const int2* items,
                        int nitems, int ninst, int steps, int grid_blocks, unsigned* bar,
                        unsigned* err, size_t lds, hipStream_t s);
int batch_max_blocks(int precision, int model, size_t lds);
// batched sweep, multi-launch form: one attempt = 5 stage launches over the
// nitems items (S5 runs the controllers folded into it) + with ctl, one
// controller launch over the ninst instances of inst_list for the others;
// smooth: the instances carry the smooth glass field (paper mode)
hipError_t launch_batch_step(int precision, int model, int smooth, const BatchDesc* desc,
                             const int2* items, int nitems, const int* inst_list, int ninst,
                             bool ctl, size_t lds, hipStream_t s);
// control blocks of the instances in inst_list, gathered into out[ninst]
// (one device-to-host copy per poll instead of one per instance)
hipError_t launch_gather_ctl(const BatchDesc* desc, const int* inst_list, int ninst,
                             DevCtl* out, hipStream_t s);
// message returned by pf_last_error(NULL) on the calling thread (calls that
// have no handle to hold it)
void set_thread_error(const std::string& msg);
}  // namespace pf

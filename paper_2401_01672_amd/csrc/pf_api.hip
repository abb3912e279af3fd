// C ABI of libpf (declarations and semantics in include/pf.h).
//
// A handle owns, per unknown (phi and/or theta): the double-buffered state
// y[0]/y[1], two stage-input buffers, and the k1/P and k3/C buffers; plus the
// per-cell neighbourhood code, the per-workgroup partial reductions and the
// device step-control block.  One attempt is five stage kernels and one
// controller kernel, all reading the control block, so a run of attempts is
// issued without host round trips (optionally as a replayed HIP graph) and
// the host only polls the control block between batches of attempts.
#include <float.h>
#include <math.h>
#include <string.h>

#include <array>
#include <chrono>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <algorithm>
#include <vector>

#include "pf_internal.h"
#include "pf_unet_internal.h"

using pf::DevCtl;
using pf::ModelConst;
using pf::StageArgs;

struct pf_handle {
  pf_params P;
  ModelConst mc;
  long long ncell = 0;
  size_t esize = 0;
  int nvar = 0;  // 1: phi (AC) or theta (Temp); 2: phi, theta (coupled)
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  void* slab = nullptr;
  void* G = nullptr;  // smooth glass field (paper mode), field precision; else null
  int smooth = 0;
  uint8_t* code = nullptr;
  void* y[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  void* a[2] = {nullptr, nullptr};
  void* b[2] = {nullptr, nullptr};
  void* k1[2] = {nullptr, nullptr};
  void* k3[2] = {nullptr, nullptr};
  double* part1 = nullptr;
  double* part5 = nullptr;
  double* diag_out = nullptr;
  unsigned* fold_ctr = nullptr;  // device: S5 partials written (controller folded into S5)
  unsigned long long* fold_acc = nullptr;  // device: their running maximum
  DevCtl* ctl = nullptr;   // device
  DevCtl* hctl = nullptr;  // pinned host mirror
  int sched = pf::kSchedFive;
  int vec = 0;  // vector stage kernels (one 16-byte vector of x1-cells per thread)
  int vec_fixed = 0;  // set by pf_set_vector: the autotuner keeps vec
  int stream_nt = 0;  // non-temporal streams: working set far above the caches
  int z_chunk = 16;  // single-stage passes (the RHS pass, batches, uniform choice)
  int tiles_p = 0, tiles_z = 0, nparts = 0, max_parts = 0;
  // per stage pass S1..S5 (index 1..5): planes per workgroup column and grid
  int st_z[6] = {0}, st_tp[6] = {0}, st_tz[6] = {0}, st_np[6] = {0};
  int pair_ts = 1, pair_zc = 16;  // paired passes: tile shape index, planes per column
  int ptx = 0, pty = 0, ptz = 0, npair = 0;
  int autotune_pending = 1;
  int steps_per_poll = 16;
  int use_graph = 1;
  hipGraphExec_t gexec = nullptr;
  int graph_steps = 0;
  double t = 0.0, dt = 0.0;
  int cur = 0;
  std::string err;
  // work tables of pf_batch_integrate calls that list this handle first:
  // kept (grown when a call needs more) so that repeat calls allocate nothing
  struct BatchWork {
    pf::BatchDesc* desc = nullptr;
    int2* items = nullptr;
    int* act = nullptr;
    unsigned* bar = nullptr;
    DevCtl* gath = nullptr;
    DevCtl* hgath = nullptr;  // pinned
    long long cap_items = 0;
    int cap_inst = 0;
    // side streams and fork/join events of a graph with parallel chains
    hipStream_t side[3] = {nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr;
    hipEvent_t join[3] = {nullptr, nullptr, nullptr};
  } bw;
};

namespace {

thread_local std::string g_create_err;

int fail(pf_handle* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  else g_create_err = msg;
  return code;
}

#define PF_HIP(h, expr)                                                              \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail((h), PF_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// The stream a call works on: the caller's (nonzero) or the handle's.  Work
// already issued on the handle's stream is finished first, so a caller
// stream never overtakes it.
hipStream_t work_stream(pf_handle* h, uintptr_t stream);

void fill_model_const(const pf_params& P, ModelConst& m) {
  memset(&m, 0, sizeof(m));
  m.n1 = P.n1;
  m.n2 = P.n2;
  m.n3 = P.n3;
  m.dirichlet_faces = P.dirichlet_faces;
  m.bc_kind = P.bc_kind;
  m.model = P.model;
  m.cL = 1.0 / (P.alpha * P.h * P.h);
  m.cR = 1.0 / (P.alpha * P.xi * P.xi);
  m.beta0 = 0.5 * P.xi * P.b * P.mu * P.alpha;
  m.betaAC = m.beta0 * P.dT;
  m.e0 = P.eps0;
  m.inv_de = 1.0 / (P.eps1 - P.eps0);
  m.iw_glass = 1.0 - P.zeta > 0.0 ? 1.0 - P.zeta : 0.0;
  m.cH = 1.0 / (P.h * P.h);
  m.lamL = P.lam[0];
  m.dlam = P.lam[1] - P.lam[0];
  m.lamG = P.lam[2];
  m.rcL = P.rhoc[0];
  m.drc = P.rhoc[1] - P.rhoc[0];
  m.rcG = P.rhoc[2];
  m.Lv = P.Lv;
  m.sep = P.rho_c_separate ? 1 : 0;
  m.rhoL = P.rho[0];
  m.drho = P.rho[1] - P.rho[0];
  m.rhoG = P.rho[2];
  m.csL = P.cs[0];
  m.dcs = P.cs[1] - P.cs[0];
  m.csG = P.cs[2];
  m.Lm = P.L;
  m.bc_T0 = P.bc_T0 - P.t_star;
  m.bc_T1 = P.bc_T1 - P.t_star;
  m.bc_t0 = P.bc_t0;
  m.bc_t1 = P.bc_t1;
  m.h3 = P.h * P.h * P.h;
  m.gamma = P.gamma;
  m.dT = P.dT;
  m.reaction = P.reaction;
  m.zeta = P.zeta;
  m.gpc = P.xi * P.xi * P.mu * P.alpha;
  m.inv_h = 1.0 / P.h;
}

// the paired and batched kernels implement the SigmaP1-P phase equation of
// the AC and coupled models on a voxel mask only
bool simple_kernels_only(const pf_params& P, int smooth) {
  return P.model == PF_MODEL_TEMP || P.reaction != PF_REACT_SIGMA || smooth;
}

// The vector kernels: n1 divisible by the vector width (4 FP32 or 2 FP64
// cells) and a plane run with its neighbour rows (of every unknown, and of
// the glass field in paper mode) within the LDS budget.  Every model,
// reaction and glass representation.
static bool vector_ok(const pf_params& P, int smooth) {
  const int nvar = P.model == PF_MODEL_COUPLED ? 2 : 1;
  const int esize = P.precision == PF_FP64 ? 8 : 4;
  return P.n1 % pf::vec_cells(esize) == 0 &&
         pf::stage4_lds_bytes(P.n1, nvar + (smooth ? 1 : 0), esize) <= pf::kStage4MaxLds;
}

int validate(const pf_params* P, const uint8_t* mask) {
  if (!P || !mask) return fail(nullptr, PF_EINVAL, "params and mask must be non-NULL");
  if (P->n1 < 1 || P->n2 < 1 || P->n3 < 1)
    return fail(nullptr, PF_EINVAL, "grid sizes must be >= 1");
  const long long nc = (long long)P->n1 * P->n2 * P->n3;
  if (nc >= (1LL << 31) - 2LL * P->n1 * P->n2)
    return fail(nullptr, PF_EINVAL, "grid too large (cell index must fit in int32)");
  if (P->model != PF_MODEL_AC && P->model != PF_MODEL_COUPLED && P->model != PF_MODEL_TEMP)
    return fail(nullptr, PF_EINVAL, "model must be PF_MODEL_AC, PF_MODEL_COUPLED or PF_MODEL_TEMP");
  if (P->precision != PF_FP64 && P->precision != PF_FP32)
    return fail(nullptr, PF_EINVAL, "precision must be PF_FP64 or PF_FP32");
  if (P->reaction != PF_REACT_SIGMA && P->reaction != PF_REACT_GRADP)
    return fail(nullptr, PF_EINVAL, "reaction must be PF_REACT_SIGMA or PF_REACT_GRADP");
  if (P->model == PF_MODEL_TEMP && P->reaction != PF_REACT_SIGMA)
    return fail(nullptr, PF_EINVAL, "the Temp model has no reaction term (use PF_REACT_SIGMA)");
  if (!(P->h > 0) || !(P->xi > 0) || !(P->alpha > 0))
    return fail(nullptr, PF_EINVAL, "h, xi and alpha must be positive");
  if (!(P->eps1 != P->eps0)) return fail(nullptr, PF_EINVAL, "eps1 must differ from eps0");
  if (P->rho_c_separate != 0 && P->rho_c_separate != 1)
    return fail(nullptr, PF_EINVAL, "rho_c_separate must be 0 or 1");
  if (P->model != PF_MODEL_AC) {
    for (int i = 0; i < 3; ++i) {
      if (P->rho_c_separate) {
        if (!(P->rho[i] > 0) || !(P->cs[i] > 0))
          return fail(nullptr, PF_EINVAL, "rho and cs must be positive");
      } else if (!(P->rhoc[i] > 0)) {
        return fail(nullptr, PF_EINVAL, "rhoc must be positive");
      }
    }
    if (P->rho_c_separate && !(P->L >= 0 && P->L < INFINITY))
      return fail(nullptr, PF_EINVAL, "L must be finite and non-negative");
  }
  if (P->dirichlet_faces < 0 || P->dirichlet_faces > 63)
    return fail(nullptr, PF_EINVAL, "dirichlet_faces must be a 6-bit mask");
  if (P->bc_kind < PF_BC_CONST || P->bc_kind > PF_BC_STEP)
    return fail(nullptr, PF_EINVAL, "bc_kind out of range");
  if (P->bc_kind == PF_BC_RAMP && !(P->bc_t1 > P->bc_t0))
    return fail(nullptr, PF_EINVAL, "ramp needs bc_t1 > bc_t0");
  if (P->tol > 0 && (!(P->safety > 0) || !(P->dt_max > 0)))
    return fail(nullptr, PF_EINVAL, "adaptive mode needs safety > 0 and dt_max > 0");
  return PF_OK;
}

StageArgs stage_args(const pf_handle* h, int stage) {
  StageArgs a;
  memset(&a, 0, sizeof(a));
  a.code = h->code;
  a.G = h->G;
  a.ctl = h->ctl;
  a.mc = h->mc;
  const bool own = stage >= 1 && stage <= 5;
  a.z_chunk = own ? h->st_z[stage] : h->z_chunk;
  a.tiles_p = own ? h->st_tp[stage] : h->tiles_p;
  a.tiles_z = own ? h->st_tz[stage] : h->tiles_z;
  a.vec = h->vec;
  a.stream_nt = h->stream_nt;
  for (int v = 0; v < 2; ++v) {
    a.y[0][v] = h->y[0][v];
    a.y[1][v] = h->y[1][v];
    a.out_y[0][v] = h->y[0][v];
    a.out_y[1][v] = h->y[1][v];
    a.k1[v] = h->k1[v];
    a.k3[v] = h->k3[v];
    if (h->vec) {
      // Vector passes: S1 y -> k1; S2 (y, k1) -> Y3 in B; S3 Y3 -> k3;
      // S4 (y, k1, k3) -> Y5 in A, P in the y_new slot, C in B; S5 (Y5, P,
      // C) -> y_new over P.  Y2 and Y4 are formed at the stencil points.
      switch (stage) {
        case 1: a.in[v] = nullptr; a.out[v] = nullptr; break;
        case 2: a.in[v] = nullptr; a.out[v] = h->b[v]; break;
        case 3: a.in[v] = h->b[v]; a.out[v] = nullptr; break;
        case 4: a.in[v] = nullptr; a.out[v] = h->a[v]; a.cbuf[v] = h->b[v]; break;
        case 5: a.in[v] = h->a[v]; a.out[v] = nullptr; a.cbuf[v] = h->b[v]; break;
        default: break;
      }
    } else {
      // One-cell passes: S1 y -> k1, Y2 in A; S2 (Y2, k1) -> Y3 in B; S3
      // (Y3, y, k1) -> k3, Y4 in A; S4 (Y4, y, k1, k3) -> Y5 in B, P over
      // k1, C over k3; S5 (Y5, P, C) -> y_new.
      switch (stage) {
        case 1: a.in[v] = nullptr; a.out[v] = h->a[v]; break;
        case 2: a.in[v] = h->a[v]; a.out[v] = h->b[v]; break;
        case 3: a.in[v] = h->b[v]; a.out[v] = h->a[v]; break;
        case 4: a.in[v] = h->a[v]; a.out[v] = h->b[v]; break;
        case 5: a.in[v] = h->b[v]; a.out[v] = nullptr; break;
        default: break;
      }
    }
  }
  a.part = (stage == 1) ? h->part1 : (stage == 5 ? h->part5 : nullptr);
  return a;
}

pf::PairArgs pair_args(const pf_handle* h, int first) {
  pf::PairArgs a;
  memset(&a, 0, sizeof(a));
  a.code = h->code;
  a.ctl = h->ctl;
  a.mc = h->mc;
  a.z_chunk = h->pair_zc;
  a.tiles_x = h->ptx;
  a.tiles_y = h->pty;
  a.tiles_z = h->ptz;
  for (int v = 0; v < 2; ++v) {
    a.y[0][v] = h->y[0][v];
    a.y[1][v] = h->y[1][v];
    a.k1[v] = h->k1[v];
    if (first == 1) {
      a.out_a[v] = h->b[v];  // Y3
    } else {
      a.in[v] = h->b[v];     // Y3
      a.out_a[v] = h->a[v];  // Y5
      a.out_p[v] = h->k3[v]; // P
    }
  }
  a.part = first == 1 ? h->part1 : nullptr;
  return a;
}

// S5 of the paired schedule: input Y5 in A, P in K3, C in the y_new slot.
StageArgs s5_paired_args(const pf_handle* h) {
  StageArgs a = stage_args(h, 5);
  for (int v = 0; v < 2; ++v) a.in[v] = h->a[v];
  a.c_from_out = 1;
  return a;
}

int num_passes(const pf_handle* h) { return h->sched == pf::kSchedFive ? 5 : 3; }

// S1 partials the controller reduces: one per S1 workgroup (five passes) or
// per first-pair workgroup (paired schedule)
int s1_parts(const pf_handle* h) { return h->sched == pf::kSchedFive ? h->st_np[1] : h->npair; }

// The step controller of a single-instance run runs in S5's last workgroup
// (no controller launch) on grids of at most kFoldMaxCells cells, whose
// passes are short enough for the launch to matter.  On large grids the
// atomic count of the workgroups' maxima, all on one word, and the
// controller's memory round trips in S5's tail cost more than the launch
// they save (256^3 FP32: S5 99 -> 110 us for a 4.6 us controller launch
// saved); on small ones the launch dominates (warm start at 96^3: 80x ->
// 94x median speed-up).  The batched sweep keeps its controller launch:
// folded per instance it measured slower over the whole sweep (6.6-6.64 s
// against 6.4 s).
constexpr long long kFoldMaxCells = 1LL << 22;

bool fold_ok(const pf_handle* h) { return h->ncell <= kFoldMaxCells; }

// The step controller folded into S5's arguments: the workgroup that writes
// the last partial runs it on `ctl`.
void set_fold(const pf_handle* h, StageArgs& a, DevCtl* ctl) {
  a.fold = 1;
  a.fold_np1 = s1_parts(h);
  a.fold_np5 = h->st_np[5];
  a.fold_p1 = h->part1;
  a.fold_ctr = h->fold_ctr;
  a.fold_acc = h->fold_acc;
  a.fold_ctl = ctl;
}

// Launch pass i (0-based) of one attempt under the handle's schedule;
// returns hipErrorInvalidValue past the last pass.  fold_ctl: if not null,
// the last pass (S5) also runs the step controller on it.
hipError_t issue_pass(const pf_handle* h, int i, hipStream_t s, DevCtl* fold_ctl = nullptr) {
  if (h->sched == pf::kSchedFive) {
    if (i >= 5) return hipErrorInvalidValue;
    StageArgs a = stage_args(h, i + 1);
    if (i == 4 && fold_ctl) set_fold(h, a, fold_ctl);
    return pf::launch_stage(h->P.precision, h->P.model, i + 1, a, s);
  }
  if (i == 0 || i == 1) {
    pf::PairArgs a = pair_args(h, i == 0 ? 1 : 3);
    return pf::launch_pair(h->P.precision, h->P.model, i == 0 ? 1 : 3, h->pair_ts, a, s);
  }
  if (i == 2) {
    StageArgs a = s5_paired_args(h);
    if (fold_ctl) set_fold(h, a, fold_ctl);
    return pf::launch_stage(h->P.precision, h->P.model, 5, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_ctl(const pf_handle* h, DevCtl* ctl, hipStream_t s) {
  return pf::launch_controller(ctl, h->part1, s1_parts(h), h->part5, h->st_np[5], h->mc.h3, s);
}

// One attempt: the passes and the step controller (in the last pass, or
// launched after it).
hipError_t issue_step(const pf_handle* h, hipStream_t s) {
  const bool fold = fold_ok(h);
  for (int i = 0; i < num_passes(h); ++i) {
    hipError_t e = issue_pass(h, i, s, (fold && i == num_passes(h) - 1) ? h->ctl : nullptr);
    if (e != hipSuccess) return e;
  }
  return fold ? hipSuccess : launch_ctl(h, h->ctl, s);
}

void drop_graph(pf_handle* h) {
  if (h->gexec) {
    (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
  }
  h->graph_steps = 0;
}

int set_tiles(pf_handle* h, int zc) {
  if (zc < 1) zc = 1;
  if (zc > h->P.n3) zc = h->P.n3;
  int tp, tz;
  int nb = pf::grid_blocks(h->mc, zc, h->vec ? pf::vec_cells(h->esize) : 1, &tp, &tz);
  if (nb > h->max_parts) return fail(h, PF_EINVAL, "tile choice exceeds partial buffer");
  h->z_chunk = zc;
  h->tiles_p = tp;
  h->tiles_z = tz;
  h->nparts = nb;
  for (int st = 1; st <= 5; ++st) {
    h->st_z[st] = zc;
    h->st_tp[st] = tp;
    h->st_tz[st] = tz;
    h->st_np[st] = nb;
  }
  drop_graph(h);
  return PF_OK;
}

// Planes per workgroup column of one stage pass (1..5) alone.
int set_stage_tiles(pf_handle* h, int st, int zc) {
  if (zc < 1) zc = 1;
  if (zc > h->P.n3) zc = h->P.n3;
  int tp, tz;
  int nb = pf::grid_blocks(h->mc, zc, h->vec ? pf::vec_cells(h->esize) : 1, &tp, &tz);
  if (nb > h->max_parts) return fail(h, PF_EINVAL, "tile choice exceeds partial buffer");
  h->st_z[st] = zc;
  h->st_tp[st] = tp;
  h->st_tz[st] = tz;
  h->st_np[st] = nb;
  drop_graph(h);
  return PF_OK;
}

int set_pair_tiles(pf_handle* h, int ts, int zc) {
  if (ts < 0 || ts > 2) return fail(h, PF_EINVAL, "pair tile index out of range");
  if (zc < 4) zc = 4;
  if (zc > h->P.n3) zc = h->P.n3;
  int tx, ty, tz;
  int nb = pf::pair_blocks(h->mc, ts, zc, &tx, &ty, &tz);
  if (nb > h->max_parts) return fail(h, PF_EINVAL, "pair tile choice exceeds partial buffer");
  h->pair_ts = ts;
  h->pair_zc = zc;
  h->ptx = tx;
  h->pty = ty;
  h->ptz = tz;
  h->npair = nb;
  drop_graph(h);
  return PF_OK;
}

void init_ctl(pf_handle* h, DevCtl& c, double t_end, long long max_steps, double eq_tol) {
  memset(&c, 0, sizeof(c));
  c.t = h->t;
  c.dt_nom = h->dt;
  c.t_end = t_end;
  c.tol = h->P.tol;
  c.safety = h->P.safety;
  c.dt_min = h->P.dt_min;
  c.dt_max = h->P.dt_max;
  c.eq_tol = eq_tol;
  c.max_steps = max_steps;
  c.cur = h->cur;
  c.dt_att = c.dt_nom;
  if (c.t_end - c.t < c.dt_att) {
    c.dt_att = c.t_end - c.t;
    c.clipped = 1;
  }
}

int push_ctl(pf_handle* h) {
  PF_HIP(h, hipMemcpyAsync(h->ctl, h->hctl, sizeof(DevCtl), hipMemcpyHostToDevice, h->stream));
  return PF_OK;
}

int pull_ctl(pf_handle* h) {
  PF_HIP(h, hipMemcpyAsync(h->hctl, h->ctl, sizeof(DevCtl), hipMemcpyDeviceToHost, h->stream));
  PF_HIP(h, hipStreamSynchronize(h->stream));
  return PF_OK;
}

// Autotuner: time the five stage kernels for each candidate z_chunk on the
// current state (no controller, so the state is untouched) and keep the
// fastest.
int autotune_measure(pf_handle* h) {
  DevCtl& c = *h->hctl;
  init_ctl(h, c, INFINITY, 1LL << 62, 0.0);
  if (!(c.dt_att > 0) || !(c.dt_att < INFINITY)) c.dt_att = 1e-12;
  int rc = push_ctl(h);
  if (rc) return rc;
  hipEvent_t e0, e1;
  PF_HIP(h, hipEventCreate(&e0));
  PF_HIP(h, hipEventCreate(&e1));
  // mean of two timed repetitions after one warm-up
  auto timed = [&](auto&& launch, float* out) -> int {
    float tot = 0.0f;
    for (int rep = 0; rep < 3; ++rep) {
      PF_HIP(h, hipEventRecord(e0, h->stream));
      PF_HIP(h, launch());
      PF_HIP(h, hipEventRecord(e1, h->stream));
      PF_HIP(h, hipEventSynchronize(e1));
      float ms = 0;
      PF_HIP(h, hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0) tot += ms;
    }
    *out = tot;
    return PF_OK;
  };
  // (1) planes per column of each single-stage pass, and (unless the caller
  // fixed it) vector or one-cell kernels.  For every candidate depth the five
  // passes run in attempt order with an event between each two (each reads
  // what its predecessor wrote, as in a run); each pass keeps its fastest
  // depth (median of three timed repetitions after a warm-up), and the kernel
  // form with the smaller sum of per-pass minima wins.  Besides powers of
  // two, the candidates include the depths whose grid is one or two whole
  // rounds of resident workgroups at 2..4 per CU (no partly filled last
  // round on large grids).
  int cus = 0, cdev = 0;
  PF_HIP(h, hipGetDevice(&cdev));
  PF_HIP(h, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, cdev));
  auto depth_cands = [&](int vec) {
    std::vector<int> zs = {1, 2, 4, 8, 16, 32};
    int tp1 = 0, tz1 = 0;
    pf::grid_blocks(h->mc, 1, vec ? pf::vec_cells(h->esize) : 1, &tp1, &tz1);
    for (int per_cu = 2; per_cu <= 4; ++per_cu)
      for (int rounds = 1; rounds <= 2; ++rounds) {
        const long long nz = ((long long)rounds * per_cu * cus + tp1 - 1) / tp1;
        if (nz < 1 || nz > h->P.n3) continue;
        const int zc = (int)((h->P.n3 + nz - 1) / nz);
        bool have = false;
        for (int z : zs) have = have || z == zc;
        if (!have) zs.push_back(zc);
      }
    return zs;
  };
  int best_vec = h->vec, best_z[6] = {0, h->z_chunk, h->z_chunk, h->z_chunk, h->z_chunk,
                                      h->z_chunk};
  float best_total = 1e30f;
  const bool try_both = !h->vec_fixed && vector_ok(h->P, h->smooth);
  hipEvent_t ev[6];
  for (int i = 0; i < 6; ++i) PF_HIP(h, hipEventCreate(&ev[i]));
  for (int vec = 1; vec >= 0; --vec) {
    if (!try_both && vec != h->vec) continue;
    h->vec = vec;
    float bst[6];
    int bz[6] = {0, 0, 0, 0, 0, 0};
    for (int st = 0; st < 6; ++st) bst[st] = 1e30f;
    for (int zc : depth_cands(vec)) {
      if (zc > h->P.n3 && zc != 1) continue;
      if (set_tiles(h, zc)) continue;
      float reps[3][6];
      for (int rep = 0; rep < 4; ++rep) {
        PF_HIP(h, hipEventRecord(ev[0], h->stream));
        for (int st = 1; st <= 5; ++st) {
          StageArgs a = stage_args(h, st);
          PF_HIP(h, pf::launch_stage(h->P.precision, h->P.model, st, a, h->stream));
          PF_HIP(h, hipEventRecord(ev[st], h->stream));
        }
        PF_HIP(h, hipEventSynchronize(ev[5]));
        if (rep == 0) continue;
        for (int st = 1; st <= 5; ++st)
          PF_HIP(h, hipEventElapsedTime(&reps[rep - 1][st], ev[st - 1], ev[st]));
      }
      for (int st = 1; st <= 5; ++st) {
        float a0 = reps[0][st], a1 = reps[1][st], a2 = reps[2][st];
        const float med = a0 > a1 ? (a1 > a2 ? a1 : (a0 > a2 ? a2 : a0))
                                  : (a0 > a2 ? a0 : (a1 > a2 ? a2 : a1));
        if (med < bst[st]) {
          bst[st] = med;
          bz[st] = zc;
        }
      }
    }
    float total = 0.0f;
    for (int st = 1; st <= 5; ++st) total += bst[st];
    if (total < best_total) {
      best_total = total;
      best_vec = vec;
      for (int st = 1; st <= 5; ++st) best_z[st] = bz[st];
    }
  }
  for (int i = 0; i < 6; ++i) (void)hipEventDestroy(ev[i]);
  h->vec = best_vec;
  rc = set_tiles(h, best_z[4]);  // the RHS pass and the reported depth follow S4
  if (rc) return rc;
  for (int st = 1; st <= 5; ++st) {
    rc = set_stage_tiles(h, st, best_z[st]);
    if (rc) return rc;
  }
  float best_ms = 1e30f;
  // (2) tile shape and planes per column of the paired passes
  if (h->sched == pf::kSchedPaired) {
    const int pz[] = {8, 16, 32, 64};
    int bts = h->pair_ts, bzc = h->pair_zc;
    best_ms = 1e30f;
    for (int ts = 0; ts < 3; ++ts) {
      for (int zc : pz) {
        if (zc > h->P.n3 && zc != pz[0]) continue;
        if (set_pair_tiles(h, ts, zc)) continue;
        float ms;
        rc = timed([&]() -> hipError_t {
          for (int i = 0; i < 2; ++i) {
            hipError_t e = issue_pass(h, i, h->stream);
            if (e != hipSuccess) return e;
          }
          return hipSuccess;
        }, &ms);
        if (rc) return rc;
        if (ms < best_ms) {
          best_ms = ms;
          bts = ts;
          bzc = zc;
        }
      }
    }
    rc = set_pair_tiles(h, bts, bzc);
    if (rc) return rc;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return PF_OK;
}

// The autotuner's choice depends on the grid's shape and on the kernel
// variant, not on the state: handles of one signature on one device reuse
// the first handle's measurement for the rest of the process.
using TuneKey = std::array<int, 12>;
struct TuneVal {
  int vec;
  int z[6];
  int pair_ts, pair_zc;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;

int autotune(pf_handle* h) {
  h->autotune_pending = 0;
  int dev = 0;
  PF_HIP(h, hipGetDevice(&dev));
  const TuneKey key = {dev, h->P.n1, h->P.n2, h->P.n3, h->P.precision, h->P.model,
                       h->P.reaction, h->smooth, h->stream_nt, h->sched, h->vec_fixed,
                       h->vec_fixed ? h->vec : -1};
  TuneVal val;
  bool hit = false;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      val = it->second;
      hit = true;
    }
  }
  if (!hit) {
    int rc = autotune_measure(h);
    if (rc) return rc;
    val.vec = h->vec;
    for (int st = 0; st <= 5; ++st) val.z[st] = st ? h->st_z[st] : h->z_chunk;
    val.pair_ts = h->pair_ts;
    val.pair_zc = h->pair_zc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.emplace(key, val);
    return PF_OK;
  }
  h->vec = val.vec;
  int rc = set_tiles(h, val.z[0]);
  for (int st = 1; st <= 5 && !rc; ++st) rc = set_stage_tiles(h, st, val.z[st]);
  if (!rc && h->sched == pf::kSchedPaired) rc = set_pair_tiles(h, val.pair_ts, val.pair_zc);
  return rc;
}

}  // namespace

namespace pf {
void set_thread_error(const std::string& msg) { g_create_err = msg; }
}  // namespace pf

namespace {
void free_batch_work(pf_handle* h) {
  pf_handle::BatchWork& b = h->bw;
  (void)hipFree(b.desc);
  (void)hipFree(b.items);
  (void)hipFree(b.act);
  (void)hipFree(b.bar);
  (void)hipFree(b.gath);
  if (b.hgath) (void)hipHostFree(b.hgath);
  for (int i = 0; i < 3; ++i) {
    if (b.side[i]) (void)hipStreamDestroy(b.side[i]);
    if (b.join[i]) (void)hipEventDestroy(b.join[i]);
  }
  if (b.fork) (void)hipEventDestroy(b.fork);
  b = pf_handle::BatchWork();
}

// the batch work tables of h for n instances and nitems work items (grown,
// never shrunk)
int batch_work(pf_handle* h, int n, long long nitems) {
  pf_handle::BatchWork& b = h->bw;
  if (b.desc && n <= b.cap_inst && nitems <= b.cap_items) return PF_OK;
  (void)hipStreamSynchronize(h->stream);
  const int ni = n > b.cap_inst ? n : b.cap_inst;
  const long long nit = nitems > b.cap_items ? nitems : b.cap_items;
  free_batch_work(h);
  if (hipMalloc(&b.desc, sizeof(pf::BatchDesc) * ni) != hipSuccess ||
      hipMalloc(&b.items, sizeof(int2) * (size_t)(nit > 0 ? nit : 1)) != hipSuccess ||
      hipMalloc(&b.act, sizeof(int) * ni) != hipSuccess ||
      hipMalloc(&b.bar, 4 * sizeof(unsigned)) != hipSuccess ||
      hipMalloc(&b.gath, sizeof(DevCtl) * ni) != hipSuccess ||
      hipHostMalloc((void**)&b.hgath, sizeof(DevCtl) * ni, hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&b.fork, hipEventDisableTiming) != hipSuccess) {
    free_batch_work(h);
    return PF_ENOMEM;
  }
  for (int i = 0; i < 3; ++i)
    if (hipStreamCreateWithFlags(&b.side[i], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b.join[i], hipEventDisableTiming) != hipSuccess) {
      free_batch_work(h);
      return PF_ENOMEM;
    }
  b.cap_inst = ni;
  b.cap_items = nit;
  return PF_OK;
}

hipStream_t work_stream(pf_handle* h, uintptr_t stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (!stream || s == h->stream) return h->stream;
  (void)hipStreamSynchronize(h->stream);
  return s;
}
}  // namespace

extern "C" {

int pf_abi_version(void) { return 2; }

int pf_warmstart(pf_handle* h, pf_unet* net, double dT, double log10_sigma_scale, int32_t mode,
                 uintptr_t stream) {
  if (!h) return PF_EINVAL;
  if (!net) return fail(h, PF_EINVAL, "network must be non-NULL");
  if (mode < PF_WARM_ALL || mode > PF_WARM_FLOOD)
    return fail(h, PF_EINVAL, "mode must be PF_WARM_ALL, PF_WARM_NUCLEUS or PF_WARM_FLOOD");
  if (h->P.model != PF_MODEL_AC && h->P.model != PF_MODEL_COUPLED)
    return fail(h, PF_EINVAL, "warm start needs a phase-field model (PF_MODEL_AC or PF_MODEL_COUPLED)");
  if (!(dT > 0.0)) return fail(h, PF_EINVAL, "dT must be positive");
  hipStream_t s = work_stream(h, stream);
  std::string e;
  const int r = pfu_forward_into(net, h->code, h->P.n1, h->P.n2, h->P.n3, dT, log10_sigma_scale,
                                 h->y[h->cur][0], h->P.precision == PF_FP64 ? 1 : 0, mode, s, &e);
  if (r != PF_OK) return fail(h, r, "warm start: " + e);
  PF_HIP(h, hipStreamSynchronize(s));
  return PF_OK;
}

const char* pf_last_error(const pf_handle* h) {
  if (!h) return g_create_err.c_str();
  return h->err.c_str();
}

namespace {

// shared by pf_create (binary mask) and pf_create_field (smooth G: mask = G >= 1/2)
int create_impl(const pf_params* params, const uint8_t* mask, const double* G,
                pf_handle** out) {
  if (!out) return fail(nullptr, PF_EINVAL, "out must be non-NULL");
  *out = nullptr;
  int rc = validate(params, mask);
  if (rc) return rc;
  pf_handle* h = new (std::nothrow) pf_handle();
  if (!h) return fail(nullptr, PF_ENOMEM, "host allocation failed");
  h->P = *params;
  fill_model_const(h->P, h->mc);
  h->smooth = G ? 1 : 0;
  h->mc.smooth = h->smooth;
  h->ncell = (long long)params->n1 * params->n2 * params->n3;
  h->esize = params->precision == PF_FP64 ? 8 : 4;
  h->nvar = params->model == PF_MODEL_COUPLED ? 2 : 1;
  // six fields per unknown; beyond twice the 256 MB last-level cache the
  // streamed fields bypass the caches (measured: faster at 256^3, slower on
  // cache-resident grids)
  h->stream_nt = (double)h->ncell * h->esize * 6 * h->nvar > 512.0e6 ? 1 : 0;
  h->vec = vector_ok(*params, G ? 1 : 0) ? 1 : 0;
  h->dt = params->dt_max > 0 ? params->dt_max : 1e-3;

  auto bail = [&](int code, const std::string& msg) {
    g_create_err = msg;
    pf_destroy(h);
    return code;
  };
  if (hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking) != hipSuccess)
    return bail(PF_EHIP, "hipStreamCreateWithFlags failed");
  h->stream = h->own_stream;

  // maximum number of workgroups over all tile choices (z_chunk >= 1)
  int tp, tz;
  h->max_parts = pf::grid_blocks(h->mc, 1, 1, &tp, &tz);  // one-cell grid bounds the vector one
  for (int ts = 0; ts < 3; ++ts) {
    int tx, ty, tzz;
    const int nb = pf::pair_blocks(h->mc, ts, 4, &tx, &ty, &tzz);
    if (nb > h->max_parts) h->max_parts = nb;
  }
  const size_t field = ((size_t)h->ncell * h->esize + 255) & ~(size_t)255;
  const size_t code_bytes = ((size_t)h->ncell + 255) & ~(size_t)255;
  const size_t part_bytes = (((size_t)h->max_parts * (pf::kPartS1 + pf::kPartS5) + 64) *
                             sizeof(double) + 255) & ~(size_t)255;
  const size_t total = field * 6 * h->nvar + code_bytes + part_bytes + 2 * 256 +  // control block + timing copy
                       256 +  // counter of the folded controller
                       (h->smooth ? field : 0);
  if (hipMalloc(&h->slab, total) != hipSuccess) return bail(PF_ENOMEM, "hipMalloc of work buffers failed");
  char* p = static_cast<char*>(h->slab);
  for (int v = 0; v < h->nvar; ++v) {
    h->y[0][v] = p; p += field;
    h->y[1][v] = p; p += field;
    h->a[v] = p; p += field;
    h->b[v] = p; p += field;
    h->k1[v] = p; p += field;
    h->k3[v] = p; p += field;
  }
  h->code = reinterpret_cast<uint8_t*>(p); p += code_bytes;
  h->part1 = reinterpret_cast<double*>(p);
  h->part5 = h->part1 + (size_t)h->max_parts * pf::kPartS1;
  h->diag_out = h->part5 + h->max_parts;
  p += part_bytes;
  h->ctl = reinterpret_cast<DevCtl*>(p);
  p += 2 * 256;
  h->fold_ctr = reinterpret_cast<unsigned*>(p);
  h->fold_acc = reinterpret_cast<unsigned long long*>(p + 128);
  p += 256;
  if (h->smooth) h->G = p;
  if (hipHostMalloc((void**)&h->hctl, sizeof(DevCtl), hipHostMallocDefault) != hipSuccess)
    return bail(PF_ENOMEM, "hipHostMalloc failed");
  if (h->smooth) {  // the glass field in the field precision
    hipError_t eg;
    if (h->esize == 8) {
      eg = hipMemcpy(h->G, G, (size_t)h->ncell * 8, hipMemcpyHostToDevice);
    } else {
      std::vector<float> gf((size_t)h->ncell);
      for (long long i = 0; i < h->ncell; ++i) gf[(size_t)i] = (float)G[i];
      eg = hipMemcpy(h->G, gf.data(), (size_t)h->ncell * 4, hipMemcpyHostToDevice);
    }
    if (eg != hipSuccess) return bail(PF_EHIP, "upload of the glass field failed");
  }

  // neighbourhood codes from the host mask
  uint8_t* dmask = nullptr;
  if (hipMalloc(&dmask, (size_t)h->ncell) != hipSuccess) return bail(PF_ENOMEM, "hipMalloc mask");
  hipError_t e = hipMemcpy(dmask, mask, (size_t)h->ncell, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = pf::launch_build_code(dmask, h->code, params->n1, params->n2, params->n3, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->slab, 0, field * 6 * h->nvar, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->fold_ctr, 0, 256, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  (void)hipFree(dmask);
  if (e != hipSuccess) return bail(PF_EHIP, std::string("setup: ") + hipGetErrorString(e));
  int zc = params->n3 >= 256 ? 32 : 16;
  if (set_tiles(h, zc)) return bail(PF_EINVAL, h->err);
  if (set_pair_tiles(h, params->n1 >= 64 ? 1 : 2, 16)) return bail(PF_EINVAL, h->err);
  init_ctl(h, *h->hctl, INFINITY, 0, 0.0);
  h->hctl->done = 1;
  if (push_ctl(h) || hipStreamSynchronize(h->stream) != hipSuccess)
    return bail(PF_EHIP, "control block init failed");
  *out = h;
  return PF_OK;
}

}  // namespace

int pf_create(const pf_params* params, const uint8_t* mask, pf_handle** out) {
  return create_impl(params, mask, nullptr, out);
}

int pf_create_field(const pf_params* params, const double* G, pf_handle** out) {
  if (!params || !G) return fail(nullptr, PF_EINVAL, "params and G must be non-NULL");
  if (params->n1 < 1 || params->n2 < 1 || params->n3 < 1)
    return fail(nullptr, PF_EINVAL, "grid sizes must be >= 1");
  const size_t n = (size_t)params->n1 * params->n2 * params->n3;
  std::vector<uint8_t> mask(n);
  for (size_t i = 0; i < n; ++i) {
    if (!(G[i] >= 0.0 && G[i] <= 1.0))
      return fail(nullptr, PF_EINVAL, "G must lie in [0, 1]");
    mask[i] = G[i] >= 0.5 ? 1 : 0;
  }
  return create_impl(params, mask.data(), G, out);
}

void pf_destroy(pf_handle* h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  drop_graph(h);
  free_batch_work(h);
  if (h->slab) (void)hipFree(h->slab);
  if (h->hctl) (void)hipHostFree(h->hctl);
  if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
  delete h;
}

int pf_set_stream(pf_handle* h, uintptr_t stream) {
  if (!h) return PF_EINVAL;
  hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : h->own_stream;
  if (s != h->stream) {
    PF_HIP(h, hipStreamSynchronize(h->stream));
    h->stream = s;
    drop_graph(h);
  }
  return PF_OK;
}

int64_t pf_num_cells(const pf_handle* h) { return h ? h->ncell : -1; }

int pf_synchronize(pf_handle* h) {
  if (!h) return PF_EINVAL;
  PF_HIP(h, hipStreamSynchronize(h->stream));
  return PF_OK;
}

int pf_set_tolerance(pf_handle* h, double tol) {
  if (!h) return PF_EINVAL;
  if (!(tol == tol)) return fail(h, PF_EINVAL, "tol must not be NaN");
  h->P.tol = tol;  // read into the control block at the start of each run
  return PF_OK;
}

int pf_set_time(pf_handle* h, double t, double dt) {
  if (!h) return PF_EINVAL;
  if (!(dt > 0) || !(t == t)) return fail(h, PF_EINVAL, "dt must be positive and t finite");
  h->t = t;
  h->dt = dt;
  return PF_OK;
}

int pf_set_state(pf_handle* h, const void* phi, const void* theta, int on_device,
                 uintptr_t stream) {
  if (!h) return PF_EINVAL;
  if (h->P.model == PF_MODEL_TEMP) {  // the single unknown theta lives in slot 0
    if (!theta) return fail(h, PF_EINVAL, "theta must be non-NULL for the Temp model");
    phi = theta;
  }
  if (!phi) return fail(h, PF_EINVAL, "phi must be non-NULL");
  if (h->nvar == 2 && !theta) return fail(h, PF_EINVAL, "theta must be non-NULL for the coupled model");
  const size_t bytes = (size_t)h->ncell * h->esize;
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  hipStream_t s = work_stream(h, stream);
  h->cur = 0;
  PF_HIP(h, hipMemcpyAsync(h->y[0][0], phi, bytes, k, s));
  if (h->nvar == 2) PF_HIP(h, hipMemcpyAsync(h->y[0][1], theta, bytes, k, s));
  PF_HIP(h, hipStreamSynchronize(s));
  return PF_OK;
}

int pf_get_state(pf_handle* h, void* phi, void* theta, int on_device, uintptr_t stream) {
  if (!h) return PF_EINVAL;
  const size_t bytes = (size_t)h->ncell * h->esize;
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (h->P.model == PF_MODEL_TEMP) {
    phi = theta;
    theta = nullptr;
  }
  hipStream_t s = work_stream(h, stream);
  if (phi) PF_HIP(h, hipMemcpyAsync(phi, h->y[h->cur][0], bytes, k, s));
  if (theta && h->nvar == 2) PF_HIP(h, hipMemcpyAsync(theta, h->y[h->cur][1], bytes, k, s));
  PF_HIP(h, hipStreamSynchronize(s));
  return PF_OK;
}

int pf_rhs(pf_handle* h, double t, const void* phi, const void* theta, void* dphi,
           void* dtheta, uintptr_t stream) {
  if (!h) return PF_EINVAL;
  hipStream_t s = work_stream(h, stream);
  if (h->P.model == PF_MODEL_TEMP) {
    // unknown theta in slot 0; the optional second output is d phi/dt
    if (!theta || !dtheta)
      return fail(h, PF_EINVAL, "theta and dtheta must be non-NULL for the Temp model");
    StageArgs a = stage_args(h, 0);
    a.ignore_done = 1;
    a.t_fixed = t;
    a.vec = 0;
    pf::grid_blocks(h->mc, h->z_chunk, 1, &a.tiles_p, &a.tiles_z);
    a.in[0] = theta;
    a.in[1] = nullptr;
    a.out[0] = dtheta;
    a.out[1] = dphi;
    PF_HIP(h, pf::launch_stage(h->P.precision, h->P.model, 0, a, s));
    return PF_OK;
  }
  if (!phi || !dphi) return fail(h, PF_EINVAL, "phi and dphi must be non-NULL");
  if (h->nvar == 2 && (!theta || !dtheta))
    return fail(h, PF_EINVAL, "theta and dtheta must be non-NULL for the coupled model");
  StageArgs a = stage_args(h, 0);
  a.ignore_done = 1;
  a.t_fixed = t;
  a.in[0] = phi;
  a.in[1] = theta;
  a.out[0] = dphi;
  a.out[1] = dtheta;
  // caller buffers: the vector kernels need 16-byte aligned fields
  auto aligned = [](const void* q) { return ((uintptr_t)q & 15u) == 0; };
  if (a.vec && !(aligned(phi) && aligned(dphi) && (h->nvar == 1 || (aligned(theta) &&
                                                                    aligned(dtheta))))) {
    a.vec = 0;
    pf::grid_blocks(h->mc, h->z_chunk, 1, &a.tiles_p, &a.tiles_z);
  }
  PF_HIP(h, pf::launch_stage(h->P.precision, h->P.model, 0, a, s));
  return PF_OK;
}

int pf_set_vector(pf_handle* h, int32_t enable) {
  if (!h) return PF_EINVAL;
  if (enable && h->P.n1 % pf::vec_cells(h->esize) != 0)
    return fail(h, PF_EINVAL, "vector kernels need n1 divisible by 4 (FP32) or 2 (FP64)");
  if (enable && !vector_ok(h->P, h->smooth))
    return fail(h, PF_EINVAL, "vector kernels: n1 too large for their LDS plane buffers");
  h->vec = enable ? 1 : 0;
  h->vec_fixed = 1;
  return set_tiles(h, h->z_chunk);
}

int pf_rkm_step(pf_handle* h, double* t, double* dt, pf_step_info* info) {
  if (!h || !t || !dt) return PF_EINVAL;
  if (!(*dt > 0)) return fail(h, PF_EINVAL, "dt must be positive");
  h->t = *t;
  h->dt = *dt;
  DevCtl& c = *h->hctl;
  init_ctl(h, c, INFINITY, 1LL << 62, 0.0);
  int rc = push_ctl(h);
  if (rc) return rc;
  PF_HIP(h, issue_step(h, h->stream));
  rc = pull_ctl(h);
  if (rc) return rc;
  h->cur = c.cur;
  h->t = c.t;
  h->dt = c.dt_nom;
  *t = c.t;
  *dt = c.dt_nom;
  if (info) {
    info->accepted = c.accepted;
    info->status = c.status;
    info->eps = c.eps;
    info->dt_used = c.dt_used;
    info->dt_next = c.dt_nom;
    info->maxk1 = c.maxk1;
    info->t = c.t;
  }
  if (c.status < 0) return fail(h, c.status, c.status == PF_ENONFINITE ? "non-finite error estimate"
                                                                      : "step fell below dt_min");
  return PF_OK;
}

int pf_diagnostics(pf_handle* h, pf_run_stats* st) {
  if (!h) return PF_EINVAL;
  return pf_diagnostics_planes(h, 0, h->P.n3, st);
}

int pf_diagnostics_planes(pf_handle* h, int32_t i3_lo, int32_t i3_hi, pf_run_stats* st) {
  if (!h || !st) return PF_EINVAL;
  if (i3_lo < 0 || i3_hi > h->P.n3 || i3_lo > i3_hi)
    return fail(h, PF_EINVAL, "planes must satisfy 0 <= i3_lo <= i3_hi <= n3");
  // the planes [i3_lo, i3_hi) are one contiguous run of cells
  const long long plane = (long long)h->P.n1 * h->P.n2;
  const long long off = plane * i3_lo, n = plane * (i3_hi - i3_lo);
  const size_t eb = (size_t)h->esize;
  auto at = [&](const void* q) -> const void* {
    return q ? static_cast<const char*>(q) + (size_t)off * eb : nullptr;
  };
  const void* G = h->G ? static_cast<const char*>(h->G) + (size_t)off * eb : nullptr;
  PF_HIP(h, pf::launch_diag(h->P.precision, h->P.model, h->code + off, G, at(h->y[h->cur][0]),
                            at(h->y[h->cur][1]), h->mc, n, h->part1,
                            h->max_parts > 1024 ? 1024 : h->max_parts, h->diag_out, h->stream));
  double out[4];
  PF_HIP(h, hipMemcpyAsync(out, h->diag_out, sizeof(out), hipMemcpyDeviceToHost, h->stream));
  PF_HIP(h, hipStreamSynchronize(h->stream));
  st->pore_count = (int64_t)out[0];
  st->sum_phi = out[1];
  st->enthalpy = out[2];
  st->ice_count = (int64_t)out[3];
  return PF_OK;
}

int pf_set_loop(pf_handle* h, int32_t steps_per_poll, int32_t use_graph) {
  if (!h || steps_per_poll < 1 || steps_per_poll > 4096) return PF_EINVAL;
  h->steps_per_poll = steps_per_poll;
  h->use_graph = use_graph ? 1 : 0;
  drop_graph(h);
  return PF_OK;
}

int pf_set_tile(pf_handle* h, int32_t z_chunk) {
  if (!h || z_chunk < 0) return PF_EINVAL;
  if (z_chunk == 0) {
    h->autotune_pending = 1;
    return PF_OK;
  }
  h->autotune_pending = 0;
  return set_tiles(h, z_chunk);
}

int pf_set_stage_tiles(pf_handle* h, const int32_t* z) {
  if (!h || !z) return PF_EINVAL;
  for (int st = 0; st < 5; ++st)
    if (z[st] < 1) return fail(h, PF_EINVAL, "stage tiles: every depth must be >= 1");
  h->autotune_pending = 0;
  int rc = set_tiles(h, z[3]);
  for (int st = 1; st <= 5 && rc == PF_OK; ++st) rc = set_stage_tiles(h, st, z[st - 1]);
  return rc;
}

int pf_integrate(pf_handle* h, double t_end, int64_t max_steps, double eq_tol,
                 pf_run_stats* stats) {
  if (!h) return PF_EINVAL;
  auto w0 = std::chrono::steady_clock::now();
  if (h->autotune_pending) {
    int rc = autotune(h);
    if (rc) return rc;
  }
  DevCtl& c = *h->hctl;
  // the equilibrium test measures the phase-field equation, which the Temp
  // model does not have
  init_ctl(h, c, t_end, max_steps, h->P.model == PF_MODEL_TEMP ? 0.0 : eq_tol);
  if (h->t >= t_end) {
    c.done = 1;
    c.status = PF_OK;
  } else if (max_steps <= 0) {
    c.done = 1;
    c.status = PF_MAXSTEPS;
  }
  int rc = push_ctl(h);
  if (rc) return rc;
  // A run with the equilibrium test may end after very few attempts (a warm
  // start at or near equilibrium): its poll interval starts at one attempt and
  // doubles up to steps_per_poll, launched directly, and the graph is built
  // only once the interval is full (instantiating it costs about as much as
  // two dozen directly launched attempts).  Fixed-horizon runs poll every
  // steps_per_poll attempts from the start.
  int poll = c.eq_tol > 0.0 ? 1 : h->steps_per_poll;
  while (!c.done) {
    // attempts left in the budget: a shorter tail is launched directly, so a
    // run issues exactly the attempts it makes (no trailing no-op attempts)
    const long long left = c.max_steps - (c.n_acc + c.n_rej);
    const int nissue = left < poll ? (int)left : poll;
    if (poll < h->steps_per_poll) poll = 2 * poll < h->steps_per_poll ? 2 * poll : h->steps_per_poll;
    if (h->use_graph && nissue == h->steps_per_poll) {
      if (!h->gexec || h->graph_steps != h->steps_per_poll) {
        drop_graph(h);
        hipGraph_t g;
        PF_HIP(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int i = 0; i < h->steps_per_poll && e == hipSuccess; ++i) e = issue_step(h, h->stream);
        hipError_t e2 = hipStreamEndCapture(h->stream, &g);
        if (e != hipSuccess) return fail(h, PF_EHIP, std::string("capture: ") + hipGetErrorString(e));
        PF_HIP(h, e2);
        hipError_t e3 = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        PF_HIP(h, e3);
        h->graph_steps = h->steps_per_poll;
      }
      PF_HIP(h, hipGraphLaunch(h->gexec, h->stream));
    } else {
      for (int i = 0; i < nissue; ++i) PF_HIP(h, issue_step(h, h->stream));
    }
    rc = pull_ctl(h);
    if (rc) return rc;
  }
  h->cur = c.cur;
  h->t = c.t;
  h->dt = c.dt_nom;
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    rc = pf_diagnostics(h, stats);
    if (rc) return rc;
    stats->steps_accepted = c.n_acc;
    stats->steps_rejected = c.n_rej;
    stats->t = c.t;
    stats->dt = c.dt_nom;
    stats->maxk1 = c.maxk1;
    stats->status = c.status;
    stats->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - w0).count();
  }
  if (c.status < 0)
    return fail(h, c.status, c.status == PF_ENONFINITE ? "non-finite error estimate"
                                                       : "step fell below dt_min");
  return c.status;
}

int pf_time_kernels(pf_handle* h, int32_t reps, double* ms) {
  if (!h || !ms || reps < 1) return PF_EINVAL;
  if (h->autotune_pending) {
    int rc = autotune(h);
    if (rc) return rc;
  }
  // The passes of one attempt run in schedule order, an event between each
  // two, repeated reps times (after one warm-up attempt), so every pass reads
  // what its predecessor has just written, as in a run.  The control block is
  // set to a live attempt, and the controller that the last pass runs works on
  // a scratch copy: y[cur] is never written by a stage kernel, so the state, t
  // and dt are unchanged (the stage buffers are scratch until the next S1).
  DevCtl& c = *h->hctl;
  init_ctl(h, c, INFINITY, 1LL << 62, 0.0);
  int rc = push_ctl(h);
  if (rc) return rc;
  const int np = num_passes(h);
  hipEvent_t ev[6];
  for (int i = 0; i <= np; ++i) PF_HIP(h, hipEventCreate(&ev[i]));
  hipEvent_t& e0 = ev[0];
  hipEvent_t& e1 = ev[1];
  for (int i = 0; i < 6; ++i) ms[i] = 0.0;
  // the last pass runs the folded controller, as in a run, on a scratch copy
  // of the control block
  DevCtl cs = c;
  cs.done = 0;
  PF_HIP(h, hipMemcpyAsync(h->ctl + 1, &cs, sizeof(DevCtl), hipMemcpyHostToDevice, h->stream));
  for (int r = 0; r <= reps; ++r) {
    PF_HIP(h, hipEventRecord(ev[0], h->stream));
    for (int i = 0; i < np; ++i) {
      PF_HIP(h, issue_pass(h, i, h->stream,
                           (i == np - 1 && fold_ok(h)) ? h->ctl + 1 : nullptr));
      PF_HIP(h, hipEventRecord(ev[i + 1], h->stream));
    }
    PF_HIP(h, hipEventSynchronize(ev[np]));
    if (r == 0) continue;  // warm-up
    for (int i = 0; i < np; ++i) {
      float x = 0;
      PF_HIP(h, hipEventElapsedTime(&x, ev[i], ev[i + 1]));
      ms[i] += (double)x / reps;
    }
  }
  // controller, on a scratch copy of the control block
  DevCtl cc = c;
  cc.done = 0;
  PF_HIP(h, hipMemcpyAsync(h->ctl + 1, &cc, sizeof(DevCtl), hipMemcpyHostToDevice, h->stream));
  PF_HIP(h, hipStreamSynchronize(h->stream));
  PF_HIP(h, hipEventRecord(e0, h->stream));
  for (int r = 0; r < reps; ++r) PF_HIP(h, launch_ctl(h, h->ctl + 1, h->stream));
  PF_HIP(h, hipEventRecord(e1, h->stream));
  PF_HIP(h, hipEventSynchronize(e1));
  float x = 0;
  PF_HIP(h, hipEventElapsedTime(&x, e0, e1));
  ms[5] = (double)x / reps;
  for (int i = 0; i <= np; ++i) (void)hipEventDestroy(ev[i]);
  return PF_OK;
}

// Items of the batched sweep over the instances in act at z planes per item.
static long long batch_items_at(pf_handle* const* inst, const std::vector<int>& act, int z) {
  long long total = 0;
  for (int i : act) {
    int tp, tz;
    total += pf::grid_blocks(inst[i]->mc, z < inst[i]->P.n3 ? z : inst[i]->P.n3,
                             pf::vec_cells(inst[i]->esize), &tp, &tz);
  }
  return total;
}

int pf_batch_integrate(pf_handle* const* inst, int32_t n, double t_end, int64_t max_steps,
                       double eq_tol, pf_run_stats* out, uintptr_t stream,
                       const pf_batch_options* opts) {
  if (!inst || n < 1 || !out) return fail(nullptr, PF_EINVAL, "batch: inst, n >= 1 and out required");
  const int mode = (opts && opts->mode) ? opts->mode : 2;
  if (mode != 1 && mode != 2) return fail(nullptr, PF_EINVAL, "batch: mode must be 1 or 2");
  if (opts && (opts->z_chunk < 0 || opts->steps_per_poll < 0 || opts->branches < 0 ||
               opts->branches > 4))
    return fail(nullptr, PF_EINVAL, "batch: negative option or more than 4 branches");
  // Parallel chains are switched off: one run with three chains (three
  // instances, staggered finishing times) ended in a host segmentation fault
  // inside this call whose cause is not found; the same case had passed five
  // times before.  Until it is, the graph holds one chain.
  if (opts && opts->branches > 1)
    return fail(nullptr, PF_EINVAL,
                "batch: parallel chains (branches > 1) are switched off in this build");
  auto w0 = std::chrono::steady_clock::now();
  for (int i = 0; i < n; ++i) {
    if (!inst[i]) return fail(nullptr, PF_EINVAL, "batch: NULL handle");
    if (inst[i]->P.precision != inst[0]->P.precision || inst[i]->P.model != inst[0]->P.model)
      return fail(nullptr, PF_EINVAL, "batch: all instances need the same model and precision");
    if (inst[i]->P.model == PF_MODEL_TEMP || inst[i]->P.reaction != PF_REACT_SIGMA)
      return fail(nullptr, PF_EINVAL, "batch: the SigmaP1-P AC and coupled models only");
    if (inst[i]->smooth != inst[0]->smooth)
      return fail(nullptr, PF_EINVAL, "batch: all instances need the same glass representation");
    if (inst[i]->smooth && mode == 1)
      return fail(nullptr, PF_EINVAL,
                  "batch: the persistent kernel takes binary masks only (paper mode: mode 2)");
    if (!vector_ok(inst[i]->P, inst[i]->smooth))
      return fail(nullptr, PF_EINVAL,
                  "batch: every instance needs n1 divisible by 4 (FP32) or 2 (FP64) and "
                  "small enough for the vector kernels");
  }
  pf_handle* h0 = inst[0];
  hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : h0->own_stream;
  // Planes per work item.  Fixed when given; otherwise 4 while the running
  // instances make at least kMinItems items, halved (down to 1) when fewer
  // remain, so that a few small instances still spread over the whole chip.
  // (Deeper items, 8 or 16 planes, read fewer halo planes but leave the last
  // round of workgroups ragged: measured slower on the 48-instance sweep.)
  const int z_fixed = (opts && opts->z_chunk) ? opts->z_chunk : 0;
  const int kBatchZ = 4;
  const long long kMinItems = 1024;
  const int kStepsPerLaunch = (opts && opts->steps_per_poll) ? opts->steps_per_poll : 32;
  // Parallel chains of the multi-launch form: the running instances are
  // split into groups of about equal work, and each group's stage launches
  // form their own chain in the graph (one on the stream, the others on side
  // streams forked from it and joined back).  A launch of one chain then runs
  // while another chain is between two of its launches.
  const bool kBranchesGiven = opts && opts->branches;
  const int kBranches = 1;
  std::vector<int> act;
  for (int i = 0; i < n; ++i) {
    pf_handle* h = inst[i];
    PF_HIP(h, hipStreamSynchronize(h->stream));
    h->vec = 1;
    DevCtl& c = *h->hctl;
    init_ctl(h, c, t_end, max_steps, eq_tol);
    if (h->t >= t_end) {
      c.done = 1;
      c.status = PF_OK;
    } else if (max_steps <= 0) {
      c.done = 1;
      c.status = PF_MAXSTEPS;
    }
    PF_HIP(h, hipMemcpyAsync(h->ctl, h->hctl, sizeof(DevCtl), hipMemcpyHostToDevice, s));
    if (!c.done) act.push_back(i);
  }
  std::vector<int> all(n);
  int n1max = 0;
  for (int i = 0; i < n; ++i) {
    all[i] = i;
    n1max = inst[i]->P.n1 > n1max ? inst[i]->P.n1 : n1max;
  }
  const size_t lds = pf::stage4_lds_bytes(n1max, h0->nvar + (h0->smooth ? 1 : 0), h0->esize);
  const long long max_items = batch_items_at(inst, all, z_fixed ? z_fixed : 1);
  if (max_items > (1LL << 30)) return fail(h0, PF_EINVAL, "batch: too many work items");
  std::vector<pf::BatchDesc> desc(n);
  memset(desc.data(), 0, sizeof(pf::BatchDesc) * n);
  std::vector<int2> items;
  // the first instance's work tables (allocated on its first batch, reused)
  if (batch_work(h0, n, max_items) != PF_OK)
    return fail(h0, PF_ENOMEM, "batch: descriptor allocation failed");
  pf::BatchDesc* ddesc = h0->bw.desc;
  int2* ditems = h0->bw.items;
  int* dact = h0->bw.act;
  unsigned* dbar = h0->bw.bar;     // [0] arrivals, [1] generation, [2] barrier-overrun flag
  DevCtl* dgath = h0->bw.gath;     // control blocks of the running instances, gathered per poll
  DevCtl* hgath = h0->bw.hgath;    // pinned host copy
  hipGraphExec_t gexec = nullptr;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(s);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
  };
  unsigned hbar[4] = {0, 0, 0, 0};
  if (hipMemcpyAsync(dbar, hbar, sizeof(hbar), hipMemcpyHostToDevice, s) != hipSuccess) {
    cleanup();
    return fail(h0, PF_EHIP, "batch: barrier upload failed");
  }
  // Tiles, descriptors and items of the running instances (act), which
  // become the table's instances (tab); the multi-launch form also captures
  // kStepsPerLaunch attempts over them.
  std::vector<int> tab;
  auto build = [&]() -> int {
    int z = z_fixed ? z_fixed : kBatchZ;
    if (!z_fixed)
      while (z > 1 && batch_items_at(inst, act, z) < kMinItems) z >>= 1;
    items.clear();
    for (int i : act) {
      pf_handle* h = inst[i];
      int rc = set_tiles(h, z);
      if (rc) return rc;
      pf::BatchDesc& d = desc[i];
      for (int st = 1; st <= 5; ++st) d.st[st - 1] = stage_args(h, st);
      d.p1 = h->part1;
      d.p5 = h->part5;
      d.ntiles = h->nparts;
      d.h3 = h->mc.h3;
    }
    // groups of about equal work: instances by decreasing tile count, each to
    // the lightest group so far; the table lists the groups one after another.
    // By default only while every chain keeps at least kMinChainItems items:
    // with fewer (the tail of a sweep, a few instances on thinned tiles) one
    // chain measured faster (48-instance sweep to equilibrium: 6.9 s with two
    // chains throughout against 6.6 s with one, 6.4 s with this rule).  A
    // count given in the options is used as given (at most one chain per
    // instance).
    long long nitems_all = 0;
    for (int i : act) nitems_all += inst[i]->nparts;
    const long long kMinChainItems = 2048;
    int nb = mode == 2 ? std::min<int>(kBranches, (int)act.size()) : 1;
    if (!kBranchesGiven)
      while (nb > 1 && nitems_all < (long long)nb * kMinChainItems) --nb;
    std::vector<int> order(act);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return inst[a]->nparts > inst[b]->nparts; });
    std::vector<std::vector<int>> grp(nb);
    std::vector<long long> load(nb, 0);
    for (int i : order) {
      int best = 0;
      for (int k = 1; k < nb; ++k)
        if (load[k] < load[best]) best = k;
      grp[best].push_back(i);
      load[best] += inst[i]->nparts;
    }
    tab.clear();
    std::vector<int> item_off(nb + 1, 0), inst_off(nb + 1, 0);
    std::vector<int> ctl_launch(nb, 0);  // a chain with instances whose controller is not folded
    for (int k = 0; k < nb; ++k) {
      for (int i : grp[k]) {
        tab.push_back(i);
        for (int t = 0; t < inst[i]->nparts; ++t) items.push_back(make_int2(i, t));
        if (!desc[i].st[4].fold) ctl_launch[k] = 1;
      }
      item_off[k + 1] = (int)items.size();
      inst_off[k + 1] = (int)tab.size();
    }
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
    if (hipMemcpyAsync(ddesc, desc.data(), sizeof(pf::BatchDesc) * n, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(ditems, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice,
                       s) != hipSuccess ||
        hipMemcpyAsync(dact, tab.data(), sizeof(int) * tab.size(), hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(h0, PF_EHIP, "batch: descriptor upload failed");
    if (mode != 2) return PF_OK;
    hipGraph_t g;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    int forked = 0;  // side streams that joined the capture
    if (e == hipSuccess && nb > 1) {
      e = hipEventRecord(h0->bw.fork, s);
      for (int k = 1; k < nb && e == hipSuccess; ++k) {
        e = hipStreamWaitEvent(h0->bw.side[k - 1], h0->bw.fork, 0);
        if (e == hipSuccess) forked = k;
      }
    }
    for (int b = 0; b < nb && e == hipSuccess; ++b) {
      hipStream_t sb = b == 0 ? s : h0->bw.side[b - 1];
      for (int k = 0; k < kStepsPerLaunch && e == hipSuccess; ++k)
        e = pf::launch_batch_step(h0->P.precision, h0->P.model, h0->smooth, ddesc,
                                  ditems + item_off[b], item_off[b + 1] - item_off[b],
                                  dact + inst_off[b], inst_off[b + 1] - inst_off[b],
                                  ctl_launch[b] != 0, lds, sb);
    }
    // every side stream that joined is joined back, also after a failed
    // launch, so that the capture ends cleanly
    for (int k = 1; k <= forked; ++k) {
      hipError_t ej = hipEventRecord(h0->bw.join[k - 1], h0->bw.side[k - 1]);
      if (ej == hipSuccess) ej = hipStreamWaitEvent(s, h0->bw.join[k - 1], 0);
      if (e == hipSuccess) e = ej;
    }
    hipGraph_t g_ = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &g_);
    g = g_;
    if (e == hipSuccess && e2 == hipSuccess) e = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0);
    if (e2 == hipSuccess && g) (void)hipGraphDestroy(g);
    if (e != hipSuccess || e2 != hipSuccess) {
      gexec = nullptr;
      return fail(h0, PF_EHIP, "batch: graph capture failed");
    }
    return PF_OK;
  };
  int grid = 0;
  if (!act.empty()) {
    // the persistent form keeps every instance in its table (finished ones
    // are skipped inside the kernel)
    if (mode == 1) act = all;
    int rc = build();
    if (rc) {
      cleanup();
      return rc;
    }
    if (mode == 1) {
      grid = pf::batch_max_blocks(h0->P.precision, h0->P.model, lds);
      if (grid < 1) {
        cleanup();
        return fail(h0, PF_EHIP, "batch: occupancy query failed");
      }
      if (grid > (int)items.size()) grid = (int)items.size();
    }
  }
  while (!act.empty()) {
    hipError_t e = mode == 1 ? pf::launch_batch(h0->P.precision, h0->P.model, ddesc,
                                                ditems, (int)items.size(), n, kStepsPerLaunch,
                                                grid, dbar, dbar + 2, lds, s)
                             : hipGraphLaunch(gexec, s);
    if (e != hipSuccess) {
      cleanup();
      return fail(h0, PF_EHIP, std::string("batch launch: ") + hipGetErrorString(e));
    }
    // the table's control blocks: one gather, one copy (dact lists them in
    // the order of tab)
    if (pf::launch_gather_ctl(ddesc, dact, (int)tab.size(), dgath, s) != hipSuccess ||
        hipMemcpyAsync(hgath, dgath, sizeof(DevCtl) * tab.size(), hipMemcpyDeviceToHost, s) !=
            hipSuccess) {
      cleanup();
      return fail(h0, PF_EHIP, "batch: control readback failed");
    }
    if (hipMemcpyAsync(hbar, dbar, sizeof(hbar), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      cleanup();
      return fail(h0, PF_EHIP, "batch: synchronize failed");
    }
    for (size_t k = 0; k < tab.size(); ++k) *inst[tab[k]]->hctl = hgath[k];
    if (hbar[2]) {
      cleanup();
      return fail(h0, PF_EHIP, "batch: a grid barrier wait overran its bound");
    }
    std::vector<int> still;
    for (int i : act)
      if (!inst[i]->hctl->done) still.push_back(i);
    if (still.size() == act.size()) continue;
    act.swap(still);
    if (act.empty()) continue;
    if (mode == 1) {  // the persistent kernel keeps its table; dact follows act for the gather
      if (hipMemcpyAsync(dact, act.data(), sizeof(int) * act.size(), hipMemcpyHostToDevice, s) !=
              hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        cleanup();
        return fail(h0, PF_EHIP, "batch: instance list upload failed");
      }
      tab = act;
      continue;
    }
    int rc = build();  // fewer instances: smaller grids, maybe thinner tiles
    if (rc) {
      cleanup();
      return rc;
    }
  }
  cleanup();
  const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - w0).count();
  int ret = PF_OK;
  for (int i = 0; i < n; ++i) {
    pf_handle* h = inst[i];
    const DevCtl& c = *h->hctl;
    h->cur = c.cur;
    h->t = c.t;
    h->dt = c.dt_nom;
    pf_run_stats& st = out[i];
    memset(&st, 0, sizeof(st));
    int rc = pf_diagnostics(h, &st);
    if (rc) return rc;
    st.steps_accepted = c.n_acc;
    st.steps_rejected = c.n_rej;
    st.t = c.t;
    st.dt = c.dt_nom;
    st.maxk1 = c.maxk1;
    st.status = c.status;
    st.wall_s = wall;
    if (c.status < 0 && ret == PF_OK) ret = c.status;
  }
  return ret;
}

int pf_set_schedule(pf_handle* h, int32_t schedule) {
  if (!h || (schedule != pf::kSchedFive && schedule != pf::kSchedPaired)) return PF_EINVAL;
  if (schedule == pf::kSchedPaired && simple_kernels_only(h->P, h->smooth))
    return fail(h, PF_EINVAL, "the paired schedule implements the SigmaP1-P AC and coupled models only");
  h->sched = schedule;
  h->autotune_pending = 1;
  drop_graph(h);
  return PF_OK;
}

int pf_set_pair_tile(pf_handle* h, int32_t tile_index, int32_t z_chunk) {
  if (!h || tile_index < 0 || tile_index > 2 || z_chunk < 1) return PF_EINVAL;
  h->autotune_pending = 0;
  return set_pair_tiles(h, tile_index, z_chunk);
}

int pf_get_config(const pf_handle* h, int32_t* out) {
  if (!h || !out) return PF_EINVAL;
  const int tsi = h->pair_ts;
  out[0] = h->sched;
  out[1] = num_passes(h);
  out[2] = h->z_chunk;
  out[3] = h->nparts;
  out[4] = pf::kPairTiles[tsi][0];
  out[5] = pf::kPairTiles[tsi][1];
  out[6] = h->pair_zc;
  out[7] = h->npair;
  out[8] = h->vec;
  for (int st = 1; st <= 5; ++st) out[8 + st] = h->st_z[st];
  return PF_OK;
}

}  // extern "C"

/*
 * pf.h - C ABI of the MI355X (gfx950) solver for the pore-scale
 * freezing/thawing phase-field model of P. Strachota, "Three-dimensional
 * phase-field simulations of water freezing and thawing at pore-scale"
 * (arXiv 2401.01672).
 *
 * The library integrates, on one GPU, the method-of-lines system obtained by
 * a finite-volume discretisation (Sec. 2.5) of
 *   - the heat equation with blended conductivity / heat capacity and latent
 *     heat release (Sec. 2.2, eq. heat-equation; blending eq.
 *     material-properties-blending-formula), and
 *   - the Allen-Cahn equation with the SigmaP1-P reaction term and the water
 *     indicator (Sec. 2.2, eqs. Allen-Cahn-equation, reaction-term-SigmaP1-P,
 *     Sigma-limiter, water-indicator),
 * or the micro-scale reduction at constant temperature (Sec. 2.4), with the
 * Runge-Kutta-Merson integrator and adaptive steps (Sec. 2.5).
 *
 * Discretisation (the paper gives the scheme only in words):
 *   - cubic cells of edge h on an n1 x n2 x n3 grid; cell (i1,i2,i3) is stored
 *     at n = i1 + n1*(i2 + n2*i3) (x1 fastest, x3 vertical);
 *   - glass is a binary voxel mask (G in {0,1});
 *   - two-point face fluxes; the face conductivity is the arithmetic mean of
 *     the two cell values; no phase-field flux through a face that touches
 *     glass or lies on the domain boundary (eq. BC-PF);
 *   - temperature faces on the domain boundary are insulated (eq.
 *     BC-temperature-wall) unless listed in dirichlet_faces, where the ghost
 *     value 2 T_D(t) - T_c is used with the cell's own conductivity (eq.
 *     BC-temperature-cap);
 *   - Merson stages k1..k5, new state y + dt (k1 + 4 k4 + k5)/6, error
 *     estimate dt (2 k1 - 9 k3 + 8 k4 - k5)/30, its max-norm over every
 *     unknown; accept when eps <= tol; next step
 *     min(dt_max, safety * dt * (tol/eps)^(1/5)); the last step is clipped to
 *     land on t_end; tol <= 0 selects fixed steps.
 *
 * State: the phase field phi and the temperature offset theta = T - T*
 * (kelvin).  Fields are stored in the handle's precision (PF_FP64 or
 * PF_FP32); the error norm, t, dt and every diagnostic sum are FP64.
 *
 * Conventions: every call returns PF_OK (0), a positive informational code,
 * or a negative error code; nothing throws across the ABI.  pf_last_error()
 * gives a message for the last failing call on a handle (pf_create failures:
 * pf_last_error(NULL)).  A handle is used from one host thread at a time.
 * Device pointers passed in are caller-owned; the handle owns its own state
 * and work buffers and frees them in pf_destroy.  Work is issued on the
 * handle's stream (pf_set_stream; default: a stream the handle creates).
 */
#ifndef PF_H_
#define PF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define PF_OK 0
#define PF_EQUILIBRIUM 1 /* run ended: max over water cells of |d phi/dt| < eq_tol */
#define PF_MAXSTEPS 2    /* run ended: step budget used                           */
#define PF_EINVAL (-1)   /* invalid argument                                      */
#define PF_ENOMEM (-2)   /* device allocation failed                              */
#define PF_EHIP (-3)     /* HIP runtime error                                     */
#define PF_ENONFINITE (-4) /* NaN/Inf in the error estimate: attempt rejected    */
#define PF_EDTMIN (-5)   /* proposed step fell below dt_min                       */

/* Models. */
#define PF_MODEL_AC 0      /* micro-scale: Allen-Cahn only, T = T* - dT (Sec. 2.4) */
#define PF_MODEL_COUPLED 1 /* heat + Allen-Cahn (Sec. 2.2)                          */
#define PF_MODEL_TEMP 2    /* Temp model: phi = varphi(T) (Sec. 2.3)                */

/* Reaction terms of the Allen-Cahn equation. */
#define PF_REACT_SIGMA 0 /* SigmaP1-P, eq. reaction-term-SigmaP1-P */
#define PF_REACT_GRADP 1 /* GradP, eq. reaction-term-GradP         */

/* Field precision. */
#define PF_FP64 0
#define PF_FP32 1

/* Dirichlet temperature schedules T_D(t) (eq. BC-temperature-cap). */
#define PF_BC_CONST 0 /* T_D = bc_T0                                           */
#define PF_BC_RAMP 1  /* linear from bc_T0 at bc_t0 to bc_T1 at bc_t1, clamped  */
#define PF_BC_STEP 2  /* bc_T0 before bc_t0, bc_T1 from bc_t0 on (freeze/thaw)  */

typedef struct pf_handle pf_handle;

/* Problem description; plain data, copied by pf_create. */
typedef struct {
  int32_t n1, n2, n3;     /* cells per axis, each >= 1                          */
  int32_t model;          /* PF_MODEL_*                                         */
  int32_t precision;      /* PF_FP64 | PF_FP32                                  */
  int32_t reaction;       /* PF_REACT_*                                         */
  int32_t dirichlet_faces;/* bit k: face k of (x1-,x1+,x2-,x2+,x3-,x3+)        */
  int32_t bc_kind;        /* PF_BC_*                                            */
  double h;               /* cell edge [m]                                      */
  double xi;              /* interface thickness parameter [m]                  */
  double alpha;           /* attachment kinetics coefficient [s m^-2]           */
  double mu;              /* interface mobility [m s^-1 K^-1]                   */
  double b;               /* SigmaP1-P factor b(eps0, eps1)                     */
  double eps0, eps1;      /* Sigma limiter knots                                */
  double zeta;            /* water indicator parameter                          */
  double t_star;          /* bulk melting point T* [K]                          */
  double dT;              /* supercooling T* - T of PF_MODEL_AC [K]             */
  double gamma;           /* Temp model rate [1/K]                              */
  double lam[3];          /* conductivity: liquid, ice, glass [W m^-1 K^-1]     */
  double rhoc[3];         /* volumetric heat capacity: liquid, ice, glass       */
  double Lv;              /* volumetric latent heat rho L [J m^-3]              */
  double bc_T0, bc_T1;    /* Dirichlet temperatures [K]                         */
  double bc_t0, bc_t1;    /* schedule times [s]                                 */
  double tol;             /* error tolerance; <= 0: fixed steps                 */
  double safety;          /* step-size safety factor                            */
  double dt_min, dt_max;  /* step bounds [s]                                    */
  /* Material model.  0: rho c blended as one volumetric quantity (rhoc) and a
   * constant latent heat per volume (Lv).  1: the paper's own form (Sec. 2.2):
   * density and specific heat blended separately by eq.
   * material-properties-blending-formula, rho c = blend(rho) blend(c), and
   * the latent term blend(rho) L in eq. heat-equation (and in eq.
   * combined-heat-xfer-phase-transition for the Temp model); rhoc and Lv are
   * then unused.  The enthalpy diagnostic uses the same per-cell values. */
  int32_t rho_c_separate;
  int32_t pad_;
  double rho[3];          /* density: liquid, ice, glass [kg m^-3]              */
  double cs[3];           /* specific heat: liquid, ice, glass [J kg^-1 K^-1]   */
  double L;               /* specific latent heat [J kg^-1]                     */
} pf_params;

/* Result of one attempt. */
typedef struct {
  int32_t accepted;  /* 1 if the attempt was accepted                         */
  int32_t status;    /* PF_OK, PF_EQUILIBRIUM, PF_ENONFINITE or PF_EDTMIN      */
  double eps;        /* max-norm of the error estimate                        */
  double dt_used;    /* step of this attempt (after clipping to t_end)       */
  double dt_next;    /* proposed next step                                    */
  double maxk1;      /* max over water cells of |k1_phi| (state at the start) */
  double t;          /* time after the attempt                                */
} pf_step_info;

/* Result of a run and diagnostics of the final state (FP64 sums; cells with
 * G = 0 are water cells, eq. water-occupied-subdomain; ice cells have
 * phi > 1/2, eq. frozen-subdomain; enthalpy = h^3 sum(rho c theta - Lv phi)). */
typedef struct {
  int64_t steps_accepted, steps_rejected;
  double t, dt;          /* time reached and next proposed step                */
  int64_t ice_count, pore_count;
  double sum_phi;        /* sum of phi over water cells                        */
  double enthalpy;       /* [J]                                                */
  double maxk1;          /* last max over water cells of |k1_phi|              */
  double wall_s;         /* host wall time of the call                         */
  int32_t status;        /* PF_OK (t_end reached), PF_EQUILIBRIUM, PF_MAXSTEPS, or an error */
  int32_t pad;
} pf_run_stats;

/* Create a solver for one grid.  mask: host pointer to n1*n2*n3 bytes,
 * nonzero = glass; read during the call only.  The state starts at
 * phi = 0, theta = 0, t = 0, dt = dt_max (use pf_set_state / pf_set_time).
 * Errors: PF_EINVAL (sizes, model/precision/reaction codes, h/xi/alpha <= 0,
 * NULL pointers), PF_ENOMEM, PF_EHIP. */
int pf_create(const pf_params* params, const uint8_t* mask, pf_handle** out);

/* Paper mode (Sec. 2.1): like pf_create, but the glass is a smooth field
 * G in [0, 1] (host pointer, n1*n2*n3 doubles, read during the call only;
 * eq. of G_balls and the cap).  The phase-field Laplacian then acts across
 * every face inside the box (no face rule at glass; the water indicator
 * I_W(G) = max(0, 1 - zeta G) masks the update), and lambda and rho c are
 * blended with each cell's G (eq. material-properties-blending-formula).
 * Water cells for the diagnostics and the equilibrium test: G < 1/2.  Runs
 * on the vector and one-cell stage kernels (no paired or batched variants).
 * Errors: as pf_create, PF_EINVAL for G outside [0, 1]. */
int pf_create_field(const pf_params* params, const double* G, pf_handle** out);

/* Free every resource of the handle.  NULL is ignored. */
void pf_destroy(pf_handle* h);

/* Message of the last failing call on h; h = NULL gives the last pf_create
 * failure of the calling thread.  Never NULL. */
const char* pf_last_error(const pf_handle* h);

/* Use a caller stream (a hipStream_t cast to uintptr_t) for all later work
 * on this handle; 0 restores the handle's own stream. */
int pf_set_stream(pf_handle* h, uintptr_t stream);

/* Stream arguments: a hipStream_t cast to uintptr_t on which the call's
 * device work is issued; 0 = the handle's stream.  A caller stream waits for
 * the work already issued on the handle's stream (the call synchronizes the
 * handle's stream first). */

/* Copy a state in: phi and theta point to n cells each in the handle's
 * precision, on the device (on_device = 1) or the host (0).  theta is
 * ignored for PF_MODEL_AC and phi for PF_MODEL_TEMP (may be NULL).
 * Synchronous with respect to the host. */
int pf_set_state(pf_handle* h, const void* phi, const void* theta, int on_device,
                 uintptr_t stream);

/* Copy the current state out (same layout rules as pf_set_state). */
int pf_get_state(pf_handle* h, void* phi, void* theta, int on_device, uintptr_t stream);

/* Change the error tolerance of later runs (params.tol at creation;
 * <= 0: fixed steps). */
int pf_set_tolerance(pf_handle* h, double tol);

/* Set the current time and the next proposed step. */
int pf_set_time(pf_handle* h, double t, double dt);

/* Right-hand side F(t, phi, theta) of the semi-discrete system (Sec. 2.5,
 * the method of lines applied to eqs. heat-equation and Allen-Cahn-equation):
 * writes dphi = d phi/dt and dtheta = d theta/dt.  All four are device
 * pointers of n cells in the handle's precision; unused fields of the model
 * may be NULL.  Asynchronous on `stream`. */
int pf_rhs(pf_handle* h, double t, const void* phi, const void* theta, void* dphi,
           void* dtheta, uintptr_t stream);

/* One Runge-Kutta-Merson attempt from (*t, current state) with proposed step
 * *dt; on return *t and *dt hold the new time and proposed step and the state
 * is advanced if the attempt was accepted.  info may be NULL.  Synchronous. */
int pf_rkm_step(pf_handle* h, double* t, double* dt, pf_step_info* info);

/* Integrate from the handle's (t, dt) until t_end, max_steps attempts, or
 * equilibrium (eq_tol > 0: max over water cells of |d phi/dt| < eq_tol at the
 * start of a step).  The step loop runs on the device (controller included);
 * the host polls it every few steps.  Returns PF_OK, PF_EQUILIBRIUM,
 * PF_MAXSTEPS or an error code; stats may be NULL.  Synchronous. */
int pf_integrate(pf_handle* h, double t_end, int64_t max_steps, double eq_tol,
                 pf_run_stats* stats);

/* Batched sweep: integrate n independent instances (same model, precision
 * and glass representation; the SigmaP1-P reaction; binary masks, or smooth
 * glass fields (pf_create_field) with mode 2; each with n1 divisible by 4
 * (FP32) or 2 (FP64), each with its own geometry,
 * constants, state, t and dt) together: every stage pass processes the tiles
 * of all unfinished instances in one launch (or one persistent cooperative
 * kernel runs all passes of a poll interval, see pf_batch_options), then each
 * instance's own controller runs (per-instance adaptive dt, equilibrium test
 * and status); finished instances drop out.  Stops each instance at t_end,
 * max_steps attempts, or equilibrium (eq_tol > 0), like pf_integrate.
 * out[i] receives instance i's statistics (wall_s: the whole batch).  stream:
 * a hipStream_t cast to uintptr_t, 0 = the first instance's stream.  The
 * first instance's handle keeps the batch's device work tables (descriptors,
 * work items, gathered control blocks) until pf_destroy, grown when a call
 * needs more: a repeat call with no more instances and work items than an
 * earlier one on the same first handle allocates no device memory of its
 * own (the HIP graph of the poll interval is instantiated per call).
 * Returns PF_OK or the first instance error code; synchronous. */
typedef struct {
  int32_t mode;           /* 1: persistent cooperative kernel: one launch
                                per poll interval, grid barriers between
                                stages;
                             2 (default): one launch per stage over the
                                instances still running, the poll
                                interval's attempts captured as a HIP graph
                                and replayed; the work table and the graph
                                are rebuilt when instances finish          */
  int32_t z_chunk;        /* planes per work item (0: 4 while the running
                             instances make at least 1024 items, halved
                             down to 1 below that)                         */
  int32_t steps_per_poll; /* attempts between host checks (0: 32)          */
  int32_t branches;       /* mode 2: parallel chains of stage launches in
                             the graph over groups of instances; switched
                             off in this build: 0 and 1 (one chain) are
                             accepted, 2 to 4 return PF_EINVAL            */
} pf_batch_options;

/* opts may be NULL (defaults). */
int pf_batch_integrate(pf_handle* const* inst, int32_t n, double t_end, int64_t max_steps,
                       double eq_tol, pf_run_stats* out, uintptr_t stream,
                       const pf_batch_options* opts);

/* Diagnostics of the current state into stats (ice/pore counts, sum_phi,
 * enthalpy); the step counters and t are left as the last run set them. */
int pf_diagnostics(pf_handle* h, pf_run_stats* stats);

/* The same diagnostics over the planes i3_lo <= i3 < i3_hi only
 * (0 <= i3_lo <= i3_hi <= n3, else PF_EINVAL).  With [0, n3/2) (integer
 * division) these are the cells whose centres lie below half the vessel
 * height, over which eq. UWC-formula (Sec. 3.3) takes the unfrozen water
 * content: UWC = 1 - ice_count / pore_count.  Synchronous. */
int pf_diagnostics_planes(pf_handle* h, int32_t i3_lo, int32_t i3_hi, pf_run_stats* stats);

/* Step-loop options: steps_per_poll attempts are issued between host polls;
 * use_graph = 1 captures them once into a HIP graph and replays it.  A
 * pf_integrate call with the equilibrium test (eq_tol > 0) polls after 1, 2,
 * 4, ... attempts, launched directly, until the interval reaches
 * steps_per_poll (a run that starts at or near equilibrium then ends after
 * a few attempts and builds no graph). */
int pf_set_loop(pf_handle* h, int32_t steps_per_poll, int32_t use_graph);

/* Tile shape of the stencil kernels: z_chunk = planes per workgroup column
 * (>= 1); 0 = choose by the built-in autotuner on the next run.  The
 * autotuner runs on a handle's first run; its choice (kernel form and the
 * depth of each pass) is kept for the rest of the process and reused by
 * every handle with the same grid shape, precision, model, reaction, glass
 * representation, streaming mode, schedule and device. */
int pf_set_tile(pf_handle* h, int32_t z_chunk);

/* Planes per workgroup column of each five-pass stage pass: z[0..4] for
 * S1..S5 (each >= 1), in the kernel form the handle has; the RHS pass and
 * the paired schedule follow z[3].  Replaces the autotuner's choice (for
 * reproducible timings and counter runs).  PF_EINVAL if z is NULL or an
 * entry is < 1. */
int pf_set_stage_tiles(pf_handle* h, const int32_t* z);

/* Stencil schedule of one attempt:
 *   0 (default): five passes, one per Merson stage (each fused with its
 *      combinations);
 *   1: three passes -- S1+S2 and S3+S4 each in one pass (the first
 *      stage of a pair is evaluated on the tile plus a one-cell ring and its
 *      output stays in LDS), then S5.
 * Both give the same arithmetic per cell.  Re-runs the tile autotuner. */
int pf_set_schedule(pf_handle* h, int32_t schedule);

/* Single-stage passes on vector kernels, one 16-byte vector of consecutive
 * x1-cells per thread (4 FP32 or 2 FP64 cells; n1 must be divisible by that
 * width, PF_EINVAL otherwise; every model, reaction and glass
 * representation), or on one-cell kernels.  The two forms store
 * different intermediate stage values (the vector passes form Y2 and Y4 at
 * the stencil points from y, k1 and k3; the one-cell passes store them) and
 * give the same results.  The default is the vector form where it applies;
 * the autotuner times both unless this call fixed one. */
int pf_set_vector(pf_handle* h, int32_t enable);

/* Tile of the paired passes: tile_index 0: 64x4, 1: 64x8, 2: 32x8 cells of
 * the x1-x2 plane per workgroup; z_chunk (>= 4) planes per column.  Turns the
 * autotuner off. */
int pf_set_pair_tile(pf_handle* h, int32_t tile_index, int32_t z_chunk);

/* Current configuration, out[0..13] = {schedule, passes per attempt,
 * single-stage z_chunk, single-stage workgroups, pair tile x, pair tile y,
 * pair z_chunk, pair workgroups, vector kernels (1) or one-cell (0),
 * z_chunk of S1, S2, S3, S4, S5} (after the autotuner, if it has run: it
 * times both kernel forms unless pf_set_vector fixed one, and picks the
 * planes per workgroup column of each stage pass separately; the
 * single-stage z_chunk is then S4's).  out must hold 14 values. */
int pf_get_config(const pf_handle* h, int32_t* out);

/* Time each kernel of one attempt from the current state and step: the
 * passes of an attempt run in order with a HIP event between each two (so
 * each pass reads what the previous one has just written, as in a run),
 * reps times after one warm-up; ms[i] receives the mean duration of pass i
 * (S1..S5, or the three passes of the paired schedule; the last pass
 * includes the step controller, which runs in its last workgroup, on a
 * scratch control block) and ms[5] that of the controller alone (reps
 * back-to-back standalone launches on a scratch control block; runs issue no
 * such launch).  The state, t and dt are left unchanged.  Synchronous. */
int pf_time_kernels(pf_handle* h, int32_t reps, double* ms);

/* Block the host until all work issued on the handle's stream is done. */
int pf_synchronize(pf_handle* h);

/* Number of cells and bytes per field of the handle (for callers that
 * allocate matching buffers). */
int64_t pf_num_cells(const pf_handle* h);

/* ------------------------------------------------------------------------
 * Learned warm start (not part of the paper's method: an accelerator for
 * sweeps to equilibrium).  A 3D U-Net maps the glass mask, the supercooling
 * dT and the surface-tension scale s (alpha = alpha_real / s) of a
 * micro-scale problem to a phase field phi0 on the water cells, which then
 * relaxes to equilibrium under the model of Sec. 2.4 (pf_integrate).
 *
 * Architecture: input channels {glass (0/1), log10(dT / 0.2 K),
 * (log10 s - 1.5) / 1.5, 5 zero channels}; levels of 16, 32, 64 channels
 * at full, half and quarter resolution; per level (and per decoder stage)
 * two 3x3x3 convolutions (zero padding) + ReLU; 2x average pooling; nearest
 * 2x upsampling; skip connections by channel concatenation [upsampled,
 * skip]; 1x1 head + sigmoid, 0 on glass cells.  Convolutions run as
 * implicit GEMMs on BF16 matrix cores with FP32 accumulation; activations
 * are BF16, parameters, gradients and Adam moments FP32.
 *
 * Flat parameter vector (pf_unet_num_params floats): for each of the ten
 * convolutions in the order enc1a, enc1b, enc2a, enc2b, enc3a, enc3b,
 * dec2a, dec2b, dec1a, dec1b: weights [cout][27][cin] with tap
 * (dz+1)*9 + (dy+1)*3 + (dx+1) (dx along x1, dz along x3), then bias
 * [cout]; then the head's 16 weights and 1 bias.  Channel counts (cin ->
 * cout): 8->16, 16->16, 16->32, 32->32, 32->64, 64->64, 96->32, 32->32,
 * 48->16, 16->16 (pf_unet_layer_info).
 *
 * Grids: n1, n2, n3 positive multiples of 4 with n1*n2*n3 < 2^24.  All
 * pointers named mask/target/out are device pointers: mask n cells of
 * uint8 (nonzero = glass), target and out n floats, layout
 * i1 + n1*(i2 + n2*i3).  Each call works on the network's stream
 * (pf_unet_set_stream; default the null stream).  A network object must not
 * be used from two threads at once.
 * ------------------------------------------------------------------------ */
typedef struct pf_unet pf_unet;

/* New network with He-normal weights drawn from SplitMix64(seed) and zero
 * biases.  Errors: PF_EINVAL (out NULL), PF_ENOMEM, PF_EHIP. */
int pf_unet_create(uint64_t seed, pf_unet** out);
void pf_unet_destroy(pf_unet* net);
const char* pf_unet_last_error(const pf_unet* net);
int pf_unet_set_stream(pf_unet* net, uintptr_t stream);
/* Forward (and data-gradient) convolution kernel of this network:
 * 2 (default): register-blocked where it is faster (16 -> 32 channels on
 * grids of at least 2^16 voxels), else as 1 -- per group of 8 input
 * channels the input block and the weights are copied into LDS
 * asynchronously (double buffered) and every staged input row feeds all the
 * output rows and planes it reaches;
 * 1: LDS-tiled -- a 16 x 4 x 4 block of output voxels per workgroup (16 x 4
 * x 8 for 16 output channels on large grids) with its input halo (and, for
 * 16 output channels, the weights) staged in LDS per chunk of input
 * channels;
 * 0: direct -- every B fragment gathered from memory.  Same products; the
 * FP32 partial sums are taken in another order. */
int pf_unet_set_conv_kernel(pf_unet* net, int32_t variant);
int64_t pf_unet_num_params(void);

/* Copy the parameter vector out / in (host pointers, pf_unet_num_params
 * floats).  Setting parameters resets the Adam state.  Synchronous. */
int pf_unet_get_params(pf_unet* net, float* host_out);
int pf_unet_set_params(pf_unet* net, const float* host_in);

/* Inference: out = network(mask, dT, s) with log10_sigma_scale = log10 s.
 * Asynchronous on the network's stream. */
int pf_unet_forward(pf_unet* net, const uint8_t* mask, int32_t n1, int32_t n2, int32_t n3,
                    double dT, double log10_sigma_scale, float* out);

/* Loss L = mean over water cells of (out - target)^2 and its gradient with
 * respect to the parameter vector (written to grad_host if non-NULL;
 * *loss if non-NULL).  No update.  Synchronous. */
int pf_unet_grad(pf_unet* net, const uint8_t* mask, const float* target, int32_t n1, int32_t n2,
                 int32_t n3, double dT, double log10_sigma_scale, float* grad_host,
                 double* loss);

/* One training step on one sample: the gradient as in pf_unet_grad, then one
 * Adam update (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with
 * learning rate lr.  Asynchronous unless loss is non-NULL (then it waits for
 * the loss of this sample, before the update). */
int pf_unet_train_step(pf_unet* net, const uint8_t* mask, const float* target, int32_t n1,
                       int32_t n2, int32_t n3, double dT, double log10_sigma_scale, double lr,
                       double* loss);

/* Mean duration of each of the ten forward convolutions on an n1 x n2 x n3
 * input (ms[0..9]; reps launches back to back between HIP events on the
 * network's stream; the activation buffers hold whatever the last call
 * left).  Synchronous. */
int pf_unet_time_layers(pf_unet* net, int32_t n1, int32_t n2, int32_t n3, int32_t reps,
                        double* ms);

/* out[0..7] = {cin, cout, weight offset, bias offset, grid level (0 full,
 * 1 half, 2 quarter), head weight offset, head bias offset, number of
 * convolutions} of convolution `layer`. */
int pf_unet_layer_info(int32_t layer, int32_t* out);

/* Warm-start modes. */
#define PF_WARM_ALL 0     /* the prediction on every cell                       */
#define PF_WARM_NUCLEUS 1 /* the prediction on the nucleus's water component     */
#define PF_WARM_FLOOD 2   /* no network: phi = 1 on the nucleus's water component */

/* Write the network's prediction for the handle's mask (PF_MODEL_AC or
 * PF_MODEL_COUPLED; dT > 0, log10_sigma_scale = log10 s) into the handle's
 * current phi (in its precision; theta, t and dt are not changed).
 * PF_WARM_NUCLEUS (the warm start proper) reads the current phi first as the
 * nucleus: the prediction is kept only on the water cells connected through
 * water-water faces to a water cell with phi > 1/2, and is 0 elsewhere (with
 * no phase-field flux through glass faces, a face-connected water component
 * without ice keeps phi = 0, since phi = 0 is a fixed point of the reaction
 * term of the phase-field equation, Sec. 2.2).  PF_WARM_FLOOD is the
 * baseline without the network: phi = 1 on that component (the network
 * object provides only its work buffers).  The handle's n1, n2, n3 must
 * satisfy the network's grid rule.  Work is issued on `stream` (0: the
 * handle's stream); synchronous. */
int pf_warmstart(pf_handle* h, pf_unet* net, double dT, double log10_sigma_scale, int32_t mode,
                 uintptr_t stream);

/* Building blocks (each call allocates and frees its own scratch; device
 * pointers; BF16 tensors channels-last [n][c], FP32 weights [cout][27][cin],
 * taps as above; the convolutions run on the kernel that
 * pf_unet_set_conv_kernel selects with 2).  y = act(conv3x3x3(x) + b) with
 * act = ReLU if relu != 0;
 * cin % 8 == 0, cout in {16, 32, 48, 64, 96}; b may be NULL.  Synchronous. */
int pf_conv3_bf16(const uint16_t* x, int32_t cin, const float* w, const float* b, int32_t relu,
                  uint16_t* y, int32_t cout, int32_t n1, int32_t n2, int32_t n3,
                  uintptr_t stream);
/* Allocation-free variant of pf_conv3_bf16, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, layouts and result as
 * pf_conv3_bf16 (the same kernels), with two differences:
 *   - the BF16 weight copy is kept in a static device array of the library
 *     (cin <= 96 and cout <= 96; 486 KiB per device, held until the process
 *     ends) instead of a per-call allocation: no hipMalloc, hipFree or
 *     allocating library call is made.  Larger cin or cout give PF_EINVAL
 *     and a message in pf_last_error(NULL);
 *   - it is asynchronous on `stream`, whose device must be the current one.
 * Every call on a device shares that device's array: calls that overlap on
 * one device (other streams, or another thread) race and give wrong
 * results.  Returns PF_OK, PF_EINVAL or PF_EHIP (message in
 * pf_last_error(NULL)). */
int pf_conv3_bf16_noalloc(const uint16_t* x, int32_t cin, const float* w, const float* b,
                          int32_t relu, uint16_t* y, int32_t cout, int32_t n1, int32_t n2,
                          int32_t n3, uintptr_t stream);
/* Gradients of y = conv3x3x3(x) + b given dy: dw [cout][27][cin], db [cout],
 * and dx [n][cin] if dx is non-NULL (then cin in {16, 32, 48, 64, 96}).
 * (cout/16) * ceil(cin/16) <= 16.  Synchronous. */
int pf_conv3_bf16_backward(const uint16_t* x, int32_t cin, const float* w, const uint16_t* dy,
                           int32_t cout, int32_t n1, int32_t n2, int32_t n3, uint16_t* dx,
                           float* dw, float* db, uintptr_t stream);
/* One 16x16x32 BF16 matrix-core product c = a b (a 16x32, b 32x16, c 16x16,
 * row-major FP32, device pointers; inputs rounded to BF16). */
int pf_mfma_probe(const float* a, const float* b, float* c, uintptr_t stream);

/* Library ABI version. */
int pf_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PF_H_ */

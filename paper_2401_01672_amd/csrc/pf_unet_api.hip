// C ABI of the warm-start network (declarations and semantics in include/pf.h).
//
// The network maps (glass mask, supercooling dT, surface-tension scale) on a
// voxel grid to a phase field phi0 in [0, 1] on the water cells, which seeds
// the Allen-Cahn relaxation.  Three resolution levels with 16, 32 and 64
// channels, two 3x3x3 convolutions with ReLU per level and per decoder
// stage, 2x average pooling, nearest 2x upsampling, skip connections by
// channel concatenation, a 1x1 head with a sigmoid, masked to water cells.
// Training minimises the mean squared error over water cells with Adam.
//
// Storage: FP32 master parameters, Adam moments and gradients (one flat
// vector each); BF16 activations and activation gradients; BF16 weight
// copies refreshed after every update.
#include <math.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "pf_internal.h"
#include "pf_unet_internal.h"

using pfu::ConvArgs;
using pfu::HeadArgs;
using pfu::View;
using pfu::WgradArgs;

namespace {

struct LayerSpec {
  int cin, cout;
};
// encoder level 1, 2, 3; decoder level 2, 1
constexpr LayerSpec kLayers[10] = {{8, 16},  {16, 16}, {16, 32}, {32, 32}, {32, 64},
                                   {64, 64}, {96, 32}, {32, 32}, {48, 16}, {16, 16}};
constexpr int kNumLayers = 10;
constexpr int kInChannels = 8;  // glass, dT feature, scale feature, 5 zero channels

inline int round32(int k) { return (k + 31) & ~31; }

struct Layer {
  int cin, cout, kpad, kpad_t;
  long long w_off, b_off;  // into the flat parameter vector
  uint16_t* wf = nullptr;  // [cout][kpad]
  uint16_t* wd = nullptr;  // [cin][kpad_t]
};

long long param_layout(Layer* L, long long* head_w, long long* head_b) {
  long long off = 0;
  for (int i = 0; i < kNumLayers; ++i) {
    L[i].cin = kLayers[i].cin;
    L[i].cout = kLayers[i].cout;
    L[i].kpad = round32(27 * L[i].cin);
    L[i].kpad_t = round32(27 * L[i].cout);
    L[i].w_off = off;
    off += 27LL * L[i].cin * L[i].cout;
    L[i].b_off = off;
    off += L[i].cout;
  }
  *head_w = off;
  off += 16;
  *head_b = off;
  off += 1;
  return off;
}

struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
  // Box-Muller
  double normal() {
    double u1 = uniform(), u2 = uniform();
    if (u1 < 1e-300) u1 = 1e-300;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
};

}  // namespace

struct pf_unet {
  std::string err;
  hipStream_t stream = nullptr;
  Layer L[kNumLayers];
  long long head_w = 0, head_b = 0, nparams = 0;
  float* params = nullptr;
  float* grad = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  uint16_t* wslab = nullptr;
  long long adam_step = 0;
  int weights_dirty = 1;
  int conv_variant = 2;  // forward-convolution kernel (2 register-blocked where it is faster, 1 LDS-tiled, 0 direct)
  // grid-dependent buffers
  int n1 = 0, n2 = 0, n3 = 0, train = 0;
  void* slab = nullptr;
  uint16_t *X0, *A1, *C1, *E1, *F1, *P1, *A2, *C2, *E2, *F2, *P2, *A3, *B3;
  uint16_t *S1, *S2;  // skip tensors (layers 1 and 3), copied into C1 / C2 with the upsampling
  uint16_t *gN16a, *gN16b, *gC1, *gP1, *gM32a, *gM32b, *gC2, *gQ32, *gQ64a, *gQ64b;
  float* wpart = nullptr;   // weight-gradient partials
  float* bpart = nullptr;   // bias-gradient partials
  float* hpart = nullptr;   // head partials
  float* hsum = nullptr;    // [kHeadParts] reduced head sums
  float* count = nullptr;   // number of water cells
  float* cpart = nullptr;   // count partials
  uint8_t* reach = nullptr; // water cells connected to the nucleus
  int* lab = nullptr;       // union-find parents of the reachability labelling
  float* hostbuf = nullptr; // pinned, 32 floats
};

namespace {

int ufail(pf_unet* n, int code, const std::string& msg) {
  if (n) n->err = msg;
  return code;
}

#define PFU_HIP(n, expr)                                                               \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return ufail((n), PF_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)

void free_grid(pf_unet* n) {
  if (n->slab) (void)hipFree(n->slab);
  n->slab = nullptr;
  n->n1 = n->n2 = n->n3 = 0;
  n->train = 0;
}

// one device slab, every sub-buffer 256-byte aligned
struct Carver {
  size_t off = 0;
  char* base = nullptr;
  template <typename T>
  T* take(size_t count) {
    const size_t at = off;
    off += (count * sizeof(T) + 255) & ~(size_t)255;
    return base ? reinterpret_cast<T*>(base + at) : nullptr;
  }
};

int ensure_grid(pf_unet* n, int n1, int n2, int n3, int train) {
  if (n1 <= 0 || n2 <= 0 || n3 <= 0 || n1 % 4 || n2 % 4 || n3 % 4)
    return ufail(n, PF_EINVAL, "grid sizes must be positive multiples of 4 (two 2x poolings)");
  if (n->slab && n->n1 == n1 && n->n2 == n2 && n->n3 == n3 && (n->train || !train)) return PF_OK;
  PFU_HIP(n, hipStreamSynchronize(n->stream));
  free_grid(n);
  const size_t N = (size_t)n1 * n2 * n3, M = N / 8, Q = N / 64;
  const int wb = pfu::wgrad_blocks((long long)N);
  const int hb = pfu::head_blocks((long long)N);
  for (int pass = 0; pass < 2; ++pass) {
    Carver c;
    c.base = static_cast<char*>(n->slab);
    n->X0 = c.take<uint16_t>(N * kInChannels);
    n->A1 = c.take<uint16_t>(N * 16);
    n->C1 = c.take<uint16_t>(N * 48);
    n->S1 = c.take<uint16_t>(N * 16);
    n->E1 = c.take<uint16_t>(N * 16);
    n->F1 = c.take<uint16_t>(N * 16);
    n->P1 = c.take<uint16_t>(M * 16);
    n->A2 = c.take<uint16_t>(M * 32);
    n->C2 = c.take<uint16_t>(M * 96);
    n->S2 = c.take<uint16_t>(M * 32);
    n->E2 = c.take<uint16_t>(M * 32);
    n->F2 = c.take<uint16_t>(M * 32);
    n->P2 = c.take<uint16_t>(Q * 32);
    n->A3 = c.take<uint16_t>(Q * 64);
    n->B3 = c.take<uint16_t>(Q * 64);
    n->hsum = c.take<float>(32);
    n->count = c.take<float>(1);
    n->cpart = c.take<float>(hb);
    n->reach = c.take<uint8_t>(N);
    n->lab = c.take<int>(N);
    if (train) {
      n->gN16a = c.take<uint16_t>(N * 16);
      n->gN16b = c.take<uint16_t>(N * 16);
      n->gC1 = c.take<uint16_t>(N * 48);
      n->gP1 = c.take<uint16_t>(M * 16);
      n->gM32a = c.take<uint16_t>(M * 32);
      n->gM32b = c.take<uint16_t>(M * 32);
      n->gC2 = c.take<uint16_t>(M * 96);
      n->gQ32 = c.take<uint16_t>(Q * 32);
      n->gQ64a = c.take<uint16_t>(Q * 64);
      n->gQ64b = c.take<uint16_t>(Q * 64);
      n->wpart = c.take<float>((size_t)wb * 27 * 64 * 96);
      n->bpart = c.take<float>((size_t)wb * 96);
      n->hpart = c.take<float>((size_t)hb * pfu::kHeadParts);
    } else {
      n->gN16a = n->gN16b = n->gC1 = n->gP1 = n->gM32a = n->gM32b = n->gC2 = n->gQ32 = nullptr;
      n->gQ64a = n->gQ64b = nullptr;
      n->wpart = n->bpart = n->hpart = nullptr;
    }
    if (pass == 0) {
      if (hipMalloc(&n->slab, c.off) != hipSuccess) {
        n->slab = nullptr;
        (void)hipGetLastError();
        return ufail(n, PF_ENOMEM, "device allocation of the network buffers failed");
      }
    }
  }
  n->n1 = n1;
  n->n2 = n2;
  n->n3 = n3;
  n->train = train;
  return PF_OK;
}

int refresh_weights(pf_unet* n) {
  if (!n->weights_dirty) return PF_OK;
  for (int i = 0; i < kNumLayers; ++i) {
    Layer& l = n->L[i];
    PFU_HIP(n, pfu::launch_weights(n->params + l.w_off, l.cout, l.cin, l.kpad, l.kpad_t, l.wf,
                                   l.wd, n->stream));
  }
  n->weights_dirty = 0;
  return PF_OK;
}

inline View V(uint16_t* p, int stride, int off) { return View{p, stride, off}; }

// forward convolution of layer i from view x to view y on grid (g1, g2, g3)
int conv(pf_unet* n, int i, View x, View y, int g1, int g2, int g3) {
  const Layer& l = n->L[i];
  ConvArgs a;
  a.in = x.p;
  a.in_stride = x.stride;
  a.in_off = x.off;
  a.cin = l.cin;
  a.w = l.wf;
  a.kpad = l.kpad;
  a.bias = n->params + l.b_off;
  a.out = y.p;
  a.out_stride = y.stride;
  a.out_off = y.off;
  a.cout = l.cout;
  a.relu = 1;
  a.n1 = g1;
  a.n2 = g2;
  a.n3 = g3;
  a.variant = n->conv_variant;
  PFU_HIP(n, pfu::launch_conv_fwd(a, n->stream));
  return PF_OK;
}

// backward of layer i: dy (pre-activation gradient, in place after the ReLU
// mask), x = layer input; writes dW, db into the gradient vector and, if dx
// is given, the input gradient
int conv_bwd(pf_unet* n, int i, View dy, View y, View x, const View* dx, int g1, int g2,
             int g3) {
  const Layer& l = n->L[i];
  const long long nv = (long long)g1 * g2 * g3;
  PFU_HIP(n, pfu::launch_relu_bwd(dy.p, dy.stride, dy.off, y.p, y.stride, y.off, l.cout, nv,
                                  n->stream));
  WgradArgs w;
  w.dy = dy.p;
  w.dy_stride = dy.stride;
  w.dy_off = dy.off;
  w.cout = l.cout;
  w.x = x.p;
  w.x_stride = x.stride;
  w.x_off = x.off;
  w.cin = l.cin;
  w.n1 = g1;
  w.n2 = g2;
  w.n3 = g3;
  w.part = n->wpart;
  w.part_bias = n->bpart;
  PFU_HIP(n, pfu::launch_conv_wgrad(w, pfu::wgrad_blocks(nv), n->grad + l.w_off,
                                    n->grad + l.b_off, n->stream));
  if (dx) {
    ConvArgs a;
    a.in = dy.p;
    a.in_stride = dy.stride;
    a.in_off = dy.off;
    a.cin = l.cout;
    a.w = l.wd;
    a.kpad = l.kpad_t;
    a.bias = nullptr;
    a.out = dx->p;
    a.out_stride = dx->stride;
    a.out_off = dx->off;
    a.cout = l.cin;
    a.relu = 0;
    a.n1 = g1;
    a.n2 = g2;
    a.n3 = g3;
    a.variant = n->conv_variant;
    PFU_HIP(n, pfu::launch_conv_fwd(a, n->stream));
  }
  return PF_OK;
}

float feature_dT(double dT) { return (float)log10(dT / 0.2); }
float feature_scale(double log10_s) { return (float)((log10_s - 1.5) / 1.5); }

#define PFU_TRY(expr)        \
  do {                       \
    int r_ = (expr);         \
    if (r_ != PF_OK) return r_; \
  } while (0)

// forward pass; with target != null also the backward pass into n->grad
int run_net(pf_unet* n, const uint8_t* glass, int from_code, double dT, double log10_s,
            void* out, int out_fp64, const float* target, const uint8_t* keep = nullptr) {
  const int N1 = n->n1, N2 = n->n2, N3 = n->n3;
  const int M1 = N1 / 2, M2 = N2 / 2, M3 = N3 / 2;
  const int Q1 = N1 / 4, Q2 = N2 / 4, Q3 = N3 / 4;
  const long long N = (long long)N1 * N2 * N3;
  hipStream_t s = n->stream;
  PFU_TRY(refresh_weights(n));
  PFU_HIP(n, pfu::launch_input(glass, from_code, feature_dT(dT), feature_scale(log10_s), n->X0, N,
                               s));
  // encoder
  PFU_TRY(conv(n, 0, V(n->X0, 8, 0), V(n->A1, 16, 0), N1, N2, N3));
  PFU_TRY(conv(n, 1, V(n->A1, 16, 0), V(n->S1, 16, 0), N1, N2, N3));
  PFU_HIP(n, pfu::launch_pool_fwd(V(n->S1, 16, 0), V(n->P1, 16, 0), 16, M1, M2, M3, s));
  PFU_TRY(conv(n, 2, V(n->P1, 16, 0), V(n->A2, 32, 0), M1, M2, M3));
  PFU_TRY(conv(n, 3, V(n->A2, 32, 0), V(n->S2, 32, 0), M1, M2, M3));
  PFU_HIP(n, pfu::launch_pool_fwd(V(n->S2, 32, 0), V(n->P2, 32, 0), 32, Q1, Q2, Q3, s));
  PFU_TRY(conv(n, 4, V(n->P2, 32, 0), V(n->A3, 64, 0), Q1, Q2, Q3));
  PFU_TRY(conv(n, 5, V(n->A3, 64, 0), V(n->B3, 64, 0), Q1, Q2, Q3));
  // decoder
  PFU_HIP(n, pfu::launch_up_cat(V(n->B3, 64, 0), V(n->S2, 32, 0), V(n->C2, 96, 0), 64, 32, M1, M2,
                                M3, s));
  PFU_TRY(conv(n, 6, V(n->C2, 96, 0), V(n->E2, 32, 0), M1, M2, M3));
  PFU_TRY(conv(n, 7, V(n->E2, 32, 0), V(n->F2, 32, 0), M1, M2, M3));
  PFU_HIP(n, pfu::launch_up_cat(V(n->F2, 32, 0), V(n->S1, 16, 0), V(n->C1, 48, 0), 32, 16, N1, N2,
                                N3, s));
  PFU_TRY(conv(n, 8, V(n->C1, 48, 0), V(n->E1, 16, 0), N1, N2, N3));
  PFU_TRY(conv(n, 9, V(n->E1, 16, 0), V(n->F1, 16, 0), N1, N2, N3));
  HeadArgs h;
  h.h = n->F1;
  h.h_stride = 16;
  h.h_off = 0;
  h.w = n->params + n->head_w;
  h.b = n->params + n->head_b;
  h.glass = glass;
  h.code_glass = from_code;
  h.keep = keep;
  h.nvox = N;
  h.out = out;
  h.out_fp64 = out_fp64;
  h.target = target;
  h.count = n->count;
  h.dh = n->gN16a;
  h.part = n->hpart;
  if (target)
    PFU_HIP(n, pfu::launch_count_water(glass, from_code, N, n->cpart, n->count, s));
  PFU_HIP(n, pfu::launch_head(h, s));
  if (!target) return PF_OK;
  // head gradients: hsum = {sum sq err, dL/db, dL/dw[16]}
  PFU_HIP(n, pfu::launch_reduce(n->hpart, pfu::head_blocks(N), pfu::kHeadParts, n->hsum, s));
  PFU_HIP(n, hipMemcpyAsync(n->grad + n->head_w, n->hsum + 2, 16 * sizeof(float),
                            hipMemcpyDeviceToDevice, s));
  PFU_HIP(n, hipMemcpyAsync(n->grad + n->head_b, n->hsum + 1, sizeof(float),
                            hipMemcpyDeviceToDevice, s));
  // decoder level 1
  const View dx9 = V(n->gN16b, 16, 0);
  PFU_TRY(conv_bwd(n, 9, V(n->gN16a, 16, 0), V(n->F1, 16, 0), V(n->E1, 16, 0), &dx9, N1, N2, N3));
  const View dx8 = V(n->gC1, 48, 0);
  PFU_TRY(conv_bwd(n, 8, V(n->gN16b, 16, 0), V(n->E1, 16, 0), V(n->C1, 48, 0), &dx8, N1, N2, N3));
  PFU_HIP(n, pfu::launch_up_bwd(V(n->gC1, 48, 0), V(n->gM32a, 32, 0), 32, M1, M2, M3, s));
  // decoder level 2
  const View dx7 = V(n->gM32b, 32, 0);
  PFU_TRY(conv_bwd(n, 7, V(n->gM32a, 32, 0), V(n->F2, 32, 0), V(n->E2, 32, 0), &dx7, M1, M2, M3));
  const View dx6 = V(n->gC2, 96, 0);
  PFU_TRY(conv_bwd(n, 6, V(n->gM32b, 32, 0), V(n->E2, 32, 0), V(n->C2, 96, 0), &dx6, M1, M2, M3));
  PFU_HIP(n, pfu::launch_up_bwd(V(n->gC2, 96, 0), V(n->gQ64a, 64, 0), 64, Q1, Q2, Q3, s));
  // level 3
  const View dx5 = V(n->gQ64b, 64, 0);
  PFU_TRY(conv_bwd(n, 5, V(n->gQ64a, 64, 0), V(n->B3, 64, 0), V(n->A3, 64, 0), &dx5, Q1, Q2, Q3));
  const View dx4 = V(n->gQ32, 32, 0);
  PFU_TRY(conv_bwd(n, 4, V(n->gQ64b, 64, 0), V(n->A3, 64, 0), V(n->P2, 32, 0), &dx4, Q1, Q2, Q3));
  // pooling adds into the skip gradient of level 2
  PFU_HIP(n, pfu::launch_pool_bwd(V(n->gQ32, 32, 0), V(n->gC2, 96, 64), 32, M1, M2, M3, 1, s));
  const View dx3 = V(n->gM32a, 32, 0);
  PFU_TRY(conv_bwd(n, 3, V(n->gC2, 96, 64), V(n->S2, 32, 0), V(n->A2, 32, 0), &dx3, M1, M2, M3));
  const View dx2 = V(n->gP1, 16, 0);
  PFU_TRY(conv_bwd(n, 2, V(n->gM32a, 32, 0), V(n->A2, 32, 0), V(n->P1, 16, 0), &dx2, M1, M2, M3));
  PFU_HIP(n, pfu::launch_pool_bwd(V(n->gP1, 16, 0), V(n->gC1, 48, 32), 16, N1, N2, N3, 1, s));
  const View dx1 = V(n->gN16a, 16, 0);
  PFU_TRY(conv_bwd(n, 1, V(n->gC1, 48, 32), V(n->S1, 16, 0), V(n->A1, 16, 0), &dx1, N1, N2, N3));
  PFU_TRY(conv_bwd(n, 0, V(n->gN16a, 16, 0), V(n->A1, 16, 0), V(n->X0, 8, 0), nullptr, N1, N2,
                   N3));
  return PF_OK;
}

int check_dims(pf_unet* n, int n1, int n2, int n3) {
  if (n1 <= 0 || n2 <= 0 || n3 <= 0 || n1 % 4 || n2 % 4 || n3 % 4)
    return ufail(n, PF_EINVAL, "grid sizes must be positive multiples of 4 (two 2x poolings)");
  if ((long long)n1 * n2 * n3 >= (1LL << 24))
    return ufail(n, PF_EINVAL, "grid too large (the water-cell count is kept exactly in FP32)");
  return PF_OK;
}

int read_loss(pf_unet* n, double* loss) {
  if (!loss) return PF_OK;
  PFU_HIP(n, hipMemcpyAsync(n->hostbuf, n->hsum, 2 * sizeof(float), hipMemcpyDeviceToHost,
                            n->stream));
  PFU_HIP(n, hipMemcpyAsync(n->hostbuf + 2, n->count, sizeof(float), hipMemcpyDeviceToHost,
                            n->stream));
  PFU_HIP(n, hipStreamSynchronize(n->stream));
  *loss = n->hostbuf[2] > 0 ? (double)n->hostbuf[0] / (double)n->hostbuf[2] : 0.0;
  return PF_OK;
}

}  // namespace

namespace {

// reach = water cells connected through water-water faces to a water cell
// with phi > 1/2: a union-find labelling of the water components, four
// launches on the stream, no host round trip
int nucleus_reach(pf_unet* n, const uint8_t* code, const void* phi, int fp64) {
  PFU_HIP(n, pfu::launch_reach(code, phi, fp64, n->lab, n->reach, n->n1, n->n2, n->n3, n->stream));
  return PF_OK;
}

}  // namespace

// internal entry used by pf_warmstart: forward pass into a solver state
int pfu_forward_into(pf_unet* n, const uint8_t* code, int n1, int n2, int n3, double dT,
                     double log10_s, void* out, int out_fp64, int mode, hipStream_t s,
                     std::string* err) {
  hipStream_t saved = n->stream;
  n->stream = s;
  const bool reach = mode == PF_WARM_NUCLEUS || mode == PF_WARM_FLOOD;
  int r = check_dims(n, n1, n2, n3);
  if (r == PF_OK) r = ensure_grid(n, n1, n2, n3, n->train);
  if (r == PF_OK && reach) r = nucleus_reach(n, code, out, out_fp64);
  if (r == PF_OK && mode == PF_WARM_FLOOD) {
    const hipError_t e =
        pfu::launch_flood(n->reach, out, out_fp64, (long long)n1 * n2 * n3, n->stream);
    if (e != hipSuccess) r = ufail(n, PF_EHIP, std::string("flood: ") + hipGetErrorString(e));
  } else if (r == PF_OK) {
    r = run_net(n, code, 1, dT, log10_s, out, out_fp64, nullptr, reach ? n->reach : nullptr);
  }
  n->stream = saved;
  if (r != PF_OK && err) *err = n->err;
  return r;
}

// Allocation-free forward convolution.  The only scratch memory of the
// forward convolution is the BF16 copy of the weights in the implicit-GEMM
// layout [cout][kpad]; here it lives in a file-scope device array sized for
// cin, cout <= 96 instead of a per-call allocation.  Host code never uses the
// array's name as an address: the device address is looked up once per
// device and kept.
namespace {
constexpr int kNoAllocMaxCin = 96;
constexpr int kNoAllocMaxCout = 96;
constexpr size_t kNoAllocWords = (size_t)kNoAllocMaxCout * ((27 * kNoAllocMaxCin + 31) & ~31);
constexpr int kNoAllocMaxDevices = 64;
std::mutex g_scratch_mu;
uint16_t* g_scratch_dev[kNoAllocMaxDevices] = {};
}  // namespace

static __device__ __align__(256) uint16_t scratch[kNoAllocWords];

namespace {
// Device address of `scratch` on the current device (looked up on the first
// call made with that device current).
int noalloc_scratch(uint16_t** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    pf::set_thread_error(std::string("pf_conv3_bf16_noalloc: hipGetDevice: ") + hipGetErrorString(e));
    return PF_EHIP;
  }
  if (dev < 0 || dev >= kNoAllocMaxDevices) {
    pf::set_thread_error("pf_conv3_bf16_noalloc: device index out of range");
    return PF_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      pf::set_thread_error(std::string("pf_conv3_bf16_noalloc: hipGetSymbolAddress: ") +
                           hipGetErrorString(e));
      return PF_EHIP;
    }
    g_scratch_dev[dev] = static_cast<uint16_t*>(p);
  }
  *out = g_scratch_dev[dev];
  return PF_OK;
}
}  // namespace

extern "C" {

int pf_unet_create(uint64_t seed, pf_unet** out) {
  if (!out) return PF_EINVAL;
  *out = nullptr;
  pf_unet* n = new pf_unet();
  n->nparams = param_layout(n->L, &n->head_w, &n->head_b);
  const size_t pb = (size_t)n->nparams * sizeof(float);
  auto bad = [&](int code) {
    pf_unet_destroy(n);
    return code;
  };
  if (hipMalloc(&n->params, pb) != hipSuccess || hipMalloc(&n->grad, pb) != hipSuccess ||
      hipMalloc(&n->adam_m, pb) != hipSuccess || hipMalloc(&n->adam_v, pb) != hipSuccess)
    return bad(PF_ENOMEM);
  size_t wel = 0;
  for (int i = 0; i < kNumLayers; ++i)
    wel += (size_t)n->L[i].cout * n->L[i].kpad + (size_t)n->L[i].cin * n->L[i].kpad_t;
  if (hipMalloc(&n->wslab, wel * sizeof(uint16_t)) != hipSuccess) return bad(PF_ENOMEM);
  size_t at = 0;
  for (int i = 0; i < kNumLayers; ++i) {
    n->L[i].wf = n->wslab + at;
    at += (size_t)n->L[i].cout * n->L[i].kpad;
    n->L[i].wd = n->wslab + at;
    at += (size_t)n->L[i].cin * n->L[i].kpad_t;
  }
  if (hipHostMalloc(&n->hostbuf, 32 * sizeof(float), hipHostMallocDefault) != hipSuccess)
    return bad(PF_ENOMEM);
  // He-normal initialisation (fan-in of the used input channels), zero biases
  std::vector<float> p((size_t)n->nparams, 0.0f);
  SplitMix64 rng{seed};
  for (int i = 0; i < kNumLayers; ++i) {
    const Layer& l = n->L[i];
    const int cin_used = i == 0 ? 3 : l.cin;
    const double sd = sqrt(2.0 / (27.0 * cin_used));
    for (int co = 0; co < l.cout; ++co)
      for (int t = 0; t < 27; ++t)
        for (int ci = 0; ci < l.cin; ++ci)
          p[(size_t)l.w_off + ((size_t)co * 27 + t) * l.cin + ci] =
              (i == 0 && ci >= 3) ? 0.0f : (float)(sd * rng.normal());
  }
  for (int c = 0; c < 16; ++c) p[(size_t)n->head_w + c] = (float)(0.25 * rng.normal());
  if (pf_unet_set_params(n, p.data()) != PF_OK) return bad(PF_EHIP);
  *out = n;
  return PF_OK;
}

void pf_unet_destroy(pf_unet* n) {
  if (!n) return;
  // teardown: errors here have no caller to report to
  if (n->stream) (void)hipStreamSynchronize(n->stream);
  else (void)hipDeviceSynchronize();
  free_grid(n);
  if (n->params) (void)hipFree(n->params);
  if (n->grad) (void)hipFree(n->grad);
  if (n->adam_m) (void)hipFree(n->adam_m);
  if (n->adam_v) (void)hipFree(n->adam_v);
  if (n->wslab) (void)hipFree(n->wslab);
  if (n->hostbuf) (void)hipHostFree(n->hostbuf);
  delete n;
}

const char* pf_unet_last_error(const pf_unet* n) { return n ? n->err.c_str() : "null network"; }

int pf_unet_set_conv_kernel(pf_unet* n, int32_t variant) {
  if (!n) return PF_EINVAL;
  if (variant < 0 || variant > 2) return ufail(n, PF_EINVAL, "variant must be 0, 1 or 2");
  n->conv_variant = variant;
  return PF_OK;
}

int pf_unet_set_stream(pf_unet* n, uintptr_t stream) {
  if (!n) return PF_EINVAL;
  n->stream = reinterpret_cast<hipStream_t>(stream);
  return PF_OK;
}

int64_t pf_unet_num_params(void) {
  Layer L[kNumLayers];
  long long hw, hb;
  return param_layout(L, &hw, &hb);
}

int pf_unet_get_params(pf_unet* n, float* host_out) {
  if (!n || !host_out) return ufail(n, PF_EINVAL, "null argument");
  PFU_HIP(n, hipMemcpyAsync(host_out, n->params, (size_t)n->nparams * sizeof(float),
                            hipMemcpyDeviceToHost, n->stream));
  PFU_HIP(n, hipStreamSynchronize(n->stream));
  return PF_OK;
}

int pf_unet_set_params(pf_unet* n, const float* host_in) {
  if (!n || !host_in) return ufail(n, PF_EINVAL, "null argument");
  const size_t pb = (size_t)n->nparams * sizeof(float);
  PFU_HIP(n, hipMemcpyAsync(n->params, host_in, pb, hipMemcpyHostToDevice, n->stream));
  PFU_HIP(n, hipMemsetAsync(n->adam_m, 0, pb, n->stream));
  PFU_HIP(n, hipMemsetAsync(n->adam_v, 0, pb, n->stream));
  PFU_HIP(n, hipStreamSynchronize(n->stream));
  n->adam_step = 0;
  n->weights_dirty = 1;
  return PF_OK;
}

int pf_unet_forward(pf_unet* n, const uint8_t* mask, int32_t n1, int32_t n2, int32_t n3,
                    double dT, double log10_sigma_scale, float* out) {
  if (!n) return PF_EINVAL;
  if (!mask || !out) return ufail(n, PF_EINVAL, "mask and out must be non-NULL device pointers");
  if (!(dT > 0.0)) return ufail(n, PF_EINVAL, "dT must be positive");
  PFU_TRY(check_dims(n, n1, n2, n3));
  PFU_TRY(ensure_grid(n, n1, n2, n3, n->train));
  return run_net(n, mask, 0, dT, log10_sigma_scale, out, 0, nullptr);
}

int pf_unet_grad(pf_unet* n, const uint8_t* mask, const float* target, int32_t n1, int32_t n2,
                 int32_t n3, double dT, double log10_sigma_scale, float* grad_host,
                 double* loss) {
  if (!n) return PF_EINVAL;
  if (!mask || !target)
    return ufail(n, PF_EINVAL, "mask and target must be non-NULL device pointers");
  if (!(dT > 0.0)) return ufail(n, PF_EINVAL, "dT must be positive");
  PFU_TRY(check_dims(n, n1, n2, n3));
  PFU_TRY(ensure_grid(n, n1, n2, n3, 1));
  PFU_TRY(run_net(n, mask, 0, dT, log10_sigma_scale, nullptr, 0, target));
  if (grad_host)
    PFU_HIP(n, hipMemcpyAsync(grad_host, n->grad, (size_t)n->nparams * sizeof(float),
                              hipMemcpyDeviceToHost, n->stream));
  PFU_TRY(read_loss(n, loss));
  PFU_HIP(n, hipStreamSynchronize(n->stream));
  return PF_OK;
}

int pf_unet_train_step(pf_unet* n, const uint8_t* mask, const float* target, int32_t n1,
                       int32_t n2, int32_t n3, double dT, double log10_sigma_scale, double lr,
                       double* loss) {
  if (!n) return PF_EINVAL;
  if (!mask || !target)
    return ufail(n, PF_EINVAL, "mask and target must be non-NULL device pointers");
  if (!(dT > 0.0) || !(lr > 0.0)) return ufail(n, PF_EINVAL, "dT and lr must be positive");
  PFU_TRY(check_dims(n, n1, n2, n3));
  PFU_TRY(ensure_grid(n, n1, n2, n3, 1));
  PFU_TRY(run_net(n, mask, 0, dT, log10_sigma_scale, nullptr, 0, target));
  // the mean over water cells: the gradient of the sum divided by the count
  // is already applied in the head; Adam with the usual constants
  const double b1 = 0.9, b2 = 0.999;
  n->adam_step += 1;
  const double bc1 = 1.0 - pow(b1, (double)n->adam_step);
  const double bc2 = 1.0 - pow(b2, (double)n->adam_step);
  PFU_HIP(n, pfu::launch_adam(n->params, n->grad, n->adam_m, n->adam_v, n->nparams, (float)lr,
                              (float)b1, (float)b2, 1e-8f, (float)bc1, (float)bc2, n->stream));
  n->weights_dirty = 1;
  PFU_TRY(read_loss(n, loss));
  return PF_OK;
}

int pf_unet_time_layers(pf_unet* n, int32_t n1, int32_t n2, int32_t n3, int32_t reps,
                        double* ms) {
  if (!n) return PF_EINVAL;
  if (!ms || reps < 1) return ufail(n, PF_EINVAL, "ms must be non-NULL and reps >= 1");
  PFU_TRY(check_dims(n, n1, n2, n3));
  PFU_TRY(ensure_grid(n, n1, n2, n3, n->train));
  PFU_TRY(refresh_weights(n));
  const int N1 = n1, N2 = n2, N3 = n3;
  struct Item {
    int layer;
    View x, y;
    int g1, g2, g3;
  };
  const Item items[kNumLayers] = {
      {0, V(n->X0, 8, 0), V(n->A1, 16, 0), N1, N2, N3},
      {1, V(n->A1, 16, 0), V(n->S1, 16, 0), N1, N2, N3},
      {2, V(n->P1, 16, 0), V(n->A2, 32, 0), N1 / 2, N2 / 2, N3 / 2},
      {3, V(n->A2, 32, 0), V(n->S2, 32, 0), N1 / 2, N2 / 2, N3 / 2},
      {4, V(n->P2, 32, 0), V(n->A3, 64, 0), N1 / 4, N2 / 4, N3 / 4},
      {5, V(n->A3, 64, 0), V(n->B3, 64, 0), N1 / 4, N2 / 4, N3 / 4},
      {6, V(n->C2, 96, 0), V(n->E2, 32, 0), N1 / 2, N2 / 2, N3 / 2},
      {7, V(n->E2, 32, 0), V(n->F2, 32, 0), N1 / 2, N2 / 2, N3 / 2},
      {8, V(n->C1, 48, 0), V(n->E1, 16, 0), N1, N2, N3},
      {9, V(n->E1, 16, 0), V(n->F1, 16, 0), N1, N2, N3}};
  hipEvent_t e0, e1;
  PFU_HIP(n, hipEventCreate(&e0));
  PFU_HIP(n, hipEventCreate(&e1));
  int rc = PF_OK;
  for (int i = 0; i < kNumLayers && rc == PF_OK; ++i) {
    const Item& it = items[i];
    rc = conv(n, it.layer, it.x, it.y, it.g1, it.g2, it.g3);  // warm-up
    if (rc != PF_OK) break;
    if (hipEventRecord(e0, n->stream) != hipSuccess) rc = ufail(n, PF_EHIP, "event record");
    for (int r = 0; r < reps && rc == PF_OK; ++r)
      rc = conv(n, it.layer, it.x, it.y, it.g1, it.g2, it.g3);
    if (rc != PF_OK) break;
    if (hipEventRecord(e1, n->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      rc = ufail(n, PF_EHIP, "event synchronize");
      break;
    }
    float t = 0.0f;
    if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
      rc = ufail(n, PF_EHIP, "event elapsed time");
      break;
    }
    ms[i] = (double)t / reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

int pf_unet_layer_info(int32_t layer, int32_t* out) {
  if (layer < 0 || layer >= kNumLayers || !out) return PF_EINVAL;
  Layer L[kNumLayers];
  long long hw, hb;
  param_layout(L, &hw, &hb);
  out[0] = L[layer].cin;
  out[1] = L[layer].cout;
  out[2] = (int32_t)L[layer].w_off;
  out[3] = (int32_t)L[layer].b_off;
  // grid level (0 full, 1 half, 2 quarter) of the layer
  static const int level[kNumLayers] = {0, 0, 1, 1, 2, 2, 1, 1, 0, 0};
  out[4] = level[layer];
  out[5] = (int32_t)hw;
  out[6] = (int32_t)hb;
  out[7] = kNumLayers;
  return PF_OK;
}

int pf_conv3_bf16(const uint16_t* x, int32_t cin, const float* w, const float* b, int32_t relu,
                  uint16_t* y, int32_t cout, int32_t n1, int32_t n2, int32_t n3,
                  uintptr_t stream) {
  if (!x || !w || !y || n1 <= 0 || n2 <= 0 || n3 <= 0 || cin % 8 || cout % 16 || cin <= 0 ||
      cout <= 0 || cout > 96 || cout / 16 == 5)
    return PF_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int kpad = round32(27 * cin);
  uint16_t* wf = nullptr;
  if (hipMalloc(&wf, (size_t)cout * kpad * sizeof(uint16_t)) != hipSuccess) return PF_ENOMEM;
  int rc = PF_OK;
  if (pfu::launch_weights(w, cout, cin, kpad, 0, wf, nullptr, s) != hipSuccess) rc = PF_EHIP;
  ConvArgs a;
  a.in = x;
  a.in_stride = cin;
  a.in_off = 0;
  a.cin = cin;
  a.w = wf;
  a.kpad = kpad;
  a.bias = b;
  a.out = y;
  a.out_stride = cout;
  a.out_off = 0;
  a.cout = cout;
  a.relu = relu ? 1 : 0;
  a.n1 = n1;
  a.n2 = n2;
  a.n3 = n3;
  a.variant = 2;
  if (rc == PF_OK && pfu::launch_conv_fwd(a, s) != hipSuccess) rc = PF_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) rc = PF_EHIP;
  (void)hipFree(wf);
  return rc;
}

int pf_conv3_bf16_noalloc(const uint16_t* x, int32_t cin, const float* w, const float* b,
                          int32_t relu, uint16_t* y, int32_t cout, int32_t n1, int32_t n2,
                          int32_t n3, uintptr_t stream) {
  if (!x || !w || !y || n1 <= 0 || n2 <= 0 || n3 <= 0 || cin % 8 || cout % 16 || cin <= 0 ||
      cout <= 0 || cout > 96 || cout / 16 == 5) {
    pf::set_thread_error("pf_conv3_bf16_noalloc: invalid argument");
    return PF_EINVAL;
  }
  if (cin > kNoAllocMaxCin || cout > kNoAllocMaxCout) {
    pf::set_thread_error("pf_conv3_bf16_noalloc: cin " + std::to_string(cin) + ", cout " +
                         std::to_string(cout) + " exceed the static weight scratch (cin <= " +
                         std::to_string(kNoAllocMaxCin) + ", cout <= " +
                         std::to_string(kNoAllocMaxCout) + ")");
    return PF_EINVAL;
  }
  uint16_t* wf = nullptr;
  int rc = noalloc_scratch(&wf);
  if (rc) return rc;
  const int kpad = round32(27 * cin);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = pfu::launch_weights(w, cout, cin, kpad, 0, wf, nullptr, s);
  ConvArgs a;
  a.in = x;
  a.in_stride = cin;
  a.in_off = 0;
  a.cin = cin;
  a.w = wf;
  a.kpad = kpad;
  a.bias = b;
  a.out = y;
  a.out_stride = cout;
  a.out_off = 0;
  a.cout = cout;
  a.relu = relu ? 1 : 0;
  a.n1 = n1;
  a.n2 = n2;
  a.n3 = n3;
  a.variant = 2;
  if (e == hipSuccess) e = pfu::launch_conv_fwd(a, s);
  if (e != hipSuccess) {
    pf::set_thread_error(std::string("pf_conv3_bf16_noalloc: launch: ") + hipGetErrorString(e));
    return PF_EHIP;
  }
  return PF_OK;
}

int pf_conv3_bf16_backward(const uint16_t* x, int32_t cin, const float* w, const uint16_t* dy,
                           int32_t cout, int32_t n1, int32_t n2, int32_t n3, uint16_t* dx,
                           float* dw, float* db, uintptr_t stream) {
  const int cin16 = (cin + 15) & ~15;
  if (!x || !w || !dy || !dw || !db || n1 <= 0 || n2 <= 0 || n3 <= 0 || cin % 8 || cout % 16 ||
      cin <= 0 || cout <= 0 || (cout / 16) * (cin16 / 16) > pfu::kConvMaxTiles)
    return PF_EINVAL;
  if (dx && (cin % 16 || cin > 96 || cin / 16 == 5)) return PF_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const long long nv = (long long)n1 * n2 * n3;
  const int nb = pfu::wgrad_blocks(nv);
  const int kpad_t = round32(27 * cout), kpad = round32(27 * cin);
  float* part = nullptr;
  uint16_t* wbuf = nullptr;
  const size_t npart = (size_t)nb * 27 * cout * cin + (size_t)nb * cout;
  if (hipMalloc(&part, npart * sizeof(float)) != hipSuccess) return PF_ENOMEM;
  if (hipMalloc(&wbuf, ((size_t)cout * kpad + (size_t)cin * kpad_t) * sizeof(uint16_t)) !=
      hipSuccess) {
    (void)hipFree(part);
    return PF_ENOMEM;
  }
  int rc = PF_OK;
  WgradArgs g;
  g.dy = dy;
  g.dy_stride = cout;
  g.dy_off = 0;
  g.cout = cout;
  g.x = x;
  g.x_stride = cin;
  g.x_off = 0;
  g.cin = cin;
  g.n1 = n1;
  g.n2 = n2;
  g.n3 = n3;
  g.part = part;
  g.part_bias = part + (size_t)nb * 27 * cout * cin;
  if (pfu::launch_conv_wgrad(g, nb, dw, db, s) != hipSuccess) rc = PF_EHIP;
  if (rc == PF_OK && dx) {
    uint16_t* wf = wbuf;
    uint16_t* wd = wbuf + (size_t)cout * kpad;
    if (pfu::launch_weights(w, cout, cin, kpad, kpad_t, wf, wd, s) != hipSuccess) rc = PF_EHIP;
    ConvArgs a;
    a.in = dy;
    a.in_stride = cout;
    a.in_off = 0;
    a.cin = cout;
    a.w = wd;
    a.kpad = kpad_t;
    a.bias = nullptr;
    a.out = dx;
    a.out_stride = cin;
    a.out_off = 0;
    a.cout = cin;
    a.relu = 0;
    a.n1 = n1;
    a.n2 = n2;
    a.n3 = n3;
    a.variant = 2;
    if (rc == PF_OK && pfu::launch_conv_fwd(a, s) != hipSuccess) rc = PF_EHIP;
  }
  if (hipStreamSynchronize(s) != hipSuccess) rc = PF_EHIP;
  (void)hipFree(part);
  (void)hipFree(wbuf);
  return rc;
}

int pf_mfma_probe(const float* a, const float* b, float* c, uintptr_t stream) {
  if (!a || !b || !c) return PF_EINVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (pfu::launch_mfma_probe(a, b, c, s) != hipSuccess) return PF_EHIP;
  return hipStreamSynchronize(s) == hipSuccess ? PF_OK : PF_EHIP;
}

}  // extern "C"

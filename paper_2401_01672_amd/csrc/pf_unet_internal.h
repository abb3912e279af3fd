// Device-side argument blocks and launchers of the warm-start network kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pfu {

// channels-last BF16 tensor view: element (voxel v, channel c) at p[v * stride + off + c]
struct View {
  uint16_t* p;
  int stride;
  int off;
};

struct ConvArgs {
  const uint16_t* in;  // input view (channels ci0 .. ci0+7 loaded as 16 bytes)
  int in_stride, in_off, cin;
  const uint16_t* w;   // BF16 weights [cout][kpad], k = tap * cin + ci
  int kpad;
  const float* bias;   // [cout] or null
  uint16_t* out;
  int out_stride, out_off, cout;
  int relu;
  int n1, n2, n3;
  int variant;         // 2: register-blocked kernel for 16 -> 32 channels on
                       // large grids, else as 1; 1: LDS-tiled kernel; 0: direct
                       // kernel (same products, FP32 sums in another order)
};

struct WgradArgs {
  const uint16_t* dy;  // output gradient view (cout channels)
  int dy_stride, dy_off, cout;
  const uint16_t* x;   // layer input view (cin channels)
  int x_stride, x_off, cin;
  int n1, n2, n3;
  float* part;         // [nblocks][cout][27][cin] per-workgroup partial weight gradients
  float* part_bias;    // [nblocks][cout] partial bias gradients (written by the centre tap)
};

struct HeadArgs {
  const uint16_t* h;   // last feature map view (16 channels)
  int h_stride, h_off;
  const float* w;      // [16] head weights (FP32 master copy)
  const float* b;      // [1]
  const uint8_t* glass;
  int code_glass;      // 1: glass flag is bit 6 of a solver cell code; 0: mask byte != 0
  const uint8_t* keep; // if non-null: the prediction is 0 where keep[v] == 0
  long long nvox;
  void* out;           // prediction (water cells; 0 on glass) or null
  int out_fp64;
  const float* target; // training target or null (inference)
  const float* count;  // number of water cells (device scalar), training only
  uint16_t* dh;        // gradient wrt h, [nvox][16]
  float* part;         // [blocks][18]: loss, dL/db, dL/dw[16]
};

constexpr int kConvMaxTiles = 16;   // (cout / 16) * ceil(cin / 16) for the weight gradient
constexpr int kHeadParts = 18;

hipError_t launch_conv_fwd(const ConvArgs& a, hipStream_t s);
hipError_t launch_conv_wgrad(const WgradArgs& a, int nblocks, float* dw, float* db,
                             hipStream_t s);
int wgrad_blocks(long long nvox);
hipError_t launch_relu_bwd(uint16_t* dy, int dys, int dyo, const uint16_t* y, int ys, int yo,
                           int c, long long nvox, hipStream_t s);
hipError_t launch_pool_fwd(const View& in, const View& out, int c, int m1, int m2, int m3,
                           hipStream_t s);
hipError_t launch_pool_bwd(const View& dout, const View& din, int c, int n1, int n2, int n3,
                           int accumulate, hipStream_t s);
// [nearest 2x upsampling of up (cu channels) | skip (cs channels)] per voxel
// into out (stride cu + cs); views without offsets, cu and cs multiples of 8
hipError_t launch_up_cat(const View& up, const View& skip, const View& out, int cu, int cs,
                         int n1, int n2, int n3, hipStream_t s);
hipError_t launch_up_fwd(const View& in, const View& out, int c, int n1, int n2, int n3,
                         hipStream_t s);
hipError_t launch_up_bwd(const View& dout, const View& din, int c, int m1, int m2, int m3,
                         hipStream_t s);
hipError_t launch_input(const uint8_t* glass, int from_code, float f1, float f2, uint16_t* out,
                        long long nvox, hipStream_t s);
hipError_t launch_count_water(const uint8_t* glass, int from_code, long long nvox, float* part,
                              float* count, hipStream_t s);
int head_blocks(long long nvox);
hipError_t launch_head(const HeadArgs& a, hipStream_t s);
hipError_t launch_weights(const float* wm, int cout, int cin, int kpad, int kpad_t, uint16_t* wf,
                          uint16_t* wd, hipStream_t s);
hipError_t launch_reduce(const float* part, int nparts, long long len, float* out, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, long long n, float lr,
                       float b1, float b2, float eps, float bc1, float bc2, hipStream_t s);
hipError_t launch_f32_to_bf16(const float* in, uint16_t* out, long long n, hipStream_t s);
hipError_t launch_bf16_to_f32(const uint16_t* in, float* out, long long n, hipStream_t s);
hipError_t launch_mfma_probe(const float* A, const float* B, float* C, hipStream_t s);
// out = 1 on the reached cells, 0 elsewhere (FP64 if fp64, else FP32)
hipError_t launch_flood(const uint8_t* reach, void* out, int fp64, long long n, hipStream_t s);
// reach = 1 on the water cells whose face-connected water component holds a
// nucleus cell (water with phi > 1/2), 0 elsewhere; lab: n1 n2 n3 ints of
// scratch (the union-find parents)
hipError_t launch_reach(const uint8_t* code, const void* phi, int fp64, int* lab, uint8_t* reach,
                        int n1, int n2, int n3, hipStream_t s);

}  // namespace pfu

#include <string>

#include "pf.h"

// forward pass of the network on a solver's cell codes (glass = bit 6),
// writing phi0 (FP32 or FP64) into out on stream s; used by pf_warmstart
// mode (PF_WARM_*): ALL writes the prediction on every cell; NUCLEUS first
// finds the water cells connected through water-water faces to a cell with
// out > 1/2 (the current nucleus) and writes the prediction there, zero on
// every other cell; FLOOD writes 1 on those cells and 0 elsewhere without
// running the network.
int pfu_forward_into(pf_unet* n, const uint8_t* code, int n1, int n2, int n3, double dT,
                     double log10_s, void* out, int out_fp64, int mode, hipStream_t s,
                     std::string* err);

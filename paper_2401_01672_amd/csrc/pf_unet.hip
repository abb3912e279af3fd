// Learned warm start: a small 3D U-Net trained and evaluated with
// hand-written BF16 MFMA kernels for gfx950 (v_mfma_f32_16x16x32_bf16).
//
// Activations are channels-last BF16: element (voxel v, channel c) of a view
// {ptr, C, stride, offset} sits at ptr[v * stride + offset + c], so the two
// halves of a skip concatenation are written in place by their producers.
// Master weights are FP32 [co][tap][ci] (tap = (dz+1)*9 + (dy+1)*3 + (dx+1));
// the kernels read BF16 copies: forward [co][k] with k = tap*Cin + ci, and
// the data-gradient copy [ci][k'] with k' = (26 - tap)*Cout + co (taps
// mirrored), both zero-padded to a multiple of 32 in k.  All accumulation is
// FP32.
//
// MFMA 16x16x32 BF16 operand layout (one wavefront, lane l, g = l / 16):
//   A (16 x 32): lane holds A[l % 16][8g .. 8g+7]
//   B (32 x 16): lane holds B[8g .. 8g+7][l % 16]
//   D (16 x 16): lane holds D[4g .. 4g+3][l % 16]
#include <float.h>
#include <math.h>
#include <stdint.h>

#include "pf_unet_internal.h"

namespace pfu {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float bf2f(uint16_t b) {
  return __uint_as_float(((uint32_t)b) << 16);
}
typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2;
// FP32 -> BF16, round to nearest even (the gfx950 conversion instruction)
__device__ __forceinline__ uint16_t f2bf(float f) {
  return __builtin_bit_cast(uint16_t, (__bf16)f);
}
// two values in one instruction: lo in bits 0..15, hi in bits 16..31
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  bf16x2 r;
  r[0] = (__bf16)lo;
  r[1] = (__bf16)hi;
  return __builtin_bit_cast(uint32_t, r);
}

__device__ __forceinline__ bf16x8 zero8() {
  bf16x8 z;
#pragma unroll
  for (int i = 0; i < 8; ++i) z[i] = (__bf16)0.0f;
  return z;
}

__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}

// ---------------------------------------------------------------------------
// Probe of the MFMA operand layout (used by a test): C = A(16x32) B(32x16)
// with A, B row-major FP32 inputs converted to BF16.
__global__ void mfma_layout_probe(const float* A, const float* B, float* C) {
  const int l = threadIdx.x, g = l >> 4, r = l & 15;
  bf16x8 a, b;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    a[j] = (__bf16)A[r * 32 + 8 * g + j];
    b[j] = (__bf16)B[(8 * g + j) * 16 + r];
  }
  f32x4 d = {0.f, 0.f, 0.f, 0.f};
  d = mfma16(a, b, d);
#pragma unroll
  for (int i = 0; i < 4; ++i) C[(4 * g + i) * 16 + r] = d[i];
}

// ---------------------------------------------------------------------------
// 3x3x3 convolution, stride 1, zero padding, as an implicit GEMM:
//   out[v][co] = act( bias[co] + sum_k W[co][k] X[k][v] ),
//   X[k = tap*Cin + ci][v] = in[v + offset(tap)][ci]  (0 outside the grid).
// A workgroup has 4 wavefronts; a wavefront owns NT tiles of 16 consecutive
// voxels and all Cout/16 output-channel tiles.  Per k-block of 32 each lane
// loads 8 input channels of one tap for one voxel (16 bytes) and the matching
// weights, and issues MT x NT MFMAs.  The epilogue adds the bias, applies the
// ReLU, and stores 4 consecutive BF16 channels per lane.

template <int MT, int NT>
__global__ __launch_bounds__(256) void conv3_fwd_kernel(ConvArgs a) {
  const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const long long nvox = (long long)a.n1 * a.n2 * a.n3;
  const long long vbase = (long long)wave * (16 * NT);
  if (vbase >= nvox) return;
  // this lane's voxel in each tile (B operand column / D column)
  int vx[NT], vy[NT], vz[NT];
  bool vin[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const long long v = vbase + 16 * t + r;
    vin[t] = v < nvox;
    const long long vv = vin[t] ? v : 0;
    vx[t] = (int)(vv % a.n1);
    vy[t] = (int)((vv / a.n1) % a.n2);
    vz[t] = (int)(vv / ((long long)a.n1 * a.n2));
  }
  f32x4 acc[MT][NT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int kblocks = a.kpad / 32;
  for (int kb = 0; kb < kblocks; ++kb) {
    const int k0 = kb * 32 + 8 * g;
    const int tap = k0 / a.cin, ci0 = k0 - tap * a.cin;
    bf16x8 bfrag[NT];
    if (tap < 27) {
      const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int x = vx[t] + dx, y = vy[t] + dy, z = vz[t] + dz;
        const bool ok = vin[t] && x >= 0 && x < a.n1 && y >= 0 && y < a.n2 && z >= 0 && z < a.n3;
        const long long src = ((long long)z * a.n2 + y) * a.n1 + x;
        bfrag[t] = ok ? ld8(a.in + src * a.in_stride + a.in_off + ci0) : zero8();
      }
    } else {
#pragma unroll
      for (int t = 0; t < NT; ++t) bfrag[t] = zero8();
    }
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const bf16x8 afrag = ld8(a.w + (long long)(m * 16 + r) * a.kpad + k0);
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[m][t] = mfma16(afrag, bfrag[t], acc[m][t]);
    }
  }
  // epilogue: lane holds channels m*16 + 4g .. +3 of voxel vbase + 16t + r
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (!vin[t]) continue;
    const long long v = vbase + 16 * t + r;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int co = m * 16 + 4 * g;
      uint16_t o[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float y = acc[m][t][i] + (a.bias ? a.bias[co + i] : 0.0f);
        if (a.relu) y = y > 0.0f ? y : 0.0f;
        o[i] = f2bf(y);
      }
      uint2 pk;
      pk.x = (uint32_t)o[0] | ((uint32_t)o[1] << 16);
      pk.y = (uint32_t)o[2] | ((uint32_t)o[3] << 16);
      *reinterpret_cast<uint2*>(a.out + v * a.out_stride + a.out_off + co) = pk;
    }
  }
}

// ---------------------------------------------------------------------------
// LDS-tiled form of the same convolution.  A workgroup owns a 16 x 4 x 4
// block of output voxels (wavefront w: the plane z0 + w; N-tile t: the x-row
// y0 + t; lane r: x0 + r) and all output channels.  The input block with its
// one-voxel halo (18 x 6 x 6 voxels) is staged in LDS one chunk of CC input
// channels at a time (row pitch CC + 8 channels, or 24 for CC = 8, so that
// the 16 lanes of a group read 16-byte fragments from distinct banks); every
// B fragment of the implicit GEMM is then one LDS read, and the input is read
// from memory once per block instead of once per tap.  One k-block of 32 is
// 32/CC taps x CC channels of the chunk, in the weight layout
// k = tap * cin + ci (no re-layout).  The A fragments (weights) come from
// memory through L1/L2, shared by all blocks.

constexpr int kTX = 16, kTY = 4, kTZ = 4;
constexpr int kHX = kTX + 2, kHY = kTY + 2, kHZ = kTZ + 2;
constexpr int kHalo = kHX * kHY * kHZ;

// Row pitch (channels) of a halo voxel in LDS.  8- and 16-channel chunks use
// the unpadded row: measured faster than the 48-byte padded one (48 -> 16 at
// 96^3: 69 against 77 us), and the smaller block lets four workgroups share
// a CU.
template <int CC>
__host__ __device__ constexpr int tile_pitch() { return CC <= 16 ? CC : CC + 8; }

// The one-group form with 8- or 16-channel chunks is held to 128 registers
// (four waves per SIMD; 48 -> 16 at 96^3: 64.5 instead of 68.5 us), no
// spills.
template <int MT, int CC>
constexpr int tile_waves() { return MT == 1 && CC <= 16 ? 4 : 1; }

// Taps past 26 (the padding of a last k-block) stand for tap 26 with zero
// weights.  halo_tap_offset: the tap's voxel offset in the halo block from
// the output voxel's (dx, dy, dz) = (-1, -1, -1) corner.
__host__ __device__ constexpr int tap_clamped(int tap) { return tap < 27 ? tap : 26; }
__host__ __device__ constexpr int halo_tap_offset(int tap) {
  return ((tap_clamped(tap) / 9) * kHY + (tap_clamped(tap) / 3) % 3) * kHX + tap_clamped(tap) % 3;
}

// TZ: output planes per workgroup, one wavefront each (64 TZ threads).
template <int MT, int CC, int TZ>
__global__ __launch_bounds__(64 * TZ) __attribute__((amdgpu_waves_per_eu(tile_waves<MT, CC>())))
void conv3_tile_kernel(ConvArgs a, int tiles_x, int tiles_y, int tiles_z) {
  constexpr int NTH = 64 * TZ;                   // threads
  constexpr int HALO = kHX * kHY * (TZ + 2);     // halo voxels
  constexpr int PITCH = tile_pitch<CC>();
  constexpr int TPB = 32 / CC;  // taps per k-block
  constexpr int KB = (27 + TPB - 1) / TPB;
  __shared__ __align__(16) uint16_t sx[HALO * PITCH];
  // One or two output groups and chunks of 8 or 16 channels: the chunk's
  // weights (27 taps x 16 MT rows, unpadded) are staged in LDS with the halo,
  // so the A fragments are LDS reads instead of L2 loads waited on inside the
  // k-block loop (48 -> 16 at 96^3: 75 instead of 83 us; 96 -> 32 at 48^3:
  // 32 instead of 46.5 us).
  constexpr bool kWL = MT <= 2 && CC <= 16;
  constexpr int WR = 16 * MT;  // weight rows staged (the workgroup's output channels)
  static_assert(!kWL || TPB > 1, "weights in LDS assume tabulated offsets");
  constexpr int WP = CC;
  __shared__ __align__(16) uint16_t sw[kWL ? 27 * WR * WP : 8];
  const int tid = threadIdx.x;
  const int lane = tid & 63, g = lane >> 4, r = lane & 15, w = tid >> 6;
  // XCD-aware order: consecutive tiles of a row stay on one XCD
  const int nblk = gridDim.x;
  const int b = blockIdx.x;
  const int q = nblk >> 3, rem = nblk & 7, xcd = b & 7, kk = b >> 3;
  const int tile = (xcd < rem) ? xcd * (q + 1) + kk : rem * (q + 1) + (xcd - rem) * q + kk;
  const int tx = tile % tiles_x, ty = (tile / tiles_x) % tiles_y, tz = tile / (tiles_x * tiles_y);
  const int x0 = tx * kTX, y0 = ty * kTY, z0 = tz * TZ;
  (void)tiles_z;
  const int mb = blockIdx.y * MT;  // first 16-channel output group of this workgroup

  f32x4 acc[MT][4];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};

  // Lane group g holds channels cig .. cig + 7 of the chunk at tap
  // kb * TPB + tg of k-block kb.  Per k-block: the lane's LDS element offset
  // of its B fragment for N-tile 0, and its weight column (tap * cin +
  // channel).  With one tap per k-block (TPB = 1) both are a base plus a
  // compile-time constant; otherwise they differ between lane groups and are
  // tabulated once.  Taps past 26 (the padding of the last k-block) read tap
  // 26 and take zero weights.
  const int cig = (8 * g) % CC, tg = (8 * g) / CC;
  const int lbase = ((w * kHY) * kHX + r) * PITCH + cig;
  int lofs[TPB == 1 ? 1 : KB], wcol[TPB == 1 ? 1 : KB];
  if constexpr (TPB > 1) {
    // a lane group's tap is one of TPB compile-time candidates per k-block:
    // select among their constant offsets (no per-lane divisions)
    const int wl = kWL ? r * WP + cig : cig;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      int hoff = halo_tap_offset(kb * TPB), tc = tap_clamped(kb * TPB);
#pragma unroll
      for (int u = 1; u < TPB; ++u)
        if (tg == u) {
          hoff = halo_tap_offset(kb * TPB + u);
          tc = tap_clamped(kb * TPB + u);
        }
      lofs[kb] = lbase + hoff * PITCH;
      // the weights in LDS: row r of tap tc; else the column in memory
      wcol[kb] = (kWL ? tc * (WR * WP) : tc * a.cin) + wl;
    }
  }
  auto lds_off = [&](int kb) -> int {
    if constexpr (TPB == 1) return lbase + (((kb / 9) * kHY + (kb / 3) % 3) * kHX + kb % 3) * PITCH;
    else return lofs[kb];
  };
  auto w_col = [&](int kb) -> int {
    if constexpr (TPB == 1) return kb * a.cin + cig;
    else return wcol[kb];
  };
  const bool pad_lane = KB * TPB > 27 && (KB - 1) * TPB + tg >= 27;
  const uint16_t* wrow[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) wrow[m] = a.w + (long long)((mb + m) * 16 + r) * a.kpad;

  // The halo block of a channel chunk (zeros outside the grid).  With chunks
  // of up to 16 channels (at most 6 slots of 16 bytes per thread) it is
  // loaded into registers while the previous chunk is computed and stored to
  // LDS between the two barriers, so the loads' latency overlaps the MFMAs
  // (48 -> 16 at 96^3: 83 instead of 91 us); wider chunks would hold too
  // many registers and load it between the barriers.
  constexpr int G8 = CC / 8;
  constexpr bool kPipe = CC <= 16;
  constexpr int NST = kPipe ? (HALO * G8 + NTH - 1) / NTH : 1;  // 16-byte slots per thread
  u32x4 st[NST];
  constexpr int NWS = kWL ? (27 * WR * G8 + NTH - 1) / NTH : 1;  // weight slots per thread
  u32x4 wst[NWS];
  auto halo_src = [&](int i, int c, const uint4** src) -> bool {
    const int c8 = i % G8, hv = i / G8;
    const int hx = hv % kHX, hy = (hv / kHX) % kHY, hz = hv / (kHX * kHY);
    const int x = x0 + hx - 1, y = y0 + hy - 1, z = z0 + hz - 1;
    if (x < 0 || x >= a.n1 || y < 0 || y >= a.n2 || z < 0 || z >= a.n3) return false;
    const long long v = ((long long)z * a.n2 + y) * a.n1 + x;
    *src = reinterpret_cast<const uint4*>(a.in + v * a.in_stride + a.in_off + c * CC + 8 * c8);
    return true;
  };
  // With chunks of up to 16 channels each thread's slots are the same halo
  // voxels and weight rows in every chunk, only c * CC channels further on:
  // their byte offsets from the input and weight bases (32-bit, checked by
  // the launcher; kNoSlot outside the grid) are computed once here instead
  // of once per chunk, which was most of the kernel's VALU work.  Their LDS
  // slots are 16 i bytes (unpadded rows: PITCH = WP = CC).  The loads go
  // through raw buffer resources, which return zeros at a byte offset at or
  // beyond the resource's size: kNoSlot is 2^31 (the launcher keeps both
  // sizes below it), so a slot outside the grid needs no branch or zero fill.
  constexpr uint32_t kNoSlot = 0x80000000u;
  const auto rin = __builtin_amdgcn_make_buffer_rsrc(
      (void*)a.in, 0, (int)(2u * (uint32_t)(a.n1 * a.n2 * a.n3) * (uint32_t)a.in_stride),
      0x00020000);
  const auto rwt =
      __builtin_amdgcn_make_buffer_rsrc((void*)a.w, 0, 2 * a.cout * a.kpad, 0x00020000);
  uint32_t hb[NST], wb[NWS];
  if constexpr (kPipe) {
#pragma unroll
    for (int j = 0; j < NST; ++j) {
      // 32-bit index arithmetic: the launcher checks that every byte offset
      // of the input view fits
      const int i = tid + NTH * j;
      const int c8 = i % G8, hv = i / G8;
      const int hx = hv % kHX, hy = (hv / kHX) % kHY, hz = hv / (kHX * kHY);
      const int x = x0 + hx - 1, y = y0 + hy - 1, z = z0 + hz - 1;
      const bool in = i < HALO * G8 && x >= 0 && x < a.n1 && y >= 0 && y < a.n2 && z >= 0 &&
                      z < a.n3;
      hb[j] = in ? 2u * (uint32_t)(((z * a.n2 + y) * a.n1 + x) * a.in_stride + a.in_off + 8 * c8)
                 : kNoSlot;
    }
    if constexpr (kWL) {
#pragma clang loop unroll(full)
      for (int j = 0; j < NWS; ++j) {
        const int i = tid + NTH * j;  // (tap, row, 8-channel group)
        const int c8 = i % G8, row = (i / G8) % WR, tap = i / (WR * G8);
        wb[j] = i < 27 * WR * G8
                    ? (uint32_t)(2 * ((mb * 16 + row) * a.kpad + tap * a.cin + 8 * c8))
                    : kNoSlot;
      }
    }
  }
  auto stage_load = [&](int c) {
    const uint32_t cb = (uint32_t)(2 * CC * c);
#pragma unroll
    for (int j = 0; j < NST; ++j) st[j] = __builtin_amdgcn_raw_buffer_load_b128(rin, hb[j] + cb, 0, 0);
    if constexpr (kWL) {
#pragma clang loop unroll(full)
      for (int j = 0; j < NWS; ++j)
        wst[j] = __builtin_amdgcn_raw_buffer_load_b128(rwt, wb[j] + cb, 0, 0);
    }
  };
  const int nchunks = a.cin / CC;
  if constexpr (kPipe) stage_load(0);
  for (int c = 0; c < nchunks; ++c) {
    __syncthreads();  // the previous chunk's LDS reads are done
    if constexpr (kPipe) {
      static_assert(!kPipe || (PITCH == CC && WP == CC), "slot i sits at 16 i bytes");
#pragma unroll
      for (int j = 0; j < NST; ++j) {
        const int i = tid + NTH * j;
        if (i < HALO * G8) *reinterpret_cast<u32x4*>(sx + 8 * i) = st[j];
      }
      if constexpr (kWL) {
#pragma clang loop unroll(full)
        for (int j = 0; j < NWS; ++j) {
          const int i = tid + NTH * j;
          if (i < 27 * WR * G8) *reinterpret_cast<u32x4*>(sw + 8 * i) = wst[j];
        }
      }
    } else {
      for (int i = tid; i < HALO * G8; i += NTH) {
        const uint4* src;
        uint4 val = make_uint4(0u, 0u, 0u, 0u);
        if (halo_src(i, c, &src)) val = *src;
        *reinterpret_cast<uint4*>(sx + (i / G8) * PITCH + 8 * (i % G8)) = val;
      }
    }
    __syncthreads();
    if constexpr (kPipe) {
      if (c + 1 < nchunks) stage_load(c + 1);
    }
    // the k-block loop is unrolled: every address below is a per-lane base
    // plus a constant (or a per-k-block entry of lofs / wcol), so the loop
    // issues little besides its loads and MFMAs
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      bf16x8 bfrag[4];
#pragma unroll
      for (int t = 0; t < 4; ++t)
        bfrag[t] = *reinterpret_cast<const bf16x8*>(sx + lds_off(kb) + t * kHX * PITCH);
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        bf16x8 afrag;
        if constexpr (kWL) afrag = *reinterpret_cast<const bf16x8*>(sw + w_col(kb) + m * 16 * WP);
        else afrag = ld8(wrow[m] + c * CC + w_col(kb));
        if (kb == KB - 1 && pad_lane) afrag = zero8();
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[m][t] = mfma16(afrag, bfrag[t], acc[m][t]);
      }
    }
  }
  // epilogue: lane holds channels m*16 + 4g .. +3 of voxel (x0 + r, y0 + t, z0 + w)
  const int x = x0 + r, z = z0 + w;
  if (x >= a.n1 || z >= a.n3) return;
  float bias[MT][4];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int i = 0; i < 4; ++i) bias[m][i] = a.bias ? a.bias[(mb + m) * 16 + 4 * g + i] : 0.0f;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int y = y0 + t;
    if (y >= a.n2) continue;
    const long long v = ((long long)z * a.n2 + y) * a.n1 + x;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int co = (mb + m) * 16 + 4 * g;
      float o[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        o[i] = acc[m][t][i] + bias[m][i];
        if (a.relu) o[i] = o[i] > 0.0f ? o[i] : 0.0f;
      }
      *reinterpret_cast<uint2*>(a.out + v * a.out_stride + a.out_off + co) =
          make_uint2(pack_bf16(o[0], o[1]), pack_bf16(o[2], o[3]));
    }
  }
}

// ---------------------------------------------------------------------------
// x-folded form for 16 output channels and 16-channel chunks.  With one
// 16-channel output group every B fragment of the tiled form feeds a single
// MFMA, so the LDS reads, not the matrix cores, bound it.  Here the three
// x-taps become the M dimension instead of part of K:
//   E[dx][co][p] = sum over (dz, dy, ci) of W[co][dz, dy, dx][ci] X[p; dz, dy][ci]
// for the 16 positions p of a row (x = x0 + p, x0 one left of the first
// output), and out[x0 + p] = E[-1][p - 1] + E[0][p] + E[+1][p + 1] for
// p = 1 .. 14.  Each B fragment (16 positions x 32 k) then feeds three MFMAs
// (one per dx), K shrinks to 9 taps x 16 channels, and the row needs no x
// halo.  The shifts by one position are row shifts of the D layout (lane r of
// a 16-lane row holds position r), done with DPP once per tile.  Costs: 14
// outputs per 16 positions and one padded tap in 10.  A workgroup owns
// 14 x 4 x TZ output voxels: wavefront w the plane z0 + w, N-tile t the row
// y0 + t.

constexpr int kFX = 16;           // positions per row
constexpr int kFOut = kFX - 2;    // outputs per row

// (every lane writes and a lane without a source reads zero, so no old value
// is needed)
__device__ __forceinline__ float dpp_row_shr1(float v) {  // lane r takes lane r - 1 (row start: 0)
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x111, 0xf, 0xf, true));
}
__device__ __forceinline__ float dpp_row_shl1(float v) {  // lane r takes lane r + 1 (row end: 0)
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x101, 0xf, 0xf, true));
}

template <int TZ>
__global__ __launch_bounds__(64 * TZ) __attribute__((amdgpu_waves_per_eu(4)))
void conv3_xfold_kernel(ConvArgs a, int tiles_x, int tiles_y) {
  constexpr int CC = 16, G8 = 2, NTH = 64 * TZ;
  constexpr int HY = kTY + 2, HZ = TZ + 2;
  constexpr int HALO = kFX * HY * HZ;  // voxels of the staged block
  constexpr int KB = 5;                // k-blocks: 9 (dz, dy) taps x 16 channels, padded to 10
  // the chunk's weights, [dx][dz, dy][co][ci], with a tenth (dz, dy) slot of
  // zeros per dx for the padding tap
  constexpr int WSZ = 3 * 10 * 16 * CC;
  __shared__ __align__(16) uint16_t sx[HALO * CC];
  __shared__ __align__(16) uint16_t sw[WSZ];
  const int tid = threadIdx.x;
  const int lane = tid & 63, g = lane >> 4, r = lane & 15, w = tid >> 6;
  // XCD-aware order: consecutive tiles of a row stay on one XCD
  const int nblk = gridDim.x, b = blockIdx.x;
  const int q = nblk >> 3, rem = nblk & 7, xcd = b & 7, kk = b >> 3;
  const int tile = (xcd < rem) ? xcd * (q + 1) + kk : rem * (q + 1) + (xcd - rem) * q + kk;
  const int tx = tile % tiles_x, ty = (tile / tiles_x) % tiles_y, tz = tile / (tiles_x * tiles_y);
  const int x0 = tx * kFOut - 1, y0 = ty * kTY, z0 = tz * TZ;

  f32x4 acc[3][4];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[d][t] = f32x4{0.f, 0.f, 0.f, 0.f};

  // lane group g: channels 8 (g & 1) .. + 7 of the (dz, dy) tap 2 kb + (g >> 1);
  // tap 9 (the padding) reads tap 8 of the input and the zero weight slot
  const int cig = 8 * (g & 1), tg = g >> 1;
  const int lbase = ((w * HY) * kFX + r) * CC + cig;
  const int wbase = r * CC + cig;
  int lofs[KB], wofs[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    const int t0 = 2 * kb < 9 ? 2 * kb : 8, t1 = 2 * kb + 1 < 9 ? 2 * kb + 1 : 8;
    const int h0 = ((t0 / 3) * HY + t0 % 3) * kFX * CC, h1 = ((t1 / 3) * HY + t1 % 3) * kFX * CC;
    lofs[kb] = lbase + (tg ? h1 : h0);
    wofs[kb] = wbase + (tg ? 2 * kb + 1 : t0) * 16 * CC;
  }
  // the zero slots (never overwritten by the staging; visible after the
  // first chunk's barrier)
  if (tid < 3 * 16 * CC / 8)
    *reinterpret_cast<u32x4*>(sw + ((tid / (16 * CC / 8)) * 10 + 9) * 16 * CC +
                              8 * (tid % (16 * CC / 8))) = u32x4{0u, 0u, 0u, 0u};

  // staging slots (the same voxels and weight rows for every chunk; 32-bit
  // byte offsets, checked by the launcher).  The loads go through raw buffer
  // resources over the input and the weights: a load at a byte offset at or
  // beyond the resource's size returns zeros, so a slot outside the grid is
  // an offset of 2^31 (the launcher keeps both sizes below it) and needs
  // neither a branch nor a zero fill.
  constexpr uint32_t kNoSlot = 0x80000000u;
  const auto rin = __builtin_amdgcn_make_buffer_rsrc(
      (void*)a.in, 0, (int)(2u * (uint32_t)(a.n1 * a.n2 * a.n3) * (uint32_t)a.in_stride),
      0x00020000);
  const auto rwt = __builtin_amdgcn_make_buffer_rsrc((void*)a.w, 0, 2 * 16 * a.kpad, 0x00020000);
  constexpr int NST = (HALO * G8 + NTH - 1) / NTH;
  constexpr int NWS = (27 * 16 * G8 + NTH - 1) / NTH;
  uint32_t hb[NST], wb[NWS];
  int wdst[NWS];
#pragma unroll
  for (int j = 0; j < NST; ++j) {
    const int i = tid + NTH * j;
    const int c8 = i % G8, hv = i / G8;
    const int hx = hv % kFX, hy = (hv / kFX) % HY, hz = hv / (kFX * HY);
    const int x = x0 + hx, y = y0 + hy - 1, z = z0 + hz - 1;
    const bool in = i < HALO * G8 && x >= 0 && x < a.n1 && y >= 0 && y < a.n2 && z >= 0 &&
                    z < a.n3;
    hb[j] = in ? 2u * (uint32_t)(((z * a.n2 + y) * a.n1 + x) * a.in_stride + a.in_off + 8 * c8)
               : kNoSlot;
  }
#pragma unroll
  for (int j = 0; j < NWS; ++j) {
    const int i = tid + NTH * j;  // (tap, row, 8-channel group), tap = 3 (dz, dy) + dx
    const int c8 = i % G8, row = (i / G8) % 16, tap = i / (16 * G8);
    wb[j] = i < 27 * 16 * G8 ? (uint32_t)(2 * (row * a.kpad + tap * a.cin + 8 * c8)) : kNoSlot;
    wdst[j] = (((tap % 3) * 10 + tap / 3) * 16 + row) * CC + 8 * c8;
  }
  u32x4 st[NST], wst[NWS];
  auto stage_load = [&](int c) {
    const uint32_t cb = (uint32_t)(2 * CC * c);
#pragma unroll
    for (int j = 0; j < NST; ++j) st[j] = __builtin_amdgcn_raw_buffer_load_b128(rin, hb[j] + cb, 0, 0);
#pragma unroll
    for (int j = 0; j < NWS; ++j) wst[j] = __builtin_amdgcn_raw_buffer_load_b128(rwt, wb[j] + cb, 0, 0);
  };
  const int nchunks = a.cin / CC;
  stage_load(0);
  for (int c = 0; c < nchunks; ++c) {
    __syncthreads();  // the previous chunk's LDS reads are done
#pragma unroll
    for (int j = 0; j < NST; ++j) {
      const int i = tid + NTH * j;
      if (i < HALO * G8) *reinterpret_cast<u32x4*>(sx + 8 * i) = st[j];
    }
#pragma unroll
    for (int j = 0; j < NWS; ++j) {
      const int i = tid + NTH * j;
      if (i < 27 * 16 * G8) *reinterpret_cast<u32x4*>(sw + wdst[j]) = wst[j];
    }
    __syncthreads();
    if (c + 1 < nchunks) stage_load(c + 1);
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      bf16x8 bfrag[4];
#pragma unroll
      for (int t = 0; t < 4; ++t)
        bfrag[t] = *reinterpret_cast<const bf16x8*>(sx + lofs[kb] + t * kFX * CC);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const bf16x8 afrag = *reinterpret_cast<const bf16x8*>(sw + d * 10 * 16 * CC + wofs[kb]);
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[d][t] = mfma16(afrag, bfrag[t], acc[d][t]);
      }
    }
  }
  // epilogue: position r of row t holds E[dx] of channels 4g .. 4g + 3
  const int x = x0 + r, z = z0 + w;
  float bias[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) bias[i] = a.bias ? a.bias[4 * g + i] : 0.0f;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    float o[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      o[i] = dpp_row_shr1(acc[0][t][i]) + acc[1][t][i] + dpp_row_shl1(acc[2][t][i]) + bias[i];
      if (a.relu) o[i] = o[i] > 0.0f ? o[i] : 0.0f;
    }
    const int y = y0 + t;
    if (r < 1 || r > kFOut || x >= a.n1 || y >= a.n2 || z >= a.n3) continue;
    // 32-bit byte offset (checked by the launcher)
    const uint32_t ob =
        2u * (uint32_t)(((z * a.n2 + y) * a.n1 + x) * a.out_stride + a.out_off + 4 * g);
    *reinterpret_cast<uint2*>(reinterpret_cast<char*>(a.out) + ob) =
        make_uint2(pack_bf16(o[0], o[1]), pack_bf16(o[2], o[3]));
  }
}

// ---------------------------------------------------------------------------
// Register-blocked form (16 and 32 output channels on large grids).  A
// wavefront owns TY x TZ rows of 16 output voxels along x (lane r: x0 + r),
// all cout; the four wavefronts of a workgroup sit 2 x 2 in (y, z), so a
// workgroup owns 16 x 2TY x 2TZ voxels.  A k-block of 32 is one group of 8
// input channels at the three x-shifts: lane group g < 3 takes dx = g - 1,
// group 3 is zero.  Per channel group the input block with its halo (16
// bytes per voxel) and the group's weight fragments (nine (dz, dy) per lane)
// are copied from global memory straight into LDS (global_load_lds, no
// registers), double buffered: the copy of group c + 1 runs while group c is
// computed.  Every input fragment -- one halo row y_in of one halo plane
// z_in -- is read from LDS once and feeds the MFMAs of every output row
// t = y_in - dy and plane w = z_in - dz it reaches (up to nine).  Voxels
// outside the grid, and the zero lane group's weights, are read from a
// zeroed line.  Same products as conv3_tile_kernel; the FP32 sums are taken
// in another order.

__device__ __align__(16) const uint4 kZeroLine = {0u, 0u, 0u, 0u};

// one 16-byte global -> LDS copy per lane; dst is the wavefront's slot 0 (the
// lane's slot is dst + lane)
__device__ __forceinline__ void copy16_lds(const void* src, uint4* dst_wave) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)dst_wave, 16, 0,
                                   0);
}

template <int MT, int TY, int TZ>
__host__ __device__ constexpr int reg_halo() { return 18 * (2 * TY + 2) * (2 * TZ + 2); }
template <int MT>
__host__ __device__ constexpr int reg_wslots() { return 9 * 64 * MT; }
template <int MT, int TY, int TZ>
__host__ __device__ constexpr int reg_lds_bytes() {
  // two buffers, each: the halo block rounded up to whole wavefront copies,
  // then the weight fragments
  return 2 * (((reg_halo<MT, TY, TZ>() + 63) / 64) * 64 + reg_wslots<MT>()) * 16;
}

template <int MT, int TY, int TZ>
__global__ __launch_bounds__(256) void conv3_reg_kernel(ConvArgs a, int tiles_x, int tiles_y,
                                                         int tiles_z) {
  constexpr int BY = 2 * TY, BZ = 2 * TZ;
  constexpr int HX = 18, HY = BY + 2, HZ = BZ + 2, HV = HX * HY * HZ;
  constexpr int HVP = ((HV + 63) / 64) * 64;  // halo slots per buffer
  constexpr int WS = reg_wslots<MT>();        // weight slots per buffer
  constexpr int BUF = HVP + WS;
  extern __shared__ __align__(16) uint4 reg_lds[];
  uint4* lds = reg_lds;
  const int tid = threadIdx.x;
  const int lane = tid & 63, g = lane >> 4, r = lane & 15;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wy = w & 1, wz = w >> 1;
  // XCD-aware order: consecutive tiles of a row stay on one XCD
  const int nblk = gridDim.x;
  const int b = blockIdx.x;
  const int q = nblk >> 3, rem = nblk & 7, xcd = b & 7, kk = b >> 3;
  const int tile = (xcd < rem) ? xcd * (q + 1) + kk : rem * (q + 1) + (xcd - rem) * q + kk;
  const int tx = tile % tiles_x, ty = (tile / tiles_x) % tiles_y, tz = tile / (tiles_x * tiles_y);
  const int x0 = tx * 16, y0 = ty * BY, z0 = tz * BZ;
  (void)tiles_z;
  const bool gact = g < 3;  // lane group 3 carries the zero quarter of each k-block

  // issue the copies of channel group c8 into buffer `buf` (asynchronous)
  auto stage = [&](int c8, int buf) {
    uint4* base = lds + (size_t)buf * BUF;
    for (int i0 = w * 64; i0 < HV; i0 += 256) {
      const int i = i0 + lane;
      if (i < HV) {
        const int hx = i % HX, hy = (i / HX) % HY, hz = i / (HX * HY);
        const int x = x0 + hx - 1, y = y0 + hy - 1, z = z0 + hz - 1;
        const void* src = &kZeroLine;
        if (x >= 0 && x < a.n1 && y >= 0 && y < a.n2 && z >= 0 && z < a.n3) {
          const long long v = ((long long)z * a.n2 + y) * a.n1 + x;
          src = a.in + v * a.in_stride + a.in_off + 8 * c8;
        }
        copy16_lds(src, base + i0);
      }
    }
    // weight slot (m, dz, dy) x lane: W[m*16 + r][tap(dz, dy, dx = g - 1)][8 c8 ..]
    for (int s0 = w * 64; s0 < WS; s0 += 256) {
      const int f = s0 / 64;  // fragment index m * 9 + dz * 3 + dy
      const int m = f / 9, dz = (f % 9) / 3, dy = f % 3;
      const void* src = &kZeroLine;
      if (gact) {
        const int tap = dz * 9 + dy * 3 + g;
        src = a.w + (long long)(m * 16 + r) * a.kpad + tap * a.cin + 8 * c8;
      }
      copy16_lds(src, base + HVP + s0);
    }
  };

  f32x4 acc[MT][TZ][TY];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int i = 0; i < TZ; ++i)
#pragma unroll
      for (int t = 0; t < TY; ++t) acc[m][i][t] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int ngroups = a.cin / 8;
  stage(0, 0);
  const int hoff = (wz * TZ * HY + wy * TY) * HX + r + (gact ? g : 0);
  for (int c8 = 0; c8 < ngroups; ++c8) {
    // this group's copies are complete and visible; every wavefront is done
    // with the other buffer (group c8 - 1), which the next copy overwrites
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (c8 + 1 < ngroups) stage(c8 + 1, (c8 + 1) & 1);
    const uint4* hb = lds + (size_t)(c8 & 1) * BUF;
    const uint4* wb = hb + HVP;
    bf16x8 afr[MT][3][3];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int dz = 0; dz < 3; ++dz)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          const uint4 u = wb[(m * 9 + dz * 3 + dy) * 64 + lane];
          afr[m][dz][dy] = *reinterpret_cast<const bf16x8*>(&u);
        }
#pragma unroll
    for (int zi = 0; zi < TZ + 2; ++zi) {
#pragma unroll
      for (int yi = 0; yi < TY + 2; ++yi) {
        const uint4 u = hb[hoff + (zi * HY + yi) * HX];
        bf16x8 f = *reinterpret_cast<const bf16x8*>(&u);
        if (!gact) f = zero8();
#pragma unroll
        for (int dz = 0; dz < 3; ++dz) {
          const int wv = zi - dz;
          if (wv < 0 || wv >= TZ) continue;
#pragma unroll
          for (int dy = 0; dy < 3; ++dy) {
            const int tv = yi - dy;
            if (tv < 0 || tv >= TY) continue;
#pragma unroll
            for (int m = 0; m < MT; ++m) acc[m][wv][tv] = mfma16(afr[m][dz][dy], f, acc[m][wv][tv]);
          }
        }
      }
    }
  }
  // epilogue: lane holds channels m*16 + 4g .. +3 of voxel (x0 + r, y, z)
  const int x = x0 + r;
  if (x >= a.n1) return;
#pragma unroll
  for (int i = 0; i < TZ; ++i) {
    const int z = z0 + wz * TZ + i;
    if (z >= a.n3) continue;
#pragma unroll
    for (int t = 0; t < TY; ++t) {
      const int y = y0 + wy * TY + t;
      if (y >= a.n2) continue;
      const long long v = ((long long)z * a.n2 + y) * a.n1 + x;
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const int co = m * 16 + 4 * g;
        float o[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          o[j] = acc[m][i][t][j] + (a.bias ? a.bias[co + j] : 0.0f);
          if (a.relu) o[j] = o[j] > 0.0f ? o[j] : 0.0f;
        }
        *reinterpret_cast<uint2*>(a.out + v * a.out_stride + a.out_off + co) =
            make_uint2(pack_bf16(o[0], o[1]), pack_bf16(o[2], o[3]));
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Weight gradient as an implicit GEMM over voxels:
//   dW[co][tap][ci] = sum_v dY[v][co] X[v + offset(tap)][ci],  db[co] = sum_v dY[v][co].
// Grid (voxel ranges) x (27 taps).  A workgroup walks its voxel range in
// chunks of CHUNK voxels: the chunk of dY and the shifted chunk of X are loaded
// 8 channels (16 bytes) at a time and stored transposed in LDS
// ([channel][voxel], rows padded by 8 elements against bank conflicts), so
// an MFMA operand (8 consecutive voxels of one channel) is one 16-byte LDS
// read.  The (cout/16) x (cin16/16) output tiles are spread over the four
// wavefronts.  Partial sums per workgroup are reduced in a fixed order by a
// second kernel, so the result is deterministic.

constexpr int wg_pitch(int chunk) { return chunk + 8; }


template <int PITCH>
__device__ __forceinline__ void stage_t(uint16_t* dst, int row0, int vv, const uint4& q) {
  const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    dst[(row0 + 2 * j) * PITCH + vv] = (uint16_t)(w[j] & 0xffffu);
    dst[(row0 + 2 * j + 1) * PITCH + vv] = (uint16_t)(w[j] >> 16);
  }
}

// CHUNK voxels per iteration (a multiple of 32): 192 where the two staged
// blocks fit in 64 KiB of LDS, else 64.  The loop waits on its global loads
// once per chunk: 192-voxel chunks took the training step at 96^3 from 4.8
// to 3.0 ms (448-voxel chunks, two workgroups per CU: 3.2 ms).
template <int CHUNK>
__global__ __launch_bounds__(256) void conv3_wgrad_kernel(WgradArgs a) {
  constexpr int PITCH = CHUNK + 8;
  extern __shared__ uint16_t lds[];
  const int cin16 = (a.cin + 15) & ~15;
  uint16_t* dyt = lds;                        // [cout][PITCH]
  uint16_t* xt = lds + a.cout * PITCH;     // [cin16][PITCH]
  const int tid = threadIdx.x;
  const int lane = tid & 63, g = lane >> 4, r = lane & 15, wave = tid >> 6;
  const int tap = blockIdx.y;
  const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
  const long long nvox = (long long)a.n1 * a.n2 * a.n3;
  const long long per = (nvox + gridDim.x - 1) / gridDim.x;
  const long long v0 = (long long)blockIdx.x * per;
  const long long v1 = v0 + per < nvox ? v0 + per : nvox;
  const int ntl = cin16 / 16, ntiles = (a.cout / 16) * ntl;
  const int cg = a.cout >> 3, xg = cin16 >> 3, xgv = a.cin >> 3;
  const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);
  f32x4 acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.0f;
  for (long long c0 = v0; c0 < v1; c0 += CHUNK) {
    __syncthreads();
    for (int i = tid; i < CHUNK * cg; i += 256) {
      const int vv = i % CHUNK, c8 = i / CHUNK;
      const long long v = c0 + vv;
      const uint4 q = v < v1 ? *reinterpret_cast<const uint4*>(a.dy + v * a.dy_stride + a.dy_off + 8 * c8)
                             : z4;
      stage_t<PITCH>(dyt, 8 * c8, vv, q);
    }
    for (int i = tid; i < CHUNK * xg; i += 256) {
      const int vv = i % CHUNK, c8 = i / CHUNK;
      const long long v = c0 + vv;
      uint4 q = z4;
      if (v < v1 && c8 < xgv) {
        // 32-bit index arithmetic (the launcher checks nvox < 2^31): the
        // 64-bit divisions were most of this loop's work
        const unsigned u = (unsigned)v, t = u / (unsigned)a.n1;
        const int x = (int)(u - t * (unsigned)a.n1) + dx;
        const int y = (int)(t % (unsigned)a.n2) + dy;
        const int z = (int)(t / (unsigned)a.n2) + dz;
        if (x >= 0 && x < a.n1 && y >= 0 && y < a.n2 && z >= 0 && z < a.n3) {
          const long long src = ((long long)z * a.n2 + y) * a.n1 + x;
          q = *reinterpret_cast<const uint4*>(a.x + src * a.x_stride + a.x_off + 8 * c8);
        }
      }
      stage_t<PITCH>(xt, 8 * c8, vv, q);
    }
    __syncthreads();
    if (tap == 13 && tid < a.cout) {
      for (int vv = 0; vv < CHUNK; ++vv) bsum += bf2f(dyt[tid * PITCH + vv]);
    }
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) {
      const int tl = wave + 4 * sl;
      if (tl < ntiles) {
        const int m = tl / ntl, n = tl - m * ntl;
#pragma unroll
        for (int kk = 0; kk < CHUNK / 32; ++kk) {
          const bf16x8 af =
              *reinterpret_cast<const bf16x8*>(dyt + (m * 16 + r) * PITCH + kk * 32 + 8 * g);
          const bf16x8 bv =
              *reinterpret_cast<const bf16x8*>(xt + (n * 16 + r) * PITCH + kk * 32 + 8 * g);
          acc[sl] = mfma16(af, bv, acc[sl]);
        }
      }
    }
  }
  // lane holds dW rows co = m*16 + 4g .. +3 of column ci = n*16 + r
  float* part = a.part + (size_t)blockIdx.x * a.cout * 27 * a.cin;
#pragma unroll
  for (int sl = 0; sl < 4; ++sl) {
    const int tl = wave + 4 * sl;
    if (tl < ntiles) {
      const int m = tl / ntl, n = tl - m * ntl;
      const int ci = n * 16 + r;
      if (ci < a.cin) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int co = m * 16 + 4 * g + i;
          part[((size_t)co * 27 + tap) * a.cin + ci] = acc[sl][i];
        }
      }
    }
  }
  if (tap == 13 && tid < a.cout) a.part_bias[(size_t)blockIdx.x * a.cout + tid] = bsum;
}

// ---------------------------------------------------------------------------
// Weight gradient with the taps sharing their staging.  The voxels are cut
// into blocks of 32 (x) x 2 (y) x 2 (z); a workgroup walks a range of blocks
// for one 16-channel chunk of the input and a group of T taps.  Per block
// dY (all cout channels) and X with its one-voxel halo (the chunk's 16
// channels) are staged once, transposed to channel-major rows in LDS, X in
// three copies pre-shifted by dx = -1, 0, +1, so that every MFMA operand of
// every tap -- 8 consecutive x of one channel -- is one aligned 16-byte LDS
// read; a K-block of 32 is one x-row of the block.  The T taps x cout/16
// output tiles are spread over the four wavefronts (at most kWtTiles each).
// The next block's loads are issued before the current block's MFMAs.
// Partials and bias partials as conv3_wgrad_kernel (same layout, reduced by
// the same kernel).

constexpr int kWtBX = 32, kWtBY = 2, kWtBZ = 2;                 // voxel block
constexpr int kWtHX = kWtBX + 2, kWtHY = kWtBY + 2, kWtHZ = kWtBZ + 2;
constexpr int kWtRows = kWtHY * kWtHZ;                         // halo rows per channel
constexpr int kWtXPitch = kWtRows * kWtBX + 8;                 // per channel (x copy), elements
constexpr int kWtYPitch = kWtBY * kWtBZ * kWtBX + 8;           // per channel (dY), elements
constexpr int kWtTiles = 9;                                    // tiles per wavefront, at most

__host__ __device__ constexpr size_t wtap_lds_bytes(int cout) {
  return (size_t)(3 * 16 * kWtXPitch + cout * kWtYPitch) * sizeof(uint16_t);
}

template <int NX, int NY>  // 16-byte loads per thread: X halo, dY
__global__ __launch_bounds__(256) void conv3_wgrad_tap_kernel(WgradArgs a, int taps_per_wg,
                                                              long long blocks_per_range) {
  extern __shared__ __align__(16) uint16_t lds[];
  uint16_t* xs = lds;                          // [3 copies][16 ch][rows][32 x]
  uint16_t* ys = lds + 3 * 16 * kWtXPitch;     // [cout][2 z][2 y][32 x]
  const int tid = threadIdx.x;
  const int lane = tid & 63, g = lane >> 4, r = lane & 15, wave = tid >> 6;
  const int range = blockIdx.x, chunk = blockIdx.y, tgrp = blockIdx.z;
  const int T = taps_per_wg, tap0 = tgrp * T;
  const int MT = a.cout / 16, ntiles = T * MT;
  const int nbx = (a.n1 + kWtBX - 1) / kWtBX, nby = (a.n2 + kWtBY - 1) / kWtBY;
  const long long nblk = (long long)nbx * nby * ((a.n3 + kWtBZ - 1) / kWtBZ);
  const long long b0 = range * blocks_per_range;
  const long long b1 = b0 + blocks_per_range < nblk ? b0 + blocks_per_range : nblk;
  const int cg = a.cout >> 3;                   // 8-channel groups of dY
  const int ci0 = chunk * 16;
  const bool bias_wg = chunk == 0 && tgrp == 0 && a.part_bias;

  f32x4 acc[kWtTiles];
#pragma unroll
  for (int j = 0; j < kWtTiles; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.0f;

  uint4 xr[NX], yr[NY];
  // loads of block b into registers (zeros outside the grid and past cin)
  auto load_block = [&](long long b) {
    const int bx = (int)(b % nbx), by = (int)((b / nbx) % nby), bz = (int)(b / ((long long)nbx * nby));
    const int x0 = bx * kWtBX, y0 = by * kWtBY, z0 = bz * kWtBZ;
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const int i = tid + 256 * j;  // (halo voxel, 8-channel group)
      xr[j] = make_uint4(0u, 0u, 0u, 0u);
      if (i < kWtHX * kWtRows * 2) {
        const int c8 = i & 1, hv = i >> 1;
        const int hx = hv % kWtHX, hr = hv / kWtHX, hy = hr % kWtHY, hz = hr / kWtHY;
        const int x = x0 + hx - 1, y = y0 + hy - 1, z = z0 + hz - 1;
        if (ci0 + 8 * c8 < a.cin && x >= 0 && x < a.n1 && y >= 0 && y < a.n2 && z >= 0 &&
            z < a.n3) {
          const long long v = ((long long)z * a.n2 + y) * a.n1 + x;
          xr[j] = *reinterpret_cast<const uint4*>(a.x + v * a.x_stride + a.x_off + ci0 + 8 * c8);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < NY; ++j) {
      const int i = tid + 256 * j;  // (block voxel, 8-channel group)
      yr[j] = make_uint4(0u, 0u, 0u, 0u);
      if (i < kWtBX * kWtBY * kWtBZ * cg) {
        const int c8 = i % cg, bv = i / cg;
        const int x = x0 + bv % kWtBX, y = y0 + (bv / kWtBX) % kWtBY, z = z0 + bv / (kWtBX * kWtBY);
        if (x < a.n1 && y < a.n2 && z < a.n3) {
          const long long v = ((long long)z * a.n2 + y) * a.n1 + x;
          yr[j] = *reinterpret_cast<const uint4*>(a.dy + v * a.dy_stride + a.dy_off + 8 * c8);
        }
      }
    }
  };
  auto put8 = [&](uint16_t* dst, int pitch, const uint4& q) {
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      dst[(2 * j) * pitch] = (uint16_t)(w[j] & 0xffffu);
      dst[(2 * j + 1) * pitch] = (uint16_t)(w[j] >> 16);
    }
  };
  if (b0 < b1) load_block(b0);
  for (long long b = b0; b < b1; ++b) {
    __syncthreads();  // the previous block's LDS reads are done
#pragma unroll
    for (int j = 0; j < NX; ++j) {
      const int i = tid + 256 * j;
      if (i < kWtHX * kWtRows * 2) {
        const int c8 = i & 1, hv = i >> 1;
        const int hx = hv % kWtHX, hr = hv / kWtHX;
        // copy d holds x' = hx - d (source x = x0 + x' + d - 1)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const int xp = hx - d;
          if (xp >= 0 && xp < kWtBX)
            put8(xs + (d * 16 + 8 * c8) * kWtXPitch + hr * kWtBX + xp, kWtXPitch, xr[j]);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < NY; ++j) {
      const int i = tid + 256 * j;
      if (i < kWtBX * kWtBY * kWtBZ * cg) {
        const int c8 = i % cg, bv = i / cg;
        put8(ys + (8 * c8) * kWtYPitch + bv, kWtYPitch, yr[j]);
      }
    }
    __syncthreads();
    if (b + 1 < b1) load_block(b + 1);
    if (bias_wg && tid < a.cout) {
      for (int bv = 0; bv < kWtBX * kWtBY * kWtBZ; ++bv) bsum += bf2f(ys[tid * kWtYPitch + bv]);
    }
    // K-block kb = the x-row (y', z') of the block
#pragma unroll
    for (int kb = 0; kb < kWtBY * kWtBZ; ++kb) {
      const int yq = kb % kWtBY, zq = kb / kWtBY;
#pragma unroll
      for (int j = 0; j < kWtTiles; ++j) {
        const int tl = wave + 4 * j;
        if (tl < ntiles) {
          const int m = tl % MT, tap = tap0 + tl / MT;
          const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
          const bf16x8 af = *reinterpret_cast<const bf16x8*>(
              ys + (m * 16 + r) * kWtYPitch + kb * kWtBX + 8 * g);
          const bf16x8 bf = *reinterpret_cast<const bf16x8*>(
              xs + ((dx + 1) * 16 + r) * kWtXPitch +
              ((zq + dz + 1) * kWtHY + (yq + dy + 1)) * kWtBX + 8 * g);
          acc[j] = mfma16(af, bf, acc[j]);
        }
      }
    }
  }
  // lane holds dW rows co = m*16 + 4g .. +3 of column ci = ci0 + r, tap
  float* part = a.part + (size_t)range * a.cout * 27 * a.cin;
#pragma unroll
  for (int j = 0; j < kWtTiles; ++j) {
    const int tl = wave + 4 * j;
    if (tl < ntiles) {
      const int m = tl % MT, tap = tap0 + tl / MT;
      const int ci = ci0 + r;
      if (ci < a.cin) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int co = m * 16 + 4 * g + i;
          part[((size_t)co * 27 + tap) * a.cin + ci] = acc[j][i];
        }
      }
    }
  }
  if (bias_wg && tid < a.cout) a.part_bias[(size_t)range * a.cout + tid] = bsum;
}

// sum of per-workgroup partials in workgroup order (deterministic); the
// loads of 16 partials are issued together before they are added in order
__global__ void reduce_parts_kernel(const float* part, int nparts, long long len, float* out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  float s = 0.0f;
  int p = 0;
  for (; p + 16 <= nparts; p += 16) {
    float v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = part[(size_t)(p + j) * len + i];
#pragma unroll
    for (int j = 0; j < 16; ++j) s += v[j];
  }
  for (; p < nparts; ++p) s += part[(size_t)p * len + i];
  out[i] = s;
}

// ---------------------------------------------------------------------------
// Elementwise pieces

// dY <- dY * (Y > 0) (ReLU backward), in place on the gradient view
__global__ void relu_bwd_kernel(uint16_t* dy, int dy_stride, int dy_off, const uint16_t* y,
                                int y_stride, int y_off, int c, long long nvox) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvox * c) return;
  const long long v = i / c;
  const int ch = (int)(i - v * c);
  const float yy = bf2f(y[v * y_stride + y_off + ch]);
  if (!(yy > 0.0f)) dy[v * dy_stride + dy_off + ch] = 0;
}

// 2x average pooling; out grid (m1, m2, m3) = input / 2
__global__ void pool_fwd_kernel(const uint16_t* in, int in_stride, int in_off, uint16_t* out,
                                int out_stride, int out_off, int c, int m1, int m2, int m3) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nv = (long long)m1 * m2 * m3;
  if (i >= nv * c) return;
  const long long v = i / c;
  const int ch = (int)(i - v * c);
  const int x = (int)(v % m1), y = (int)((v / m1) % m2), z = (int)(v / ((long long)m1 * m2));
  const int n1 = 2 * m1, n2 = 2 * m2;
  float s = 0.0f;
  for (int d = 0; d < 8; ++d) {
    const long long src = ((long long)(2 * z + (d >> 2)) * n2 + (2 * y + ((d >> 1) & 1))) * n1 +
                          (2 * x + (d & 1));
    s += bf2f(in[src * in_stride + in_off + ch]);
  }
  out[v * out_stride + out_off + ch] = f2bf(0.125f * s);
}

// pooling backward: dIn[child] (+)= dOut[parent] / 8
__global__ void pool_bwd_kernel(const uint16_t* dout, int dout_stride, int dout_off,
                                uint16_t* din, int din_stride, int din_off, int c, int n1, int n2,
                                int n3, int accumulate) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nv = (long long)n1 * n2 * n3;
  if (i >= nv * c) return;
  const long long v = i / c;
  const int ch = (int)(i - v * c);
  const int x = (int)(v % n1), y = (int)((v / n1) % n2), z = (int)(v / ((long long)n1 * n2));
  const int m1 = n1 / 2, m2 = n2 / 2;
  const long long p = ((long long)(z / 2) * m2 + y / 2) * m1 + x / 2;
  float g = 0.125f * bf2f(dout[p * dout_stride + dout_off + ch]);
  uint16_t* dst = din + v * din_stride + din_off + ch;
  if (accumulate) g += bf2f(*dst);
  *dst = f2bf(g);
}

// Vector forms of 2x average pooling and nearest upsampling: one thread per
// voxel and group of 8 channels (16 bytes), 32-bit index arithmetic (grids
// below 2^24 voxels).  Per channel the same sums in the same order as the
// one-element kernels, so the results are bitwise the same.
__device__ __forceinline__ uint4 ld16(const uint16_t* p) { return *reinterpret_cast<const uint4*>(p); }

__global__ void pool_fwd8_kernel(const uint16_t* in, int in_stride, int in_off, uint16_t* out,
                                 int out_stride, int out_off, int c8, int m1, int m2,
                                 unsigned total) {
  const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const unsigned v = i / (unsigned)c8, g = i - v * (unsigned)c8;
  const unsigned x = v % (unsigned)m1, t = v / (unsigned)m1;
  const unsigned y = t % (unsigned)m2, z = t / (unsigned)m2;
  const unsigned n1 = 2u * m1, n2 = 2u * m2;
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int d = 0; d < 8; ++d) {
    const unsigned src = ((2u * z + (d >> 2)) * n2 + (2u * y + ((d >> 1) & 1))) * n1 + (2u * x + (d & 1));
    const uint4 q = ld16(in + (size_t)src * in_stride + in_off + 8 * g);
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      acc[2 * k] += bf2f((uint16_t)(w[k] & 0xffffu));
      acc[2 * k + 1] += bf2f((uint16_t)(w[k] >> 16));
    }
  }
  uint32_t o[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    o[k] = (uint32_t)f2bf(0.125f * acc[2 * k]) | ((uint32_t)f2bf(0.125f * acc[2 * k + 1]) << 16);
  *reinterpret_cast<uint4*>(out + (size_t)v * out_stride + out_off + 8 * g) =
      make_uint4(o[0], o[1], o[2], o[3]);
}

__global__ void up_fwd8_kernel(const uint16_t* in, int in_stride, int in_off, uint16_t* out,
                               int out_stride, int out_off, int c8, int n1, int n2,
                               unsigned total) {
  const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const unsigned v = i / (unsigned)c8, g = i - v * (unsigned)c8;
  const unsigned x = v % (unsigned)n1, t = v / (unsigned)n1;
  const unsigned y = t % (unsigned)n2, z = t / (unsigned)n2;
  const unsigned p = ((z >> 1) * ((unsigned)n2 >> 1) + (y >> 1)) * ((unsigned)n1 >> 1) + (x >> 1);
  *reinterpret_cast<uint4*>(out + (size_t)v * out_stride + out_off + 8 * g) =
      ld16(in + (size_t)p * in_stride + in_off + 8 * g);
}

// The decoder's input at one level: nearest 2x upsampling of the coarser
// path (cu channels) and the skip tensor of this level (cs channels),
// concatenated per voxel into out (stride cu + cs).  One thread per 8
// channels of a voxel, so consecutive threads write each voxel's whole row:
// the skip half is not written on its own as a strided partial row (on grids
// past the last-level cache those partial lines cost a read-modify-write
// each).
__global__ void up_cat8_kernel(const uint16_t* up, int up_stride, const uint16_t* skip,
                               int skip_stride, uint16_t* out, int cu8, int cs8, int n1, int n2,
                               unsigned total) {
  const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const unsigned c8 = (unsigned)(cu8 + cs8);
  const unsigned v = i / c8, g = i - v * c8;
  uint4 q;
  if (g < (unsigned)cu8) {
    const unsigned x = v % (unsigned)n1, t = v / (unsigned)n1;
    const unsigned y = t % (unsigned)n2, z = t / (unsigned)n2;
    const unsigned p =
        ((z >> 1) * ((unsigned)n2 >> 1) + (y >> 1)) * ((unsigned)n1 >> 1) + (x >> 1);
    q = ld16(up + (size_t)p * up_stride + 8 * g);
  } else {
    q = ld16(skip + (size_t)v * skip_stride + 8 * (g - (unsigned)cu8));
  }
  *reinterpret_cast<uint4*>(out + (size_t)v * (8 * c8) + 8 * g) = q;
}

// nearest 2x upsampling (output grid n = 2 m)
__global__ void up_fwd_kernel(const uint16_t* in, int in_stride, int in_off, uint16_t* out,
                              int out_stride, int out_off, int c, int n1, int n2, int n3) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nv = (long long)n1 * n2 * n3;
  if (i >= nv * c) return;
  const long long v = i / c;
  const int ch = (int)(i - v * c);
  const int x = (int)(v % n1), y = (int)((v / n1) % n2), z = (int)(v / ((long long)n1 * n2));
  const int m1 = n1 / 2, m2 = n2 / 2;
  const long long p = ((long long)(z / 2) * m2 + y / 2) * m1 + x / 2;
  out[v * out_stride + out_off + ch] = in[p * in_stride + in_off + ch];
}

// upsampling backward: dIn[parent] = sum of the 8 children's gradients
__global__ void up_bwd_kernel(const uint16_t* dout, int dout_stride, int dout_off, uint16_t* din,
                              int din_stride, int din_off, int c, int m1, int m2, int m3) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nv = (long long)m1 * m2 * m3;
  if (i >= nv * c) return;
  const long long v = i / c;
  const int ch = (int)(i - v * c);
  const int x = (int)(v % m1), y = (int)((v / m1) % m2), z = (int)(v / ((long long)m1 * m2));
  const int n1 = 2 * m1, n2 = 2 * m2;
  float s = 0.0f;
  for (int d = 0; d < 8; ++d) {
    const long long src = ((long long)(2 * z + (d >> 2)) * n2 + (2 * y + ((d >> 1) & 1))) * n1 +
                          (2 * x + (d & 1));
    s += bf2f(dout[src * dout_stride + dout_off + ch]);
  }
  din[v * din_stride + din_off + ch] = f2bf(s);
}

// network input: channel 0 glass mask, 1 supercooling feature, 2 surface
// tension feature, 3..7 zero (the first convolution takes 8 channels)
__global__ void input_kernel(const uint8_t* glass, int glass_from_code, float f1, float f2,
                             uint16_t* out, long long nvox) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvox) return;
  const uint8_t gb = glass[v];
  const float gm = glass_from_code ? ((gb & 0x40u) ? 1.0f : 0.0f) : (gb ? 1.0f : 0.0f);
  uint16_t* o = out + v * 8;
  o[0] = f2bf(gm);
  o[1] = f2bf(f1);
  o[2] = f2bf(f2);
  for (int c = 3; c < 8; ++c) o[c] = 0;
}

// number of water cells: per-workgroup partial counts (exact in FP32 below 2^24)
__global__ __launch_bounds__(256) void count_water_kernel(const uint8_t* glass, int from_code,
                                                         long long nvox, float* part) {
  __shared__ float red[256];
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  float c = 0.0f;
  if (v < nvox) c = (from_code ? !(glass[v] & 0x40u) : !glass[v]) ? 1.0f : 0.0f;
  red[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// head: yhat = sigmoid(b + sum_c w[c] h[v][c]) on water cells, 0 on glass.
// With a target: squared error on water cells, the gradient wrt h of the
// mean over water cells, and per-workgroup partial sums of the squared error
// and of the head's weight and bias gradients (fixed-order tree sums).
__global__ __launch_bounds__(256) void head_kernel(HeadArgs a) {
  __shared__ float red[kHeadParts][256];
  const long long v = (long long)blockIdx.x * 256 + threadIdx.x;
  const bool in = v < a.nvox;
  float hv[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) hv[c] = 0.0f;
  float dz = 0.0f, loss = 0.0f;
  if (in) {
    const bool water = a.code_glass ? !(a.glass[v] & 0x40u) : !a.glass[v];
    float z = a.b[0];
    const uint4* hp = reinterpret_cast<const uint4*>(a.h + v * a.h_stride + a.h_off);
    const uint4 q0 = hp[0], q1 = hp[1];
    const uint32_t w8[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      hv[2 * j] = bf2f((uint16_t)(w8[j] & 0xffffu));
      hv[2 * j + 1] = bf2f((uint16_t)(w8[j] >> 16));
    }
#pragma unroll
    for (int c = 0; c < 16; ++c) z += a.w[c] * hv[c];
    const float sg = 1.0f / (1.0f + expf(-z));
    const float yhat = (water && !(a.keep && !a.keep[v])) ? sg : 0.0f;
    if (a.out) {
      if (a.out_fp64) static_cast<double*>(a.out)[v] = (double)yhat;
      else static_cast<float*>(a.out)[v] = yhat;
    }
    if (a.target && water) {
      const float e = sg - a.target[v];
      loss = e * e;
      dz = 2.0f * e * sg * (1.0f - sg) / a.count[0];
    }
    if (a.target) {
      uint32_t o[8];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        o[j] = (uint32_t)f2bf(dz * a.w[2 * j]) | ((uint32_t)f2bf(dz * a.w[2 * j + 1]) << 16);
      uint4* dp = reinterpret_cast<uint4*>(a.dh + v * 16);
      dp[0] = make_uint4(o[0], o[1], o[2], o[3]);
      dp[1] = make_uint4(o[4], o[5], o[6], o[7]);
    }
  }
  if (!a.target) return;
  red[0][threadIdx.x] = loss;
  red[1][threadIdx.x] = dz;
#pragma unroll
  for (int c = 0; c < 16; ++c) red[2 + c][threadIdx.x] = dz * hv[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int j = 0; j < kHeadParts; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < kHeadParts) a.part[(size_t)blockIdx.x * kHeadParts + threadIdx.x] = red[threadIdx.x][0];
}

// master FP32 weights [co][27][ci] -> BF16 forward copy [co][kpad] and
// data-gradient copy [ci][kpad_t] (taps mirrored: k' = (26 - tap) * cout + co)
__global__ void weights_kernel(const float* wm, int cout, int cin, int kpad, int kpad_t,
                               uint16_t* wf, uint16_t* wd) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nf = (long long)cout * kpad, nd = (long long)cin * kpad_t;
  if (i < nf) {
    const int co = (int)(i / kpad), k = (int)(i - (long long)co * kpad);
    wf[i] = k < 27 * cin ? f2bf(wm[((size_t)co * 27 + k / cin) * cin + k % cin]) : (uint16_t)0;
  } else if (wd && i < nf + nd) {
    const long long j = i - nf;
    const int ci = (int)(j / kpad_t), k = (int)(j - (long long)ci * kpad_t);
    uint16_t val = 0;
    if (k < 27 * cout) {
      const int tapf = k / cout, co = k % cout, tap = 26 - tapf;
      val = f2bf(wm[((size_t)co * 27 + tap) * cin + ci]);
    }
    wd[j] = val;
  }
}

// Adam with bias correction (Kingma and Ba 2015) on the flat FP32 parameters
__global__ void adam_kernel(float* p, const float* g, float* m, float* v, long long n, float lr,
                            float b1, float b2, float eps, float bc1, float bc2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

__global__ void f32_to_bf16_kernel(const float* in, uint16_t* out, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = f2bf(in[i]);
}

__global__ void bf16_to_f32_kernel(const uint16_t* in, float* out, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = bf2f(in[i]);
}

// ---------------------------------------------------------------------------
// Water cells reachable from the nucleus.  Under the phase-field equation
// with zero phi-flux across glass faces, a face-connected component of water
// cells that holds no ice keeps phi = 0 for ever (no flux in, and phi = 0 is
// a fixed point of the reaction term), so ice can only appear in the
// components that contain the initial nucleus.

// No-network baseline of the warm start: phi = 1 on the reached cells (the
// nucleus's water component), 0 elsewhere.
__global__ void flood_kernel(const uint8_t* reach, void* out, int fp64, long long n) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  if (fp64)
    static_cast<double*>(out)[v] = reach[v] ? 1.0 : 0.0;
  else
    static_cast<float*>(out)[v] = reach[v] ? 1.0f : 0.0f;
}

// Connected components of the water cells by union-find (face neighbours
// joined across water-water faces, bits 0..5 of the cell code), in two
// levels.  A workgroup first labels the components inside its 16^3 tile with
// a union-find in LDS and writes, for every cell, the global index of its
// tile-local root (so every tree in lab is flat at first).  A second kernel
// then unites only across tile faces, in global memory.  lab[v] is v's parent
// and a root has lab[v] == v; a link always hangs the root with the larger
// index under the one with the smaller index, and a find replaces a cell's
// parent by its grandparent as it climbs, so lab[v] <= v holds throughout:
// every path descends in index and every find ends.  A failed link means
// another thread linked that root first, so the retries of a union are
// bounded by the links made meanwhile (no thread waits on another).
//
// The links are agent-scope compare-and-swaps.  The finds of the merge read
// lab through the caches, which may return an older value of an entry: an
// older parent is still an ancestor (parents only ever move up), and an entry
// read as a root that has been linked meanwhile fails the compare-and-swap,
// whose result is the current parent, from which the union goes on upwards.
// Reading every step from memory instead (the XCDs' L2s are not coherent
// with each other) made each step a memory round trip: a single-level
// union-find over all 3 n faces took 319 us at 96^3.  The kernels after the
// merge read lab with agent-scope loads.
constexpr int kUT = 16;  // tile edge of the local labelling

__device__ __forceinline__ int uf_load(const int* lab, int x) {
  return __hip_atomic_load(lab + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// CACHED: plain loads and stores (the merge); else agent-scope ones
template <bool CACHED>
__device__ __forceinline__ int uf_find(int* lab, int x) {
  for (;;) {
    const int p = CACHED ? lab[x] : uf_load(lab, x);
    if (p == x) return x;
    const int g = CACHED ? lab[p] : uf_load(lab, p);
    if (g == p) return p;
    if (CACHED) lab[x] = g;
    else __hip_atomic_store(lab + x, g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = g;
  }
}

__device__ __forceinline__ void uf_union(int* lab, int a, int b) {
  a = uf_find<true>(lab, a);
  b = uf_find<true>(lab, b);
  while (a != b) {
    if (a > b) {
      const int t = a;
      a = b;
      b = t;
    }
    int expected = b;
    if (__hip_atomic_compare_exchange_strong(lab + b, &expected, a, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return;
    // b was linked meanwhile: continue from its new parent
    b = uf_find<true>(lab, expected);
    a = uf_find<true>(lab, a);
  }
}

// the same in LDS, on tile-local indices (workgroup scope)
__device__ __forceinline__ int lf_find(int* ll, int x) {
  for (;;) {
    const int p = __hip_atomic_load(ll + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (p == x) return x;
    const int g = __hip_atomic_load(ll + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (g == p) return p;
    __hip_atomic_store(ll + x, g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    x = g;
  }
}

__device__ __forceinline__ void lf_union(int* ll, int a, int b) {
  a = lf_find(ll, a);
  b = lf_find(ll, b);
  while (a != b) {
    if (a > b) {
      const int t = a;
      a = b;
      b = t;
    }
    int expected = b;
    if (__hip_atomic_compare_exchange_strong(ll + b, &expected, a, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
      return;
    b = lf_find(ll, expected);
    a = lf_find(ll, a);
  }
}

// Level 1: the components inside each 16^3 tile (cells outside the grid
// count as glass); lab = global index of the cell's tile-local root, and no
// cell reached yet.
__global__ __launch_bounds__(1024) void reach_local_kernel(const uint8_t* code, int* lab,
                                                          uint8_t* reach, int n1, int n2, int n3,
                                                          int tx, int ty) {
  constexpr int T = kUT * kUT * kUT;
  __shared__ int ll[T];
  __shared__ uint8_t sc[T];
  const int b = blockIdx.x;
  const int x0 = (b % tx) * kUT, y0 = ((b / tx) % ty) * kUT, z0 = (b / (tx * ty)) * kUT;
  const long long pl = (long long)n1 * n2;
  for (int i = threadIdx.x; i < T; i += 1024) {
    const int x = x0 + (i % kUT), y = y0 + (i / kUT) % kUT, z = z0 + i / (kUT * kUT);
    const bool in = x < n1 && y < n2 && z < n3;
    sc[i] = in ? code[z * pl + (long long)y * n1 + x] : (uint8_t)0x40u;
    ll[i] = i;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < T; i += 1024) {
    const unsigned c = sc[i];
    if (c & 0x40u) continue;
    const int lx = i % kUT, ly = (i / kUT) % kUT, lz = i / (kUT * kUT);
    if ((c & 2u) && lx + 1 < kUT) lf_union(ll, i, i + 1);
    if ((c & 8u) && ly + 1 < kUT) lf_union(ll, i, i + kUT);
    if ((c & 32u) && lz + 1 < kUT) lf_union(ll, i, i + kUT * kUT);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < T; i += 1024) {
    const int x = x0 + (i % kUT), y = y0 + (i / kUT) % kUT, z = z0 + i / (kUT * kUT);
    if (x >= n1 || y >= n2 || z >= n3) continue;
    const int r = lf_find(ll, i);
    const long long v = z * pl + (long long)y * n1 + x;
    lab[v] = (int)((z0 + r / (kUT * kUT)) * pl + (long long)(y0 + (r / kUT) % kUT) * n1 +
                   (x0 + r % kUT));
    reach[v] = 0;
  }
}

// Level 2: water cells on the +x1, +x2, +x3 face of their tile unite with
// their water neighbour in the next tile.
__global__ void reach_merge_kernel(const uint8_t* code, int* lab, int n1, int n2, long long n) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const long long pl = (long long)n1 * n2;
  const unsigned u = (unsigned)v, t = u / (unsigned)n1;  // n < 2^31
  const unsigned x = u - t * (unsigned)n1, y = t % (unsigned)n2, z = t / (unsigned)n2;
  const bool ex = x % kUT == kUT - 1, ey = y % kUT == kUT - 1, ez = z % kUT == kUT - 1;
  if (!(ex || ey || ez)) return;
  const unsigned c = code[v];
  if (c & 0x40u) return;
  if (ex && (c & 2u)) uf_union(lab, (int)v, (int)(v + 1));
  if (ey && (c & 8u)) uf_union(lab, (int)v, (int)(v + n1));
  if (ez && (c & 32u)) uf_union(lab, (int)v, (int)(v + pl));
}

// the components of the nucleus (water cells with phi > 1/2): flag at the root
__global__ void reach_seed_kernel(const uint8_t* code, const void* phi, int fp64, int* lab,
                                  uint8_t* reach, long long n) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const double p = fp64 ? static_cast<const double*>(phi)[v]
                        : (double)static_cast<const float*>(phi)[v];
  if (!(code[v] & 0x40u) && p > 0.5) reach[uf_find<false>(lab, (int)v)] = 1;
}

// every water cell takes its root's flag (a root keeps its own; the flags of
// non-root cells are read by no one)
__global__ void reach_resolve_kernel(const uint8_t* code, int* lab, uint8_t* reach, long long n) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  if (code[v] & 0x40u) return;
  const int r = uf_find<false>(lab, (int)v);
  if (r != (int)v) reach[v] = reach[r];
}

__global__ void clear_int_kernel(int* p) { *p = 0; }

// ---------------------------------------------------------------------------
// Host launchers

static inline unsigned blocks_for(long long n, int t) { return (unsigned)((n + t - 1) / t); }

constexpr long long kSplitBelow = 256;  // workgroups: one per CU

template <int CC>
static hipError_t launch_tile_cc(const ConvArgs& a, hipStream_t s) {
  const int tx = (a.n1 + kTX - 1) / kTX, ty = (a.n2 + kTY - 1) / kTY, tz = (a.n3 + kTZ - 1) / kTZ;
  // Output channels per workgroup: all of them, unless the grid then has
  // fewer workgroups than the chip has CUs (the coarsest level of the
  // network); then the most 16-channel groups per workgroup that still give
  // one workgroup per CU, else one group, with the groups over gridDim.y
  // (each workgroup stages the same input block; such small grids stay in
  // the L2).
  const long long tiles = (long long)tx * ty * tz;
  const int groups = a.cout / 16;
  int mt = groups;
  if (tiles < kSplitBelow) {
    mt = 1;
    for (int d = groups; d > 1; --d)
      if (groups % d == 0 && tiles * (groups / d) >= kSplitBelow) {
        mt = d;
        break;
      }
  }
  const dim3 grid((unsigned)tiles, (unsigned)(groups / mt)), block(256);
  if constexpr (CC == 16) {
    if (a.cout == 16) {
      // 16 output channels: the x-folded form, where each B fragment feeds
      // three MFMAs (48 -> 16 at 96^3: 48.4 instead of 49.7 us by events)
      const int fx = (a.n1 + kFOut - 1) / kFOut, fz = (a.n3 + 7) / 8;
      const long long ftiles = (long long)fx * ty * fz;
      const long long nv = (long long)a.n1 * a.n2 * a.n3;
      const bool out32 = 2 * (nv * a.out_stride + a.out_off) < 0xffffffffLL;
      // its staging loads mark slots outside the grid with offset 2^31
      const bool in31 = 2 * nv * a.in_stride < (1LL << 31) && 2LL * 16 * a.kpad < (1LL << 31);
      if (ftiles >= 2 * kSplitBelow && ftiles < (1LL << 31) && out32 && in31) {
        hipLaunchKernelGGL((conv3_xfold_kernel<8>), dim3((unsigned)ftiles), dim3(512), 0, s, a,
                           fx, ty);
        return hipGetLastError();
      }
    }
  }
  if constexpr (CC <= 16) {
    if (mt == 1 && tiles >= 2 * kSplitBelow) {
      // the one-group form on large grids: 8 planes (8 wavefronts) per
      // workgroup, so that the halo and the weights are staged once for
      // twice the outputs (48 -> 16 at 96^3: 58 instead of 64.5 us; 8 -> 16:
      // 23 instead of 26 us)
      const int tz8 = (a.n3 + 7) / 8;
      const long long tiles8 = (long long)tx * ty * tz8;
      hipLaunchKernelGGL((conv3_tile_kernel<1, CC, 8>), dim3((unsigned)tiles8, (unsigned)groups),
                         dim3(512), 0, s, a, tx, ty, tz8);
      return hipGetLastError();
    }
  }
  switch (mt) {
    case 1: hipLaunchKernelGGL((conv3_tile_kernel<1, CC, kTZ>), grid, block, 0, s, a, tx, ty, tz); break;
    case 2: hipLaunchKernelGGL((conv3_tile_kernel<2, CC, kTZ>), grid, block, 0, s, a, tx, ty, tz); break;
    case 3: hipLaunchKernelGGL((conv3_tile_kernel<3, CC, kTZ>), grid, block, 0, s, a, tx, ty, tz); break;
    case 4: hipLaunchKernelGGL((conv3_tile_kernel<4, CC, kTZ>), grid, block, 0, s, a, tx, ty, tz); break;
    case 6: hipLaunchKernelGGL((conv3_tile_kernel<6, CC, kTZ>), grid, block, 0, s, a, tx, ty, tz); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int MT, int TY, int TZ>
static hipError_t launch_reg_mt(const ConvArgs& a, hipStream_t s) {
  const int tx = (a.n1 + 15) / 16, ty = (a.n2 + 2 * TY - 1) / (2 * TY),
            tz = (a.n3 + 2 * TZ - 1) / (2 * TZ);
  constexpr size_t lds = reg_lds_bytes<MT, TY, TZ>();
  static_assert(lds <= 65536, "register-blocked convolution: LDS block too large");
  hipLaunchKernelGGL((conv3_reg_kernel<MT, TY, TZ>), dim3((unsigned)(tx * ty * tz)), dim3(256),
                     lds, s, a, tx, ty, tz);
  return hipGetLastError();
}

template <int TY, int TZ>
static hipError_t launch_reg(const ConvArgs& a, hipStream_t s) {
  switch (a.cout / 16) {
    case 1: return launch_reg_mt<1, TY, TZ>(a, s);
    case 2: return launch_reg_mt<2, TY, TZ>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_conv_fwd(const ConvArgs& a, hipStream_t s) {
  if (a.cin % 8 || a.cout % 16 || a.in_stride % 8 || a.in_off % 8 || a.out_stride % 4 ||
      a.out_off % 4 || a.kpad % 32 || a.kpad < 27 * a.cin)
    return hipErrorInvalidValue;
  const long long nvox = (long long)a.n1 * a.n2 * a.n3;
  if (nvox == 0) return hipSuccess;
  if (a.variant == 2 && a.cin == 16 && a.cout == 32 && nvox >= (1LL << 16)) {
    // register-blocked where it is measured faster: 16 -> 32 channels on
    // grids with enough blocks to fill the chip (48^3: 15 us against 18 us).
    // 16 -> 16 runs faster on the LDS-tiled form since its weights are staged
    // in LDS and its workgroups own 8 planes (96^3: 36 against 40 us), and
    // with 8 or 48 and more input channels the per-group copy latency of the
    // register-blocked form costs more than its LDS savings.
    return launch_reg<2, 2>(a, s);
  }
  // the tiled form addresses its staging slots by 32-bit byte offsets and
  // marks slots outside the grid with offset 2^31
  const bool off32 = 2 * (nvox * a.in_stride + a.in_off) < 0xffffffffLL &&
                     2 * nvox * a.in_stride < (1LL << 31) && 2LL * a.cout * a.kpad < (1LL << 31);
  if (a.variant >= 1 && off32) {
    // 16-channel chunks up to 64 output channels: their weights fit in LDS
    // beside the halo (one or two output groups per workgroup; 64 outputs on
    // small grids are split into one group per workgroup)
    if (a.cin % 32 == 0 && a.cout > 64) return launch_tile_cc<32>(a, s);
    if (a.cin % 16 == 0) return launch_tile_cc<16>(a, s);
    return launch_tile_cc<8>(a, s);
  }
  const int mt = a.cout / 16;
  const dim3 block(256);
#define PFU_CONV(MT, NT)                                                          \
  do {                                                                            \
    const long long waves = (nvox + 16 * (NT)-1) / (16 * (NT));                   \
    hipLaunchKernelGGL((conv3_fwd_kernel<MT, NT>), dim3(blocks_for(waves, 4)), block, 0, s, a); \
  } while (0)
  switch (mt) {
    case 1: PFU_CONV(1, 4); break;
    case 2: PFU_CONV(2, 4); break;
    case 3: PFU_CONV(3, 2); break;
    case 4: PFU_CONV(4, 2); break;
    case 6: PFU_CONV(6, 2); break;
    default: return hipErrorInvalidValue;
  }
#undef PFU_CONV
  return hipGetLastError();
}

// voxel ranges of the weight gradient (workgroups per tap and channel chunk,
// and partial copies to reduce): one per 2048 voxels, at most 256
int wgrad_blocks(long long nvox) {
  long long nb = nvox / 2048;
  if (nb < 1) nb = 1;
  if (nb > 256) nb = 256;
  return (int)nb;
}

hipError_t launch_conv_wgrad(const WgradArgs& a, int nblocks, float* dw, float* db,
                             hipStream_t s) {
  const int cin16 = (a.cin + 15) & ~15;
  if (a.cin % 8 || a.cout % 16 || (a.cout / 16) * (cin16 / 16) > kConvMaxTiles ||
      a.dy_stride % 8 || a.dy_off % 8 || a.x_stride % 8 || a.x_off % 8 || nblocks < 1 ||
      (long long)a.n1 * a.n2 * a.n3 >= (1LL << 31))
    return hipErrorInvalidValue;
  const size_t lds192 = (size_t)(a.cout + cin16) * wg_pitch(192) * sizeof(uint16_t);
  const int mt = a.cout / 16;
  if (mt <= 3 && wtap_lds_bytes(a.cout) <= 65536 && (long long)a.n1 * a.n2 * a.n3 > 0) {
    // nine taps share their staging (a third of the 27 for parallelism: at
    // most 27 output tiles per workgroup)
    const int T = 9;
    const long long nblk = (long long)((a.n1 + kWtBX - 1) / kWtBX) * ((a.n2 + kWtBY - 1) / kWtBY) *
                           ((a.n3 + kWtBZ - 1) / kWtBZ);
    const long long per = (nblk + nblocks - 1) / nblocks;
    const dim3 grid((unsigned)nblocks, (unsigned)(cin16 / 16), (unsigned)(27 / T));
    const size_t lds = wtap_lds_bytes(a.cout);
    switch (mt) {
      case 1: hipLaunchKernelGGL((conv3_wgrad_tap_kernel<5, 1>), grid, dim3(256), lds, s, a, T, per); break;
      case 2: hipLaunchKernelGGL((conv3_wgrad_tap_kernel<5, 2>), grid, dim3(256), lds, s, a, T, per); break;
      default: hipLaunchKernelGGL((conv3_wgrad_tap_kernel<5, 3>), grid, dim3(256), lds, s, a, T, per); break;
    }
  } else if (lds192 <= 65536) {
    hipLaunchKernelGGL(conv3_wgrad_kernel<192>, dim3(nblocks, 27), dim3(256), lds192, s, a);
  } else {
    const size_t lds = (size_t)(a.cout + cin16) * wg_pitch(64) * sizeof(uint16_t);
    hipLaunchKernelGGL(conv3_wgrad_kernel<64>, dim3(nblocks, 27), dim3(256), lds, s, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long len = 27LL * a.cout * a.cin;
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(blocks_for(len, 256)), dim3(256), 0, s, a.part,
                     nblocks, len, dw);
  e = hipGetLastError();
  if (e != hipSuccess || !db) return e;
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(blocks_for(a.cout, 256)), dim3(256), 0, s,
                     a.part_bias, nblocks, (long long)a.cout, db);
  return hipGetLastError();
}

hipError_t launch_relu_bwd(uint16_t* dy, int dys, int dyo, const uint16_t* y, int ys, int yo,
                           int c, long long nvox, hipStream_t s) {
  if (nvox * c == 0) return hipSuccess;
  hipLaunchKernelGGL(relu_bwd_kernel, dim3(blocks_for(nvox * c, 256)), dim3(256), 0, s, dy, dys,
                     dyo, y, ys, yo, c, nvox);
  return hipGetLastError();
}

hipError_t launch_pool_fwd(const View& in, const View& out, int c, int m1, int m2, int m3,
                           hipStream_t s) {
  const long long n = (long long)m1 * m2 * m3 * c;
  if (n == 0) return hipSuccess;
  if (c % 8 == 0 && in.stride % 8 == 0 && in.off % 8 == 0 && out.stride % 8 == 0 &&
      out.off % 8 == 0 && n < (1LL << 32)) {
    const unsigned total = (unsigned)(n / 8);
    hipLaunchKernelGGL(pool_fwd8_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, in.p,
                       in.stride, in.off, out.p, out.stride, out.off, c / 8, m1, m2, total);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(pool_fwd_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, in.p, in.stride,
                     in.off, out.p, out.stride, out.off, c, m1, m2, m3);
  return hipGetLastError();
}

hipError_t launch_pool_bwd(const View& dout, const View& din, int c, int n1, int n2, int n3,
                           int accumulate, hipStream_t s) {
  const long long n = (long long)n1 * n2 * n3 * c;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(pool_bwd_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, dout.p,
                     dout.stride, dout.off, din.p, din.stride, din.off, c, n1, n2, n3, accumulate);
  return hipGetLastError();
}

hipError_t launch_up_cat(const View& up, const View& skip, const View& out, int cu, int cs,
                         int n1, int n2, int n3, hipStream_t s) {
  const long long nv = (long long)n1 * n2 * n3;
  if (nv == 0) return hipSuccess;
  const long long total = nv * ((cu + cs) / 8);
  if (cu % 8 || cs % 8 || up.off || skip.off || out.off || up.stride % 8 ||
      skip.stride % 8 || out.stride != cu + cs || n1 % 2 || n2 % 2 || n3 % 2 ||
      total >= (1LL << 32))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(up_cat8_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, up.p,
                     up.stride, skip.p, skip.stride, out.p, cu / 8, cs / 8, n1, n2,
                     (unsigned)total);
  return hipGetLastError();
}

hipError_t launch_up_fwd(const View& in, const View& out, int c, int n1, int n2, int n3,
                         hipStream_t s) {
  const long long n = (long long)n1 * n2 * n3 * c;
  if (n == 0) return hipSuccess;
  if (c % 8 == 0 && in.stride % 8 == 0 && in.off % 8 == 0 && out.stride % 8 == 0 &&
      out.off % 8 == 0 && n < (1LL << 32)) {
    const unsigned total = (unsigned)(n / 8);
    hipLaunchKernelGGL(up_fwd8_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, s, in.p,
                       in.stride, in.off, out.p, out.stride, out.off, c / 8, n1, n2, total);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(up_fwd_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, in.p, in.stride,
                     in.off, out.p, out.stride, out.off, c, n1, n2, n3);
  return hipGetLastError();
}

hipError_t launch_up_bwd(const View& dout, const View& din, int c, int m1, int m2, int m3,
                         hipStream_t s) {
  const long long n = (long long)m1 * m2 * m3 * c;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(up_bwd_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, dout.p,
                     dout.stride, dout.off, din.p, din.stride, din.off, c, m1, m2, m3);
  return hipGetLastError();
}

hipError_t launch_input(const uint8_t* glass, int from_code, float f1, float f2, uint16_t* out,
                        long long nvox, hipStream_t s) {
  if (nvox == 0) return hipSuccess;
  hipLaunchKernelGGL(input_kernel, dim3(blocks_for(nvox, 256)), dim3(256), 0, s, glass, from_code,
                     f1, f2, out, nvox);
  return hipGetLastError();
}

hipError_t launch_count_water(const uint8_t* glass, int from_code, long long nvox, float* part,
                              float* count, hipStream_t s) {
  const int nb = (int)blocks_for(nvox, 256);
  hipLaunchKernelGGL(count_water_kernel, dim3(nb), dim3(256), 0, s, glass, from_code, nvox, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce(part, nb, 1, count, s);
}

int head_blocks(long long nvox) { return (int)blocks_for(nvox, 256); }

hipError_t launch_head(const HeadArgs& a, hipStream_t s) {
  if (a.h_stride % 8 || a.h_off % 8) return hipErrorInvalidValue;
  if (a.nvox == 0) return hipSuccess;
  hipLaunchKernelGGL(head_kernel, dim3(head_blocks(a.nvox)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_weights(const float* wm, int cout, int cin, int kpad, int kpad_t, uint16_t* wf,
                          uint16_t* wd, hipStream_t s) {
  const long long n = (long long)cout * kpad + (wd ? (long long)cin * kpad_t : 0);
  hipLaunchKernelGGL(weights_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, wm, cout, cin, kpad,
                     kpad_t, wf, wd);
  return hipGetLastError();
}

hipError_t launch_reduce(const float* part, int nparts, long long len, float* out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(blocks_for(len, 256)), dim3(256), 0, s, part, nparts,
                     len, out);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, long long n, float lr,
                       float b1, float b2, float eps, float bc1, float bc2, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, g, m, v, n, lr, b1,
                     b2, eps, bc1, bc2);
  return hipGetLastError();
}

hipError_t launch_f32_to_bf16(const float* in, uint16_t* out, long long n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(f32_to_bf16_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_bf16_to_f32(const uint16_t* in, float* out, long long n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(bf16_to_f32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_flood(const uint8_t* reach, void* out, int fp64, long long n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(flood_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, reach, out, fp64, n);
  return hipGetLastError();
}

hipError_t launch_reach(const uint8_t* code, const void* phi, int fp64, int* lab, uint8_t* reach,
                        int n1, int n2, int n3, hipStream_t s) {
  const long long n = (long long)n1 * n2 * n3;
  if (n == 0) return hipSuccess;
  if (n >= (1LL << 31)) return hipErrorInvalidValue;  // cell indices are int
  const dim3 grid(blocks_for(n, 256)), block(256);
  const int tx = (n1 + kUT - 1) / kUT, ty = (n2 + kUT - 1) / kUT, tz = (n3 + kUT - 1) / kUT;
  hipLaunchKernelGGL(reach_local_kernel, dim3((unsigned)(tx * ty * tz)), dim3(1024), 0, s, code,
                     lab, reach, n1, n2, n3, tx, ty);
  hipLaunchKernelGGL(reach_merge_kernel, grid, block, 0, s, code, lab, n1, n2, n);
  hipLaunchKernelGGL(reach_seed_kernel, grid, block, 0, s, code, phi, fp64, lab, reach, n);
  hipLaunchKernelGGL(reach_resolve_kernel, grid, block, 0, s, code, lab, reach, n);
  return hipGetLastError();
}

hipError_t launch_mfma_probe(const float* A, const float* B, float* C, hipStream_t s) {
  hipLaunchKernelGGL(mfma_layout_probe, dim3(1), dim3(64), 0, s, A, B, C);
  return hipGetLastError();
}

}  // namespace pfu

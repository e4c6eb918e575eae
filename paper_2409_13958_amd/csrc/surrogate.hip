// Kernels and host object of the learned surrogate of the AIM grid
// convolution (layout and conventions in surrogate.h).
#include "surrogate.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace pmfem {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kT = 256;
constexpr int kRedBlocks = 1024;   // blocks of the device reductions (partials in dred)
constexpr int kSgWS = 48;          // LDS point stride (floats) of the weight-gradient kernel
constexpr size_t kSgWgradLds = (size_t)(kSgTX * kSgTY + kSgHalo) * kSgWS * sizeof(float);

// FP32 -> BF16, round to nearest even (finite inputs)
__device__ __forceinline__ uint32_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float bf16_float(uint32_t h) { return __uint_as_float(h << 16); }

inline uint16_t bf16_bits_host(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ int wrapi(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

__device__ __forceinline__ int64_t vox_of(const SgGrid& g, int z, int y, int x) {
  return ((int64_t)z * g.ny + y) * g.nx + x;
}

// ---------------------------------------------------------------------------
// First-layer form (one input channel -> kSgC outputs), FP32 FMA. Also the
// data gradient of the last layer (weights flipped). Tile: 8 rows of 32
// points of one z-plane per 256-thread workgroup; the 3 input planes of the
// tile with a one-point halo staged in LDS.
__global__ __launch_bounds__(kT) void k_sg_in(SgGrid g, const float* __restrict__ x, float xs,
                                               const float* __restrict__ w,
                                               const float* __restrict__ b,
                                               float* __restrict__ out, int relu,
                                               const float* __restrict__ mask) {
  __shared__ float sx[3 * kSgHalo];
  __shared__ __align__(16) float sw[kSgC * 27];
  const int tiles_x = (g.nx + kSgTX - 1) / kSgTX;
  const int x0 = (int)(blockIdx.x % tiles_x) * kSgTX, y0 = (int)(blockIdx.x / tiles_x) * kSgTY;
  const int z = blockIdx.y, t = threadIdx.x;
  for (int i = t; i < kSgC * 27; i += kT) sw[(i % 27) * kSgC + i / 27] = w[i];  // [o][co]
  for (int i = t; i < 3 * kSgHalo; i += kT) {
    const int pl = i / kSgHalo, h = i - pl * kSgHalo;
    const int hy = h / kSgHX, hx = h - hy * kSgHX, gz = z + pl - 1;
    float v = 0.f;
    if (gz >= 0 && gz < g.nz)
      v = x[vox_of(g, gz, wrapi(y0 + hy - 1, g.ny), wrapi(x0 + hx - 1, g.nx))] * xs;
    sx[i] = v;
  }
  __syncthreads();
  const int ty = t / kSgTX, tx = t % kSgTX;
  float acc[kSgC];
#pragma unroll
  for (int co = 0; co < kSgC; ++co) acc[co] = b ? b[co] : 0.f;
  for (int dz = 0; dz < 3; ++dz)
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const float v = sx[dz * kSgHalo + (ty + dy) * kSgHX + tx + dx];
        const float4* w4 = reinterpret_cast<const float4*>(&sw[(dz * 9 + dy * 3 + dx) * kSgC]);
#pragma unroll
        for (int q = 0; q < kSgC / 4; ++q) {
          const float4 ww = w4[q];
          acc[4 * q] = fmaf(ww.x, v, acc[4 * q]);
          acc[4 * q + 1] = fmaf(ww.y, v, acc[4 * q + 1]);
          acc[4 * q + 2] = fmaf(ww.z, v, acc[4 * q + 2]);
          acc[4 * q + 3] = fmaf(ww.w, v, acc[4 * q + 3]);
        }
      }
  const int gx = x0 + tx, gy = y0 + ty;
  if (gx >= g.nx || gy >= g.ny) return;
  const int64_t v = vox_of(g, z, gy, gx);
  float4* o4 = reinterpret_cast<float4*>(out + v * kSgC);
  const float4* m4 = mask ? reinterpret_cast<const float4*>(mask + v * kSgC) : nullptr;
#pragma unroll
  for (int q = 0; q < kSgC / 4; ++q) {
    float4 r = make_float4(acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]);
    if (m4) {
      const float4 mk = m4[q];
      r.x = mk.x > 0.f ? r.x : 0.f;
      r.y = mk.y > 0.f ? r.y : 0.f;
      r.z = mk.z > 0.f ? r.z : 0.f;
      r.w = mk.w > 0.f ? r.w : 0.f;
    }
    if (relu) {
      r.x = fmaxf(r.x, 0.f);
      r.y = fmaxf(r.y, 0.f);
      r.z = fmaxf(r.z, 0.f);
      r.w = fmaxf(r.w, 0.f);
    }
    o4[q] = r;
  }
}

// Last-layer form (kSgC inputs -> one output), FP32 FMA: y = (conv + b) ys.
// The input planes are staged one at a time with a padded point stride (36
// floats: 16-byte aligned, and 16 consecutive points of a 16-byte read fall
// in distinct banks); weights as [offset][channel], both read as float4.
__global__ __launch_bounds__(kT) void k_sg_out(SgGrid g, const float* __restrict__ a,
                                                const float* __restrict__ w,
                                                const float* __restrict__ b, float ys,
                                                float* __restrict__ y) {
  constexpr int S = kSgC + 4;
  __shared__ __align__(16) float sa[kSgHalo * S];
  __shared__ __align__(16) float sw[kSgC * 27];
  const int tiles_x = (g.nx + kSgTX - 1) / kSgTX;
  const int x0 = (int)(blockIdx.x % tiles_x) * kSgTX, y0 = (int)(blockIdx.x / tiles_x) * kSgTY;
  const int z = blockIdx.y, t = threadIdx.x;
  const int ty = t / kSgTX, tx = t % kSgTX;
  for (int i = t; i < kSgC * 27; i += kT) sw[(i % 27) * kSgC + i / 27] = w[i];  // [o][ci]
  float acc = 0.f;
  for (int dz = 0; dz < 3; ++dz) {
    const int gz = z + dz - 1;
    if (gz < 0 || gz >= g.nz) continue;  // the same for the whole workgroup
    __syncthreads();
    for (int i = t; i < kSgHalo * (kSgC / 4); i += kT) {
      const int h = i / (kSgC / 4), q = i % (kSgC / 4);
      const int hy = h / kSgHX, hx = h - hy * kSgHX;
      const float4 v = reinterpret_cast<const float4*>(
          a + vox_of(g, gz, wrapi(y0 + hy - 1, g.ny), wrapi(x0 + hx - 1, g.nx)) * kSgC)[q];
      reinterpret_cast<float4*>(&sa[h * S])[q] = v;
    }
    __syncthreads();
    for (int dy = 0; dy < 3; ++dy)
      for (int dx = 0; dx < 3; ++dx) {
        const float4* s4 = reinterpret_cast<const float4*>(&sa[((ty + dy) * kSgHX + tx + dx) * S]);
        const float4* w4 = reinterpret_cast<const float4*>(&sw[(dz * 9 + dy * 3 + dx) * kSgC]);
#pragma unroll
        for (int q = 0; q < kSgC / 4; ++q) {
          const float4 av = s4[q], ww = w4[q];
          acc = fmaf(ww.x, av.x, acc);
          acc = fmaf(ww.y, av.y, acc);
          acc = fmaf(ww.z, av.z, acc);
          acc = fmaf(ww.w, av.w, acc);
        }
      }
  }
  const int gx = x0 + tx, gy = y0 + ty;
  if (gx >= g.nx || gy >= g.ny) return;
  y[vox_of(g, z, gy, gx)] = (acc + b[0]) * ys;
}

// Middle layer (kSgC -> kSgC) on the matrix cores, as an implicit GEMM: M =
// grid points, N = output channels, K = 27 offsets x kSgC input channels,
// with v_mfma_f32_16x16x32_bf16 (A: 16 points x 32 channels of one offset;
// B: 32 input x 16 output channels). A workgroup computes 8 rows x 32 points
// of two consecutive z-planes; each of its four waves owns two rows (four
// 16-point M tiles) times both 16-channel N tiles of both planes, sixteen
// independent accumulators. The input planes z0-1 .. z0+2 are staged in LDS
// one at a time as BF16 (and, with SPLIT, the BF16 remainder x - bf16(x),
// which a second product adds), 16-byte channel chunks XOR-swizzled by point
// so that 16 consecutive points of one chunk fall in distinct banks; every A
// fragment read from LDS serves both output planes, and the next plane's
// loads are in flight (in registers) while the current one is multiplied.
// Also the data gradient (weights transposed and flipped, no bias) with the
// ReLU mask of the layer below.
template <bool SPLIT>
__global__ __launch_bounds__(kT, 2) void k_sg_mid(SgGrid g, const float* __restrict__ a,
                                                   const uint16_t* __restrict__ w,
                                                   const float* __restrict__ b,
                                                   float* __restrict__ out, int relu,
                                                   const float* __restrict__ mask) {
  constexpr int kLoads = (kSgHalo * (kSgC / 4) + kT - 1) / kT;  // float4 per thread per plane
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  __shared__ uint4 shi[kSgHalo * 4];
  __shared__ uint4 slo[SPLIT ? kSgHalo * 4 : 1];
  const int tiles_x = (g.nx + kSgTX - 1) / kSgTX;
  const int x0 = (int)(blockIdx.x % tiles_x) * kSgTX, y0 = (int)(blockIdx.x / tiles_x) * kSgTY;
  const int z0 = 2 * (int)blockIdx.y, nout = min(2, g.nz - z0);
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6, li = lane & 15, kg = lane >> 4;
  // input planes of the two outputs inside the grid
  const int p_lo = max(0, z0 - 1), p_hi = min(g.nz - 1, z0 + nout);
  float4 pre[kLoads];
  auto load_plane = [&](int gz) {
#pragma unroll
    for (int k = 0; k < kLoads; ++k) {
      const int i = t + k * kT;
      if (i < kSgHalo * (kSgC / 4)) {
        const int h = i >> 3, q = i & 7, hy = h / kSgHX, hx = h - hy * kSgHX;
        pre[k] = reinterpret_cast<const float4*>(
            a + vox_of(g, gz, wrapi(y0 + hy - 1, g.ny), wrapi(x0 + hx - 1, g.nx)) * kSgC)[q];
      }
    }
  };
  auto store_plane = [&]() {
#pragma unroll
    for (int k = 0; k < kLoads; ++k) {
      const int i = t + k * kT;
      if (i < kSgHalo * (kSgC / 4)) {
        const int h = i >> 3, q = i & 7, chunk = (q >> 1) ^ ((h >> 2) & 3);
        const float4 v = pre[k];
        const bf16x4 hv = {(__bf16)v.x, (__bf16)v.y, (__bf16)v.z, (__bf16)v.w};
        reinterpret_cast<bf16x4*>(&shi[h * 4 + chunk])[q & 1] = hv;
        if (SPLIT) {
          const bf16x4 lv = {(__bf16)(v.x - (float)hv[0]), (__bf16)(v.y - (float)hv[1]),
                             (__bf16)(v.z - (float)hv[2]), (__bf16)(v.w - (float)hv[3])};
          reinterpret_cast<bf16x4*>(&slo[h * 4 + chunk])[q & 1] = lv;
        }
      }
    }
  };
  f32x4 acc[2][4][2];
#pragma unroll
  for (int zo = 0; zo < 2; ++zo)
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) acc[zo][mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  load_plane(p_lo);
  for (int p = p_lo; p <= p_hi; ++p) {
    __syncthreads();  // the previous plane has been multiplied
    store_plane();
    __syncthreads();
    if (p < p_hi) load_plane(p + 1);  // the next plane, in flight meanwhile
    // offset dz of this plane for output z0 + zo (valid if 0..2)
    const int dz0 = p - z0 + 1, dz1 = p - z0;
    const bool on0 = dz0 <= 2, on1 = nout > 1 && dz1 >= 0;
#pragma unroll 3
    for (int j = 0; j < 9; ++j) {
      const int dy = j / 3, dx = j % 3;
      bf16x8 ah[4], al[4];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        const int h = (2 * wv + (mt >> 1) + dy) * kSgHX + (mt & 1) * 16 + li + dx;
        const int chunk = kg ^ ((h >> 2) & 3);
        ah[mt] = *reinterpret_cast<const bf16x8*>(&shi[h * 4 + chunk]);
        if (SPLIT) al[mt] = *reinterpret_cast<const bf16x8*>(&slo[h * 4 + chunk]);
      }
#pragma unroll
      for (int zo = 0; zo < 2; ++zo) {
        if (!(zo == 0 ? on0 : on1)) continue;
        // B fragments of offset (dz, j): output channels li and 16 + li, inputs 8 kg ..
        const bf16x8* wz = reinterpret_cast<const bf16x8*>(
            w + ((int64_t)((zo == 0 ? dz0 : dz1) * 9 + j) * kSgC + li) * kSgC + kg * 8);
        const bf16x8 bw0 = wz[0], bw1 = wz[16 * (kSgC / 8)];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          acc[zo][mt][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mt], bw0, acc[zo][mt][0], 0, 0, 0);
          acc[zo][mt][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[mt], bw1, acc[zo][mt][1], 0, 0, 0);
        }
        if (SPLIT) {
#pragma unroll
          for (int mt = 0; mt < 4; ++mt) {
            acc[zo][mt][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[mt], bw0, acc[zo][mt][0], 0, 0, 0);
            acc[zo][mt][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[mt], bw1, acc[zo][mt][1], 0, 0, 0);
          }
        }
      }
    }
  }
  // D tile of 16 points x 16 channels: lane holds points 4 kg + r, channel li
#pragma unroll
  for (int zo = 0; zo < 2; ++zo) {
    if (zo >= nout) continue;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const int gy = y0 + 2 * wv + (mt >> 1);
      if (gy >= g.ny) continue;
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        const int co = nt * 16 + li;
        const float bias = b ? b[co] : 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gx = x0 + (mt & 1) * 16 + kg * 4 + r;
          if (gx >= g.nx) continue;
          const int64_t v = vox_of(g, z0 + zo, gy, gx);
          float val = acc[zo][mt][nt][r] + bias;
          if (mask && !(mask[v * kSgC + co] > 0.f)) val = 0.f;
          if (relu) val = fmaxf(val, 0.f);
          out[v * kSgC + co] = val;
        }
      }
    }
  }
}

// Weight gradient of a kSgC -> kSgC layer: gW[co][ci][o] = sum over points v
// of gr[v][co] a[v + o][ci] (circular in x, y; zero outside in z), on the
// matrix cores with FP32 operands (v_mfma_f32_16x16x4f32: M = 16 output
// channels, N = 16 input channels, K = 4 points, FP32 products and sums).
// Grid (P, 3): blockIdx.y is dz; each 512-thread workgroup walks the tiles
// blockIdx.x, +P, ...; wave w owns the 16 x 16 channel block (w & 3) for the
// nine (dy, dx) of its dz (nine independent accumulators) and every other
// group of four points (w >> 2). The tile's output gradient and the input
// plane are staged in LDS at a point stride of kSgWS floats, so that four
// consecutive points of one 16-channel block fall in distinct banks. Partial
// sums per workgroup and half go to part[2 P][C*C*27]. The next tile's loads
// are in flight (in registers) while the current one is multiplied.
__global__ __launch_bounds__(512) void k_sg_wgrad(SgGrid g, const float* __restrict__ gr,
                                                   const float* __restrict__ a,
                                                   float* __restrict__ part) {
  extern __shared__ float4 wsm4[];
  float* sg = reinterpret_cast<float*>(wsm4);        // [kSgTX * kSgTY][kSgWS]
  float* sa = sg + kSgTX * kSgTY * kSgWS;             // [kSgHalo][kSgWS]
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6, li = lane & 15, kq = lane >> 4;
  const int mt = (wv >> 1) & 1, nt = wv & 1, half = wv >> 2, dz = blockIdx.y;
  const int tiles_x = (g.nx + kSgTX - 1) / kSgTX, tiles_y = (g.ny + kSgTY - 1) / kSgTY;
  const int tpp = tiles_x * tiles_y, ntiles = tpp * g.nz;
  constexpr int kLg = kSgTX * kSgTY * 8 / 512;            // float4 of the tile per thread
  constexpr int kLa = (kSgHalo * 8 + 511) / 512;           // float4 of the plane per thread
  static_assert(kLg * 512 == kSgTX * kSgTY * 8, "tile float4 count");
  // the workgroup's tiles whose plane z + dz - 1 lies inside the grid
  auto next_tile = [&](int tl) {
    while (tl < ntiles && (tl / tpp + dz - 1 < 0 || tl / tpp + dz - 1 >= g.nz)) tl += gridDim.x;
    return tl;
  };
  float4 pg[kLg], pa[kLa];
  auto load_tile = [&](int tl) {
    const int z = tl / tpp, r = tl - z * tpp;
    const int x0 = (r % tiles_x) * kSgTX, y0 = (r / tiles_x) * kSgTY, gz = z + dz - 1;
#pragma unroll
    for (int k = 0; k < kLg; ++k) {
      const int i = t + k * 512, v = i >> 3, q = i & 7;
      const int gx = x0 + (v & (kSgTX - 1)), gy = y0 + v / kSgTX;
      pg[k] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (gx < g.nx && gy < g.ny) pg[k] = reinterpret_cast<const float4*>(gr + vox_of(g, z, gy, gx) * kSgC)[q];
    }
#pragma unroll
    for (int k = 0; k < kLa; ++k) {
      const int i = t + k * 512;
      pa[k] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (i < kSgHalo * 8) {
        const int h = i >> 3, q = i & 7, hy = h / kSgHX, hx = h - hy * kSgHX;
        pa[k] = reinterpret_cast<const float4*>(
            a + vox_of(g, gz, wrapi(y0 + hy - 1, g.ny), wrapi(x0 + hx - 1, g.nx)) * kSgC)[q];
      }
    }
  };
  f32x4 acc[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  int tile = next_tile(blockIdx.x);  // the same for the whole workgroup
  if (tile < ntiles) load_tile(tile);
  while (tile < ntiles) {
    __syncthreads();  // the previous tile has been used
#pragma unroll
    for (int k = 0; k < kLg; ++k) {
      const int i = t + k * 512;
      reinterpret_cast<float4*>(sg + (i >> 3) * kSgWS)[i & 7] = pg[k];
    }
#pragma unroll
    for (int k = 0; k < kLa; ++k) {
      const int i = t + k * 512;
      if (i < kSgHalo * 8) reinterpret_cast<float4*>(sa + (i >> 3) * kSgWS)[i & 7] = pa[k];
    }
    __syncthreads();
    const int nxt = next_tile(tile + gridDim.x);
    if (nxt < ntiles) load_tile(nxt);  // in flight while this tile is multiplied
    tile = nxt;
    for (int st = half; st < kSgTX * kSgTY / 4; st += 2) {
      const int v = 4 * st + kq, ty = v / kSgTX, tx = v % kSgTX;
      const float ga = sg[v * kSgWS + mt * 16 + li];     // A: output channel x point
      const float* sb = sa + (ty * kSgHX + tx) * kSgWS + nt * 16 + li;
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        const float bb = sb[((j / 3) * kSgHX + j % 3) * kSgWS];  // B: point x input channel
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ga, bb, acc[j], 0, 0, 0);
      }
    }
  }
  // D block: lane holds output channels 16 mt + 4 kq + r, input channel 16 nt + li;
  // partial sums as [offset][co][ci], so that 16 lanes store 64 contiguous bytes
  float* P = part + ((int64_t)blockIdx.x * 2 + half) * (kSgC * kSgC * 27);
#pragma unroll
  for (int j = 0; j < 9; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      P[((dz * 9 + j) * kSgC + mt * 16 + 4 * kq + r) * kSgC + nt * 16 + li] = acc[j][r];
}

// Sum of the weight-gradient partial sums part[P][27][C][C] into a layer's
// W[co][ci][27] (ci < Ci, co < Co). A workgroup takes 64 consecutive partial
// entries (contiguous loads) and four quarters of the P sums; the quarters
// are added in a fixed order (FP64 throughout).
__global__ __launch_bounds__(256) void k_sg_reduce_w(int P, const float* __restrict__ part, int Ci,
                                                      int Co, float* __restrict__ dst) {
  __shared__ double red[4][64];
  const int el = threadIdx.x & 63, qt = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + el;
  const int o = e / (kSgC * kSgC), co = (e / kSgC) % kSgC, ci = e % kSgC;
  const bool used = e < 27 * kSgC * kSgC && co < Co && ci < Ci;
  double sum = 0.0;
  if (used) {
#pragma unroll 8
    for (int p = qt; p < P; p += 4) sum += part[(int64_t)p * (27 * kSgC * kSgC) + e];
  }
  red[qt][el] = sum;
  __syncthreads();
  if (qt == 0 && used)
    dst[(co * Ci + ci) * 27 + o] = (float)(((red[0][el] + red[1][el]) + red[2][el]) + red[3][el]);
}

// Column sums of g[V][C] (C divides 256): partial per workgroup -> part[P][C].
__global__ __launch_bounds__(kT) void k_sg_colsum(int64_t V, int C, const float* __restrict__ g,
                                                   float* __restrict__ part) {
  __shared__ float red[kT];
  const int t = threadIdx.x, c = t % C, grp = t / C, ng = kT / C;
  float acc = 0.f;
  for (int64_t v = (int64_t)blockIdx.x * ng + grp; v < V; v += (int64_t)gridDim.x * ng)
    acc += g[v * C + c];
  red[t] = acc;
  __syncthreads();
  if (t < C) {
    float s = 0.f;
    for (int k = 0; k < ng; ++k) s += red[k * C + t];
    part[(int64_t)blockIdx.x * C + t] = s;
  }
}

// dst[i] = sum_p part[p * n + src(i)], src(i) = (i / run) * stride + i % run:
// one workgroup per output, the P partial sums split over its threads and
// added by a fixed-order tree (FP64)
__global__ __launch_bounds__(256) void k_sg_reduce(int P, int64_t n, const float* __restrict__ part,
                                                    int64_t count, int run, int64_t stride,
                                                    float* __restrict__ dst) {
  __shared__ double red[256];
  const int64_t i = blockIdx.x;
  if (i >= count) return;  // the same for the whole workgroup
  const int64_t src = (i / run) * stride + i % run;
  double sum = 0.0;
  for (int p = threadIdx.x; p < P; p += blockDim.x) sum += part[(int64_t)p * n + src];
  red[threadIdx.x] = sum;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) dst[i] = (float)red[0];
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  return red[0];
}

// Mean-squared loss against t tscale: gy = dL/dy = 2 (y - t tscale) / V
// (also into channel 0 of gpad), per-workgroup sums of squares to part.
__global__ __launch_bounds__(kT) void k_sg_loss(int64_t V, const float* __restrict__ y,
                                                 const float* __restrict__ tg, float tscale,
                                                 float* __restrict__ gy, float* __restrict__ gpad,
                                                 double* __restrict__ part) {
  __shared__ double red[kT];
  double s = 0.0;
  const float k = 2.f / (float)V;
  for (int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x; v < V; v += (int64_t)gridDim.x * kT) {
    const float d = y[v] - tg[v] * tscale;
    s += (double)d * d;
    gy[v] = k * d;
    gpad[v * kSgC] = k * d;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kT) void k_sg_sumd(int P, const double* __restrict__ part,
                                                 double scale, double* __restrict__ out) {
  __shared__ double red[kT];
  double s = 0.0;
  for (int p = threadIdx.x; p < P; p += kT) s += part[p];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *out = s * scale;
}

// per-workgroup sums of |a - b|^2 (b may be null: |a|^2) and |b|^2
__global__ __launch_bounds__(kT) void k_sg_sq2(int64_t n, const float* __restrict__ a,
                                                const float* __restrict__ b,
                                                double* __restrict__ part) {
  __shared__ double red[kT];
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    const double bv = b ? (double)b[i] : 0.0, d = (double)a[i] - bv;
    s0 += d * d;
    s1 += bv * bv;
  }
  s0 = block_sum(s0, red);
  __syncthreads();
  s1 = block_sum(s1, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s0;
    part[2 * blockIdx.x + 1] = s1;
  }
}

__global__ void k_sg_pad(int64_t V, const float* __restrict__ x, float xs, float* __restrict__ dst) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < V) dst[v * kSgC] = x[v] * xs;
}

__global__ void k_sg_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g,
                          float* __restrict__ m1, float* __restrict__ m2, float lr_t, float b1,
                          float b2, float eps) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi, v = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = v;
  p[i] -= lr_t * a / (sqrtf(v) + eps);
}

// middle-layer weights W[co][ci][27] -> forward [27][co][ci] and, for the
// data gradient, [27][ci][co] with the offset reversed; both BF16
__global__ void k_sg_pack_mid(const float* __restrict__ W, uint16_t* __restrict__ wf,
                              uint16_t* __restrict__ wt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 27 * kSgC * kSgC) return;
  const int o = i / (kSgC * kSgC), r = i % (kSgC * kSgC), u = r / kSgC, v = r % kSgC;
  wf[i] = (uint16_t)bf16_bits(W[(u * kSgC + v) * 27 + o]);
  wt[i] = (uint16_t)bf16_bits(W[(v * kSgC + u) * 27 + 26 - o]);
}

// first/last-layer weights [C][27] -> BF16 values (and reversed offsets)
__global__ void k_sg_pack_io(const float* __restrict__ W, float* __restrict__ w,
                             float* __restrict__ wflip) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kSgC * 27) return;
  const int c = i / 27, o = i % 27;
  w[i] = bf16_float(bf16_bits(W[i]));
  if (wflip) wflip[i] = bf16_float(bf16_bits(W[c * 27 + 26 - o]));
}

// SplitMix64 finaliser (Steele, Lea and Flood, 2014) as a counter-based hash
__device__ __host__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_sg_texture(int64_t n, const double* __restrict__ pos, SgTexture tx,
                             double* __restrict__ m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = pos[3 * i], y = pos[3 * i + 1];
  double mx, my, mz;
  if (tx.kind == 0) {
    const uint64_t h1 = mix64(((uint64_t)tx.seed << 32) ^ (uint64_t)(2 * i));
    const uint64_t h2 = mix64(((uint64_t)tx.seed << 32) ^ (uint64_t)(2 * i + 1));
    const double u1 = (double)(h1 >> 11) * 0x1p-53, u2 = (double)(h2 >> 11) * 0x1p-53;
    mz = 2.0 * u1 - 1.0;
    const double r = sqrt(fmax(0.0, 1.0 - mz * mz)), ph = 2.0 * 3.14159265358979323846 * u2;
    mx = r * cos(ph);
    my = r * sin(ph);
  } else if (tx.kind == 1) {
    double dx = x - tx.cx, dy = y - tx.cy;
    dx -= tx.Lx * rint(dx / tx.Lx);
    dy -= tx.Ly * rint(dy / tx.Ly);
    const double r = sqrt(dx * dx + dy * dy);
    mz = tx.pol * exp(-(r * r) / (tx.rc * tx.rc));
    const double ip = sqrt(fmax(0.0, 1.0 - mz * mz));
    if (r > 0.0) {
      mx = -tx.chir * dy / r * ip;
      my = tx.chir * dx / r * ip;
    } else {
      mx = my = 0.0;
      mz = tx.pol;
    }
  } else {
    const double L = tx.nx != 0.0 ? tx.Lx : tx.Ly;
    const double u = x * tx.nx + y * tx.ny - tx.cx;
    const double d1 = u - L * rint(u / L), d2 = (u - 0.5 * L) - L * rint((u - 0.5 * L) / L);
    const double th = fabs(d1) < fabs(d2) ? 2.0 * atan(exp(d1 / tx.rc)) : 2.0 * atan(exp(-d2 / tx.rc));
    const double c = cos(th), s = sin(th);
    mx = c * tx.ed[0] + s * tx.er[0];
    my = c * tx.ed[1] + s * tx.er[1];
    mz = c * tx.ed[2] + s * tx.er[2];
  }
  const double nrm = 1.0 / sqrt(mx * mx + my * my + mz * mz);
  m[3 * i] = mx * nrm;
  m[3 * i + 1] = my * nrm;
  m[3 * i + 2] = mz * nrm;
}

__global__ void k_sg_f32(int64_t n3, const double* __restrict__ a, float* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n3) b[i] = (float)a[i];
}

unsigned blocks(int64_t n, int t = kT) { return (unsigned)((n + t - 1) / t); }

dim3 tile_grid(const SgGrid& g) {
  return dim3((unsigned)(((g.nx + kSgTX - 1) / kSgTX) * ((g.ny + kSgTY - 1) / kSgTY)),
              (unsigned)g.nz);
}

template <class T>
hipError_t alloc(T** p, int64_t count) {
  return hipMalloc((void**)p, (size_t)count * sizeof(T));
}

void launch_mid(const Surrogate* s, hipStream_t st, const float* a, const uint16_t* w,
                const float* b, float* out, int relu, const float* mask) {
  const dim3 grid(tile_grid(s->gd).x, (unsigned)((s->gd.nz + 1) / 2));  // two planes per workgroup
  if (s->split)
    hipLaunchKernelGGL(k_sg_mid<true>, grid, dim3(kT), 0, st, s->gd, a, w, b, out, relu, mask);
  else
    hipLaunchKernelGGL(k_sg_mid<false>, grid, dim3(kT), 0, st, s->gd, a, w, b, out, relu, mask);
}

float* act_of(const Surrogate* s, int l, bool train) {
  return s->act + (int64_t)(train ? l : (l & 1)) * s->nvox * kSgC;
}

// forward pass; the output grid gets (net + b) * ys. ev (or null): events
// recorded before and after every layer, [2 * depth].
void forward(Surrogate* s, hipStream_t st, const float* Q, bool train, float* yout, float ys,
             hipEvent_t* ev = nullptr) {
  const int D = s->depth;
  const dim3 grid = tile_grid(s->gd);
  if (ev) (void)hipEventRecord(ev[0], st);
  hipLaunchKernelGGL(k_sg_in, grid, dim3(kT), 0, st, s->gd, Q, s->s_in, s->win, s->p + s->boff[0],
                     act_of(s, 0, train), 1, (const float*)nullptr);
  if (ev) (void)hipEventRecord(ev[1], st);
  for (int l = 1; l <= D - 2; ++l) {
    if (ev) (void)hipEventRecord(ev[2 * l], st);
    launch_mid(s, st, act_of(s, l - 1, train), s->wmid + (int64_t)(l - 1) * 27 * kSgC * kSgC,
               s->p + s->boff[l], act_of(s, l, train), 1, nullptr);
    if (ev) (void)hipEventRecord(ev[2 * l + 1], st);
  }
  if (ev) (void)hipEventRecord(ev[2 * (D - 1)], st);
  hipLaunchKernelGGL(k_sg_out, grid, dim3(kT), 0, st, s->gd, act_of(s, D - 2, train), s->wout,
                     s->p + s->boff[D - 1], ys, yout);
  if (ev) (void)hipEventRecord(ev[2 * D - 1], st);
}

// weight and bias gradients of a layer from its output gradient g [V][C]
// (channel 0 only for the last layer) and its input a [V][C]
void layer_grads(Surrogate* s, hipStream_t st, int l, const float* g, const float* a) {
  const SgGrid& gd = s->gd;
  const int ntiles = (int)tile_grid(gd).x * gd.nz;
  const int P = std::min(kSgWPart / 2, ntiles);  // two partial sums per workgroup
  const int64_t nW = (int64_t)kSgC * kSgC * 27;
  hipLaunchKernelGGL(k_sg_wgrad, dim3((unsigned)P, 3), dim3(512), kSgWgradLds, st, gd, g, a,
                     s->part);
  const int D = s->depth;
  const int ci = l == 0 ? 1 : kSgC, co = l == D - 1 ? 1 : kSgC;
  hipLaunchKernelGGL(k_sg_reduce_w, dim3((unsigned)((nW + 63) / 64)), dim3(kT), 0, st, 2 * P,
                     s->part, ci, co, s->grad + s->woff[l]);
  // bias: column sums of the output gradient
  float* bpart = s->part;  // reused after the reduction above (same stream)
  if (co == 1) {
    hipLaunchKernelGGL(k_sg_colsum, dim3(kRedBlocks), dim3(kT), 0, st, s->nvox, 1, s->gy, bpart);
  } else {
    hipLaunchKernelGGL(k_sg_colsum, dim3(kRedBlocks), dim3(kT), 0, st, s->nvox, kSgC, g, bpart);
  }
  hipLaunchKernelGGL(k_sg_reduce, dim3((unsigned)co), dim3(kT), 0, st, kRedBlocks, (int64_t)co, bpart,
                     (int64_t)co, co, (int64_t)0, s->grad + s->boff[l]);
}

}  // namespace

hipError_t sg_create(Surrogate* s, int depth, SgGrid gd, int64_t n, const double* pos_host,
                     bool split) {
  s->depth = depth;
  s->split = split;
  s->gd = gd;
  s->nvox = (int64_t)gd.nx * gd.ny * gd.nz;
  s->n = n;
  s->woff.assign(depth, 0);
  s->boff.assign(depth, 0);
  int64_t cur = 0;
  for (int l = 0; l < depth; ++l) {
    const int ci = l == 0 ? 1 : kSgC, co = l == depth - 1 ? 1 : kSgC;
    s->woff[l] = cur;
    cur += (int64_t)co * ci * 27;
    s->boff[l] = cur;
    cur += co;
  }
  s->nparam = cur;
  hipError_t e;
  const int nmid = std::max(0, depth - 2);
  if ((e = alloc(&s->p, cur)) || (e = alloc(&s->grad, cur)) || (e = alloc(&s->m1, cur)) ||
      (e = alloc(&s->m2, cur)))
    return e;
  if ((e = hipMemset(s->m1, 0, cur * 4)) || (e = hipMemset(s->m2, 0, cur * 4))) return e;
  if ((e = alloc(&s->wmid, std::max<int64_t>(1, (int64_t)nmid * 27 * kSgC * kSgC))) ||
      (e = alloc(&s->wmidt, std::max<int64_t>(1, (int64_t)nmid * 27 * kSgC * kSgC))) ||
      (e = alloc(&s->win, kSgC * 27)) || (e = alloc(&s->wout, kSgC * 27)) ||
      (e = alloc(&s->woutt, kSgC * 27)))
    return e;
  if ((e = hipFuncSetAttribute((const void*)k_sg_wgrad, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kSgWgradLds)))
    return e;
  if ((e = alloc(&s->act, 2 * s->nvox * kSgC))) return e;
  if ((e = alloc(&s->dred, 2 * kRedBlocks + 8))) return e;
  if ((e = alloc(&s->pos, 3 * n)) || (e = alloc(&s->m64, 3 * n)) || (e = alloc(&s->m32, 3 * n)) ||
      (e = alloc(&s->ha, 3 * n)) || (e = alloc(&s->hs, 3 * n)))
    return e;
  return hipMemcpy(s->pos, pos_host, (size_t)n * 3 * sizeof(double), hipMemcpyHostToDevice);
}

hipError_t sg_ensure_training(Surrogate* s, int n_loss) {
  hipError_t e;
  if (!s->trained_buffers) {
    (void)hipFree(s->act);
    s->act = nullptr;
    const int64_t nb = (int64_t)std::max(2, s->depth - 1) * s->nvox * kSgC;
    const int64_t vc = s->nvox * kSgC;
    if ((e = alloc(&s->act, nb)) || (e = alloc(&s->gA, vc)) || (e = alloc(&s->gB, vc)) ||
        (e = alloc(&s->xpad, vc)) || (e = alloc(&s->gpad, vc)) || (e = alloc(&s->y, s->nvox)) ||
        (e = alloc(&s->gy, s->nvox)) || (e = alloc(&s->qbuf, s->nvox)) ||
        (e = alloc(&s->ubuf, s->nvox)) ||
        (e = alloc(&s->part, std::max<int64_t>((int64_t)kSgWPart * kSgC * kSgC * 27,
                                               (int64_t)kRedBlocks * kSgC))))
      return e;
    if ((e = hipMemset(s->xpad, 0, vc * 4)) || (e = hipMemset(s->gpad, 0, vc * 4))) return e;
    s->trained_buffers = true;
  }
  if (n_loss > s->loss_cap) {
    (void)hipFree(s->loss);
    s->loss = nullptr;
    s->loss_cap = 0;
    if ((e = alloc(&s->loss, n_loss))) return e;
    s->loss_cap = n_loss;
  }
  return hipSuccess;
}

void sg_destroy(Surrogate* s) {
  void* bufs[] = {s->p,   s->grad, s->m1,   s->m2,   s->wmid, s->wmidt, s->win, s->wout,
                  s->woutt, s->act, s->gA,  s->gB,   s->xpad, s->gpad, s->y,    s->gy,
                  s->qbuf, s->ubuf, s->part, s->dred, s->loss, s->pos,  s->m64, s->m32,
                  s->ha,  s->hs};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  *s = Surrogate{};
}

void sg_default_params(const Surrogate* s, uint64_t seed, std::vector<float>& out) {
  // He-normal weights (variance 2 / fan-in; 1 / fan-in for the linear last
  // layer), zero biases; normal deviates by Box-Muller from the hash above
  out.assign((size_t)s->nparam, 0.f);
  uint64_t ctr = 0;
  auto uni = [&]() { return ((double)(mix64(seed * 0x100000001B3ull + ctr++) >> 11) + 0.5) * 0x1p-53; };
  for (int l = 0; l < s->depth; ++l) {
    const int ci = l == 0 ? 1 : kSgC, co = l == s->depth - 1 ? 1 : kSgC;
    const double sd = std::sqrt((l == s->depth - 1 ? 1.0 : 2.0) / (27.0 * ci));
    for (int64_t k = 0; k < (int64_t)co * ci * 27; ++k) {
      const double u1 = uni(), u2 = uni();
      const double gsn = std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * 3.14159265358979323846 * u2);
      out[(size_t)(s->woff[l] + k)] = (float)(sd * gsn);
    }
  }
}

hipError_t sg_set_params(Surrogate* s, const float* host, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(s->p, host, (size_t)s->nparam * 4, hipMemcpyHostToDevice, st);
  if (e) return e;
  if ((e = hipMemsetAsync(s->m1, 0, (size_t)s->nparam * 4, st)) ||
      (e = hipMemsetAsync(s->m2, 0, (size_t)s->nparam * 4, st)))
    return e;
  s->adam_t = 0;
  return sg_pack(s, st);
}

hipError_t sg_pack(Surrogate* s, hipStream_t st) {
  const int D = s->depth;
  hipLaunchKernelGGL(k_sg_pack_io, dim3(blocks(kSgC * 27)), dim3(kT), 0, st, s->p + s->woff[0],
                     s->win, (float*)nullptr);
  hipLaunchKernelGGL(k_sg_pack_io, dim3(blocks(kSgC * 27)), dim3(kT), 0, st, s->p + s->woff[D - 1],
                     s->wout, s->woutt);
  for (int l = 1; l <= D - 2; ++l) {
    const int64_t off = (int64_t)(l - 1) * 27 * kSgC * kSgC;
    hipLaunchKernelGGL(k_sg_pack_mid, dim3(blocks(27 * kSgC * kSgC)), dim3(kT), 0, st,
                       s->p + s->woff[l], s->wmid + off, s->wmidt + off);
  }
  return hipGetLastError();
}

hipError_t sg_get_params(const Surrogate* s, float* host, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(host, s->p, (size_t)s->nparam * 4, hipMemcpyDeviceToHost, st);
  if (e) return e;
  return hipStreamSynchronize(st);
}

hipError_t sg_apply(Surrogate* s, hipStream_t st, const float* Q, float* U) {
  forward(s, st, Q, s->trained_buffers, U, s->s_out);
  return hipGetLastError();
}

hipError_t sg_profile(Surrogate* s, hipStream_t st, const float* Q, float* U, int reps, double* ms) {
  const int D = s->depth;
  std::vector<hipEvent_t> ev(2 * D, nullptr);
  hipError_t e = hipSuccess;
  for (auto& x : ev)
    if ((e = hipEventCreate(&x))) break;
  for (int l = 0; l < D; ++l) ms[l] = 0.0;
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    forward(s, st, Q, s->trained_buffers, U, s->s_out, ev.data());
    if ((e = hipGetLastError()) || (e = hipStreamSynchronize(st))) break;
    for (int l = 0; l < D; ++l) {
      float t = 0.f;
      if ((e = hipEventElapsedTime(&t, ev[2 * l], ev[2 * l + 1]))) break;
      ms[l] += (double)t / reps;
    }
  }
  for (auto& x : ev)
    if (x) (void)hipEventDestroy(x);
  return e;
}

hipError_t sg_loss_grad(Surrogate* s, hipStream_t st, const float* Q, const float* tg, float tscale,
                        int slot) {
  const int D = s->depth;
  const SgGrid& gd = s->gd;
  const dim3 grid = tile_grid(gd);
  forward(s, st, Q, true, s->y, 1.f);
  hipLaunchKernelGGL(k_sg_pad, dim3(blocks(s->nvox)), dim3(kT), 0, st, s->nvox, Q, s->s_in, s->xpad);
  hipLaunchKernelGGL(k_sg_loss, dim3(kRedBlocks), dim3(kT), 0, st, s->nvox, s->y, tg, tscale, s->gy,
                     s->gpad, s->dred);
  hipLaunchKernelGGL(k_sg_sumd, dim3(1), dim3(kT), 0, st, kRedBlocks, s->dred,
                     1.0 / (double)s->nvox, s->loss + slot);
  // last layer
  layer_grads(s, st, D - 1, s->gpad, act_of(s, D - 2, true));
  hipLaunchKernelGGL(k_sg_in, grid, dim3(kT), 0, st, gd, s->gy, 1.f, s->woutt, (const float*)nullptr,
                     s->gB, 0, act_of(s, D - 2, true));
  float *gcur = s->gB, *gnext = s->gA;
  for (int l = D - 2; l >= 1; --l) {
    layer_grads(s, st, l, gcur, act_of(s, l - 1, true));
    launch_mid(s, st, gcur, s->wmidt + (int64_t)(l - 1) * 27 * kSgC * kSgC, nullptr, gnext, 0,
               act_of(s, l - 1, true));
    std::swap(gcur, gnext);
  }
  layer_grads(s, st, 0, gcur, s->xpad);
  return hipGetLastError();
}

hipError_t sg_adam(Surrogate* s, hipStream_t st, double lr) {
  const double b1 = 0.9, b2 = 0.999;
  s->adam_t++;
  const double lr_t = lr * std::sqrt(1.0 - std::pow(b2, (double)s->adam_t)) /
                      (1.0 - std::pow(b1, (double)s->adam_t));
  hipLaunchKernelGGL(k_sg_adam, dim3(blocks(s->nparam)), dim3(kT), 0, st, s->nparam, s->p, s->grad,
                     s->m1, s->m2, (float)lr_t, (float)b1, (float)b2, 1e-8f);
  return sg_pack(s, st);
}

hipError_t sg_texture(Surrogate* s, hipStream_t st, const SgTexture& tx, double* m_dev) {
  hipLaunchKernelGGL(k_sg_texture, dim3(blocks(s->n)), dim3(kT), 0, st, s->n, s->pos, tx, m_dev);
  return hipGetLastError();
}

hipError_t sg_to_f32(Surrogate* s, hipStream_t st, const double* m64, float* m32) {
  hipLaunchKernelGGL(k_sg_f32, dim3(blocks(3 * s->n)), dim3(kT), 0, st, 3 * s->n, m64, m32);
  return hipGetLastError();
}

hipError_t sg_field_error(Surrogate* s, hipStream_t st, const float* a, const float* b,
                          double* out2) {
  hipLaunchKernelGGL(k_sg_sq2, dim3(kRedBlocks), dim3(kT), 0, st, 3 * s->n, a, b, s->dred);
  std::vector<double> h(2 * kRedBlocks);
  hipError_t e = hipMemcpyAsync(h.data(), s->dred, h.size() * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e || (e = hipStreamSynchronize(st))) return e;
  out2[0] = out2[1] = 0.0;
  for (int i = 0; i < kRedBlocks; ++i) {
    out2[0] += h[2 * i];
    out2[1] += h[2 * i + 1];
  }
  return hipSuccess;
}

hipError_t sg_sumsq(Surrogate* s, hipStream_t st, const float* x, int64_t count, double* out) {
  hipLaunchKernelGGL(k_sg_sq2, dim3(kRedBlocks), dim3(kT), 0, st, count, x, (const float*)nullptr,
                     s->dred);
  std::vector<double> h(2 * kRedBlocks);
  hipError_t e = hipMemcpyAsync(h.data(), s->dred, h.size() * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e || (e = hipStreamSynchronize(st))) return e;
  *out = 0.0;
  for (int i = 0; i < kRedBlocks; ++i) *out += h[2 * i];
  return hipSuccess;
}

}  // namespace pmfem

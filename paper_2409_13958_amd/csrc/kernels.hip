// gfx950 kernels of the PM-FEM effective-field evaluation.
//
// One H_eff evaluation (paper Eqs. heff, hex, hms_d1 - hms_d3):
//   k_rowdot3      q = D m (Eq. hms_d1); on a second stream u_Z = Z0 m (Eq. hms_d2b)
//   k_anterp_scatter, k_anterp_sum  Q = W^T q      (Sec. 3.2.2, step 1; other forms:
//                  k_anterp_line by grid lines, k_anterp by tiles, both gathers)
//   k_fft_xy_fwd   real-to-complex FFT along x, FFT along y, per z-plane (step 2)
//   k_fft_z_mul    FFT along z, multiply by the PGF spectrum, inverse along z
//   k_fft_yx_inv   inverse FFT along y, complex-to-real along x -> U = (1/4 pi) K * Q
//                  (k_r2c_x, k_fft_y, k_c2r_x: the same passes one axis at a time)
//   k_interp_tile  u = W U + P q + u_Z            (steps 3 and 4)
//   k_exch         H_ex = L m, as differences     (Eqs. hex, lapl_2; second stream)
//   k_gsum         H = H_ex - G u (+ H_applied)   (Eq. hms_d3, heff)
// All arithmetic is FP32; every reduction is done in a fixed order inside a
// wavefront or a thread, so results are bitwise reproducible (no atomics).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace pmfem {

// ---------------------------------------------------------------------------
// helpers

__device__ __forceinline__ float lagrange(int a, float xi, int p) {
  // basis function a of the Lagrange interpolant through 0..p at xi:
  // prod_{c != a} (xi - c) times 1 / prod_{c != a} (a - c) = (-1)^(p-a) / (a! (p-a)!)
  const float invf[6] = {1.0f, 1.0f, 0.5f, 1.0f / 6.0f, 1.0f / 24.0f, 1.0f / 120.0f};
  float v = ((p - a) & 1 ? -1.0f : 1.0f) * invf[a] * invf[p - a];
  for (int c = 0; c <= p; ++c)
    if (c != a) v *= (xi - (float)c);
  return v;
}

// Cubic (p = 3) Lagrange basis through xi = 0, 1, 2, 3 as a polynomial in the
// centred variable t = xi - 3/2 (|t| <= 3/2, so no cancellation beyond a few
// ulps): L_a(t) = c0 + c1 t + c2 t^2 + c3 t^3.
struct Cubic {
  float c0, c1, c2, c3;
};

__device__ __forceinline__ Cubic cubic_basis(int a) {
  Cubic c;
  c.c0 = (a == 0 || a == 3) ? -0.0625f : 0.5625f;
  c.c1 = a == 0 ? (1.0f / 24.0f) : a == 1 ? -1.125f : a == 2 ? 1.125f : -(1.0f / 24.0f);
  c.c2 = (a == 0 || a == 3) ? 0.25f : -0.25f;
  c.c3 = a == 0 ? -(1.0f / 6.0f) : a == 1 ? 0.5f : a == 2 ? -0.5f : (1.0f / 6.0f);
  return c;
}

__device__ __forceinline__ float cubic_eval(const Cubic& c, float xi) {
  const float t = xi - 1.5f;
  return fmaf(fmaf(fmaf(c.c3, t, c.c2), t, c.c1), t, c.c0);
}

__device__ __forceinline__ void wave_lds_sync() {
  // make this wavefront's LDS writes visible to its own other lanes
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Grid storage (GridParams::gmode). BF16 is the upper half of an FP32 word,
// rounded to nearest even (the grid values are finite); the pair form keeps
// the rounding residual as a second BF16 value, so hi + lo carries 16
// significant bits. Arithmetic stays FP32: values are widened on load.
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float((uint32_t)h << 16);
}

__device__ __forceinline__ int64_t grid_points(const GridParams& g) {
  return (int64_t)g.N[0] * g.N[1] * g.N[2];
}

__device__ __forceinline__ void grid_store(float* G, int64_t i, float v, const GridParams& g) {
  if (g.gmode == 0) {
    G[i] = v;
    return;
  }
  uint16_t* H = reinterpret_cast<uint16_t*>(G);
  const uint16_t hi = f32_to_bf16(v);
  H[i] = hi;
  if (g.gmode == 2) H[grid_points(g) + i] = f32_to_bf16(v - bf16_to_f32(hi));
}

__device__ __forceinline__ float grid_load(const float* G, int64_t i, const GridParams& g) {
  if (g.gmode == 0) return G[i];
  const uint16_t* H = reinterpret_cast<const uint16_t*>(G);
  float v = bf16_to_f32(H[i]);
  if (g.gmode == 2) v += bf16_to_f32(H[grid_points(g) + i]);
  return v;
}

__device__ __forceinline__ int st_of(uint32_t packed, int axis) {
  return (int)((packed >> (10 * axis)) & 1023u);
}

// cumulative node index of source row `srow` at unwrapped box x (the node
// index of its first node, continued across a periodic wrap)
__device__ __forceinline__ int row_cum(const int32_t* box_start, int64_t srow, int nbx, int per,
                                       int tot, int x) {
  if (per) {
    int wrap = 0;
    if (x < 0) {
      x += nbx;
      wrap = -1;
    } else if (x > nbx) {
      x -= nbx;
      wrap = 1;
    }
    return wrap * tot + box_start[srow + x];
  }
  return box_start[srow + min(max(x, 0), nbx)];
}

// Block-strided copy loop with K loads in flight per thread: load(i) for K
// indices first, then store(i, value) for the same K.
template <int K, class Load, class Store>
__device__ __forceinline__ void batched(int n, Load&& load, Store&& store) {
  for (int i0 = threadIdx.x; i0 < n; i0 += K * blockDim.x) {
    decltype(load(0)) v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = i0 + k * blockDim.x;
      if (i < n) v[k] = load(i);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = i0 + k * blockDim.x;
      if (i < n) store(i, v[k]);
    }
  }
}

// node index of staged element e: rows [base[j], base[j+1]) hold the nodes
// of box row j from cumulative index c0[j] on (wrapping inside the row on a
// periodic x axis, where the row has tot[j] nodes starting at b0[j])
__device__ __forceinline__ int staged_node(int e, int nrow, const int* base, const int* c0,
                                           const int* b0, const int* tot, int per, int& row) {
  int lo = 0, hi = nrow;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (base[mid] <= e) lo = mid;
    else hi = mid;
  }
  row = lo;
  const int c = c0[lo] + (e - base[lo]);
  if (!per) return c;
  int rel = (c - b0[lo]) % tot[lo];
  if (rel < 0) rel += tot[lo];
  return b0[lo] + rel;
}

template <int W>
__device__ __forceinline__ float group_sum(float v) {
  // butterfly sum over groups of W consecutive lanes (W divides 64)
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
  return v;
}

// Entries e0 + lane, e0 + lane + G, ... of a row, K records of a lane in
// flight at once: all K record loads, then the K uses (which issue their
// gathers together). A record past the row end re-reads entry e (valid) and
// is passed on with ok = false; the sum order is the entry order.
template <int G, int K, class Rec, class Use>
__device__ __forceinline__ void row_entries(int e0, int e1, int lane, const Rec* __restrict__ rec,
                                            Use&& use) {
  for (int e = e0 + lane; e < e1; e += K * G) {
    Rec r[K];
#pragma unroll
    for (int k = 0; k < K; ++k) r[k] = rec[e + k * G < e1 ? e + k * G : e];
#pragma unroll
    for (int k = 0; k < K; ++k) use(r[k], e + k * G < e1);
  }
}

// ---------------------------------------------------------------------------
// charges and element-exact correction, G lanes per row, one 16-byte record
// {column, x, y, z} per entry (one vector load):
//   k_charges:  q_n   = sum_k D_nk . m_k     (local pattern)
//   k_zcorr:    u_Z,n = sum_j Z0_nj . m_j     (element-correction pattern)
// The two are independent; the library runs k_zcorr on a second stream,
// beside anterpolation and the FFT.

template <int G>
__global__ void __launch_bounds__(256) k_rowdot3(int64_t n, const float* __restrict__ m,
                                                 const int32_t* __restrict__ rp,
                                                 const int4* __restrict__ rec,
                                                 float* __restrict__ out) {
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int lane = threadIdx.x & (G - 1);
  if (row >= n) return;  // whole groups leave together
  float acc = 0.f;
  row_entries<G, 4>(rp[row], rp[row + 1], lane, rec, [&](const int4& r, bool ok) {
    const float* mk = m + 3 * (int64_t)r.x;
    const float m0 = mk[0], m1 = mk[1], m2 = mk[2];
    acc = fmaf(ok ? __int_as_float(r.y) : 0.f, m0, acc);
    acc = fmaf(ok ? __int_as_float(r.z) : 0.f, m1, acc);
    acc = fmaf(ok ? __int_as_float(r.w) : 0.f, m2, acc);
  });
  acc = group_sum<G>(acc);
  if (lane == 0) out[row] = acc;
}

template __global__ void k_rowdot3<4>(int64_t, const float*, const int32_t*, const int4*, float*);
template __global__ void k_rowdot3<8>(int64_t, const float*, const int32_t*, const int4*, float*);
template __global__ void k_rowdot3<16>(int64_t, const float*, const int32_t*, const int4*, float*);

// ---------------------------------------------------------------------------
// anterpolation: one workgroup per tile of kAntTX x kAntTY x kAntTZ grid
// points. The nodes of every box whose stencil can reach the tile (the
// tile's halo) are staged once in LDS; then each thread gathers, in a fixed
// order, the contributions of the boxes covering its grid point (per-axis
// box ranges precomputed on the host). No atomics; the sum order per grid
// point is fixed, so the result is reproducible bit for bit.

__device__ void block_exclusive_scan(int* a, int n, int* tmp) {
  // in-place exclusive scan of a[0..n) by blockDim.x threads; tmp holds
  // blockDim.x ints; a[n] receives the total
  const int T = blockDim.x, t = threadIdx.x;
  const int per = (n + T - 1) / T;
  const int lo = t * per, hi = min(n, lo + per);
  int sum = 0;
  for (int i = lo; i < hi; ++i) sum += a[i];
  tmp[t] = sum;
  __syncthreads();
  for (int d = 1; d < T; d <<= 1) {
    int v = (t >= d) ? tmp[t - d] : 0;
    __syncthreads();
    tmp[t] += v;
    __syncthreads();
  }
  int run = tmp[t] - sum;
  for (int i = lo; i < hi; ++i) {
    int c = a[i];
    a[i] = run;
    run += c;
  }
  if (t == T - 1) a[n] = tmp[T - 1];
  __syncthreads();
}

// stencil start of box b along an axis (unwrapped for periodic axes)
__device__ __forceinline__ int box_stencil_start(int b, int N, int p, int per) {
  const int s0 = b - (p - 1) / 2;
  return per ? s0 : min(max(s0, 0), N - p - 1);
}

__global__ void __launch_bounds__(256) k_anterp(
    GridParams g, const float* __restrict__ q, const float4* __restrict__ pos4,
    const int32_t* __restrict__ box_start, const int2* __restrict__ brx,
    const int2* __restrict__ bry, const int2* __restrict__ brz, float* __restrict__ Q) {
  __shared__ int s_off[kAntHalo];
  __shared__ int s_tmp[256];
  __shared__ float4 s_nd[kAntCap];  // xi_x, xi_y, xi_z, q of the staged nodes
  const int ntx = (g.N[0] + kAntTX - 1) / kAntTX, nty = (g.N[1] + kAntTY - 1) / kAntTY;
  const int tile = blockIdx.x;
  const int t0[3] = {(tile % ntx) * kAntTX, ((tile / ntx) % nty) * kAntTY,
                     (tile / (ntx * nty)) * kAntTZ};
  const int te[3] = {min(kAntTX, g.N[0] - t0[0]), min(kAntTY, g.N[1] - t0[1]),
                     min(kAntTZ, g.N[2] - t0[2])};
  const int2* br[3] = {brx, bry, brz};
  int hs[3], hc[3];
  for (int a = 0; a < 3; ++a) {
    const int2 f = br[a][t0[a]], l = br[a][t0[a] + te[a] - 1];
    hs[a] = f.x;
    hc[a] = g.per[a] ? (te[a] - 1) + g.p + 1 : l.x + l.y - f.x;
  }
  const int H = hc[0] * hc[1] * hc[2];
  auto box_of = [&](int h) -> int64_t {
    const int ix = h % hc[0], iy = (h / hc[0]) % hc[1], iz = h / (hc[0] * hc[1]);
    const int bx = (hs[0] + ix) % g.nbox[0], by = (hs[1] + iy) % g.nbox[1],
              bz = (hs[2] + iz) % g.nbox[2];
    return ((int64_t)bz * g.nbox[1] + by) * g.nbox[0] + bx;
  };
  for (int h = threadIdx.x; h < H; h += blockDim.x) {
    const int64_t b = box_of(h);
    s_off[h] = box_start[b + 1] - box_start[b];
  }
  __syncthreads();
  block_exclusive_scan(s_off, H, s_tmp);
  const int total = s_off[H];
  const int lx = threadIdx.x % kAntTX, ly = (threadIdx.x / kAntTX) % kAntTY,
            lz = threadIdx.x / (kAntTX * kAntTY);
  const bool inside = lx < te[0] && ly < te[1] && lz < te[2];
  const int gx = t0[0] + lx, gy = t0[1] + ly, gz = t0[2] + lz;
  if (total == 0) {  // no node reaches this tile (uniform across the block)
    if (inside) grid_store(Q, ((int64_t)gz * g.N[1] + gy) * g.N[0] + gx, 0.f, g);
    return;
  }
  const bool staged = total <= kAntCap;
  if (staged) {
    for (int h = threadIdx.x; h < H; h += blockDim.x) {
      const int64_t b = box_of(h);
      const int k0 = box_start[b], k1 = box_start[b + 1], o = s_off[h];
      for (int k = k0; k < k1; ++k) {
        const float4 pp = pos4[k];
        s_nd[o + k - k0] = make_float4(pp.x, pp.y, pp.z, q[k]);
      }
    }
  }
  __syncthreads();
  if (!inside) return;
  const int2 rx = brx[gx], ry = bry[gy], rz = brz[gz];
  // halo-relative first box of this point's ranges
  const int ox = g.per[0] ? lx : rx.x - hs[0];
  const int oy = g.per[1] ? ly : ry.x - hs[1];
  const int oz = g.per[2] ? lz : rz.x - hs[2];
  float acc = 0.f;
  // stencil index of the point in the k-th box of its range: on a periodic
  // axis the k-th box starts its stencil k - p points before the point; on a
  // non-periodic axis the (clamped) stencil start of that box decides
  for (int iz = 0; iz < rz.y; ++iz) {
    const int az = g.per[2] ? g.p - iz : gz - box_stencil_start(rz.x + iz, g.N[2], g.p, 0);
    for (int iy = 0; iy < ry.y; ++iy) {
      const int ay = g.per[1] ? g.p - iy : gy - box_stencil_start(ry.x + iy, g.N[1], g.p, 0);
      const int hrow = ((oz + iz) * hc[1] + (oy + iy)) * hc[0] + ox;
      for (int ix = 0; ix < rx.y; ++ix) {
        const int ax = g.per[0] ? g.p - ix : gx - box_stencil_start(rx.x + ix, g.N[0], g.p, 0);
        const int k0 = s_off[hrow + ix], k1 = s_off[hrow + ix + 1];
        if (k0 == k1) continue;
        // nodes of one box: all share (ax, ay, az)
        const bool cubic = g.p == 3;
        Cubic cx, cy, cz;
        if (cubic) {
          cx = cubic_basis(ax);
          cy = cubic_basis(ay);
          cz = cubic_basis(az);
        }
        for (int k = k0; k < k1; ++k) {
          float4 nd;
          if (staged) {
            nd = s_nd[k];
          } else {
            const int64_t b = box_of(hrow + ix);
            const int kg = box_start[b] + (k - k0);
            const float4 pp = pos4[kg];
            nd = make_float4(pp.x, pp.y, pp.z, q[kg]);
          }
          const float w = cubic ? cubic_eval(cx, nd.x) * cubic_eval(cy, nd.y) * cubic_eval(cz, nd.z)
                                : lagrange(ax, nd.x, g.p) * lagrange(ay, nd.y, g.p) *
                                      lagrange(az, nd.z, g.p);
          acc = fmaf(nd.w, w, acc);
        }
      }
    }
  }
  grid_store(Q, ((int64_t)gz * g.N[1] + gy) * g.N[0] + gx, acc, g);
}

// ---------------------------------------------------------------------------
// anterpolation by grid lines. A workgroup takes `xa` consecutive points of
// one (y, z) grid line, one thread per point. The boxes whose stencils reach
// the line form at most (p + 1)^2 box rows. Their nodes in the segment's x
// range are listed on the host, column-major (x box outermost, then box row,
// then node order), each entry tagged with its box row; the box table does
// not change between evaluations, so the list is built once. The workgroup
// stages the listed nodes in LDS, each reduced to what the line needs: its
// xi_x and the product c = q L_ay(xi_y) L_az(xi_z) of its charge with its y
// and z weights at the line (a_y, a_z are fixed per box row). A point then
// sums c L_ax(xi_x) over the p + 1 box columns covering it; a_x is fixed per
// column, so the inner loop runs over one contiguous LDS range per column.
// The sum order is fixed (no atomics).

__device__ __forceinline__ float basis(int a, float xi, int p) {
  return p == 3 ? cubic_eval(cubic_basis(a), xi) : lagrange(a, xi, p);
}

__global__ void __launch_bounds__(128) k_anterp_line(
    GridParams g, AntPlan pl, const float* __restrict__ q, const float4* __restrict__ pos4,
    const int32_t* __restrict__ list, const int32_t* __restrict__ lstart,
    const int32_t* __restrict__ colst, const int2* __restrict__ brx,
    const int2* __restrict__ bry, const int2* __restrict__ brz, float* __restrict__ Q) {
  extern __shared__ float4 smem4[];
  unsigned char* smem = reinterpret_cast<unsigned char*>(smem4);
  float2* s_nd = reinterpret_cast<float2*>(smem + pl.o_x);  // (xi_x, c) per listed node
  int* s_col0 = reinterpret_cast<int*>(smem + pl.o_off);    // [sbx + 1] column starts
  int* s_ayz = reinterpret_cast<int*>(smem + pl.o_meta);    // [nrow] a_y | a_z << 8
  const int tid = threadIdx.x, T = blockDim.x;
  const int w = blockIdx.x;
  const int sx = w % pl.nsx, line = w / pl.nsx;
  const int gy = line % g.N[1], gz = line / g.N[1];
  const int x0 = sx * pl.xa, xa = min(pl.xa, g.N[0] - x0);
  const int2 ry = bry[gy], rz = brz[gz];
  const int nrow = ry.y * rz.y;
  const int p = g.p, shift = (p - 1) / 2;
  const int fb = g.per[0] ? x0 - p + shift : brx[x0].x;  // first listed box column
  const int l0 = lstart[w];
  const int n = min(lstart[w + 1] - l0, pl.ncap);
  if (tid < nrow) {
    const int iy = tid % ry.y, iz = tid / ry.y;
    int by = ry.x + iy, bz = rz.x + iz;
    if (by >= g.nbox[1]) by -= g.nbox[1];
    if (bz >= g.nbox[2]) bz -= g.nbox[2];
    int ay = gy - box_stencil_start(by, g.N[1], p, g.per[1]);
    int az = gz - box_stencil_start(bz, g.N[2], p, g.per[2]);
    if (g.per[1]) ay = ((ay % g.N[1]) + g.N[1]) % g.N[1];
    if (g.per[2]) az = ((az % g.N[2]) + g.N[2]) % g.N[2];
    s_ayz[tid] = ay | (az << 8);
  }
  for (int k = tid; k <= pl.sbx; k += T) s_col0[k] = colst[(int64_t)w * (pl.sbx + 1) + k];
  __syncthreads();
  // stage the listed nodes with their y/z weights at this line, K in flight
  {
    constexpr int K = 8;
    for (int e0 = tid; e0 < n; e0 += K * T) {
      int ent[K];
#pragma unroll
      for (int j = 0; j < K; ++j) ent[j] = e0 + j * T < n ? list[l0 + e0 + j * T] : 0;
      float4 nd[K];
      float qq[K];
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const int gi = ent[j] & 0x3FFFFFF;
        nd[j] = pos4[gi];
        qq[j] = q[gi];
      }
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const int e = e0 + j * T;
        if (e < n) {
          const int ayz = s_ayz[(unsigned)ent[j] >> 26];
          s_nd[e] = make_float2(nd[j].x, qq[j] * basis(ayz & 255, nd[j].y, p) *
                                             basis(ayz >> 8, nd[j].z, p));
        }
      }
    }
  }
  __syncthreads();
  if (tid >= xa) return;
  // gather for the point gx, column by column
  const int gx = x0 + tid;
  const int2 rx = brx[gx];
  const int k0 = g.per[0] ? tid : rx.x - fb;
  const int kc = g.per[0] ? p + 1 : rx.y;
  float acc = 0.f;
  for (int c4 = 0; c4 < kc; ++c4) {
    const int k = k0 + c4;
    const int a = g.per[0] ? p - c4 : gx - box_stencil_start(fb + k, g.N[0], p, 0);
    const int n1 = min(s_col0[k + 1], n);
    if (p == 3) {
      const Cubic cb = cubic_basis(a);
#pragma unroll 2
      for (int e = s_col0[k]; e < n1; ++e) {
        const float2 v = s_nd[e];
        acc = fmaf(v.y, cubic_eval(cb, v.x), acc);
      }
    } else {
      for (int e = s_col0[k]; e < n1; ++e) {
        const float2 v = s_nd[e];
        acc = fmaf(v.y, lagrange(a, v.x, p), acc);
      }
    }
  }
  grid_store(Q, ((int64_t)gz * g.N[1] + gy) * g.N[0] + gx, acc, g);
}

// ---------------------------------------------------------------------------
// anterpolation by scatter. One 64-lane workgroup per tile of boxes: its
// nodes (listed on the host in box order, each with the offset of its box's
// stencil in the tile footprint) come in batches of 64, one per lane, and the
// 16 nodes of a 16-lane row go to that row's lane group (DPP broadcasts
// within the row; one 64-lane group for p > 3). A lane of a group owns one
// (a, b) pair of x and y stencil offsets and adds, for every node of its
// group, q L_a(xi_x) L_b(xi_y) L_c(xi_z), c = 0..p, to the grid points of the
// node's stencil in the group's own LDS copy of the tile footprint (the
// grid points the stencils of the tile's boxes cover). Within an instruction
// the lanes of a group address distinct points and the groups distinct
// copies, and each group takes its nodes in a fixed order, so the sums do
// not depend on timing. The copies are then added in group order and the
// footprint written out; k_anterp_sum adds, for every grid point, the
// footprints of the (at most two per axis) tiles that cover it.

// L_a(xi) for compile-time p and a
template <int P>
__device__ __forceinline__ float basis_ct(int a, float xi) {
  if constexpr (P == 3) return cubic_eval(cubic_basis(a), xi);
  else return lagrange(a, xi, P);
}

// value of lane I of this lane's 16-lane row (DPP row broadcast)
template <int I>
__device__ __forceinline__ float row_lane(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x150 + I, 0xf, 0xf, false));
}

template <int P>
__device__ __forceinline__ void anterp_scatter_body(
    GridParams g, ScPlan pl, const float* __restrict__ q, const float4* __restrict__ pos4,
    const int2* __restrict__ list, const int32_t* __restrict__ lstart,
    float* __restrict__ part, const int blk) {
  constexpr int P1 = P + 1, GS = P1 * P1 <= 16 ? 16 : 64, NG = 64 / GS;
  extern __shared__ float s_acc[];  // [NG][fsize] footprint copies
  const int lane = threadIdx.x, grp = lane / GS, gl = lane - grp * GS;
  const bool act = gl < P1 * P1;
  // the lane's x and y stencil offsets; lane c of a group (b = 0) also
  // evaluates the z weight of index c for the group
  const int a = gl % P1, b = gl / P1;
  const int w = blk;
  const int l0 = lstart[w], cnt = lstart[w + 1] - l0;
  // nodes come in batches of 64, lane L holding entry f0 + L of the tile's
  // list {node, footprint offset of its stencil}; the next batch is requested
  // while the current one is added
  auto fetch = [&](int f0, float4& ps, float& qq, int& off) {
    const int f = f0 + lane;
    const int2 e = list[l0 + (f < cnt ? f : 0)];
    ps = pos4[e.x];
    qq = f < cnt ? q[e.x] : 0.f;
    off = e.y;
  };
  float4 ps = make_float4(0.f, 0.f, 0.f, 0.f);
  float qq = 0.f;
  int ofs = 0;
  if (cnt > 0) fetch(0, ps, qq, ofs);
  const int FXY = pl.fd[0] * pl.fd[1], fsize = pl.fsize;
  for (int i = lane; i < NG * fsize; i += 64) s_acc[i] = 0.f;
  __syncthreads();
  float* acc = s_acc + grp * fsize + b * pl.fd[0] + a;
  Cubic cxa{}, cyb{};
  if constexpr (P == 3) {
    cxa = cubic_basis(a);
    cyb = cubic_basis(b);
  }
  auto lane_basis = [&](int k, const Cubic& ck, float xi) {
    if constexpr (P == 3) return cubic_eval(ck, xi);
    else return lagrange(k, xi, P);
  };
  // one node: its stencil's contributions on the lane's (a, b) column, a
  // plain read-add-write (the lanes of a group address distinct points of
  // the group's own copy, and one wavefront's LDS accesses complete in order)
  auto add = [&](float px, float py, float qv, int off, const float* lz) {
    const float wab = qv * lane_basis(a, cxa, px) * lane_basis(b, cyb, py);
    float* base = acc + off;
    float v[P1];
#pragma unroll
    for (int c = 0; c < P1; ++c) v[c] = base[c * FXY];
#pragma unroll
    for (int c = 0; c < P1; ++c) base[c * FXY] = fmaf(wab, lz[c], v[c]);
    // keep the next node's reads behind these writes (other lanes' points)
    __builtin_amdgcn_wave_barrier();
  };
  for (int f0 = 0; f0 < cnt; f0 += 64) {
    float4 psn = make_float4(0.f, 0.f, 0.f, 0.f);
    float qqn = 0.f;
    int ofsn = 0;
    if (f0 + 64 < cnt) fetch(f0 + 64, psn, qqn, ofsn);
    const int nb = min(64, cnt - f0);
    if constexpr (GS == 16) {
      // group g adds the nodes of its row's lanes 0..15 in order
      const int mine = nb - 16 * grp;  // nodes of this batch in the group's row
#define PMFEM_SC_NODE(I)                                                                     \
  {                                                                                          \
    const float px = row_lane<I>(ps.x), py = row_lane<I>(ps.y), pz = row_lane<I>(ps.z);     \
    const float qv = row_lane<I>(qq);                                                        \
    const int off = __float_as_int(row_lane<I>(__int_as_float(ofs)));                        \
    const float lzm = lane_basis(a, cxa, pz);                                                \
    float lz[P1];                                                                            \
    lz[0] = row_lane<0>(lzm);                                                                \
    if constexpr (P1 > 1) lz[1 % P1] = row_lane<1>(lzm);                                     \
    if constexpr (P1 > 2) lz[2 % P1] = row_lane<2>(lzm);                                     \
    if constexpr (P1 > 3) lz[3 % P1] = row_lane<3>(lzm);                                     \
    if (act && I < mine) add(px, py, qv, off, lz);                                           \
  }
      PMFEM_SC_NODE(0) PMFEM_SC_NODE(1) PMFEM_SC_NODE(2) PMFEM_SC_NODE(3)
      PMFEM_SC_NODE(4) PMFEM_SC_NODE(5) PMFEM_SC_NODE(6) PMFEM_SC_NODE(7)
      PMFEM_SC_NODE(8) PMFEM_SC_NODE(9) PMFEM_SC_NODE(10) PMFEM_SC_NODE(11)
      PMFEM_SC_NODE(12) PMFEM_SC_NODE(13) PMFEM_SC_NODE(14) PMFEM_SC_NODE(15)
#undef PMFEM_SC_NODE
    } else {
      // one group: every lane adds node i of the batch
      for (int i = 0; i < nb; ++i) {
        auto bc = [&](float v) {
          return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), i));
        };
        const float px = bc(ps.x), py = bc(ps.y), pz = bc(ps.z), qv = bc(qq);
        const int off = __builtin_amdgcn_readlane(ofs, i);
        const float lzm = lane_basis(a, cxa, pz);
        float lz[P1];
#pragma unroll
        for (int c = 0; c < P1; ++c)
          lz[c] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lzm), c));
        if (act) add(px, py, qv, off, lz);
      }
    }
    ps = psn;
    qq = qqn;
    ofs = ofsn;
  }
  __syncthreads();
  float* out = part + (int64_t)w * fsize;
  for (int i = lane; i < fsize; i += 64) {
    float v = s_acc[i];
#pragma unroll
    for (int k = 1; k < NG; ++k) v += s_acc[k * fsize + i];
    out[i] = v;
  }
}

template <int P>
__global__ void __launch_bounds__(64) k_anterp_scatter(
    GridParams g, ScPlan pl, const float* __restrict__ q, const float4* __restrict__ pos4,
    const int2* __restrict__ list, const int32_t* __restrict__ lstart,
    float* __restrict__ part) {
  anterp_scatter_body<P>(g, pl, q, pos4, list, lstart, part, blockIdx.x);
}

template <int P>
__global__ void __launch_bounds__(64) k_anterp_scatter_cells(const CellTab* __restrict__ tab,
                                                            const int32_t* __restrict__ bcell,
                                                            const int32_t* __restrict__ boff) {
  const int c = bcell[blockIdx.x];
  const CellTab& t = tab[c];
  anterp_scatter_body<P>(t.g, t.sp, t.q, t.pos4, t.sc_list, t.sc_lstart, t.sc_part,
                         blockIdx.x - boff[c]);
}

#define PMFEM_ANTERP_SCATTER(P)                                                               \
  template __global__ void k_anterp_scatter<P>(GridParams, ScPlan, const float*, const float4*, \
                                               const int2*, const int32_t*, float*);         \
  template __global__ void k_anterp_scatter_cells<P>(const CellTab*, const int32_t*,          \
                                                     const int32_t*);
PMFEM_ANTERP_SCATTER(1)
PMFEM_ANTERP_SCATTER(2)
PMFEM_ANTERP_SCATTER(3)
PMFEM_ANTERP_SCATTER(4)
PMFEM_ANTERP_SCATTER(5)

// Q at every grid point: the sum, z tile outermost, then y, then x, of the
// footprint values of the tiles covering it; tab_a[2 g + i] = (tile, offset)
// along axis a, tile < 0 when absent. A thread takes PT consecutive x points
// of one grid line (PT divides Nx), sharing their y and z entries.
template <int PT>
__device__ __forceinline__ void anterp_sum_body(GridParams g, ScPlan pl,
                                                    const int2* __restrict__ tabx,
                                                    const int2* __restrict__ taby,
                                                    const int2* __restrict__ tabz,
                                                    const float* __restrict__ part,
                                                    float* __restrict__ Q, const int blk) {
  const int Nx = g.N[0], Ny = g.N[1];
  const int64_t i0 = ((int64_t)blk * blockDim.x + threadIdx.x) * PT;
  if (i0 >= (int64_t)Nx * Ny * g.N[2]) return;
  const int gx0 = (int)(i0 % Nx);
  const int64_t r = i0 / Nx;
  const int gy = (int)(r % Ny), gz = (int)(r / Ny);
  int2 ex[PT][2];
#pragma unroll
  for (int k = 0; k < PT; ++k) {
    ex[k][0] = tabx[2 * (gx0 + k)];
    ex[k][1] = tabx[2 * (gx0 + k) + 1];
  }
  const int2 ey0 = taby[2 * gy], ey1 = taby[2 * gy + 1];
  const int2 ez0 = tabz[2 * gz], ez1 = tabz[2 * gz + 1];
  const int FX = pl.fd[0], FY = pl.fd[1];
  // all 8 PT candidate values are loaded at once (an absent tile reads entry
  // 0 and counts as zero), so that no load waits behind a branch
  float val[2][2][PT][2];
#pragma unroll
  for (int kz = 0; kz < 2; ++kz) {
    const int2 ez = kz ? ez1 : ez0;
#pragma unroll
    for (int ky = 0; ky < 2; ++ky) {
      const int2 ey = ky ? ey1 : ey0;
      const int64_t t0 = ((int64_t)ez.x * pl.nt[1] + ey.x) * pl.nt[0];
      const int o0 = (ez.y * FY + ey.y) * FX;
#pragma unroll
      for (int k = 0; k < PT; ++k)
#pragma unroll
        for (int kx = 0; kx < 2; ++kx) {
          const int2 e = ex[k][kx];
          const bool ok = ez.x >= 0 && ey.x >= 0 && e.x >= 0;
          val[kz][ky][k][kx] = part[ok ? (t0 + e.x) * pl.fsize + o0 + e.y : 0];
          if (!ok) val[kz][ky][k][kx] = 0.f;
        }
    }
  }
  float sum[PT];
#pragma unroll
  for (int k = 0; k < PT; ++k) {
    sum[k] = 0.f;
#pragma unroll
    for (int kz = 0; kz < 2; ++kz)
#pragma unroll
      for (int ky = 0; ky < 2; ++ky)
#pragma unroll
        for (int kx = 0; kx < 2; ++kx) sum[k] += val[kz][ky][k][kx];
  }
#pragma unroll
  for (int k = 0; k < PT; ++k) grid_store(Q, i0 + k, sum[k], g);
}

template <int PT>
__global__ void __launch_bounds__(256) k_anterp_sum(GridParams g, ScPlan pl,
                                                    const int2* __restrict__ tabx,
                                                    const int2* __restrict__ taby,
                                                    const int2* __restrict__ tabz,
                                                    const float* __restrict__ part,
                                                    float* __restrict__ Q) {
  anterp_sum_body<PT>(g, pl, tabx, taby, tabz, part, Q, blockIdx.x);
}

template <int PT>
__global__ void __launch_bounds__(256) k_anterp_sum_cells(const CellTab* __restrict__ tab,
                                                         const int32_t* __restrict__ bcell,
                                                         const int32_t* __restrict__ boff) {
  const int c = bcell[blockIdx.x];
  const CellTab& t = tab[c];
  anterp_sum_body<PT>(t.g, t.sp, t.sc_tab[0], t.sc_tab[1], t.sc_tab[2], t.sc_part, t.grid,
                      blockIdx.x - boff[c]);
}

template __global__ void k_anterp_sum<1>(GridParams, ScPlan, const int2*, const int2*,
                                         const int2*, const float*, float*);
template __global__ void k_anterp_sum<4>(GridParams, ScPlan, const int2*, const int2*,
                                         const int2*, const float*, float*);
template __global__ void k_anterp_sum_cells<1>(const CellTab*, const int32_t*, const int32_t*);
template __global__ void k_anterp_sum_cells<4>(const CellTab*, const int32_t*, const int32_t*);

// ---------------------------------------------------------------------------
// LDS radix-2 FFT on `lines` lines of length n, lines `stride` elements apart
// (a stride of n + 1 keeps column-wise access free of bank conflicts), input
// in bit-reversed order; decimation in time, natural-order output. lds_fft is
// the contiguous case.

__device__ __forceinline__ void radix2(float2& a, float2& b, float2 w) {
  const float2 t = make_float2(b.x * w.x - b.y * w.y, b.x * w.y + b.y * w.x);
  b = make_float2(a.x - t.x, a.y - t.y);
  a = make_float2(a.x + t.x, a.y + t.y);
}

__device__ void lds_fft_s(float2* buf, int n, int logn, int lines, int stride, const float2* tw,
                          float sign) {
  // radix-2 decimation in time; n = 2^logn, so every index split is a shift.
  // Three stages s, s + 1, s + 2 are done together by one thread per 8
  // elements (the same twelve butterflies, in registers), then a pair, then a
  // single stage as needed, so every pass costs one LDS round trip and one
  // barrier.
  int s = 1;
  for (; s + 2 <= logn; s += 3) {
    const int ls = s - 1;  // log2(h), h the half of stage s
    const int h = 1 << ls;
    const int total = lines << (logn - 3);
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      const int line = idx >> (logn - 3);
      const int j = idx & ((1 << (logn - 3)) - 1);
      const int k = j & (h - 1);
      const int i0 = line * stride + ((j >> ls) << (ls + 3)) + k;
      float2 w1 = tw[k << (logn - s)];
      float2 w2 = tw[k << (logn - s - 1)], w3 = tw[(k + h) << (logn - s - 1)];
      float2 w4 = tw[k << (logn - s - 2)], w5 = tw[(k + h) << (logn - s - 2)];
      float2 w6 = tw[(k + 2 * h) << (logn - s - 2)], w7 = tw[(k + 3 * h) << (logn - s - 2)];
      w1.y *= sign;
      w2.y *= sign;
      w3.y *= sign;
      w4.y *= sign;
      w5.y *= sign;
      w6.y *= sign;
      w7.y *= sign;
      float2 a[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) a[m] = buf[i0 + m * h];
      radix2(a[0], a[1], w1);
      radix2(a[2], a[3], w1);
      radix2(a[4], a[5], w1);
      radix2(a[6], a[7], w1);
      radix2(a[0], a[2], w2);
      radix2(a[1], a[3], w3);
      radix2(a[4], a[6], w2);
      radix2(a[5], a[7], w3);
      radix2(a[0], a[4], w4);
      radix2(a[1], a[5], w5);
      radix2(a[2], a[6], w6);
      radix2(a[3], a[7], w7);
#pragma unroll
      for (int m = 0; m < 8; ++m) buf[i0 + m * h] = a[m];
    }
    __syncthreads();
  }
  for (; s + 1 <= logn; s += 2) {
    const int ls = s - 1;  // log2(h), h the half of stage s
    const int h = 1 << ls;
    const int total = lines << (logn - 2);
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      const int line = idx >> (logn - 2);
      const int j = idx & ((1 << (logn - 2)) - 1);
      const int k = j & (h - 1);
      const int i0 = line * stride + ((j >> ls) << (ls + 2)) + k;
      float2 w1 = tw[k << (logn - s)];
      float2 w2 = tw[k << (logn - s - 1)];
      float2 w3 = tw[(k + h) << (logn - s - 1)];
      w1.y *= sign;
      w2.y *= sign;
      w3.y *= sign;
      float2 a0 = buf[i0], a1 = buf[i0 + h], a2 = buf[i0 + 2 * h], a3 = buf[i0 + 3 * h];
      radix2(a0, a1, w1);
      radix2(a2, a3, w1);
      radix2(a0, a2, w2);
      radix2(a1, a3, w3);
      buf[i0] = a0;
      buf[i0 + h] = a1;
      buf[i0 + 2 * h] = a2;
      buf[i0 + 3 * h] = a3;
    }
    __syncthreads();
  }
  if (s == logn) {  // a last single stage
    const int ls = s - 1;
    const int half = 1 << ls;
    const int lh = logn - 1;
    const int total = lines << lh;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      const int line = idx >> lh;
      const int j = idx & ((1 << lh) - 1);
      const int k = j & (half - 1);
      const int i0 = line * stride + ((j >> ls) << (ls + 1)) + k;
      float2 w = tw[k];  // tw step 1 in the last stage
      w.y *= sign;
      float2 a = buf[i0], b = buf[i0 + half];
      radix2(a, b, w);
      buf[i0] = a;
      buf[i0 + half] = b;
    }
    __syncthreads();
  }
}

__device__ void lds_fft(float2* buf, int n, int logn, int lines, const float2* tw, float sign) {
  lds_fft_s(buf, n, logn, lines, n, tw, sign);
}

__device__ __forceinline__ int bitrev(int i, int logn) { return (int)(__brev((unsigned)i) >> (32 - logn)); }

// R2C along x: pairs of real rows (y, y+1) of plane z form one complex line.
// grid [Nz][Ny][Nx] real -> spec [Nz][My][Hx] complex (rows y < Ny written).
__device__ __forceinline__ void r2c_x_body(GridParams g, const float* __restrict__ Q,
                                               float2* __restrict__ spec, const float2* __restrict__ twx,
                                               int lines_per_block, const int blk) {
  extern __shared__ float2 sh[];
  const int Mx = g.M[0], logM = g.logM[0], Hx = Mx / 2 + 1;
  float2* tw = sh;
  float2* buf = sh + Mx / 2;
  for (int i = threadIdx.x; i < Mx / 2; i += blockDim.x) tw[i] = twx[i];
  const int pairs = (g.N[1] + 1) / 2;
  const int64_t total_lines = (int64_t)pairs * g.N[2];
  const int64_t l0 = (int64_t)blk * lines_per_block;
  int nl = (int)((total_lines - l0) < lines_per_block ? (total_lines - l0) : lines_per_block);
  for (int idx = threadIdx.x; idx < nl * Mx; idx += blockDim.x) {
    int li = idx / Mx, x = idx - li * Mx;
    int64_t L = l0 + li;
    int z = (int)(L / pairs), y = 2 * (int)(L % pairs);
    float re = 0.f, im = 0.f;
    if (x < g.N[0]) {
      re = grid_load(Q, ((int64_t)z * g.N[1] + y) * g.N[0] + x, g);
      if (y + 1 < g.N[1]) im = grid_load(Q, ((int64_t)z * g.N[1] + y + 1) * g.N[0] + x, g);
    }
    buf[li * Mx + bitrev(x, logM)] = make_float2(re, im);
  }
  __syncthreads();
  lds_fft(buf, Mx, logM, nl, tw, 1.0f);
  for (int idx = threadIdx.x; idx < nl * Hx; idx += blockDim.x) {
    int li = idx / Hx, k = idx - li * Hx;
    int64_t L = l0 + li;
    int z = (int)(L / pairs), y = 2 * (int)(L % pairs);
    float2 a = buf[li * Mx + k];
    float2 b = buf[li * Mx + ((Mx - k) & (Mx - 1))];
    // X_y = (Z[k] + conj Z[-k]) / 2, X_{y+1} = (Z[k] - conj Z[-k]) / (2i)
    float2 x0 = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));
    float2 x1 = make_float2(0.5f * (a.y + b.y), -0.5f * (a.x - b.x));
    spec[((int64_t)z * g.M[1] + y) * Hx + k] = x0;
    if (y + 1 < g.N[1]) spec[((int64_t)z * g.M[1] + y + 1) * Hx + k] = x1;
  }
}

__global__ void __launch_bounds__(256) k_r2c_x(GridParams g, const float* __restrict__ Q,
                                               float2* __restrict__ spec, const float2* __restrict__ twx,
                                               int lines_per_block) {
  r2c_x_body(g, Q, spec, twx, lines_per_block, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_r2c_x_cells(const CellTab* __restrict__ tab,
                                                     const int32_t* __restrict__ bcell,
                                                     const int32_t* __restrict__ boff) {
  const int c = bcell[blockIdx.x];
  const CellTab& t = tab[c];
  r2c_x_body(t.g, t.grid, t.spec, t.twx, t.lpb, blockIdx.x - boff[c]);
}

// n / d for 0 <= n < 2^22 and 1 <= d < 2^10 without an integer divide: the
// float quotient is off by at most one, which the correction removes.
__device__ __forceinline__ int fdiv(int n, int d, float inv_d) {
  int q = (int)((float)n * inv_d);
  if (q * d > n) --q;
  else if ((q + 1) * d <= n) ++q;
  return q;
}

// Forward transform of one z-plane held whole in LDS: real rows y < Ny are
// paired into complex lines (R2C along x), separated into the half spectrum
// kx < Hx, transposed into columns (stride My + 1) and transformed along y.
// Q[z][y][x] -> spec[z][ky][kx] for all ky < My. nsplit workgroups share a
// plane: each does the x pass and the y pass of its share of the columns.
__device__ __forceinline__ void fft_xy_fwd_body(GridParams g, const float* __restrict__ Q,
                                                     float2* __restrict__ spec,
                                                     const float2* __restrict__ twx,
                                                     const float2* __restrict__ twy,
                                                     int nsplit, const int blk) {
  extern __shared__ float2 sh[];
  const int Mx = g.M[0], My = g.M[1], Hx = Mx / 2 + 1, lx = g.logM[0], ly = g.logM[1];
  const int Nx = g.N[0], Ny = g.N[1], pairs = (Ny + 1) / 2, cs = My + 1;
  float2* tx = sh;
  float2* ty = tx + Mx / 2;
  float2* A = ty + My / 2;        // [pairs][Mx]
  float2* C = A + pairs * Mx;     // [Hx][My + 1]
  const int z = blk / nsplit, part = blk - z * nsplit;
  const int kw = (Hx + nsplit - 1) / nsplit, k0 = part * kw, nk = min(Hx, k0 + kw) - k0;
  const float invnk = 1.0f / (float)nk;
  for (int i = threadIdx.x; i < Mx / 2; i += blockDim.x) tx[i] = twx[i];
  for (int i = threadIdx.x; i < My / 2; i += blockDim.x) ty[i] = twy[i];
  const int64_t qz = (int64_t)z * Ny * Nx;
  const float invHx = 1.0f / (float)Hx;
  batched<8>(
      pairs * Mx,
      [&](int idx) {
        const int li = idx >> lx, x = idx & (Mx - 1), y = 2 * li;
        float2 v = make_float2(0.f, 0.f);
        if (x < Nx) {
          v.x = grid_load(Q, qz + (int64_t)y * Nx + x, g);
          if (y + 1 < Ny) v.y = grid_load(Q, qz + (int64_t)(y + 1) * Nx + x, g);
        }
        return v;
      },
      [&](int idx, float2 v) {
        const int li = idx >> lx, x = idx & (Mx - 1);
        A[li * Mx + bitrev(x, lx)] = v;
      });
  // rows Ny..My-1 of the columns are the zero padding
  for (int idx = threadIdx.x; idx < nk * (My - 2 * pairs); idx += blockDim.x) {
    const int yq = fdiv(idx, nk, invnk);
    const int k = k0 + idx - yq * nk, y = 2 * pairs + yq;
    C[k * cs + bitrev(y, ly)] = make_float2(0.f, 0.f);
  }
  __syncthreads();
  lds_fft_s(A, Mx, lx, pairs, Mx, tx, 1.0f);
  for (int idx = threadIdx.x; idx < pairs * nk; idx += blockDim.x) {
    const int li = fdiv(idx, nk, invnk), k = k0 + idx - li * nk, y = 2 * li;
    const float2 a = A[li * Mx + k];
    const float2 b = A[li * Mx + ((Mx - k) & (Mx - 1))];
    // X_y = (Z[k] + conj Z[-k]) / 2, X_{y+1} = (Z[k] - conj Z[-k]) / (2i)
    C[k * cs + bitrev(y, ly)] = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));
    C[k * cs + bitrev(y + 1, ly)] =
        y + 1 < Ny ? make_float2(0.5f * (a.y + b.y), -0.5f * (a.x - b.x)) : make_float2(0.f, 0.f);
  }
  __syncthreads();
  lds_fft_s(C + k0 * cs, My, ly, nk, cs, ty, 1.0f);
  float2* Sz = spec + (int64_t)z * My * Hx;
  for (int idx = threadIdx.x; idx < My * nk; idx += blockDim.x) {
    const int ky = fdiv(idx, nk, invnk), k = k0 + idx - ky * nk;
    Sz[ky * Hx + k] = C[k * cs + ky];
  }
}

__global__ void __launch_bounds__(1024) k_fft_xy_fwd(GridParams g, const float* __restrict__ Q,
                                                     float2* __restrict__ spec,
                                                     const float2* __restrict__ twx,
                                                     const float2* __restrict__ twy,
                                                     int nsplit) {
  fft_xy_fwd_body(g, Q, spec, twx, twy, nsplit, blockIdx.x);
}

__global__ void __launch_bounds__(1024) k_fft_xy_fwd_cells(const CellTab* __restrict__ tab,
                                                           const int32_t* __restrict__ bcell,
                                                           const int32_t* __restrict__ boff,
                                                           int nsplit) {
  const int c = bcell[blockIdx.x];
  const CellTab& t = tab[c];
  fft_xy_fwd_body(t.g, t.grid, t.spec, t.twx, t.twy, nsplit, blockIdx.x - boff[c]);
}

// Inverse of k_fft_xy_fwd for one z-plane: inverse FFT along y of the half
// spectrum columns, rows y < Ny paired into complex lines with Hermitian
// extension (C2R along x), inverse FFT along x. spec[z] -> U[z][y][x].
// nsplit workgroups share a plane: each does the y pass and the x pass of
// its share of the row pairs.
__device__ __forceinline__ void fft_yx_inv_body(GridParams g, const float2* __restrict__ spec,
                                                     float* __restrict__ U,
                                                     const float2* __restrict__ twx,
                                                     const float2* __restrict__ twy,
                                                     int nsplit, const int blk) {
  extern __shared__ float2 sh[];
  const int Mx = g.M[0], My = g.M[1], Hx = Mx / 2 + 1, lx = g.logM[0], ly = g.logM[1];
  const int Nx = g.N[0], Ny = g.N[1], pairs = (Ny + 1) / 2, cs = My + 1;
  float2* tx = sh;
  float2* ty = tx + Mx / 2;
  float2* A = ty + My / 2;
  float2* C = A + pairs * Mx;
  const int z = blk / nsplit, part = blk - z * nsplit;
  const int lw = (pairs + nsplit - 1) / nsplit, l0 = part * lw, nl = min(pairs, l0 + lw) - l0;
  for (int i = threadIdx.x; i < Mx / 2; i += blockDim.x) tx[i] = twx[i];
  for (int i = threadIdx.x; i < My / 2; i += blockDim.x) ty[i] = twy[i];
  const float2* Sz = spec + (int64_t)z * My * Hx;
  const float invHx = 1.0f / (float)Hx;
  batched<8>(
      My * Hx, [&](int idx) { return Sz[idx]; },
      [&](int idx, float2 v) {
        const int ky = fdiv(idx, Hx, invHx), k = idx - ky * Hx;
        C[k * cs + bitrev(ky, ly)] = v;
      });
  __syncthreads();
  lds_fft_s(C, My, ly, Hx, cs, ty, -1.0f);
  for (int idx = threadIdx.x; idx < nl * Mx; idx += blockDim.x) {
    const int li = l0 + (idx >> lx), k = idx & (Mx - 1), y = 2 * li;
    const int kk = k <= Mx / 2 ? k : Mx - k;
    float2 a = C[kk * cs + y];
    float2 b = y + 1 < Ny ? C[kk * cs + y + 1] : make_float2(0.f, 0.f);
    if (k > Mx / 2) {
      a.y = -a.y;
      b.y = -b.y;
    }
    // Z = X_y + i X_{y+1}
    A[li * Mx + bitrev(k, lx)] = make_float2(a.x - b.y, a.y + b.x);
  }
  __syncthreads();
  lds_fft_s(A + l0 * Mx, Mx, lx, nl, Mx, tx, -1.0f);
  const int64_t uzo = (int64_t)z * Ny * Nx;
  const float invNx = 1.0f / (float)Nx;
  for (int idx = threadIdx.x; idx < nl * Nx; idx += blockDim.x) {
    const int li = l0 + fdiv(idx, Nx, invNx), x = idx - (li - l0) * Nx, y = 2 * li;
    const float2 v = A[li * Mx + x];
    grid_store(U, uzo + (int64_t)y * Nx + x, v.x, g);
    if (y + 1 < Ny) grid_store(U, uzo + (int64_t)(y + 1) * Nx + x, v.y, g);
  }
}

__global__ void __launch_bounds__(1024) k_fft_yx_inv(GridParams g, const float2* __restrict__ spec,
                                                     float* __restrict__ U,
                                                     const float2* __restrict__ twx,
                                                     const float2* __restrict__ twy,
                                                     int nsplit) {
  fft_yx_inv_body(g, spec, U, twx, twy, nsplit, blockIdx.x);
}

__global__ void __launch_bounds__(1024) k_fft_yx_inv_cells(const CellTab* __restrict__ tab,
                                                           const int32_t* __restrict__ bcell,
                                                           const int32_t* __restrict__ boff,
                                                           int nsplit) {
  const int c = bcell[blockIdx.x];
  const CellTab& t = tab[c];
  fft_yx_inv_body(t.g, t.spec, t.grid, t.twx, t.twy, nsplit, blockIdx.x - boff[c]);
}

// FFT along y for lines (z < Nz, kx): groups of B consecutive kx per block.
// Forward: input rows y < Ny (others zero), all My outputs written.
// Inverse: all My inputs, outputs y < n_out written.
__device__ __forceinline__ void fft_y_body(GridParams g, float2* __restrict__ spec,
                                               const float2* __restrict__ twy, int B, int inverse,
                                               int n_in, int n_out, const int blk) {
  extern __shared__ float2 sh[];
  const int My = g.M[1], logM = g.logM[1], Hx = g.M[0] / 2 + 1;
  float2* tw = sh;
  float2* buf = sh + My / 2;
  for (int i = threadIdx.x; i < My / 2; i += blockDim.x) tw[i] = twy[i];
  const int groups_per_plane = (Hx + B - 1) / B;
  const int z = blk / groups_per_plane;
  const int kx0 = (blk - z * groups_per_plane) * B;
  const int nb = (Hx - kx0) < B ? (Hx - kx0) : B;
  for (int idx = threadIdx.x; idx < nb * My; idx += blockDim.x) {
    int y = idx / nb, li = idx - y * nb;
    float2 v = make_float2(0.f, 0.f);
    if (y < n_in) v = spec[((int64_t)z * My + y) * Hx + kx0 + li];
    buf[li * My + bitrev(y, logM)] = v;
  }
  __syncthreads();
  lds_fft(buf, My, logM, nb, tw, inverse ? -1.0f : 1.0f);
  for (int idx = threadIdx.x; idx < nb * n_out; idx += blockDim.x) {
    int y = idx / nb, li = idx - y * nb;
    spec[((int64_t)z * My + y) * Hx + kx0 + li] = buf[li * My + y];
  }
}

__global__ void __launch_bounds__(256) k_fft_y(GridParams g, float2* __restrict__ spec,
                                               const float2* __restrict__ twy, int B, int inverse,
                                               int n_in, int n_out) {
  fft_y_body(g, spec, twy, B, inverse, n_in, n_out, blockIdx.x);
}

// inverse = 0: rows y < N_y in, all M_y out; inverse = 1: all in, y < N_y out
__global__ void __launch_bounds__(256) k_fft_y_cells(const CellTab* __restrict__ tab,
                                                     const int32_t* __restrict__ bcell,
                                                     const int32_t* __restrict__ boff,
                                                     int inverse) {
  const int c = bcell[blockIdx.x];
  const CellTab& t = tab[c];
  const int ny = t.g.N[1], my = t.g.M[1];
  fft_y_body(t.g, t.spec, t.twy, t.by, inverse, inverse ? my : ny, inverse ? ny : my,
             blockIdx.x - boff[c]);
}

// FFT along z of lines c = ky*Hx + kx (B consecutive per block), multiply by
// the real spectrum khat[kz][c], inverse FFT, write z < Nz.
__device__ __forceinline__ void fft_z_mul_body(GridParams g, float2* __restrict__ spec,
                                                   const float* __restrict__ khat,
                                                   const float2* __restrict__ twz, int B, const int blk) {
  extern __shared__ float2 sh[];
  const int Mz = g.M[2], logM = g.logM[2], Hx = g.M[0] / 2 + 1;
  const int64_t plane = (int64_t)g.M[1] * Hx;
  float2* tw = sh;
  float2* buf = sh + Mz / 2;
  for (int i = threadIdx.x; i < Mz / 2; i += blockDim.x) tw[i] = twz[i];
  const int64_t c0 = (int64_t)blk * B;
  const int nb = (int)((plane - c0) < B ? (plane - c0) : B);
  batched<8>(
      nb * Mz,
      [&](int idx) {
        const int z = idx / nb, li = idx - z * nb;
        return z < g.N[2] ? spec[(int64_t)z * plane + c0 + li] : make_float2(0.f, 0.f);
      },
      [&](int idx, float2 v) {
        const int z = idx / nb, li = idx - z * nb;
        buf[li * Mz + bitrev(z, logM)] = v;
      });
  __syncthreads();
  lds_fft(buf, Mz, logM, nb, tw, 1.0f);
  // multiply and scatter back in bit-reversed order for the inverse
  batched<8>(
      nb * Mz,
      [&](int idx) {
        const int kz = idx / nb, li = idx - kz * nb;
        return khat[(int64_t)kz * plane + c0 + li];
      },
      [&](int idx, float kk) {
        const int kz = idx / nb, li = idx - kz * nb;
        const float2 v = buf[li * Mz + kz];
        buf[li * Mz + kz] = make_float2(v.x * kk, v.y * kk);  // same element, same thread
      });
  __syncthreads();
  // bit-reverse permutation in place
  for (int idx = threadIdx.x; idx < nb * Mz; idx += blockDim.x) {
    int i = idx / nb, li = idx - i * nb;
    int j = bitrev(i, logM);
    if (i < j) {
      float2 a = buf[li * Mz + i];
      buf[li * Mz + i] = buf[li * Mz + j];
      buf[li * Mz + j] = a;
    }
  }
  __syncthreads();
  lds_fft(buf, Mz, logM, nb, tw, -1.0f);
  for (int idx = threadIdx.x; idx < nb * g.N[2]; idx += blockDim.x) {
    int z = idx / nb, li = idx - z * nb;
    spec[(int64_t)z * plane + c0 + li] = buf[li * Mz + z];
  }
}

__global__ void __launch_bounds__(256) k_fft_z_mul(GridParams g, float2* __restrict__ spec,
                                                   const float* __restrict__ khat,
                                                   const float2* __restrict__ twz, int B) {
  fft_z_mul_body(g, spec, khat, twz, B, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_fft_z_mul_cells(const CellTab* __restrict__ tab,
                                                         const int32_t* __restrict__ bcell,
                                                         const int32_t* __restrict__ boff,
                                                         int B) {
  const int c = bcell[blockIdx.x];
  const CellTab& t = tab[c];
  fft_z_mul_body(t.g, t.spec, t.khat, t.twz, B, blockIdx.x - boff[c]);
}

// C2R along x: rows (y, y+1) of plane z from their half spectra -> U[z][y][x].
__device__ __forceinline__ void c2r_x_body(GridParams g, const float2* __restrict__ spec,
                                               float* __restrict__ U, const float2* __restrict__ twx,
                                               int lines_per_block, const int blk) {
  extern __shared__ float2 sh[];
  const int Mx = g.M[0], logM = g.logM[0], Hx = Mx / 2 + 1;
  float2* tw = sh;
  float2* buf = sh + Mx / 2;
  for (int i = threadIdx.x; i < Mx / 2; i += blockDim.x) tw[i] = twx[i];
  const int pairs = (g.N[1] + 1) / 2;
  const int64_t total_lines = (int64_t)pairs * g.N[2];
  const int64_t l0 = (int64_t)blk * lines_per_block;
  int nl = (int)((total_lines - l0) < lines_per_block ? (total_lines - l0) : lines_per_block);
  for (int idx = threadIdx.x; idx < nl * Mx; idx += blockDim.x) {
    int li = idx / Mx, k = idx - li * Mx;
    int64_t L = l0 + li;
    int z = (int)(L / pairs), y = 2 * (int)(L % pairs);
    int kk = k <= Mx / 2 ? k : Mx - k;
    float2 a = spec[((int64_t)z * g.M[1] + y) * Hx + kk];
    float2 b = make_float2(0.f, 0.f);
    if (y + 1 < g.N[1]) b = spec[((int64_t)z * g.M[1] + y + 1) * Hx + kk];
    if (k > Mx / 2) {
      a.y = -a.y;
      b.y = -b.y;
    }
    // Z = X_y + i X_{y+1}
    buf[li * Mx + bitrev(k, logM)] = make_float2(a.x - b.y, a.y + b.x);
  }
  __syncthreads();
  lds_fft(buf, Mx, logM, nl, tw, -1.0f);
  for (int idx = threadIdx.x; idx < nl * g.N[0]; idx += blockDim.x) {
    int li = idx / g.N[0], x = idx - li * g.N[0];
    int64_t L = l0 + li;
    int z = (int)(L / pairs), y = 2 * (int)(L % pairs);
    float2 v = buf[li * Mx + x];
    grid_store(U, ((int64_t)z * g.N[1] + y) * g.N[0] + x, v.x, g);
    if (y + 1 < g.N[1]) grid_store(U, ((int64_t)z * g.N[1] + y + 1) * g.N[0] + x, v.y, g);
  }
}

__global__ void __launch_bounds__(256) k_c2r_x(GridParams g, const float2* __restrict__ spec,
                                               float* __restrict__ U, const float2* __restrict__ twx,
                                               int lines_per_block) {
  c2r_x_body(g, spec, U, twx, lines_per_block, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_c2r_x_cells(const CellTab* __restrict__ tab,
                                                     const int32_t* __restrict__ bcell,
                                                     const int32_t* __restrict__ boff) {
  const int c = bcell[blockIdx.x];
  const CellTab& t = tab[c];
  c2r_x_body(t.g, t.spec, t.grid, t.twx, t.lpb, blockIdx.x - boff[c]);
}

// ---------------------------------------------------------------------------
// Mixed-radix FFT passes (extents that are products of 2, 3, 5 and 7):
// Stockham autosort in LDS, natural order in and out, ping-pong between two
// buffers, radices 4, 2, 3, 5, 7 taken in that order of preference. Pass
// with Ns = product of the radices done so far and radix R: element j of
// the n/R groups reads a_q = src[j + q n/R], q < R, multiplies a_q by the
// twiddle w^(q k) with k = j mod Ns and w = exp(-2 pi i / (Ns R)) (conjugated
// for the inverse), forms the R-point DFT b_p = sum_q a_q exp(-2 pi i q p / R)
// and writes b_p to dst[(j / Ns) Ns R + k + p Ns]. tw[t] = exp(-2 pi i t / n).

__device__ __forceinline__ float2 cmulf(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// R-point DFT in place, sign +1 forward (exp(-i ...)), -1 inverse
template <int R>
__device__ __forceinline__ void dft_small(float2* v, float sign) {
  // cos and sin of 2 pi m / R, m < R
  float c[R], sn[R];
  if constexpr (R == 2) {
    c[0] = 1.f; sn[0] = 0.f; c[1] = -1.f; sn[1] = 0.f;
  } else if constexpr (R == 3) {
    c[0] = 1.f; sn[0] = 0.f;
    c[1] = -0.5f; sn[1] = 0.86602540378443865f;
    c[2] = -0.5f; sn[2] = -0.86602540378443865f;
  } else if constexpr (R == 4) {
    c[0] = 1.f; sn[0] = 0.f; c[1] = 0.f; sn[1] = 1.f;
    c[2] = -1.f; sn[2] = 0.f; c[3] = 0.f; sn[3] = -1.f;
  } else if constexpr (R == 5) {
    c[0] = 1.f; sn[0] = 0.f;
    c[1] = 0.30901699437494742f; sn[1] = 0.95105651629515357f;
    c[2] = -0.80901699437494742f; sn[2] = 0.58778525229247313f;
    c[3] = -0.80901699437494742f; sn[3] = -0.58778525229247313f;
    c[4] = 0.30901699437494742f; sn[4] = -0.95105651629515357f;
  } else {
    c[0] = 1.f; sn[0] = 0.f;
    c[1] = 0.62348980185873353f; sn[1] = 0.78183148246802981f;
    c[2] = -0.22252093395631440f; sn[2] = 0.97492791218182361f;
    c[3] = -0.90096886790241913f; sn[3] = 0.43388373911755812f;
    c[4] = -0.90096886790241913f; sn[4] = -0.43388373911755812f;
    c[5] = -0.22252093395631440f; sn[5] = -0.97492791218182361f;
    c[6] = 0.62348980185873353f; sn[6] = -0.78183148246802981f;
  }
  float2 out[R];
#pragma unroll
  for (int p = 0; p < R; ++p) {
    float2 acc = v[0];
#pragma unroll
    for (int q = 1; q < R; ++q) {
      const int m = (q * p) % R;
      // exp(-i sign 2 pi m / R)
      const float2 w = make_float2(c[m], -sign * sn[m]);
      const float2 t = cmulf(v[q], w);
      acc.x += t.x;
      acc.y += t.y;
    }
    out[p] = acc;
  }
#pragma unroll
  for (int p = 0; p < R; ++p) v[p] = out[p];
}

template <int R>
__device__ __forceinline__ void stockham_pass(const float2* src, float2* dst, int n, int Ns,
                                              int lines, int ld, const float2* tw, float sign) {
  const int nR = n / R, step = n / (Ns * R);
  const int total = lines * nR;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int line = idx / nR, j = idx - line * nR;
    const float2* s = src + line * ld;
    float2* d = dst + line * ld;
    const int k = j % Ns;
    float2 v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = s[j + q * nR];
#pragma unroll
    for (int q = 1; q < R; ++q) {
      float2 w = tw[q * k * step];  // q k step < n
      w.y *= sign;
      v[q] = cmulf(v[q], w);
    }
    dft_small<R>(v, sign);
    const int base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int p = 0; p < R; ++p) d[base + p * Ns] = v[p];
  }
}

// lines of length n, line stride ld, in a; returns the buffer (a or b)
// holding the transform
__device__ float2* lds_fft_mr(float2* a, float2* b, int n, int lines, int ld, const float2* tw,
                              float sign) {
  int Ns = 1;
  while (Ns < n) {
    const int rem = n / Ns;
    if (rem % 4 == 0) {
      stockham_pass<4>(a, b, n, Ns, lines, ld, tw, sign);
      Ns *= 4;
    } else if (rem % 2 == 0) {
      stockham_pass<2>(a, b, n, Ns, lines, ld, tw, sign);
      Ns *= 2;
    } else if (rem % 3 == 0) {
      stockham_pass<3>(a, b, n, Ns, lines, ld, tw, sign);
      Ns *= 3;
    } else if (rem % 5 == 0) {
      stockham_pass<5>(a, b, n, Ns, lines, ld, tw, sign);
      Ns *= 5;
    } else {
      stockham_pass<7>(a, b, n, Ns, lines, ld, tw, sign);
      Ns *= 7;
    }
    __syncthreads();
    float2* t = a;
    a = b;
    b = t;
  }
  return a;
}

// Whole z-plane x and y passes, mixed radix (as k_fft_xy_fwd / k_fft_yx_inv
// for powers of two): one workgroup per plane; LDS: the two twiddle tables
// and two buffers of max(pairs Mx, Hx My) values. Forward: the pairs of real
// rows as complex lines along x, their half spectra unpacked into the
// columns of the plane, the columns along y. Inverse: the columns along y,
// the pairs of rows rebuilt as complex lines with the Hermitian half, the
// lines along x.
__device__ __forceinline__ void fft_xy_fwd_mr_body(GridParams g, const float* __restrict__ Q,
                                                   float2* __restrict__ spec,
                                                   const float2* __restrict__ twfx,
                                                   const float2* __restrict__ twfy,
                                                   const int blk) {
  extern __shared__ float2 sh[];
  const int Mx = g.M[0], My = g.M[1], Hx = Mx / 2 + 1, Ny = g.N[1];
  const int pairs = (Ny + 1) / 2;
  const int cap = max(pairs * Mx, Hx * My);
  float2* twx = sh;
  float2* twy = twx + Mx;
  float2* A = twy + My;
  float2* Bf = A + cap;
  for (int i = threadIdx.x; i < Mx; i += blockDim.x) twx[i] = twfx[i];
  for (int i = threadIdx.x; i < My; i += blockDim.x) twy[i] = twfy[i];
  const int z = blk;
  for (int idx = threadIdx.x; idx < pairs * Mx; idx += blockDim.x) {
    const int l = idx / Mx, x = idx - l * Mx, y = 2 * l;
    float re = 0.f, im = 0.f;
    if (x < g.N[0]) {
      re = grid_load(Q, ((int64_t)z * Ny + y) * g.N[0] + x, g);
      if (y + 1 < Ny) im = grid_load(Q, ((int64_t)z * Ny + y + 1) * g.N[0] + x, g);
    }
    A[idx] = make_float2(re, im);
  }
  __syncthreads();
  const float2* R = lds_fft_mr(A, Bf, Mx, pairs, Mx, twx, 1.0f);
  float2* C = R == A ? Bf : A;
  float2* D = R == A ? A : Bf;
  // X_y = (Z[k] + conj Z[-k]) / 2, X_{y+1} = (Z[k] - conj Z[-k]) / (2i), as
  // the columns C[kx My + y], zero past the rows
  for (int idx = threadIdx.x; idx < Hx * My; idx += blockDim.x) {
    const int kx = idx / My, y = idx - kx * My;
    float2 v = make_float2(0.f, 0.f);
    if (y < Ny) {
      const int l = y >> 1;
      const float2 a = R[l * Mx + kx];
      const float2 b = R[l * Mx + (kx == 0 ? 0 : Mx - kx)];
      v = (y & 1) ? make_float2(0.5f * (a.y + b.y), -0.5f * (a.x - b.x))
                  : make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));
    }
    C[idx] = v;
  }
  __syncthreads();
  const float2* S = lds_fft_mr(C, D, My, Hx, My, twy, 1.0f);
  for (int idx = threadIdx.x; idx < My * Hx; idx += blockDim.x) {
    const int ky = idx / Hx, kx = idx - ky * Hx;
    spec[((int64_t)z * My + ky) * Hx + kx] = S[kx * My + ky];
  }
}

__device__ __forceinline__ void fft_yx_inv_mr_body(GridParams g, const float2* __restrict__ spec,
                                                   float* __restrict__ U,
                                                   const float2* __restrict__ twfx,
                                                   const float2* __restrict__ twfy,
                                                   const int blk) {
  extern __shared__ float2 sh[];
  const int Mx = g.M[0], My = g.M[1], Hx = Mx / 2 + 1, Ny = g.N[1];
  const int pairs = (Ny + 1) / 2;
  const int cap = max(pairs * Mx, Hx * My);
  float2* twx = sh;
  float2* twy = twx + Mx;
  float2* A = twy + My;
  float2* Bf = A + cap;
  for (int i = threadIdx.x; i < Mx; i += blockDim.x) twx[i] = twfx[i];
  for (int i = threadIdx.x; i < My; i += blockDim.x) twy[i] = twfy[i];
  const int z = blk;
  for (int idx = threadIdx.x; idx < My * Hx; idx += blockDim.x) {
    const int ky = idx / Hx, kx = idx - ky * Hx;
    A[kx * My + ky] = spec[((int64_t)z * My + ky) * Hx + kx];
  }
  __syncthreads();
  const float2* R = lds_fft_mr(A, Bf, My, Hx, My, twy, -1.0f);
  float2* L = R == A ? Bf : A;
  float2* D = R == A ? A : Bf;
  // Z = X_y + i X_{y+1} over the full line, X[k] = conj X[Mx - k] for k >= Hx
  for (int idx = threadIdx.x; idx < pairs * Mx; idx += blockDim.x) {
    const int l = idx / Mx, k = idx - l * Mx, y = 2 * l;
    const int kk = k < Hx ? k : Mx - k;
    float2 a = R[kk * My + y];
    float2 b = make_float2(0.f, 0.f);
    if (y + 1 < Ny) b = R[kk * My + y + 1];
    if (k >= Hx) {
      a.y = -a.y;
      b.y = -b.y;
    }
    L[idx] = make_float2(a.x - b.y, a.y + b.x);
  }
  __syncthreads();
  const float2* S = lds_fft_mr(L, D, Mx, pairs, Mx, twx, -1.0f);
  for (int idx = threadIdx.x; idx < pairs * g.N[0]; idx += blockDim.x) {
    const int l = idx / g.N[0], x = idx - l * g.N[0], y = 2 * l;
    const float2 v = S[l * Mx + x];
    grid_store(U, ((int64_t)z * Ny + y) * g.N[0] + x, v.x, g);
    if (y + 1 < Ny) grid_store(U, ((int64_t)z * Ny + y + 1) * g.N[0] + x, v.y, g);
  }
}

__global__ void __launch_bounds__(512) k_fft_xy_fwd_mr(GridParams g, const float* __restrict__ Q,
                                                       float2* __restrict__ spec,
                                                       const float2* __restrict__ twfx,
                                                       const float2* __restrict__ twfy) {
  fft_xy_fwd_mr_body(g, Q, spec, twfx, twfy, blockIdx.x);
}

__global__ void __launch_bounds__(512) k_fft_yx_inv_mr(GridParams g,
                                                       const float2* __restrict__ spec,
                                                       float* __restrict__ U,
                                                       const float2* __restrict__ twfx,
                                                       const float2* __restrict__ twfy) {
  fft_yx_inv_mr_body(g, spec, U, twfx, twfy, blockIdx.x);
}

__global__ void __launch_bounds__(512) k_fft_xy_fwd_mr_cells(const CellTab* __restrict__ tab,
                                                             const int32_t* __restrict__ bcell,
                                                             const int32_t* __restrict__ boff) {
  const int c = bcell[blockIdx.x];
  const CellTab& t = tab[c];
  fft_xy_fwd_mr_body(t.g, t.grid, t.spec, t.twfx, t.twfy, blockIdx.x - boff[c]);
}

__global__ void __launch_bounds__(512) k_fft_yx_inv_mr_cells(const CellTab* __restrict__ tab,
                                                             const int32_t* __restrict__ bcell,
                                                             const int32_t* __restrict__ boff) {
  const int c = bcell[blockIdx.x];
  const CellTab& t = tab[c];
  fft_yx_inv_mr_body(t.g, t.spec, t.grid, t.twfx, t.twfy, blockIdx.x - boff[c]);
}

// R2C along x, mixed radix: as k_r2c_x (pairs of real rows y, y + 1 as one
// complex line, half spectrum of each), LDS: twiddles [Mx], two line buffers.
__device__ __forceinline__ void r2c_x_mr_body(GridParams g, const float* __restrict__ Q,
                                              float2* __restrict__ spec,
                                              const float2* __restrict__ twf,
                                              int lines_per_block, const int blk) {
  extern __shared__ float2 sh[];
  const int Mx = g.M[0], Hx = Mx / 2 + 1;
  float2* tw = sh;
  float2* A = sh + Mx;
  float2* Bf = A + lines_per_block * Mx;
  for (int i = threadIdx.x; i < Mx; i += blockDim.x) tw[i] = twf[i];
  const int pairs = (g.N[1] + 1) / 2;
  const int64_t total_lines = (int64_t)pairs * g.N[2];
  const int64_t l0 = (int64_t)blk * lines_per_block;
  const int nl = (int)((total_lines - l0) < lines_per_block ? (total_lines - l0) : lines_per_block);
  for (int idx = threadIdx.x; idx < nl * Mx; idx += blockDim.x) {
    const int li = idx / Mx, x = idx - li * Mx;
    const int64_t L = l0 + li;
    const int z = (int)(L / pairs), y = 2 * (int)(L % pairs);
    float re = 0.f, im = 0.f;
    if (x < g.N[0]) {
      re = grid_load(Q, ((int64_t)z * g.N[1] + y) * g.N[0] + x, g);
      if (y + 1 < g.N[1]) im = grid_load(Q, ((int64_t)z * g.N[1] + y + 1) * g.N[0] + x, g);
    }
    A[li * Mx + x] = make_float2(re, im);
  }
  __syncthreads();
  const float2* R = lds_fft_mr(A, Bf, Mx, nl, Mx, tw, 1.0f);
  for (int idx = threadIdx.x; idx < nl * Hx; idx += blockDim.x) {
    const int li = idx / Hx, k = idx - li * Hx;
    const int64_t L = l0 + li;
    const int z = (int)(L / pairs), y = 2 * (int)(L % pairs);
    const float2 a = R[li * Mx + k];
    const float2 b = R[li * Mx + (k == 0 ? 0 : Mx - k)];
    // X_y = (Z[k] + conj Z[-k]) / 2, X_{y+1} = (Z[k] - conj Z[-k]) / (2i)
    spec[((int64_t)z * g.M[1] + y) * Hx + k] = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));
    if (y + 1 < g.N[1])
      spec[((int64_t)z * g.M[1] + y + 1) * Hx + k] =
          make_float2(0.5f * (a.y + b.y), -0.5f * (a.x - b.x));
  }
}

__global__ void __launch_bounds__(256) k_r2c_x_mr(GridParams g, const float* __restrict__ Q,
                                                  float2* __restrict__ spec,
                                                  const float2* __restrict__ twf,
                                                  int lines_per_block) {
  r2c_x_mr_body(g, Q, spec, twf, lines_per_block, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_r2c_x_mr_cells(const CellTab* __restrict__ tab,
                                                        const int32_t* __restrict__ bcell,
                                                        const int32_t* __restrict__ boff) {
  const int c = bcell[blockIdx.x];
  const CellTab& t = tab[c];
  r2c_x_mr_body(t.g, t.grid, t.spec, t.twfx, t.lpb, blockIdx.x - boff[c]);
}

// FFT along y, mixed radix, as k_fft_y (B columns kx per block)
__device__ __forceinline__ void fft_y_mr_body(GridParams g, float2* __restrict__ spec,
                                              const float2* __restrict__ twf, int B, int inverse,
                                              int n_in, int n_out, const int blk) {
  extern __shared__ float2 sh[];
  const int My = g.M[1], Hx = g.M[0] / 2 + 1;
  float2* tw = sh;
  float2* A = sh + My;
  float2* Bf = A + B * My;
  for (int i = threadIdx.x; i < My; i += blockDim.x) tw[i] = twf[i];
  const int groups_per_plane = (Hx + B - 1) / B;
  const int z = blk / groups_per_plane;
  const int kx0 = (blk - z * groups_per_plane) * B;
  const int nb = (Hx - kx0) < B ? (Hx - kx0) : B;
  for (int idx = threadIdx.x; idx < nb * My; idx += blockDim.x) {
    const int y = idx / nb, li = idx - y * nb;
    float2 v = make_float2(0.f, 0.f);
    if (y < n_in) v = spec[((int64_t)z * My + y) * Hx + kx0 + li];
    A[li * My + y] = v;
  }
  __syncthreads();
  const float2* R = lds_fft_mr(A, Bf, My, nb, My, tw, inverse ? -1.0f : 1.0f);
  for (int idx = threadIdx.x; idx < nb * n_out; idx += blockDim.x) {
    const int y = idx / nb, li = idx - y * nb;
    spec[((int64_t)z * My + y) * Hx + kx0 + li] = R[li * My + y];
  }
}

__global__ void __launch_bounds__(256) k_fft_y_mr(GridParams g, float2* __restrict__ spec,
                                                  const float2* __restrict__ twf, int B,
                                                  int inverse, int n_in, int n_out) {
  fft_y_mr_body(g, spec, twf, B, inverse, n_in, n_out, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_fft_y_mr_cells(const CellTab* __restrict__ tab,
                                                        const int32_t* __restrict__ bcell,
                                                        const int32_t* __restrict__ boff,
                                                        int inverse) {
  const int c = bcell[blockIdx.x];
  const CellTab& t = tab[c];
  const int ny = t.g.N[1], my = t.g.M[1];
  fft_y_mr_body(t.g, t.spec, t.twfy, t.by, inverse, inverse ? my : ny, inverse ? ny : my,
                blockIdx.x - boff[c]);
}

// FFT along z, K multiply, inverse FFT along z, mixed radix, as k_fft_z_mul
__device__ __forceinline__ void fft_z_mul_mr_body(GridParams g, float2* __restrict__ spec,
                                                  const float* __restrict__ khat,
                                                  const float2* __restrict__ twf, int B,
                                                  const int blk) {
  extern __shared__ float2 sh[];
  const int Mz = g.M[2], Hx = g.M[0] / 2 + 1;
  const int64_t plane = (int64_t)g.M[1] * Hx;
  float2* tw = sh;
  float2* A = sh + Mz;
  float2* Bf = A + B * Mz;
  for (int i = threadIdx.x; i < Mz; i += blockDim.x) tw[i] = twf[i];
  const int64_t c0 = (int64_t)blk * B;
  const int nb = (int)((plane - c0) < B ? (plane - c0) : B);
  for (int idx = threadIdx.x; idx < nb * Mz; idx += blockDim.x) {
    const int z = idx / nb, li = idx - z * nb;
    A[li * Mz + z] = z < g.N[2] ? spec[(int64_t)z * plane + c0 + li] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  float2* F = lds_fft_mr(A, Bf, Mz, nb, Mz, tw, 1.0f);
  float2* other = F == A ? Bf : A;
  for (int idx = threadIdx.x; idx < nb * Mz; idx += blockDim.x) {
    const int kz = idx / nb, li = idx - kz * nb;
    const float kk = khat[(int64_t)kz * plane + c0 + li];
    const float2 v = F[li * Mz + kz];
    F[li * Mz + kz] = make_float2(v.x * kk, v.y * kk);  // same element, same thread
  }
  __syncthreads();
  const float2* R = lds_fft_mr(F, other, Mz, nb, Mz, tw, -1.0f);
  for (int idx = threadIdx.x; idx < nb * g.N[2]; idx += blockDim.x) {
    const int z = idx / nb, li = idx - z * nb;
    spec[(int64_t)z * plane + c0 + li] = R[li * Mz + z];
  }
}

__global__ void __launch_bounds__(256) k_fft_z_mul_mr(GridParams g, float2* __restrict__ spec,
                                                      const float* __restrict__ khat,
                                                      const float2* __restrict__ twf, int B) {
  fft_z_mul_mr_body(g, spec, khat, twf, B, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_fft_z_mul_mr_cells(const CellTab* __restrict__ tab,
                                                            const int32_t* __restrict__ bcell,
                                                            const int32_t* __restrict__ boff,
                                                            int B) {
  const int c = bcell[blockIdx.x];
  const CellTab& t = tab[c];
  fft_z_mul_mr_body(t.g, t.spec, t.khat, t.twfz, B, blockIdx.x - boff[c]);
}

// C2R along x, mixed radix, as k_c2r_x
__device__ __forceinline__ void c2r_x_mr_body(GridParams g, const float2* __restrict__ spec,
                                              float* __restrict__ U,
                                              const float2* __restrict__ twf,
                                              int lines_per_block, const int blk) {
  extern __shared__ float2 sh[];
  const int Mx = g.M[0], Hx = Mx / 2 + 1;
  float2* tw = sh;
  float2* A = sh + Mx;
  float2* Bf = A + lines_per_block * Mx;
  for (int i = threadIdx.x; i < Mx; i += blockDim.x) tw[i] = twf[i];
  const int pairs = (g.N[1] + 1) / 2;
  const int64_t total_lines = (int64_t)pairs * g.N[2];
  const int64_t l0 = (int64_t)blk * lines_per_block;
  const int nl = (int)((total_lines - l0) < lines_per_block ? (total_lines - l0) : lines_per_block);
  for (int idx = threadIdx.x; idx < nl * Mx; idx += blockDim.x) {
    const int li = idx / Mx, k = idx - li * Mx;
    const int64_t L = l0 + li;
    const int z = (int)(L / pairs), y = 2 * (int)(L % pairs);
    const int kk = k < Hx ? k : Mx - k;
    float2 a = spec[((int64_t)z * g.M[1] + y) * Hx + kk];
    float2 b = make_float2(0.f, 0.f);
    if (y + 1 < g.N[1]) b = spec[((int64_t)z * g.M[1] + y + 1) * Hx + kk];
    if (k >= Hx) {
      a.y = -a.y;
      b.y = -b.y;
    }
    // Z = X_y + i X_{y+1}
    A[li * Mx + k] = make_float2(a.x - b.y, a.y + b.x);
  }
  __syncthreads();
  const float2* R = lds_fft_mr(A, Bf, Mx, nl, Mx, tw, -1.0f);
  for (int idx = threadIdx.x; idx < nl * g.N[0]; idx += blockDim.x) {
    const int li = idx / g.N[0], x = idx - li * g.N[0];
    const int64_t L = l0 + li;
    const int z = (int)(L / pairs), y = 2 * (int)(L % pairs);
    const float2 v = R[li * Mx + x];
    grid_store(U, ((int64_t)z * g.N[1] + y) * g.N[0] + x, v.x, g);
    if (y + 1 < g.N[1]) grid_store(U, ((int64_t)z * g.N[1] + y + 1) * g.N[0] + x, v.y, g);
  }
}

__global__ void __launch_bounds__(256) k_c2r_x_mr(GridParams g, const float2* __restrict__ spec,
                                                  float* __restrict__ U,
                                                  const float2* __restrict__ twf,
                                                  int lines_per_block) {
  c2r_x_mr_body(g, spec, U, twf, lines_per_block, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_c2r_x_mr_cells(const CellTab* __restrict__ tab,
                                                        const int32_t* __restrict__ bcell,
                                                        const int32_t* __restrict__ boff) {
  const int c = bcell[blockIdx.x];
  const CellTab& t = tab[c];
  c2r_x_mr_body(t.g, t.spec, t.grid, t.twfx, t.lpb, blockIdx.x - boff[c]);
}

// ---------------------------------------------------------------------------
// interpolation + precorrection (steps 3 and 4), tile form. A workgroup
// takes the observer boxes x in [x0, x0 + xs), y = by, z in [z0, z0 + tz).
// Every source box their near regions touch lies in the block
//   x in [x0 - r_b, x0 + xs + r_b), y in [by - r_b, by + r_b],
//   z in [z0 - r_b, z0 + tz + r_b)
// whose nodes are listed on the host column-major: x box column outermost,
// then z, then y, then node order (the box table is fixed, so the list is
// built once). The workgroup stages the charges of its list in LDS. The
// precorrection values of every row are stored in the matching order (x
// offset, then z, then y), so the near columns of a row are 2 r_b + 1
// contiguous runs of the staged charges, one per x offset; each row carries
// the (start, length) of its runs. The (p + 1) y-lines of U over the tile's z
// range are staged too. Each group of G lanes then takes one observer row:
// u_n = W_n U + sum over the runs of P q + u_Z, in a fixed order.
//
// A row's values are one padded array (each run rounded up to 4 values with
// zeros), read as 4-value chunks: lane l of the group takes chunks l, l + G,
// ..., the first KC of them held in registers at once, so the lanes stay busy
// whatever the run lengths are; a chunk finds its run from the cumulative
// chunk counts of the row.

// five waves per SIMD (at most 96 registers) where the row state fits them
// without spilling, else four
#define PMFEM_IC_OCC __attribute__((amdgpu_waves_per_eu(WT * KC <= 30 ? 5 : 4)))
template <int WT, int KC>
__device__ __forceinline__ void interp_tile_body(
    GridParams g, IcPlan pl, const float* __restrict__ U, const float4* __restrict__ pos4,
    const int32_t* __restrict__ list, const int32_t* __restrict__ lstart,
    const int32_t* __restrict__ wseg, const uint32_t* __restrict__ rdesc,
    const int32_t* __restrict__ prp, const float* __restrict__ pval,
    const float* __restrict__ q, const float* __restrict__ uz, float* __restrict__ u, const int blk) {
  extern __shared__ float4 smem4[];
  unsigned char* smem = reinterpret_cast<unsigned char*>(smem4);
  float* s_q = reinterpret_cast<float*>(smem + pl.o_q);   // staged charges
  float* s_U = reinterpret_cast<float*>(smem + pl.o_u);   // [uzl][p + 1][ux]
  int* s_seg = reinterpret_cast<int*>(smem + pl.o_seg);   // [tz + 1] row prefix, [tz] first row
  const int tid = threadIdx.x, T = blockDim.x;
  const int nby = g.nbox[1];
  const int p = g.p, p1 = p + 1;
  const int w = blk;
  const int sx = w % pl.nsx, rest = w / pl.nsx;
  const int by = rest % nby, sz = rest / nby;
  const int x0 = sx * pl.xs, z0 = sz * pl.tz;
  const int tz = min(pl.tz, g.nbox[2] - z0);
  // [0, pl.tz]: row prefix over the z segments; [pl.tz + 1, 2 pl.tz]: first row of each
  const int segw = 2 * pl.tz + 1;
  for (int i = tid; i < segw; i += T) s_seg[i] = wseg[(int64_t)w * segw + i];
  const int l0 = lstart[w];
  const int n = min(lstart[w + 1] - l0, pl.qcap);
  // the first list entries are requested before the potential lines are
  // staged, so that both wait on memory together
  constexpr int KQ = 8;
  int gi[KQ];
#pragma unroll
  for (int j = 0; j < KQ; ++j) gi[j] = tid + j * T < n ? list[l0 + tid + j * T] : 0;
  // stencil lines of U: z-lines [stz(z0), stz(z0) + tz + p), y-lines [sty, sty + p]
  const int ux0 = box_stencil_start(x0, g.N[0], p, g.per[0]);
  const int sty = box_stencil_start(by, g.N[1], p, g.per[1]);
  const int stz = box_stencil_start(z0, g.N[2], p, g.per[2]);
  {
    // thread -> one x point t of the lines l = l00, l00 + lpp, ... (lpp whole
    // lines per pass); y and z follow l incrementally, so no division per value
    const int Nx = g.N[0], Ny = g.N[1], Nz = g.N[2];
    const int ux = pl.ux, nl = pl.uzl * p1, lpp = T / ux;
    const int l00 = tid / ux, t = tid - l00 * ux;
    if (l00 < lpp) {
      // a periodic line wraps at most once (ux, p + 1 and uzl never exceed N)
      int x = ux0 + t;
      if (g.per[0]) x = x < 0 ? x + Nx : (x >= Nx ? x - Nx : x);
      const bool okx = x < Nx;
      const int wy = g.per[1] ? Ny : 0, wz = g.per[2] ? Nz : 0;
      const int dly = lpp % p1, dlz = lpp / p1;
      int ly = l00 % p1, lz = l00 / p1;
      constexpr int KU = 8;
      for (int l0 = l00; l0 < nl; l0 += KU * lpp) {
        float v[KU];
#pragma unroll
        for (int k = 0; k < KU; ++k) {
          int y = sty + ly, z = stz + lz;
          y += y < 0 ? wy : 0;
          y -= y >= Ny ? wy : 0;
          z += z < 0 ? wz : 0;
          z -= z >= Nz ? wz : 0;
          const bool ok = okx && z < Nz && l0 + k * lpp < nl;
          v[k] = ok ? grid_load(U, (int64_t)(z * Ny + y) * Nx + x, g) : 0.f;
          ly += dly;
          lz += dlz;
          if (ly >= p1) {
            ly -= p1;
            ++lz;
          }
        }
#pragma unroll
        for (int k = 0; k < KU; ++k)
          if (l0 + k * lpp < nl) s_U[(l0 + k * lpp) * ux + t] = v[k];
      }
    }
  }
  // stage the listed charges, KQ loads in flight, the next list entries
  // requested while the charges arrive; 4 zeros after them
  if (tid < 4) s_q[n + tid] = 0.f;
  for (int e0 = tid; e0 < n; e0 += KQ * T) {
    float v[KQ];
#pragma unroll
    for (int j = 0; j < KQ; ++j) v[j] = q[gi[j]];
    const int e1 = e0 + KQ * T;
#pragma unroll
    for (int j = 0; j < KQ; ++j) gi[j] = e1 + j * T < n ? list[l0 + e1 + j * T] : 0;
#pragma unroll
    for (int j = 0; j < KQ; ++j)
      if (e0 + j * T < n) s_q[e0 + j * T] = v[j];
  }
  __syncthreads();
  const int nrows = s_seg[tz];
  const int* s_first = s_seg + pl.tz + 1;

  // rows: G lanes per row; the next row's descriptors are fetched while the
  // current row is formed
  constexpr int G = kIcLanes;
  constexpr int W = WT;                 // 2 r_b + 1
  const int lane = tid & (G - 1), grp = tid / G, ngrp = T / G;
  const bool cubic = p == 3;
  // lane-constant parts of the interpolation weights (p = 3): lane -> x point
  // ax = lane % 4 and the NY = 16 / G y points from ay0 = NY (lane / 4)
  constexpr int NY = 16 / G;
  const int ax = lane & 3, ay0 = (lane >> 2) * NY;
  const Cubic cbx = cubic_basis(ax);
  Cubic cby[NY];
#pragma unroll
  for (int i = 0; i < NY; ++i) cby[i] = cubic_basis(ay0 + i);
  // slot sl of the tile -> its row: segment kz by bisection over the prefix
  // (pl.tz is a power of two; prefix entries past the tile equal nrows)
  auto fetch = [&](int sl, uint32_t* dsc, int& pp, float4& xi, int& r) {
    int kz = 0;
    for (int s = pl.tz >> 1; s > 0; s >>= 1) kz = s_seg[kz + s] <= sl ? kz + s : kz;
    r = s_first[kz] + (sl - s_seg[kz]);
#pragma unroll
    for (int dx = 0; dx < W; ++dx) dsc[dx] = rdesc[(int64_t)r * W + dx];
    pp = prp[r];
    xi = pos4[r];
  };
  uint32_t dsc[W];
  int pp = 0, r = 0;
  float4 xi = make_float4(0.f, 0.f, 0.f, 0.f);
  if (grp < nrows) fetch(grp, dsc, pp, xi, r);
  for (int sl = grp; sl < nrows; sl += ngrp) {
    // cumulative chunk counts cb of the runs and the staged index of chunk j
    // of run d, qb_d + 4 j with qb_d = start_d - 4 cb_d, kept as qb_0 and the
    // steps dq_d = qb_d - qb_(d-1) (a sum of selects, not an indexed array)
    int cb[W + 1], dq[W];
    cb[0] = 0;
    int qprev = 0;
#pragma unroll
    for (int d = 0; d < W; ++d) {
      const int qbd = (int)(dsc[d] & 0xFFFFu) - 4 * cb[d];
      dq[d] = qbd - qprev;
      qprev = qbd;
      cb[d + 1] = cb[d] + (((int)(dsc[d] >> 16) + 3) >> 2);
    }
    const int C = cb[W];
    // the first KC chunks of every lane in flight at once; a chunk past the
    // row reads valid (finite) values of the next rows, or the zeros that pad
    // the matrix, and pairs them with the zeros after the staged charges
    const float4* prow = reinterpret_cast<const float4*>(pval + pp) + lane;
    float4 v[KC];
#pragma unroll
    for (int t = 0; t < KC; ++t) v[t] = prow[G * t];
    uint32_t dn[W];
    int ppn = 0, rn = 0;
    float4 xin = make_float4(0.f, 0.f, 0.f, 0.f);
    if (sl + ngrp < nrows) fetch(sl + ngrp, dn, ppn, xin, rn);
    float acc = 0.f;
    // padding values are zero and 4 zeros follow the staged charges, so the
    // 4 products of a chunk need no per-value test
    auto chunk = [&](int j, const float4& pv) {
      int b = dq[0] + 4 * j;
#pragma unroll
      for (int d = 1; d < W; ++d) b += j >= cb[d] ? dq[d] : 0;
      const float* sq = s_q + (j < C ? b : n);
      acc = fmaf(pv.x, sq[0], acc);
      acc = fmaf(pv.y, sq[1], acc);
      acc = fmaf(pv.z, sq[2], acc);
      acc = fmaf(pv.w, sq[3], acc);
    };
#pragma unroll
    for (int t = 0; t < KC; ++t) chunk(lane + G * t, v[t]);
    for (int j = lane + G * KC; j < C; j += G) chunk(j, prow[j - lane]);
    // W U from the staged lines; the box of the row from its packed coordinates
    const uint32_t bc = __float_as_uint(xi.w);
    const int bx = (int)(bc & 1023u), bz = (int)((bc >> 20) & 1023u);
    const int relx = g.per[0] ? bx - x0 : box_stencil_start(bx, g.N[0], p, 0) - ux0;
    const int relz = g.per[2] ? bz - z0 : box_stencil_start(bz, g.N[2], p, 0) - stz;
    if (cubic) {
      const int zs = p1 * pl.ux;
      const float* su = s_U + (relz * p1 + ay0) * pl.ux + relx + ax;
      const float wz0 = cubic_eval(cubic_basis(0), xi.z), wz1 = cubic_eval(cubic_basis(1), xi.z);
      const float wz2 = cubic_eval(cubic_basis(2), xi.z), wz3 = cubic_eval(cubic_basis(3), xi.z);
      float sy = 0.f;
#pragma unroll
      for (int i = 0; i < NY; ++i) {
        const float* s0 = su + i * pl.ux;
        const float t = wz0 * s0[0] + wz1 * s0[zs] + wz2 * s0[2 * zs] + wz3 * s0[3 * zs];
        sy = fmaf(cubic_eval(cby[i], xi.y), t, sy);
      }
      acc = fmaf(cubic_eval(cbx, xi.x), sy, acc);
    } else {
      const int nst = p1 * p1 * p1;
      for (int l = lane; l < nst; l += G) {
        const int lx = l % p1, ly = (l / p1) % p1, lz = l / (p1 * p1);
        acc = fmaf(lagrange(lx, xi.x, p) * lagrange(ly, xi.y, p) * lagrange(lz, xi.z, p),
                   s_U[((relz + lz) * p1 + ly) * pl.ux + relx + lx], acc);
      }
    }
    acc = group_sum<G>(acc);
    if (lane == 0) u[r] = acc + uz[r];
#pragma unroll
    for (int dx = 0; dx < W; ++dx) dsc[dx] = dn[dx];
    pp = ppn;
    xi = xin;
    r = rn;
  }
}

template <int WT, int KC>
__global__ void __launch_bounds__(256) PMFEM_IC_OCC k_interp_tile(
    GridParams g, IcPlan pl, const float* __restrict__ U, const float4* __restrict__ pos4,
    const int32_t* __restrict__ list, const int32_t* __restrict__ lstart,
    const int32_t* __restrict__ wseg, const uint32_t* __restrict__ rdesc,
    const int32_t* __restrict__ prp, const float* __restrict__ pval,
    const float* __restrict__ q, const float* __restrict__ uz, float* __restrict__ u) {
  interp_tile_body<WT, KC>(g, pl, U, pos4, list, lstart, wseg, rdesc, prp, pval, q, uz, u,
                           blockIdx.x);
}

template <int WT, int KC>
__global__ void __launch_bounds__(256) PMFEM_IC_OCC k_interp_tile_cells(
    const CellTab* __restrict__ tab, const int32_t* __restrict__ bcell,
    const int32_t* __restrict__ boff) {
  const int c = bcell[blockIdx.x];
  const CellTab& t = tab[c];
  interp_tile_body<WT, KC>(t.g, t.icp, t.grid, t.pos4, t.ic_list, t.ic_lstart, t.ic_wseg,
                           t.ic_rdesc, t.prp, t.pv, t.q, t.uz, t.u, blockIdx.x - boff[c]);
}

#define PMFEM_INTERP_TILE(WT, KC)                                                             \
  template __global__ void k_interp_tile<WT, KC>(                                             \
      GridParams, IcPlan, const float*, const float4*, const int32_t*, const int32_t*,        \
      const int32_t*, const uint32_t*, const int32_t*, const float*, const float*, const float*, \
      float*);                                                                                \
  template __global__ void k_interp_tile_cells<WT, KC>(const CellTab*, const int32_t*,        \
                                                       const int32_t*);
#define PMFEM_INTERP_TILES(WT) \
  PMFEM_INTERP_TILE(WT, 2)     \
  PMFEM_INTERP_TILE(WT, 4)     \
  PMFEM_INTERP_TILE(WT, 6)     \
  PMFEM_INTERP_TILE(WT, 8)
PMFEM_INTERP_TILES(1)
PMFEM_INTERP_TILES(3)
PMFEM_INTERP_TILES(5)
PMFEM_INTERP_TILES(7)
#undef PMFEM_INTERP_TILE

// ---------------------------------------------------------------------------
// exchange and gradient over the shared local pattern, G lanes per row:
//   k_exch:  H_ex,n = sum_k L_nk (m_k - m_n)         (records {col, L})
//   k_gsum:  H_n = H_ex,n - sum_k G_nk u_k + H_applied  (records {col, Gx, Gy, Gz})
// The exchange needs only m, so the library runs it on the second stream
// beside the grid steps; k_gsum then adds the magnetostatic gradient.

template <int G, typename MT>
__global__ void __launch_bounds__(256) k_exch(int64_t n, const int32_t* __restrict__ rp,
                                              const int2* __restrict__ lrec,
                                              const MT* __restrict__ m,
                                              float* __restrict__ hex) {
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int lane = threadIdx.x & (G - 1);
  if (row >= n) return;  // whole groups leave together
  // difference form: the rows of L sum to zero (constants are in its null
  // space), so H_ex,n = sum_k L_nk (m_k - m_n); a uniform m gives exactly
  // zero and the FP32 rounding scales with the variation of m, not with m.
  // With an FP64 m (MT = double) the differences are formed before the one
  // rounding to FP32, so the rounding of m itself, which the exchange
  // operator would amplify by its largest eigenvalue, never enters.
  const MT* mn = m + 3 * row;
  const MT n0 = mn[0], n1 = mn[1], n2 = mn[2];
  float hx = 0.f, hy = 0.f, hz = 0.f;
  row_entries<G, 4>(rp[row], rp[row + 1], lane, lrec, [&](const int2& r, bool ok) {
    const MT* mk = m + 3 * (int64_t)r.x;
    const float d0 = (float)(mk[0] - n0), d1 = (float)(mk[1] - n1), d2 = (float)(mk[2] - n2);
    const float w = ok ? __int_as_float(r.y) : 0.f;
    hx = fmaf(w, d0, hx);
    hy = fmaf(w, d1, hy);
    hz = fmaf(w, d2, hz);
  });
  hx = group_sum<G>(hx);
  hy = group_sum<G>(hy);
  hz = group_sum<G>(hz);
  if (lane == 0) {
    hex[3 * row] = hx;
    hex[3 * row + 1] = hy;
    hex[3 * row + 2] = hz;
  }
}

template <int G>
__global__ void __launch_bounds__(256) k_gsum(int64_t n, const int32_t* __restrict__ rp,
                                              const int4* __restrict__ grec,
                                              const float* __restrict__ u,
                                              const float* __restrict__ hex,
                                              float* __restrict__ h, float hax, float hay,
                                              float haz, int with_hex, int with_ms) {
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const int lane = threadIdx.x & (G - 1);
  if (row >= n) return;  // whole groups leave together
  float hx = 0.f, hy = 0.f, hz = 0.f;
  if (with_ms) {
    row_entries<G, 4>(rp[row], rp[row + 1], lane, grec, [&](const int4& r, bool ok) {
      const float uv = u[r.x];
      const float uk = ok ? uv : 0.f;
      hx = fmaf(-__int_as_float(r.y), uk, hx);
      hy = fmaf(-__int_as_float(r.z), uk, hy);
      hz = fmaf(-__int_as_float(r.w), uk, hz);
    });
    hx = group_sum<G>(hx);
    hy = group_sum<G>(hy);
    hz = group_sum<G>(hz);
  }
  if (lane == 0) {
    if (with_hex) {
      hx += hex[3 * row];
      hy += hex[3 * row + 1];
      hz += hex[3 * row + 2];
    }
    h[3 * row] = hx + hax;
    h[3 * row + 1] = hy + hay;
    h[3 * row + 2] = hz + haz;
  }
}

#define PMFEM_LOCAL_KERNELS(G)                                                                  \
  template __global__ void k_exch<G, float>(int64_t, const int32_t*, const int2*, const float*,   \
                                            float*);                                             \
  template __global__ void k_exch<G, double>(int64_t, const int32_t*, const int2*, const double*, \
                                             float*);                                            \
  template __global__ void k_gsum<G>(int64_t, const int32_t*, const int4*, const float*,         \
                                     const float*, float*, float, float, float, int, int);
PMFEM_LOCAL_KERNELS(4)
PMFEM_LOCAL_KERNELS(8)
PMFEM_LOCAL_KERNELS(16)
#undef PMFEM_LOCAL_KERNELS

// ---------------------------------------------------------------------------
// LLG (unit-vector Landau-Lifshitz form), classic RK4 in FP64

__global__ void k_rk_stage(int64_t n, const double* __restrict__ m, const double* __restrict__ k,
                           double c, double* __restrict__ mst, float* __restrict__ m32) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * n) return;
  double v = m[i];
  if (k) v += c * k[i];
  if (mst) mst[i] = v;
  m32[i] = (float)v;
}

__global__ void k_rk_rhs(int64_t n, const double* __restrict__ mst, const float* __restrict__ h,
                         double pref, double alpha, double* __restrict__ kout,
                         double* __restrict__ acc, double weight, int first) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double mx = mst[3 * i], my = mst[3 * i + 1], mz = mst[3 * i + 2];
  double hx = h[3 * i], hy = h[3 * i + 1], hz = h[3 * i + 2];
  double cx = my * hz - mz * hy, cy = mz * hx - mx * hz, cz = mx * hy - my * hx;   // m x H
  double dx = my * cz - mz * cy, dy = mz * cx - mx * cz, dz = mx * cy - my * cx;   // m x (m x H)
  double kx = pref * (cx + alpha * dx), ky = pref * (cy + alpha * dy), kz = pref * (cz + alpha * dz);
  kout[3 * i] = kx;
  kout[3 * i + 1] = ky;
  kout[3 * i + 2] = kz;
  if (first) {
    acc[3 * i] = weight * kx;
    acc[3 * i + 1] = weight * ky;
    acc[3 * i + 2] = weight * kz;
  } else {
    acc[3 * i] += weight * kx;
    acc[3 * i + 1] += weight * ky;
    acc[3 * i + 2] += weight * kz;
  }
}

__global__ void k_rk_final(int64_t n, double* __restrict__ m, const double* __restrict__ acc,
                           double dt6) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = m[3 * i] + dt6 * acc[3 * i];
  double y = m[3 * i + 1] + dt6 * acc[3 * i + 1];
  double z = m[3 * i + 2] + dt6 * acc[3 * i + 2];
  double r = 1.0 / sqrt(x * x + y * y + z * z);
  m[3 * i] = x * r;
  m[3 * i + 1] = y * r;
  m[3 * i + 2] = z * r;
}

// energy partial sums: block b writes {sum mu m.Hex, sum q u}
// ---------------------------------------------------------------------------
// Implicit LLG steps (Sec. 2.2: implicit time stepping with a Newton
// iteration and a preconditioned Krylov solver). One step solves
//   G(x) = x - r - dt f(mb) = 0,   mb = (1 - theta) m + theta x,
//   f(v) = c [v x H(v) + alpha v x (v x H(v))],  c = -gamma0 / (1 + alpha^2),
// with r = m, theta = 1/2 for the midpoint rule and r a combination of past
// states, dt the step times the BDF coefficient, theta = 1 for BDF; by
// Newton, the linear systems dG/dx d = G by GMRES with the Jacobian applied
// matrix-free (the field is linear in m, H(v) = A v + H_app):
//   dG/dx w = w - theta dt c [w x H + mb x (A w)
//                            + alpha (w x (mb x H) + mb x (w x H) + mb x (mb x (A w)))].
// All vectors are FP64; A w is one FP32 field evaluation. (Below, "m" of
// the residual kernel is r.)

__device__ __forceinline__ void cross3(double ax, double ay, double az, double bx, double by,
                                       double bz, double& cx, double& cy, double& cz) {
  cx = ay * bz - az * by;
  cy = az * bx - ax * bz;
  cz = ax * by - ay * bx;
}

// the evaluation point mb = (1 - theta) m + theta x (theta = 1/2: the
// midpoint rule; theta = 1: BDF, mb = x) and its FP32 copy for the field
__global__ void k_mid_point(int64_t n3, const double* __restrict__ m, const double* __restrict__ x,
                            double theta, double* __restrict__ mb, float* __restrict__ mb32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  const double v = theta == 1.0 ? x[i] : (1.0 - theta) * m[i] + theta * x[i];
  mb[i] = v;
  mb32[i] = (float)v;
}

// Residual G at the field H of the evaluation point and, per node, the inverse of the 3x3
// diagonal block of dG/dx with A replaced by its exchange diagonal a_n
// (the block-inverse preconditioner); part[b] = block b's share of |G|^2,
// summed in a fixed order (grid-stride, then a tree in LDS).
__global__ void __launch_bounds__(256) k_mid_residual(int64_t n, const double* __restrict__ m,
                                                      const double* __restrict__ x,
                                                      const double* __restrict__ mb,
                                                      const float* __restrict__ H,
                                                      const double* __restrict__ adiag, double dt,
                                                      double c, double alpha, double theta,
                                                      double* __restrict__ G,
                                                      double* __restrict__ Minv,
                                                      double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double bx = mb[3 * i], by = mb[3 * i + 1], bz = mb[3 * i + 2];
    const double hx = H[3 * i], hy = H[3 * i + 1], hz = H[3 * i + 2];
    double px, py, pz, qx, qy, qz;
    cross3(bx, by, bz, hx, hy, hz, px, py, pz);   // mb x H
    cross3(bx, by, bz, px, py, pz, qx, qy, qz);   // mb x (mb x H)
    const double gx = x[3 * i] - m[3 * i] - dt * c * (px + alpha * qx);
    const double gy = x[3 * i + 1] - m[3 * i + 1] - dt * c * (py + alpha * qy);
    const double gz = x[3 * i + 2] - m[3 * i + 2] - dt * c * (pz + alpha * qz);
    G[3 * i] = gx;
    G[3 * i + 1] = gy;
    G[3 * i + 2] = gz;
    acc += gx * gx + gy * gy + gz * gz;
    // columns of the block: D e_k = e_k x H + a mb x e_k
    //   + alpha (e_k x (mb x H) + mb x (e_k x H) + a mb x (mb x e_k))
    const double a = adiag[i];
    double B[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double ex = k == 0, ey = k == 1, ez = k == 2;
      double t1x, t1y, t1z, t2x, t2y, t2z, t3x, t3y, t3z, t4x, t4y, t4z, t5x, t5y, t5z, ux, uy, uz;
      cross3(ex, ey, ez, hx, hy, hz, t1x, t1y, t1z);        // e x H
      cross3(bx, by, bz, ex, ey, ez, t2x, t2y, t2z);        // mb x e
      cross3(ex, ey, ez, px, py, pz, t3x, t3y, t3z);        // e x (mb x H)
      cross3(bx, by, bz, t1x, t1y, t1z, t4x, t4y, t4z);     // mb x (e x H)
      cross3(bx, by, bz, t2x, t2y, t2z, t5x, t5y, t5z);     // mb x (mb x e)
      ux = t1x + a * t2x + alpha * (t3x + t4x + a * t5x);
      uy = t1y + a * t2y + alpha * (t3y + t4y + a * t5y);
      uz = t1z + a * t2z + alpha * (t3z + t4z + a * t5z);
      const double s = -theta * dt * c;
      B[0][k] = (k == 0) + s * ux;
      B[1][k] = (k == 1) + s * uy;
      B[2][k] = (k == 2) + s * uz;
    }
    // inverse by the adjugate
    const double c00 = B[1][1] * B[2][2] - B[1][2] * B[2][1];
    const double c01 = B[1][2] * B[2][0] - B[1][0] * B[2][2];
    const double c02 = B[1][0] * B[2][1] - B[1][1] * B[2][0];
    const double det = B[0][0] * c00 + B[0][1] * c01 + B[0][2] * c02;
    const double r = 1.0 / det;
    double* Mi = Minv + 9 * i;
    Mi[0] = c00 * r;
    Mi[1] = (B[0][2] * B[2][1] - B[0][1] * B[2][2]) * r;
    Mi[2] = (B[0][1] * B[1][2] - B[0][2] * B[1][1]) * r;
    Mi[3] = c01 * r;
    Mi[4] = (B[0][0] * B[2][2] - B[0][2] * B[2][0]) * r;
    Mi[5] = (B[0][2] * B[1][0] - B[0][0] * B[1][2]) * r;
    Mi[6] = c02 * r;
    Mi[7] = (B[0][1] * B[2][0] - B[0][0] * B[2][1]) * r;
    Mi[8] = (B[0][0] * B[1][1] - B[0][1] * B[1][0]) * r;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// x / |x| per node (an accepted adaptive step: the rule keeps |m| only up to
// the Newton residual, which is an rms over all nodes, so a few nodes could
// otherwise drift over many steps)
__global__ void k_mid_normalize(int64_t n, double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = x[3 * i], b = x[3 * i + 1], c = x[3 * i + 2];
  const double r = 1.0 / sqrt(a * a + b * b + c * c);
  x[3 * i] = a * r;
  x[3 * i + 1] = b * r;
  x[3 * i + 2] = c * r;
}

// z = Minv v per node; z32 its FP32 copy (NULL: not written)
template <typename VT>
__global__ void k_mid_precond(int64_t n, const double* __restrict__ Minv,
                              const VT* __restrict__ v, double* __restrict__ z,
                              float* __restrict__ z32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* Mi = Minv + 9 * i;
  const double vx = (double)v[3 * i], vy = (double)v[3 * i + 1], vz = (double)v[3 * i + 2];
  const double a = Mi[0] * vx + Mi[1] * vy + Mi[2] * vz;
  const double b = Mi[3] * vx + Mi[4] * vy + Mi[5] * vz;
  const double d = Mi[6] * vx + Mi[7] * vy + Mi[8] * vz;
  z[3 * i] = a;
  z[3 * i + 1] = b;
  z[3 * i + 2] = d;
  if (z32) {
    z32[3 * i] = (float)a;
    z32[3 * i + 1] = (float)b;
    z32[3 * i + 2] = (float)d;
  }
}
template __global__ void k_mid_precond<double>(int64_t, const double*, const double*, double*,
                                               float*);
template __global__ void k_mid_precond<float>(int64_t, const double*, const float*, double*,
                                              float*);

// w = dG/dx z, with Az = A z from one FP32 field evaluation
__global__ void k_mid_jvp(int64_t n, const double* __restrict__ z, const float* __restrict__ Az,
                          const double* __restrict__ mb, const float* __restrict__ H, double s,
                          double alpha, double* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double bx = mb[3 * i], by = mb[3 * i + 1], bz = mb[3 * i + 2];
  const double hx = H[3 * i], hy = H[3 * i + 1], hz = H[3 * i + 2];
  const double zx = z[3 * i], zy = z[3 * i + 1], zz = z[3 * i + 2];
  const double ax = Az[3 * i], ay = Az[3 * i + 1], az = Az[3 * i + 2];
  double px, py, pz, t1x, t1y, t1z, t2x, t2y, t2z, t3x, t3y, t3z, t4x, t4y, t4z, t5x, t5y, t5z;
  cross3(bx, by, bz, hx, hy, hz, px, py, pz);          // mb x H
  cross3(zx, zy, zz, hx, hy, hz, t1x, t1y, t1z);       // z x H
  cross3(bx, by, bz, ax, ay, az, t2x, t2y, t2z);       // mb x (A z)
  cross3(zx, zy, zz, px, py, pz, t3x, t3y, t3z);       // z x (mb x H)
  cross3(bx, by, bz, t1x, t1y, t1z, t4x, t4y, t4z);    // mb x (z x H)
  cross3(bx, by, bz, t2x, t2y, t2z, t5x, t5y, t5z);    // mb x (mb x (A z))
  w[3 * i] = zx + s * (t1x + t2x + alpha * (t3x + t4x + t5x));
  w[3 * i + 1] = zy + s * (t1y + t2y + alpha * (t3y + t4y + t5y));
  w[3 * i + 2] = zz + s * (t1z + t2z + alpha * (t3z + t4z + t5z));
}

// Gram-Schmidt of the implicit solver's GMRES. The Krylov basis V is held
// in FP32 (its rounding, 6e-8 relative, lies below the relative residual
// GMRES is asked for, and each basis vector is one FP32 field evaluation's
// input anyway); w and every sum are FP64, each sum in a fixed order
// (grid-stride per thread, a fixed shuffle tree per wavefront, the four
// wavefronts in order, then k_sum_parts).
constexpr int kGsChunk = 16;

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  return v;
}

// part[j * gridDim.x + b] = block b's share of V_j . w for j < nv and of
// w . w for j = nv
__global__ void __launch_bounds__(256) k_gs_dots(int64_t n3, const float* __restrict__ V,
                                                 int64_t ldv, int nv, const double* __restrict__ w,
                                                 double* __restrict__ part) {
  __shared__ double red[4][kGsChunk];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int j0 = 0; j0 <= nv; j0 += kGsChunk) {
    const int jn = min(kGsChunk, nv + 1 - j0);
    double acc[kGsChunk];
#pragma unroll
    for (int k = 0; k < kGsChunk; ++k) acc[k] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3;
         i += (int64_t)gridDim.x * blockDim.x) {
      const double wi = w[i];
#pragma unroll
      for (int k = 0; k < kGsChunk; ++k) {
        const int j = j0 + k;
        if (k < jn) acc[k] = fma(j < nv ? (double)V[(int64_t)j * ldv + i] : wi, wi, acc[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < kGsChunk; ++k) {
      if (k < jn) {
        const double sv = wave_sum_d(acc[k]);
        if (lane == 0) red[wv][k] = sv;
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < jn)
      part[(int64_t)(j0 + threadIdx.x) * gridDim.x + blockIdx.x] =
          ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
    __syncthreads();
  }
}

// w -= sum_j h[j] V_j (j < nv, ascending); part[b] = block b's share of
// |w|^2 after the update
__global__ void __launch_bounds__(256) k_gs_update(int64_t n3, const float* __restrict__ V,
                                                   int64_t ldv, int nv,
                                                   const double* __restrict__ h,
                                                   double* __restrict__ w,
                                                   double* __restrict__ part) {
  __shared__ double hs[kGsMaxVectors];
  __shared__ double red[4];
  for (int t = threadIdx.x; t < nv; t += blockDim.x) hs[t] = h[t];
  __syncthreads();
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v = w[i];
    for (int j = 0; j < nv; ++j) v = fma(-hs[j], (double)V[(int64_t)j * ldv + i], v);
    w[i] = v;
    acc = fma(v, v, acc);
  }
  const double sv = wave_sum_d(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sv;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// out = (float)(s w)
__global__ void k_gs_store(int64_t n3, const double* __restrict__ w, double s,
                           float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n3) out[i] = (float)(s * w[i]);
}

// out = sum_j coef[j] V_j (j < nv, ascending)
__global__ void k_gs_combine(int64_t n3, const float* __restrict__ V, int64_t ldv, int nv,
                             const double* __restrict__ coef, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  double v = 0.0;
  for (int j = 0; j < nv; ++j) v = fma(coef[j], (double)V[(int64_t)j * ldv + i], v);
  out[i] = v;
}

// part[j * gridDim.x + b] = block b's share of V_j . w for j < nv (fixed
// order: grid-stride per thread, then a tree in LDS)
__global__ void __launch_bounds__(256) k_mdot(int64_t n3, const double* __restrict__ V,
                                              int64_t ldv, int nv, const double* __restrict__ w,
                                              double* __restrict__ part) {
  __shared__ double red[256];
  for (int j = 0; j < nv; ++j) {
    const double* Vj = V + (int64_t)j * ldv;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n3;
         i += (int64_t)gridDim.x * blockDim.x)
      acc = fma(Vj[i], w[i], acc);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)j * gridDim.x + blockIdx.x] = red[0];
    __syncthreads();
  }
}

// out[j] = sum over b < nparts of part[j * nparts + b], one block per j,
// fixed order
__global__ void __launch_bounds__(256) k_sum_parts(const double* __restrict__ part, int nparts,
                                                   double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x) acc += part[(int64_t)blockIdx.x * nparts + b];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// out = aw w + sum_j coef[j] V_j (j < nv); out may alias w
__global__ void k_lincomb(int64_t n3, const double* __restrict__ V, int64_t ldv, int nv,
                          const double* __restrict__ coef, double aw, const double* w,
                          double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  double v = aw != 0.0 ? aw * w[i] : 0.0;
  for (int j = 0; j < nv; ++j) v = fma(coef[j], V[(int64_t)j * ldv + i], v);
  out[i] = v;
}

__global__ void __launch_bounds__(256) k_energy(int64_t n, const double* __restrict__ m,
                                                const double* __restrict__ mu,
                                                const float* __restrict__ hex,
                                                const float* __restrict__ q,
                                                const float* __restrict__ u,
                                                double* __restrict__ part) {
  __shared__ double s0[256], s1[256];
  double a = 0.0, b = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    a += mu[i] * (m[3 * i] * hex[3 * i] + m[3 * i + 1] * hex[3 * i + 1] +
                  m[3 * i + 2] * hex[3 * i + 2]);
    b += (double)q[i] * (double)u[i];
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s0[threadIdx.x] += s0[threadIdx.x + o];
      s1[threadIdx.x] += s1[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s0[0];
    part[2 * blockIdx.x + 1] = s1[0];
  }
}

}  // namespace pmfem

// gfx950 kernels of the PM-FEM effective-field evaluation.
//
// One H_eff evaluation (paper Eqs. heff, hex, hms_d1 - hms_d3):
//   k_local        q = D m (Eq. hms_d1), u_Z = Z0 m (Eq. hms_d2b)
//   k_anterp       Q = W^T q                      (Sec. 3.2.2, step 1)
//   k_r2c_x        real-to-complex FFT along x    (step 2)
//   k_fft_y        FFT along y (forward)
//   k_fft_z_mul    FFT along z, multiply by the PGF spectrum, inverse along z
//   k_fft_y        FFT along y (inverse)
//   k_c2r_x        complex-to-real FFT along x -> U = (1/4 pi) K * Q
//   k_interp_corr  u = W U + P q + u_Z            (steps 3 and 4)
//   k_grad         H = L m - G u (+ H_applied)    (Eqs. hex/lapl_2, hms_d3)
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

template <int W>
__device__ __forceinline__ float group_sum(float v) {
  // butterfly sum over groups of W consecutive lanes (W divides 64)
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
  return v;
}

// ---------------------------------------------------------------------------
// charges and element-exact correction: 16 lanes per row
//   q_n   = sum_k D_nk . m_k          (local pattern, D stored as three arrays)
//   u_Z,n = sum_j Z0_nj . m_j          (element-correction pattern)

__global__ void __launch_bounds__(256) k_local(
    int64_t n, const float* __restrict__ m, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ col, const float* __restrict__ dx, const float* __restrict__ dy,
    const float* __restrict__ dz, const int32_t* __restrict__ zrp,
    const int32_t* __restrict__ zcol, const float* __restrict__ zx,
    const float* __restrict__ zy, const float* __restrict__ zz, float* __restrict__ q,
    float* __restrict__ uz) {
  int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  int lane = threadIdx.x & 15;
  if (row >= n) return;
  float qq = 0.f, uu = 0.f;
  const int e0 = rp[row], e1 = rp[row + 1];
  const int z0 = zrp[row], z1 = zrp[row + 1];
  for (int e = e0 + lane; e < e1; e += 16) {
    const int64_t k = col[e];
    qq += dx[e] * m[3 * k] + dy[e] * m[3 * k + 1] + dz[e] * m[3 * k + 2];
  }
  for (int e = z0 + lane; e < z1; e += 16) {
    const int64_t k = zcol[e];
    uu += zx[e] * m[3 * k] + zy[e] * m[3 * k + 1] + zz[e] * m[3 * k + 2];
  }
  qq = group_sum<16>(qq);
  uu = group_sum<16>(uu);
  if (lane == 0) {
    q[row] = qq;
    uz[row] = uu;
  }
}

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
    if (inside) Q[((int64_t)gz * g.N[1] + gy) * g.N[0] + gx] = 0.f;
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
  Q[((int64_t)gz * g.N[1] + gy) * g.N[0] + gx] = acc;
}

// ---------------------------------------------------------------------------
// anterpolation by grid lines. A workgroup takes `xa` consecutive points of
// one (y, z) grid line, one thread per point. The boxes whose stencils reach
// the line form at most (p + 1)^2 box rows; their nodes in the x-range of
// the segment are staged once in LDS with coalesced loads, each reduced to
// what the line needs: xi_x, its stencil start along x, and the product
// q L_ay(xi_y) L_az(xi_z) of its charge with its y and z weights at the
// line. Each thread then sums, row by row and in box order (a fixed order,
// no atomics), q L_ay L_az L_ax over the nodes of the boxes covering its
// point.

__device__ __forceinline__ float basis(int a, float xi, int p) {
  return p == 3 ? cubic_eval(cubic_basis(a), xi) : lagrange(a, xi, p);
}

__global__ void __launch_bounds__(256) k_anterp_line(
    GridParams g, AntPlan pl, const float* __restrict__ q, const float4* __restrict__ pos4,
    const int32_t* __restrict__ box_start, const int2* __restrict__ brx,
    const int2* __restrict__ bry, const int2* __restrict__ brz, float* __restrict__ Q) {
  extern __shared__ float4 smem4[];
  unsigned char* smem = reinterpret_cast<unsigned char*>(smem4);
  float* s_x = reinterpret_cast<float*>(smem + pl.o_x);
  float* s_c = reinterpret_cast<float*>(smem + pl.o_c);
  uint16_t* s_st = reinterpret_cast<uint16_t*>(smem + pl.o_st);
  int* s_base = reinterpret_cast<int*>(smem + pl.o_meta);  // nrow + 1
  int* s_c0 = s_base + (pl.nrow + 1);
  int* s_b0 = s_c0 + pl.nrow;
  int* s_tot = s_b0 + pl.nrow;
  int* s_ay = s_tot + pl.nrow;
  int* s_az = s_ay + pl.nrow;
  int* s_yz = s_az + pl.nrow;
  int* s_off = reinterpret_cast<int*>(smem + pl.o_off);  // nrow x (sbx + 1)
  const int tid = threadIdx.x;
  const int nbx = g.nbox[0], nby = g.nbox[1], nbz = g.nbox[2];
  const int sx = blockIdx.x % pl.nsx, line = blockIdx.x / pl.nsx;
  const int gy = line % g.N[1], gz = line / g.N[1];
  const int x0 = sx * pl.xa, xa = min(pl.xa, g.N[0] - x0);
  const int2 ry = bry[gy], rz = brz[gz];
  const int nrow = ry.y * rz.y;
  const int p = g.p, shift = (p - 1) / 2;
  // first staged box (unwrapped on a periodic x) and the staged box count
  const int2 fx = brx[x0], lxr = brx[x0 + xa - 1];
  const int fb = g.per[0] ? x0 - p + shift : fx.x;
  const int nbs = g.per[0] ? xa + p : lxr.x + lxr.y - fx.x;
  const int sb1 = pl.sbx + 1;
  // 1. box rows: by = ry.x + iy, bz = rz.x + iz (wrapped on periodic axes)
  if (tid < nrow) {
    const int iy = tid % ry.y, iz = tid / ry.y;
    int by = ry.x + iy, bz = rz.x + iz;
    if (by >= nby) by -= nby;
    if (bz >= nbz) bz -= nbz;
    const int64_t srow = ((int64_t)bz * nby + by) * nbx;
    const int b0 = box_start[srow], tot = box_start[srow + nbx] - b0;
    s_b0[tid] = b0;
    s_tot[tid] = tot;
    s_c0[tid] = tot > 0 ? row_cum(box_start, srow, nbx, g.per[0], tot, fb) : 0;
    s_yz[tid] = tot > 0 ? bz * nby + by : -1;
    // stencil index of the line in this box row's stencils
    int ay = gy - box_stencil_start(by, g.N[1], p, g.per[1]);
    int az = gz - box_stencil_start(bz, g.N[2], p, g.per[2]);
    if (g.per[1]) ay = ((ay % g.N[1]) + g.N[1]) % g.N[1];
    if (g.per[2]) az = ((az % g.N[2]) + g.N[2]) % g.N[2];
    s_ay[tid] = ay;
    s_az[tid] = az;
  }
  __syncthreads();
  for (int e = tid; e < nrow * sb1; e += blockDim.x) {
    const int j = e / sb1, k = e - j * sb1;
    int off = 0;
    if (s_yz[j] >= 0)
      off = row_cum(box_start, (int64_t)s_yz[j] * nbx, nbx, g.per[0], s_tot[j],
                    fb + min(k, nbs)) - s_c0[j];
    s_off[e] = off;
  }
  __syncthreads();
  if (tid < 64) {
    const int len = tid < nrow ? s_off[tid * sb1 + nbs] : 0;
    int x = len;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(x, d, 64);
      if (tid >= d) x += y;
    }
    if (tid < nrow) s_base[tid] = x - len;
    if (tid == nrow - 1) s_base[nrow] = x;
  }
  __syncthreads();
  // 2. stage the nodes with their y/z weights at this line
  const int total = min(s_base[nrow], pl.ncap);
  for (int e = tid; e < total; e += blockDim.x) {
    int lo = 0, hi = nrow;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_base[mid] <= e) lo = mid;
      else hi = mid;
    }
    const int c = s_c0[lo] + (e - s_base[lo]);
    int gi = c;
    if (g.per[0]) {
      int rel = (c - s_b0[lo]) % s_tot[lo];
      if (rel < 0) rel += s_tot[lo];
      gi = s_b0[lo] + rel;
    }
    const float4 nd = pos4[gi];
    const float qq = q[gi];
    const uint32_t packed = __float_as_uint(nd.w);
    s_x[e] = nd.x;
    s_st[e] = (uint16_t)st_of(packed, 0);
    s_c[e] = qq * basis(s_ay[lo], nd.y, p) * basis(s_az[lo], nd.z, p);
  }
  __syncthreads();
  if (tid >= xa) return;
  // 3. gather for the point gx
  const int gx = x0 + tid;
  const int2 rx = brx[gx];
  const int k0 = g.per[0] ? tid : rx.x - fb;
  const int kc = g.per[0] ? p + 1 : rx.y;
  float acc = 0.f;
  for (int j = 0; j < nrow; ++j) {
    const int* off = s_off + j * sb1;
    const int nb = s_base[j];
    const int n1 = nb + off[k0 + kc];
    for (int nn = nb + off[k0]; nn < n1; ++nn) {
      int a = gx - (int)s_st[nn];
      if (g.per[0] && a < 0) a += g.N[0];
      acc = fmaf(s_c[nn], basis(a, s_x[nn], p), acc);
    }
  }
  Q[((int64_t)gz * g.N[1] + gy) * g.N[0] + gx] = acc;
}

// ---------------------------------------------------------------------------
// LDS radix-2 FFT on `lines` lines of length n stored contiguously in LDS in
// bit-reversed order; decimation in time, natural-order output.

__device__ void lds_fft(float2* buf, int n, int logn, int lines, const float2* tw, float sign) {
  int half_n = n >> 1;
  int total = lines * half_n;
  for (int s = 1; s <= logn; ++s) {
    int half = 1 << (s - 1);
    int tstep = n >> s;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      int line = idx / half_n;
      int j = idx - line * half_n;
      int grp = j / half;
      int k = j - grp * half;
      int i0 = line * n + grp * 2 * half + k;
      int i1 = i0 + half;
      float2 w = tw[k * tstep];
      w.y *= sign;
      float2 a = buf[i0], b = buf[i1];
      float2 t = make_float2(b.x * w.x - b.y * w.y, b.x * w.y + b.y * w.x);
      buf[i0] = make_float2(a.x + t.x, a.y + t.y);
      buf[i1] = make_float2(a.x - t.x, a.y - t.y);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ int bitrev(int i, int logn) { return (int)(__brev((unsigned)i) >> (32 - logn)); }

// R2C along x: pairs of real rows (y, y+1) of plane z form one complex line.
// grid [Nz][Ny][Nx] real -> spec [Nz][My][Hx] complex (rows y < Ny written).
__global__ void __launch_bounds__(256) k_r2c_x(GridParams g, const float* __restrict__ Q,
                                               float2* __restrict__ spec, const float2* __restrict__ twx,
                                               int lines_per_block) {
  extern __shared__ float2 sh[];
  const int Mx = g.M[0], logM = g.logM[0], Hx = Mx / 2 + 1;
  float2* tw = sh;
  float2* buf = sh + Mx / 2;
  for (int i = threadIdx.x; i < Mx / 2; i += blockDim.x) tw[i] = twx[i];
  const int pairs = (g.N[1] + 1) / 2;
  const int64_t total_lines = (int64_t)pairs * g.N[2];
  const int64_t l0 = (int64_t)blockIdx.x * lines_per_block;
  int nl = (int)((total_lines - l0) < lines_per_block ? (total_lines - l0) : lines_per_block);
  for (int idx = threadIdx.x; idx < nl * Mx; idx += blockDim.x) {
    int li = idx / Mx, x = idx - li * Mx;
    int64_t L = l0 + li;
    int z = (int)(L / pairs), y = 2 * (int)(L % pairs);
    float re = 0.f, im = 0.f;
    if (x < g.N[0]) {
      re = Q[((int64_t)z * g.N[1] + y) * g.N[0] + x];
      if (y + 1 < g.N[1]) im = Q[((int64_t)z * g.N[1] + y + 1) * g.N[0] + x];
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

// LDS radix-2 FFT as lds_fft, lines `stride` elements apart (a stride of
// n + 1 keeps column-wise access free of bank conflicts).
__device__ void lds_fft_s(float2* buf, int n, int logn, int lines, int stride, const float2* tw,
                          float sign) {
  const int half_n = n >> 1;
  const int total = lines * half_n;
  for (int s = 1; s <= logn; ++s) {
    const int half = 1 << (s - 1);
    const int tstep = n >> s;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      const int line = idx / half_n;
      const int j = idx - line * half_n;
      const int grp = j / half;
      const int k = j - grp * half;
      const int i0 = line * stride + grp * 2 * half + k;
      const int i1 = i0 + half;
      float2 w = tw[k * tstep];
      w.y *= sign;
      const float2 a = buf[i0], b = buf[i1];
      const float2 t = make_float2(b.x * w.x - b.y * w.y, b.x * w.y + b.y * w.x);
      buf[i0] = make_float2(a.x + t.x, a.y + t.y);
      buf[i1] = make_float2(a.x - t.x, a.y - t.y);
    }
    __syncthreads();
  }
}

// Forward transform of one z-plane held whole in LDS: real rows y < Ny are
// paired into complex lines (R2C along x), separated into the half spectrum
// kx < Hx, transposed into columns (stride My + 1) and transformed along y.
// Q[z][y][x] -> spec[z][ky][kx] for all ky < My.
__global__ void __launch_bounds__(1024) k_fft_xy_fwd(GridParams g, const float* __restrict__ Q,
                                                     float2* __restrict__ spec,
                                                     const float2* __restrict__ twx,
                                                     const float2* __restrict__ twy) {
  extern __shared__ float2 sh[];
  const int Mx = g.M[0], My = g.M[1], Hx = Mx / 2 + 1, lx = g.logM[0], ly = g.logM[1];
  const int Nx = g.N[0], Ny = g.N[1], pairs = (Ny + 1) / 2, cs = My + 1;
  float2* tx = sh;
  float2* ty = tx + Mx / 2;
  float2* A = ty + My / 2;        // [pairs][Mx]
  float2* C = A + pairs * Mx;     // [Hx][My + 1]
  const int z = blockIdx.x;
  for (int i = threadIdx.x; i < Mx / 2; i += blockDim.x) tx[i] = twx[i];
  for (int i = threadIdx.x; i < My / 2; i += blockDim.x) ty[i] = twy[i];
  const float* Qz = Q + (int64_t)z * Ny * Nx;
  for (int idx = threadIdx.x; idx < pairs * Mx; idx += blockDim.x) {
    const int li = idx / Mx, x = idx - li * Mx, y = 2 * li;
    float re = 0.f, im = 0.f;
    if (x < Nx) {
      re = Qz[(int64_t)y * Nx + x];
      if (y + 1 < Ny) im = Qz[(int64_t)(y + 1) * Nx + x];
    }
    A[li * Mx + bitrev(x, lx)] = make_float2(re, im);
  }
  // rows Ny..My-1 of the columns are the zero padding
  for (int idx = threadIdx.x; idx < Hx * (My - 2 * pairs); idx += blockDim.x) {
    const int k = idx % Hx, y = 2 * pairs + idx / Hx;
    C[k * cs + bitrev(y, ly)] = make_float2(0.f, 0.f);
  }
  __syncthreads();
  lds_fft_s(A, Mx, lx, pairs, Mx, tx, 1.0f);
  for (int idx = threadIdx.x; idx < pairs * Hx; idx += blockDim.x) {
    const int li = idx / Hx, k = idx - li * Hx, y = 2 * li;
    const float2 a = A[li * Mx + k];
    const float2 b = A[li * Mx + ((Mx - k) & (Mx - 1))];
    // X_y = (Z[k] + conj Z[-k]) / 2, X_{y+1} = (Z[k] - conj Z[-k]) / (2i)
    C[k * cs + bitrev(y, ly)] = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));
    C[k * cs + bitrev(y + 1, ly)] =
        y + 1 < Ny ? make_float2(0.5f * (a.y + b.y), -0.5f * (a.x - b.x)) : make_float2(0.f, 0.f);
  }
  __syncthreads();
  lds_fft_s(C, My, ly, Hx, cs, ty, 1.0f);
  float2* Sz = spec + (int64_t)z * My * Hx;
  for (int idx = threadIdx.x; idx < My * Hx; idx += blockDim.x) {
    const int ky = idx / Hx, k = idx - ky * Hx;
    Sz[idx] = C[k * cs + ky];
  }
}

// Inverse of k_fft_xy_fwd for one z-plane: inverse FFT along y of the half
// spectrum columns, rows y < Ny paired into complex lines with Hermitian
// extension (C2R along x), inverse FFT along x. spec[z] -> U[z][y][x].
__global__ void __launch_bounds__(1024) k_fft_yx_inv(GridParams g, const float2* __restrict__ spec,
                                                     float* __restrict__ U,
                                                     const float2* __restrict__ twx,
                                                     const float2* __restrict__ twy) {
  extern __shared__ float2 sh[];
  const int Mx = g.M[0], My = g.M[1], Hx = Mx / 2 + 1, lx = g.logM[0], ly = g.logM[1];
  const int Nx = g.N[0], Ny = g.N[1], pairs = (Ny + 1) / 2, cs = My + 1;
  float2* tx = sh;
  float2* ty = tx + Mx / 2;
  float2* A = ty + My / 2;
  float2* C = A + pairs * Mx;
  const int z = blockIdx.x;
  for (int i = threadIdx.x; i < Mx / 2; i += blockDim.x) tx[i] = twx[i];
  for (int i = threadIdx.x; i < My / 2; i += blockDim.x) ty[i] = twy[i];
  const float2* Sz = spec + (int64_t)z * My * Hx;
  for (int idx = threadIdx.x; idx < My * Hx; idx += blockDim.x) {
    const int ky = idx / Hx, k = idx - ky * Hx;
    C[k * cs + bitrev(ky, ly)] = Sz[idx];
  }
  __syncthreads();
  lds_fft_s(C, My, ly, Hx, cs, ty, -1.0f);
  for (int idx = threadIdx.x; idx < pairs * Mx; idx += blockDim.x) {
    const int li = idx / Mx, k = idx - li * Mx, y = 2 * li;
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
  lds_fft_s(A, Mx, lx, pairs, Mx, tx, -1.0f);
  float* Uz = U + (int64_t)z * Ny * Nx;
  for (int idx = threadIdx.x; idx < pairs * Nx; idx += blockDim.x) {
    const int li = idx / Nx, x = idx - li * Nx, y = 2 * li;
    const float2 v = A[li * Mx + x];
    Uz[(int64_t)y * Nx + x] = v.x;
    if (y + 1 < Ny) Uz[(int64_t)(y + 1) * Nx + x] = v.y;
  }
}

// FFT along y for lines (z < Nz, kx): groups of B consecutive kx per block.
// Forward: input rows y < Ny (others zero), all My outputs written.
// Inverse: all My inputs, outputs y < n_out written.
__global__ void __launch_bounds__(256) k_fft_y(GridParams g, float2* __restrict__ spec,
                                               const float2* __restrict__ twy, int B, int inverse,
                                               int n_in, int n_out) {
  extern __shared__ float2 sh[];
  const int My = g.M[1], logM = g.logM[1], Hx = g.M[0] / 2 + 1;
  float2* tw = sh;
  float2* buf = sh + My / 2;
  for (int i = threadIdx.x; i < My / 2; i += blockDim.x) tw[i] = twy[i];
  const int groups_per_plane = (Hx + B - 1) / B;
  const int z = blockIdx.x / groups_per_plane;
  const int kx0 = (blockIdx.x - z * groups_per_plane) * B;
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

// FFT along z of lines c = ky*Hx + kx (B consecutive per block), multiply by
// the real spectrum khat[kz][c], inverse FFT, write z < Nz.
__global__ void __launch_bounds__(256) k_fft_z_mul(GridParams g, float2* __restrict__ spec,
                                                   const float* __restrict__ khat,
                                                   const float2* __restrict__ twz, int B) {
  extern __shared__ float2 sh[];
  const int Mz = g.M[2], logM = g.logM[2], Hx = g.M[0] / 2 + 1;
  const int64_t plane = (int64_t)g.M[1] * Hx;
  float2* tw = sh;
  float2* buf = sh + Mz / 2;
  for (int i = threadIdx.x; i < Mz / 2; i += blockDim.x) tw[i] = twz[i];
  const int64_t c0 = (int64_t)blockIdx.x * B;
  const int nb = (int)((plane - c0) < B ? (plane - c0) : B);
  for (int idx = threadIdx.x; idx < nb * Mz; idx += blockDim.x) {
    int z = idx / nb, li = idx - z * nb;
    float2 v = make_float2(0.f, 0.f);
    if (z < g.N[2]) v = spec[(int64_t)z * plane + c0 + li];
    buf[li * Mz + bitrev(z, logM)] = v;
  }
  __syncthreads();
  lds_fft(buf, Mz, logM, nb, tw, 1.0f);
  // multiply and scatter back in bit-reversed order for the inverse
  for (int idx = threadIdx.x; idx < nb * Mz; idx += blockDim.x) {
    int kz = idx / nb, li = idx - kz * nb;
    float kk = khat[(int64_t)kz * plane + c0 + li];
    float2 v = buf[li * Mz + kz];
    buf[li * Mz + kz] = make_float2(v.x * kk, v.y * kk);  // same element, same thread
  }
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

// C2R along x: rows (y, y+1) of plane z from their half spectra -> U[z][y][x].
__global__ void __launch_bounds__(256) k_c2r_x(GridParams g, const float2* __restrict__ spec,
                                               float* __restrict__ U, const float2* __restrict__ twx,
                                               int lines_per_block) {
  extern __shared__ float2 sh[];
  const int Mx = g.M[0], logM = g.logM[0], Hx = Mx / 2 + 1;
  float2* tw = sh;
  float2* buf = sh + Mx / 2;
  for (int i = threadIdx.x; i < Mx / 2; i += blockDim.x) tw[i] = twx[i];
  const int pairs = (g.N[1] + 1) / 2;
  const int64_t total_lines = (int64_t)pairs * g.N[2];
  const int64_t l0 = (int64_t)blockIdx.x * lines_per_block;
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
    U[((int64_t)z * g.N[1] + y) * g.N[0] + x] = v.x;
    if (y + 1 < g.N[1]) U[((int64_t)z * g.N[1] + y + 1) * g.N[0] + x] = v.y;
  }
}

// ---------------------------------------------------------------------------
// interpolation + precorrection. All rows of one observer box have the same
// near boxes, hence the same precorrection columns: for each of the
// (2 r_b + 1)^2 (dy, dz) pairs, the nodes of the 2 r_b + 1 consecutive boxes
// along x (a run that splits in two where a periodic x axis wraps), in box
// order. The matrix therefore stores values only; the columns are rebuilt
// from the box table. Each group of 16 lanes takes one occupied observer
// box: it gathers the box's source charges into its own LDS slice in column
// order, prefetches the first row's matrix values, then for every row of
// the box forms W U (64 stencil values of the box, weights from the row's
// local coordinates) plus P q, reduced in a fixed order.

template <int W>
__device__ __forceinline__ int group_excl_scan(int v, int lane, int& total) {
  int x = v;
#pragma unroll
  for (int d = 1; d < W; d <<= 1) {
    const int y = __shfl_up(x, d, W);
    if (lane >= d) x += y;
  }
  total = __shfl(x, W - 1, W);
  return x - v;
}

struct Window {
  int sA, nA, sB, nB;  // node runs [sA, sA + nA) then [sB, sB + nB)
};

// source nodes of pair i (dy, dz) for observer box (bx, by, bz)
__device__ __forceinline__ Window pair_window(const GridParams& g, const int32_t* box_start,
                                              int i, int bx, int by, int bz) {
  Window w{0, 0, 0, 0};
  const int W = 2 * g.rb + 1;
  int y = by + i % W - g.rb, z = bz + i / W - g.rb;
  if (g.per[1]) {
    if (y < 0) y += g.nbox[1];
    if (y >= g.nbox[1]) y -= g.nbox[1];
  } else if (y < 0 || y >= g.nbox[1]) {
    return w;
  }
  if (g.per[2]) {
    if (z < 0) z += g.nbox[2];
    if (z >= g.nbox[2]) z -= g.nbox[2];
  } else if (z < 0 || z >= g.nbox[2]) {
    return w;
  }
  const int64_t row = ((int64_t)z * g.nbox[1] + y) * g.nbox[0];
  const int nbx = g.nbox[0];
  int lo = bx - g.rb, hi = bx + g.rb;
  int a0, a1, b0 = 0, b1 = -1;
  if (g.per[0]) {
    if (lo < 0) {
      a0 = lo + nbx; a1 = nbx - 1; b0 = 0; b1 = hi;
    } else if (hi >= nbx) {
      a0 = lo; a1 = nbx - 1; b0 = 0; b1 = hi - nbx;
    } else {
      a0 = lo; a1 = hi;
    }
  } else {
    a0 = max(lo, 0);
    a1 = min(hi, nbx - 1);
  }
  w.sA = box_start[row + a0];
  w.nA = box_start[row + a1 + 1] - w.sA;
  if (b1 >= b0) {
    w.sB = box_start[row + b0];
    w.nB = box_start[row + b1 + 1] - w.sB;
  }
  return w;
}

__global__ void __launch_bounds__(256) k_interp_corr(
    GridParams g, int n_occ, const int32_t* __restrict__ occ, const float* __restrict__ U,
    const float4* __restrict__ pos4, const int32_t* __restrict__ box_start,
    const int32_t* __restrict__ prp, const float* __restrict__ pval,
    const float* __restrict__ q, const float* __restrict__ uz, float* __restrict__ u) {
  constexpr int G = kIcGroup;
  constexpr int KP = 16;  // prefetched matrix values per lane (rows up to 256 entries)
  __shared__ float s_qg[kIcGroups][kIcGQ];
  const int lane = threadIdx.x & (G - 1);
  const int grp = threadIdx.x / G;
  const int gid = blockIdx.x * kIcGroups + grp;
  const bool live = gid < n_occ;
  const int B = live ? occ[gid] : 0;
  const int bx = B % g.nbox[0], by = (B / g.nbox[0]) % g.nbox[1], bz = B / (g.nbox[0] * g.nbox[1]);
  const int r0 = live ? box_start[B] : 0, r1 = live ? box_start[B + 1] : 0;
  // prefetch the first row's matrix values
  const int pr0 = live ? prp[r0] : 0;
  const int rl0 = live ? prp[r0 + 1] - pr0 : 0;
  float pv[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int j = lane + G * k;
    pv[k] = j < rl0 ? pval[pr0 + j] : 0.f;
  }
  // gather the source charges of the box's windows in column order
  const int W = 2 * g.rb + 1, npair = W * W;
  int S = 0;
  for (int t = 0; t * G < npair; ++t) {
    const int i = t * G + lane;
    Window w{0, 0, 0, 0};
    if (live && i < npair) w = pair_window(g, box_start, i, bx, by, bz);
    int tot;
    const int off = S + group_excl_scan<G>(w.nA + w.nB, lane, tot);
    S += tot;
    if (off + w.nA + w.nB <= kIcGQ) {
      for (int c = 0; c < w.nA; ++c) s_qg[grp][off + c] = q[w.sA + c];
      for (int c = 0; c < w.nB; ++c) s_qg[grp][off + w.nA + c] = q[w.sB + c];
    }
  }
  const bool staged = S <= kIcGQ;
  wave_lds_sync();
  // stencil of the box: lane holds the 4 values (ax, ay) = (lane % 4, lane / 4), az = 0..3
  const int shift = (g.p - 1) / 2;
  const bool cubic = g.p == 3;
  int sta[3];
  const int bxyz[3] = {bx, by, bz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int st = bxyz[a] - shift;
    if (g.per[a]) {
      if (st < 0) st += g.N[a];
    } else {
      st = min(max(st, 0), g.N[a] - g.p - 1);
    }
    sta[a] = st;
  }
  const int lax = lane & 3, lay = lane >> 2;
  float uv[4] = {0.f, 0.f, 0.f, 0.f};
  if (cubic && live) {
    int gx = sta[0] + lax, gy = sta[1] + lay;
    if (gx >= g.N[0]) gx -= g.N[0];
    if (gy >= g.N[1]) gy -= g.N[1];
#pragma unroll
    for (int az = 0; az < 4; ++az) {
      int gz = sta[2] + az;
      if (gz >= g.N[2]) gz -= g.N[2];
      uv[az] = U[((int64_t)gz * g.N[1] + gy) * g.N[0] + gx];
    }
  }
  const Cubic cx = cubic_basis(lax), cy = cubic_basis(lay);
  const Cubic cz0 = cubic_basis(0), cz1 = cubic_basis(1), cz2 = cubic_basis(2), cz3 = cubic_basis(3);
  // rows: the wave runs as many rounds as its largest box has rows
  int nr = r1 - r0;
  int maxr = nr;
#pragma unroll
  for (int o = 32; o >= G; o >>= 1) maxr = max(maxr, __shfl_xor(maxr, o, 64));
  for (int rr = 0; rr < maxr; ++rr) {
    const bool act = rr < nr;
    const int r = r0 + rr;
    float acc = 0.f;
    if (act) {
      const int pr = rr == 0 ? pr0 : prp[r];
      // the row length equals S by construction; the min keeps every read in bounds
      const int rl = min(S, rr == 0 ? rl0 : prp[r + 1] - pr);
      if (staged) {
        if (rr == 0) {
#pragma unroll
          for (int k = 0; k < KP; ++k) {
            const int j = lane + G * k;
            if (j < rl) acc = fmaf(pv[k], s_qg[grp][j], acc);
          }
          for (int j = lane + G * KP; j < rl; j += G) acc = fmaf(pval[pr + j], s_qg[grp][j], acc);
        } else {
          for (int j = lane; j < rl; j += G) acc = fmaf(pval[pr + j], s_qg[grp][j], acc);
        }
      } else {
        // very large rows: walk the windows in global memory
        for (int j = lane; j < rl; j += G) {
          int loc = j;
          float qj = 0.f;
          for (int i = 0; i < npair; ++i) {
            const Window w = pair_window(g, box_start, i, bx, by, bz);
            if (loc < w.nA) { qj = q[w.sA + loc]; break; }
            loc -= w.nA;
            if (loc < w.nB) { qj = q[w.sB + loc]; break; }
            loc -= w.nB;
          }
          acc = fmaf(pval[pr + j], qj, acc);
        }
      }
      const float4 xi = pos4[r];
      if (cubic) {
        const float wxy = cubic_eval(cx, xi.x) * cubic_eval(cy, xi.y);
        acc = fmaf(wxy * cubic_eval(cz0, xi.z), uv[0], acc);
        acc = fmaf(wxy * cubic_eval(cz1, xi.z), uv[1], acc);
        acc = fmaf(wxy * cubic_eval(cz2, xi.z), uv[2], acc);
        acc = fmaf(wxy * cubic_eval(cz3, xi.z), uv[3], acc);
      } else {
        const int p1 = g.p + 1, nst = p1 * p1 * p1;
        for (int l = lane; l < nst; l += G) {
          const int ax = l % p1, ay = (l / p1) % p1, az = l / (p1 * p1);
          int gx = sta[0] + ax, gy = sta[1] + ay, gz = sta[2] + az;
          if (gx >= g.N[0]) gx -= g.N[0];
          if (gy >= g.N[1]) gy -= g.N[1];
          if (gz >= g.N[2]) gz -= g.N[2];
          acc = fmaf(lagrange(ax, xi.x, g.p) * lagrange(ay, xi.y, g.p) * lagrange(az, xi.z, g.p),
                     U[((int64_t)gz * g.N[1] + gy) * g.N[0] + gx], acc);
        }
      }
    }
    acc = group_sum<G>(acc);
    if (act && lane == 0) u[r] = acc + uz[r];
  }
}

// ---------------------------------------------------------------------------
// interpolation + precorrection, segment form. A workgroup takes `xs`
// consecutive boxes of one (y, z) box row; their rows are contiguous. Every
// source charge those rows need lies in the (2 r_b + 1)^2 neighbouring box
// rows, boxes x0 - r_b .. x0 + xs + r_b - 1 (unwrapped along a periodic x),
// so these are staged once in LDS with coalesced loads, together with the
// (p + 1)^2 stencil lines of U the segment reads. Then each 16-lane group
// takes one observer row at a time: it copies the row's window charges from
// the staged rows into column order (pair-major, each x-run in unwrapped box
// order, which is the storage order of the precorrection values), streams
// the row's matrix values, and adds W U from the staged lines.

__global__ void __launch_bounds__(256) k_interp_seg(
    GridParams g, IcPlan pl, const float* __restrict__ U, const float4* __restrict__ pos4,
    const int32_t* __restrict__ box_start, const int32_t* __restrict__ prp,
    const float* __restrict__ pval, const float* __restrict__ q, const float* __restrict__ uz,
    float* __restrict__ u) {
  extern __shared__ float4 smem4[];
  unsigned char* smem = reinterpret_cast<unsigned char*>(smem4);
  float* s_q = reinterpret_cast<float*>(smem + pl.o_q);
  float* s_U = reinterpret_cast<float*>(smem + pl.o_u);
  int* s_base = reinterpret_cast<int*>(smem + pl.o_meta);  // np + 1 staged row starts
  int* s_c0 = s_base + (pl.np + 1);                          // cumulative index at x0 - r_b
  int* s_b0 = s_c0 + pl.np;                                  // first node of the row
  int* s_tot = s_b0 + pl.np;                                 // nodes in the row
  int* s_yz = s_tot + pl.np;                                 // row index, -1 if outside
  uint16_t* s_off = reinterpret_cast<uint16_t*>(smem + pl.o_off);  // np x (sb + 1)
  uint16_t* s_row = reinterpret_cast<uint16_t*>(smem + pl.o_row);  // box of each row
  const int tid = threadIdx.x;
  const int nbx = g.nbox[0], nby = g.nbox[1], nbz = g.nbox[2];
  const int sx = blockIdx.x % pl.nsx, byz = blockIdx.x / pl.nsx;
  const int by = byz % nby, bz = byz / nby;
  const int x0 = sx * pl.xs, xs = min(pl.xs, nbx - x0);
  const int64_t orow = ((int64_t)bz * nby + by) * nbx;
  const int r_lo = box_start[orow + x0], r_hi = box_start[orow + x0 + xs];
  if (r_lo == r_hi) return;  // uniform across the workgroup
  const int rb = g.rb, W = 2 * rb + 1, np = pl.np, sb1 = pl.sb + 1, p1 = g.p + 1;
  const int shift = (g.p - 1) / 2;

  // 1. source rows
  if (tid < np) {
    int y = by + tid % W - rb, z = bz + tid / W - rb;
    bool ok = true;
    if (g.per[1]) y = (y + nby) % nby;
    else ok = ok && y >= 0 && y < nby;
    if (g.per[2]) z = (z + nbz) % nbz;
    else ok = ok && z >= 0 && z < nbz;
    int b0 = 0, tot = 0, c0 = 0, yz = -1;
    if (ok) {
      yz = z * nby + y;
      const int64_t srow = (int64_t)yz * nbx;
      b0 = box_start[srow];
      tot = box_start[srow + nbx] - b0;
      c0 = row_cum(box_start, srow, nbx, g.per[0], tot, x0 - rb);
    }
    s_b0[tid] = b0;
    s_tot[tid] = tot;
    s_c0[tid] = c0;
    s_yz[tid] = tot > 0 ? yz : -1;
  }
  __syncthreads();
  // 2. per source row, staged offset of each unwrapped box x0 - r_b + k
  for (int e = tid; e < np * sb1; e += blockDim.x) {
    const int i = e / sb1, k = e - i * sb1;
    int off = 0;
    if (s_yz[i] >= 0)
      off = row_cum(box_start, (int64_t)s_yz[i] * nbx, nbx, g.per[0], s_tot[i], x0 - rb + k) -
            s_c0[i];
    s_off[e] = (uint16_t)off;
  }
  // observer row -> box of the segment
  for (int k = tid; k < xs; k += blockDim.x) {
    const int a = box_start[orow + x0 + k] - r_lo, b = box_start[orow + x0 + k + 1] - r_lo;
    for (int r = a; r < b && r < pl.rcap; ++r) s_row[r] = (uint16_t)k;
  }
  // stencil lines of U: (ay, az) in [0, p]^2, x from the segment's first stencil start
  const int sty = box_stencil_start(by, g.N[1], g.p, g.per[1]);
  const int stz = box_stencil_start(bz, g.N[2], g.p, g.per[2]);
  const int ux0 = box_stencil_start(x0, g.N[0], g.p, g.per[0]);
  for (int e = tid; e < p1 * p1 * pl.ux; e += blockDim.x) {
    const int l = e / pl.ux, t = e - l * pl.ux;
    int y = sty + l % p1, z = stz + l / p1, x = ux0 + t;
    if (g.per[1]) y = (y + g.N[1]) % g.N[1];
    if (g.per[2]) z = (z + g.N[2]) % g.N[2];
    float v = 0.f;
    if (g.per[0]) {
      x = (x + g.N[0]) % g.N[0];
      v = U[((int64_t)z * g.N[1] + y) * g.N[0] + x];
    } else if (x < g.N[0]) {
      v = U[((int64_t)z * g.N[1] + y) * g.N[0] + x];
    }
    s_U[e] = v;
  }
  __syncthreads();
  // 3. staged row starts (one wave scans np <= 49 lengths)
  if (tid < 64) {
    const int len = tid < np ? (int)s_off[tid * sb1 + pl.sb] : 0;
    int x = len;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(x, d, 64);
      if (tid >= d) x += y;
    }
    if (tid < np) s_base[tid] = x - len;
    if (tid == np - 1) s_base[np] = x;
  }
  __syncthreads();
  // 4. stage the source charges (coalesced per source row)
  const int total = min(s_base[np], pl.qcap);
  for (int e = tid; e < total; e += blockDim.x) {
    int lo = 0, hi = np;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_base[mid] <= e) lo = mid;
      else hi = mid;
    }
    const int c = s_c0[lo] + (e - s_base[lo]);
    int gi = c;
    if (g.per[0]) {
      int rel = (c - s_b0[lo]) % s_tot[lo];
      if (rel < 0) rel += s_tot[lo];
      gi = s_b0[lo] + rel;
    }
    s_q[e] = q[gi];
  }
  __syncthreads();

  // 5. rows: one per 16-lane group
  constexpr int G = 16, KP = 16;
  const int lane = tid & (G - 1), grp = tid / G, ngrp = blockDim.x / G;
  float* col = reinterpret_cast<float*>(smem + pl.o_col) + grp * pl.scap;
  const bool cubic = g.p == 3;
  const Cubic cx = cubic_basis(lane & 3), cy = cubic_basis(lane >> 2);
  const Cubic cz0 = cubic_basis(0), cz1 = cubic_basis(1), cz2 = cubic_basis(2), cz3 = cubic_basis(3);
  for (int r = r_lo + grp; r < r_hi; r += ngrp) {
    const int pr = prp[r];
    const int S = prp[r + 1] - pr;
    float pv[KP];
#pragma unroll
    for (int j = 0; j < KP; ++j) {
      const int idx = lane + G * j;
      pv[j] = idx < S ? pval[pr + idx] : 0.f;
    }
    const float4 xi = pos4[r];
    const int k = r - r_lo < pl.rcap ? (int)s_row[r - r_lo] : 0;
    // window charges into column order
    int sacc = 0;
    for (int i0 = 0; i0 < np; i0 += G) {
      const int i = i0 + lane;
      int len = 0, src = 0;
      if (i < np) {
        const int a = s_off[i * sb1 + k], b = s_off[i * sb1 + k + W];
        len = b - a;
        src = s_base[i] + a;
      }
      int tot;
      const int dst = sacc + group_excl_scan<G>(len, lane, tot);
      sacc += tot;
      for (int c = 0; c < len; ++c)
        if (dst + c < pl.scap) col[dst + c] = s_q[src + c];
    }
    wave_lds_sync();
    const int rl = min(min(S, sacc), pl.scap);
    float acc = 0.f;
#pragma unroll
    for (int j = 0; j < KP; ++j) {
      const int idx = lane + G * j;
      if (idx < rl) acc = fmaf(pv[j], col[idx], acc);
    }
    for (int idx = lane + G * KP; idx < rl; idx += G) acc = fmaf(pval[pr + idx], col[idx], acc);
    // W U from the staged stencil lines
    const int bx = x0 + k;
    const int rel = g.per[0] ? k : box_stencil_start(bx, g.N[0], g.p, 0) - ux0;
    if (cubic) {
      const float* su = s_U + (lane >> 2) * pl.ux + rel + (lane & 3);
      const int zs = 4 * pl.ux;
      const float wxy = cubic_eval(cx, xi.x) * cubic_eval(cy, xi.y);
      acc = fmaf(wxy * cubic_eval(cz0, xi.z), su[0], acc);
      acc = fmaf(wxy * cubic_eval(cz1, xi.z), su[zs], acc);
      acc = fmaf(wxy * cubic_eval(cz2, xi.z), su[2 * zs], acc);
      acc = fmaf(wxy * cubic_eval(cz3, xi.z), su[3 * zs], acc);
    } else {
      const int nst = p1 * p1 * p1;
      for (int l = lane; l < nst; l += G) {
        const int ax = l % p1, ay = (l / p1) % p1, az = l / (p1 * p1);
        acc = fmaf(lagrange(ax, xi.x, g.p) * lagrange(ay, xi.y, g.p) * lagrange(az, xi.z, g.p),
                   s_U[(az * p1 + ay) * pl.ux + rel + ax], acc);
      }
    }
    acc = group_sum<G>(acc);
    if (lane == 0) u[r] = acc + uz[r];
    wave_lds_sync();  // the column buffer is rewritten for the next row
  }
}

// ---------------------------------------------------------------------------
// exchange + gradient + sum over the shared local pattern, 16 lanes per row:
//   H_n = sum_k ( L_nk m_k - G_nk u_k ) + H_applied,  gl = {Gx, Gy, Gz, L}

__global__ void __launch_bounds__(256) k_grad(int64_t n, const int32_t* __restrict__ rp,
                                              const int32_t* __restrict__ col,
                                              const float4* __restrict__ gl,
                                              const float* __restrict__ m,
                                              const float* __restrict__ u,
                                              float* __restrict__ h, float hax, float hay,
                                              float haz, int with_ex, int with_ms) {
  int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  int lane = threadIdx.x & 15;
  if (row >= n) return;
  float hx = 0.f, hy = 0.f, hz = 0.f;
  const int e0 = rp[row], e1 = rp[row + 1];
  for (int e = e0 + lane; e < e1; e += 16) {
    const int64_t k = col[e];
    const float4 w = gl[e];
    if (with_ex) {
      hx += w.w * m[3 * k];
      hy += w.w * m[3 * k + 1];
      hz += w.w * m[3 * k + 2];
    }
    if (with_ms) {
      const float uk = u[k];
      hx -= w.x * uk;
      hy -= w.y * uk;
      hz -= w.z * uk;
    }
  }
  hx = group_sum<16>(hx);
  hy = group_sum<16>(hy);
  hz = group_sum<16>(hz);
  if (lane == 0) {
    h[3 * row] = hx + hax;
    h[3 * row + 1] = hy + hay;
    h[3 * row + 2] = hz + haz;
  }
}

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

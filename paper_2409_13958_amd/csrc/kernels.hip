// gfx950 kernels of the PM-FEM effective-field evaluation.
//
// One H_eff evaluation (paper Eqs. heff, hex, hms_d1 - hms_d3):
//   k_local        H_ex = L m, q = D m (Eq. hms_d1), u_Z = Z0 m (Eq. hms_d2b)
//   k_anterp       Q = W^T q                      (Sec. 3.2.2, step 1)
//   k_r2c_x        real-to-complex FFT along x    (step 2)
//   k_fft_y        FFT along y (forward)
//   k_fft_z_mul    FFT along z, multiply by the PGF spectrum, inverse along z
//   k_fft_y        FFT along y (inverse)
//   k_c2r_x        complex-to-real FFT along x -> U = (1/4 pi) K * Q
//   k_interp_corr  u = W U + P q + u_Z            (steps 3 and 4)
//   k_grad         H = H_ex - G u (+ H_applied)   (Eq. hms_d3)
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

__device__ __forceinline__ int st_of(uint32_t packed, int axis) {
  return (int)((packed >> (10 * axis)) & 1023u);
}

template <int W>
__device__ __forceinline__ float group_sum(float v) {
  // butterfly sum over groups of W consecutive lanes (W divides 64)
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
  return v;
}

// ---------------------------------------------------------------------------
// local operators: 16 lanes per row

__global__ void __launch_bounds__(256) k_local(
    int64_t n, const float* __restrict__ m, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ col, const float4* __restrict__ ld,
    const int32_t* __restrict__ zrp, const int32_t* __restrict__ zcol,
    const float4* __restrict__ zv, float4* __restrict__ hex, float* __restrict__ q,
    float* __restrict__ uz, int with_ex, int with_ms) {
  int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  int lane = threadIdx.x & 15;
  if (row >= n) return;
  float hx = 0.f, hy = 0.f, hz = 0.f, qq = 0.f, zz = 0.f;
  int e0 = rp[row], e1 = rp[row + 1];
  for (int e = e0 + lane; e < e1; e += 16) {
    int k = col[e];
    float4 w = ld[e];
    float mx = m[3 * (int64_t)k], my = m[3 * (int64_t)k + 1], mz = m[3 * (int64_t)k + 2];
    hx += w.x * mx;
    hy += w.x * my;
    hz += w.x * mz;
    qq += w.y * mx + w.z * my + w.w * mz;
  }
  if (with_ms) {
    int z0 = zrp[row], z1 = zrp[row + 1];
    for (int e = z0 + lane; e < z1; e += 16) {
      int k = zcol[e];
      float4 w = zv[e];
      zz += w.x * m[3 * (int64_t)k] + w.y * m[3 * (int64_t)k + 1] + w.z * m[3 * (int64_t)k + 2];
    }
  }
  hx = group_sum<16>(hx);
  hy = group_sum<16>(hy);
  hz = group_sum<16>(hz);
  qq = group_sum<16>(qq);
  zz = group_sum<16>(zz);
  if (lane == 0) {
    hex[row] = with_ex ? make_float4(hx, hy, hz, 0.f) : make_float4(0.f, 0.f, 0.f, 0.f);
    q[row] = qq;
    uz[row] = zz;
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

__device__ __forceinline__ int halo_start(const int2* br, int g0, int nbox, int per) {
  (void)nbox;
  (void)per;
  return br[g0].x;
}

__global__ void __launch_bounds__(256) k_anterp(
    GridParams g, const float* __restrict__ q, const float4* __restrict__ pos4,
    const int32_t* __restrict__ box_start, const int2* __restrict__ brx,
    const int2* __restrict__ bry, const int2* __restrict__ brz, float* __restrict__ Q) {
  __shared__ int s_off[kAntHalo];
  __shared__ int s_tmp[256];
  __shared__ float4 s_nd[kAntCap];
  __shared__ uint32_t s_st[kAntCap];
  const int ntx = (g.N[0] + kAntTX - 1) / kAntTX, nty = (g.N[1] + kAntTY - 1) / kAntTY;
  const int tile = blockIdx.x;
  const int t0[3] = {(tile % ntx) * kAntTX, ((tile / ntx) % nty) * kAntTY,
                     (tile / (ntx * nty)) * kAntTZ};
  const int te[3] = {min(kAntTX, g.N[0] - t0[0]), min(kAntTY, g.N[1] - t0[1]),
                     min(kAntTZ, g.N[2] - t0[2])};
  const int2* br[3] = {brx, bry, brz};
  int hs[3], hc[3];
  for (int a = 0; a < 3; ++a) {
    int2 f = br[a][t0[a]], l = br[a][t0[a] + te[a] - 1];
    hs[a] = f.x;
    if (g.per[a]) {
      hc[a] = (te[a] - 1) + g.p + 1;
    } else {
      hc[a] = l.x + l.y - f.x;
    }
  }
  const int H = hc[0] * hc[1] * hc[2];
  auto box_of = [&](int h) -> int64_t {
    int ix = h % hc[0], iy = (h / hc[0]) % hc[1], iz = h / (hc[0] * hc[1]);
    int bx = (hs[0] + ix) % g.nbox[0], by = (hs[1] + iy) % g.nbox[1],
        bz = (hs[2] + iz) % g.nbox[2];
    return ((int64_t)bz * g.nbox[1] + by) * g.nbox[0] + bx;
  };
  for (int h = threadIdx.x; h < H; h += blockDim.x) {
    int64_t b = box_of(h);
    s_off[h] = box_start[b + 1] - box_start[b];
  }
  __syncthreads();
  block_exclusive_scan(s_off, H, s_tmp);
  const int total = s_off[H];
  if (total == 0) {
    // no node reaches this tile
    const int lx = threadIdx.x % kAntTX, ly = (threadIdx.x / kAntTX) % kAntTY,
              lz = threadIdx.x / (kAntTX * kAntTY);
    if (lx < te[0] && ly < te[1] && lz < te[2])
      Q[((int64_t)(t0[2] + lz) * g.N[1] + (t0[1] + ly)) * g.N[0] + (t0[0] + lx)] = 0.f;
    return;
  }
  const bool staged = total <= kAntCap;
  if (staged) {
    for (int h = threadIdx.x; h < H; h += blockDim.x) {
      int64_t b = box_of(h);
      int k0 = box_start[b], k1 = box_start[b + 1], o = s_off[h];
      for (int k = k0; k < k1; ++k) {
        float4 pp = pos4[k];
        s_nd[o + k - k0] = make_float4(pp.x, pp.y, pp.z, q[k]);
        s_st[o + k - k0] = __float_as_uint(pp.w);
      }
    }
  }
  __syncthreads();
  const int lx = threadIdx.x % kAntTX, ly = (threadIdx.x / kAntTX) % kAntTY,
            lz = threadIdx.x / (kAntTX * kAntTY);
  if (lx >= te[0] || ly >= te[1] || lz >= te[2]) return;
  const int gx = t0[0] + lx, gy = t0[1] + ly, gz = t0[2] + lz;
  const int2 rx = brx[gx], ry = bry[gy], rz = brz[gz];
  // halo-relative first box of this point's ranges (periodic: the halo
  // starts at the box range of the tile's first point, shifted by one box
  // per grid point)
  const int ox = g.per[0] ? lx : rx.x - hs[0];
  const int oy = g.per[1] ? ly : ry.x - hs[1];
  const int oz = g.per[2] ? lz : rz.x - hs[2];
  float acc = 0.f;
  for (int iz = 0; iz < rz.y; ++iz)
    for (int iy = 0; iy < ry.y; ++iy) {
      // the x-boxes of one (y, z) row are consecutive in the halo and their
      // nodes consecutive in the staged arrays
      const int h0 = ((oz + iz) * hc[1] + (oy + iy)) * hc[0] + ox;
      const int k0 = s_off[h0], k1 = s_off[h0 + rx.y];
      for (int k = k0; k < k1; ++k) {
        float4 nd;
        uint32_t pk;
        if (staged) {
          nd = s_nd[k];
          pk = s_st[k];
        } else {
          // locate node k of the halo in global memory
          int lo = h0, hi = h0 + rx.y - 1;
          while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= k) lo = mid; else hi = mid - 1;
          }
          int64_t b = box_of(lo);
          int kg = box_start[b] + (k - s_off[lo]);
          float4 pp = pos4[kg];
          nd = make_float4(pp.x, pp.y, pp.z, q[kg]);
          pk = __float_as_uint(pp.w);
        }
        int ax = gx - st_of(pk, 0), ay = gy - st_of(pk, 1), az = gz - st_of(pk, 2);
        if (ax < 0) ax += g.N[0];
        if (ay < 0) ay += g.N[1];
        if (az < 0) az += g.N[2];
        acc += nd.w * (lagrange(ax, nd.x, g.p) * lagrange(ay, nd.y, g.p) * lagrange(az, nd.z, g.p));
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
// along x, in box order. The matrix therefore stores values only (row
// pointer + values); columns are rebuilt from the box table. One workgroup
// handles kIcXS observer boxes of one (y, z) box row: it stages the source
// charges of all windows it needs in LDS once, then each wavefront takes
// whole observer boxes: it caches the box's window charges and its 64
// stencil values of U in registers and streams the P rows of the box.

template <int W>
__device__ __forceinline__ int wave_excl_scan(int v, int lane, int& total) {
  int x = v;
#pragma unroll
  for (int d = 1; d < W; d <<= 1) {
    int y = __shfl_up(x, d, W);
    if (lane >= d) x += y;
  }
  total = __shfl(x, W - 1, W);
  return x - v;
}

__device__ __forceinline__ int wrap_box(int b, int nb, int per, bool& ok) {
  if (per) {
    if (b < 0) b += nb;
    if (b >= nb) b -= nb;
    ok = true;
  } else {
    ok = (b >= 0 && b < nb);
  }
  return b;
}

__global__ void __launch_bounds__(256) k_interp_corr(
    GridParams g, const float* __restrict__ U, const float4* __restrict__ pos4,
    const int32_t* __restrict__ box_start, const int32_t* __restrict__ prp,
    const float* __restrict__ pval, const float* __restrict__ q, const float* __restrict__ uz,
    float* __restrict__ u) {
  __shared__ int s_off[kIcPairs * kIcCols + 1];
  __shared__ int s_tmp[256];
  __shared__ float s_q[kIcQCap];
  const int rb = g.rb, W = 2 * rb + 1, npair = W * W;
  const int nseg = (g.nbox[0] + kIcXS - 1) / kIcXS;
  const int seg = blockIdx.x % nseg;
  const int by = (blockIdx.x / nseg) % g.nbox[1];
  const int bz = blockIdx.x / (nseg * g.nbox[1]);
  const int bx0 = seg * kIcXS;
  const int nobs = min(kIcXS, g.nbox[0] - bx0);
  const int C = nobs + 2 * rb;  // staged columns: boxes bx0 - rb .. bx0 + nobs - 1 + rb
  // observer rows of this segment
  const int64_t brow = ((int64_t)bz * g.nbox[1] + by) * g.nbox[0];
  const int r_first = box_start[brow + bx0], r_last = box_start[brow + bx0 + nobs];
  if (r_first == r_last) return;  // uniform across the block
  auto src_box = [&](int i, int c, bool& ok) -> int64_t {
    int dy = i % W - rb, dz = i / W - rb;
    bool okx, oky, okz;
    int sx = wrap_box(bx0 - rb + c, g.nbox[0], g.per[0], okx);
    int sy = wrap_box(by + dy, g.nbox[1], g.per[1], oky);
    int sz = wrap_box(bz + dz, g.nbox[2], g.per[2], okz);
    ok = okx && oky && okz;
    return ((int64_t)sz * g.nbox[1] + sy) * g.nbox[0] + sx;
  };
  const int NE = npair * C;
  for (int t = threadIdx.x; t < NE; t += blockDim.x) {
    bool ok;
    int64_t b = src_box(t / C, t % C, ok);
    s_off[t] = ok ? box_start[b + 1] - box_start[b] : 0;
  }
  __syncthreads();
  block_exclusive_scan(s_off, NE, s_tmp);
  const bool staged = s_off[NE] <= kIcQCap;
  if (staged) {
    for (int t = threadIdx.x; t < NE; t += blockDim.x) {
      bool ok;
      int64_t b = src_box(t / C, t % C, ok);
      if (!ok) continue;
      int k0 = box_start[b], k1 = box_start[b + 1], o = s_off[t];
      for (int k = k0; k < k1; ++k) s_q[o + k - k0] = q[k];
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p1 = g.p + 1, nst = p1 * p1 * p1;
  const int shift = (g.p - 1) / 2;
  for (int ob = wave; ob < nobs; ob += 4) {
    const int bx = bx0 + ob;
    const int r0 = box_start[brow + bx], r1 = box_start[brow + bx + 1];
    if (r0 == r1) continue;
    // window of pair i: staged columns [ob, ob + 2 rb]
    int len = 0, wst = 0;
    if (lane < npair) {
      wst = s_off[lane * C + ob];
      len = s_off[lane * C + ob + 2 * rb + 1] - wst;
    }
    int S;
    const int woff = wave_excl_scan<64>(len, lane, S);
    const int wend = lane < npair ? woff + len : 0x7fffffff;
    // source charges of this box's windows, cached per lane (j = lane + 64 k)
    float qv[kIcKQ];
    const int nk = (S + 63) >> 6;
    const bool cached = nk <= kIcKQ;
    auto charge = [&](int j) -> float {
      // pair holding local index j: first lane whose window end exceeds j
      int lo = 0;
#pragma unroll
      for (int step = 32; step >= 1; step >>= 1) {
        int cand = lo + step - 1;
        int e = __shfl(wend, cand < 63 ? cand : 63, 64);
        if (e <= j) lo += step;
      }
      int i = lo;
      int o = __shfl(woff, i, 64), st = __shfl(wst, i, 64);
      int loc = j - o;
      if (staged) return s_q[st + loc];
      // unstaged: walk the window's boxes in global memory
      for (int c = 0; c <= 2 * rb; ++c) {
        bool ok;
        int64_t b = src_box(i, ob + c, ok);
        if (!ok) continue;
        int nb = box_start[b + 1] - box_start[b];
        if (loc < nb) return q[box_start[b] + loc];
        loc -= nb;
      }
      return 0.f;
    };
    if (cached) {
#pragma unroll
      for (int k = 0; k < kIcKQ; ++k) {
        float v = 0.f;
        if (k < nk) {
          int j = lane + 64 * k;
          float c = charge(j < S ? j : 0);
          v = j < S ? c : 0.f;
        }
        qv[k] = v;
      }
    }
    // stencil values of U for this box (same start for every row of the box)
    int sta[3];
    const int bxyz[3] = {bx, by, bz};
    for (int a = 0; a < 3; ++a) {
      int st = bxyz[a] - shift;
      if (g.per[a]) {
        if (st < 0) st += g.N[a];
      } else {
        st = min(max(st, 0), g.N[a] - g.p - 1);
      }
      sta[a] = st;
    }
    float uv[4];
    int lax[4], lay[4], laz[4];
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      int l = lane + 64 * s2;
      uv[s2] = 0.f;
      lax[s2] = lay[s2] = laz[s2] = 0;
      if (l < nst) {
        int ax = l % p1, ay = (l / p1) % p1, az = l / (p1 * p1);
        int gx = sta[0] + ax, gy = sta[1] + ay, gz = sta[2] + az;
        if (gx >= g.N[0]) gx -= g.N[0];
        if (gy >= g.N[1]) gy -= g.N[1];
        if (gz >= g.N[2]) gz -= g.N[2];
        uv[s2] = U[((int64_t)gz * g.N[1] + gy) * g.N[0] + gx];
        lax[s2] = ax;
        lay[s2] = ay;
        laz[s2] = az;
      }
    }
    for (int r = r0; r < r1; ++r) {
      const int pr = prp[r];
      const int rl = min(S, prp[r + 1] - pr);  // equal by construction; guards the reads
      float acc = 0.f;
      if (cached) {
        float pv[kIcKQ];
#pragma unroll
        for (int k = 0; k < kIcKQ; ++k) {
          int j = lane + 64 * k;
          pv[k] = (k < nk && j < rl) ? pval[pr + j] : 0.f;
        }
#pragma unroll
        for (int k = 0; k < kIcKQ; ++k) acc += pv[k] * qv[k];
      } else {
        for (int k = 0; k < nk; ++k) {
          int j = lane + 64 * k;
          float c = charge(j < S ? j : 0);
          if (j < rl) acc += pval[pr + j] * c;
        }
      }
      const float4 xi = pos4[r];
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2) {
        if (lane + 64 * s2 < nst)
          acc += uv[s2] * (lagrange(lax[s2], xi.x, g.p) * lagrange(lay[s2], xi.y, g.p) *
                           lagrange(laz[s2], xi.z, g.p));
      }
      acc = group_sum<64>(acc);
      if (lane == 0) u[r] = acc + uz[r];
    }
  }
}

// ---------------------------------------------------------------------------
// gradient + sum: 16 lanes per row; writes h[n][3]

__global__ void __launch_bounds__(256) k_grad(int64_t n, const int32_t* __restrict__ rp,
                                              const int32_t* __restrict__ col,
                                              const float4* __restrict__ gv,
                                              const float* __restrict__ u,
                                              const float4* __restrict__ hex,
                                              float* __restrict__ h, float hax, float hay,
                                              float haz, int with_ms) {
  int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  int lane = threadIdx.x & 15;
  if (row >= n) return;
  float gx = 0.f, gy = 0.f, gz = 0.f;
  if (with_ms) {
    int e0 = rp[row], e1 = rp[row + 1];
    for (int e = e0 + lane; e < e1; e += 16) {
      float4 w = gv[e];
      float uk = u[col[e]];
      gx += w.x * uk;
      gy += w.y * uk;
      gz += w.z * uk;
    }
  }
  gx = group_sum<16>(gx);
  gy = group_sum<16>(gy);
  gz = group_sum<16>(gz);
  if (lane == 0) {
    float4 he = hex[row];
    h[3 * row] = he.x - gx + hax;
    h[3 * row + 1] = he.y - gy + hay;
    h[3 * row + 2] = he.z - gz + haz;
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
                                                const float4* __restrict__ hex,
                                                const float* __restrict__ q,
                                                const float* __restrict__ u,
                                                double* __restrict__ part) {
  __shared__ double s0[256], s1[256];
  double a = 0.0, b = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    float4 he = hex[i];
    a += mu[i] * (m[3 * i] * he.x + m[3 * i + 1] * he.y + m[3 * i + 2] * he.z);
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

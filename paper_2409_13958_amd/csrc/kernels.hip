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
  // basis function a of the Lagrange interpolant through 0..p, at xi
  float v = 1.0f;
  for (int c = 0; c <= p; ++c) {
    if (c == a) continue;
    v *= (xi - (float)c) / (float)(a - c);
  }
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
// anterpolation: one thread per grid point gathers from the boxes whose
// stencils cover it (box ranges per axis precomputed on the host)

__global__ void __launch_bounds__(256) k_anterp(
    GridParams g, const float* __restrict__ q, const float4* __restrict__ pos4,
    const int32_t* __restrict__ box_start, const int2* __restrict__ brx,
    const int2* __restrict__ bry, const int2* __restrict__ brz, float* __restrict__ Q) {
  int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t ng = (int64_t)g.N[0] * g.N[1] * g.N[2];
  if (gid >= ng) return;
  int gx = (int)(gid % g.N[0]);
  int gy = (int)((gid / g.N[0]) % g.N[1]);
  int gz = (int)(gid / ((int64_t)g.N[0] * g.N[1]));
  int2 rx = brx[gx], ry = bry[gy], rz = brz[gz];
  float acc = 0.f;
  for (int iz = 0; iz < rz.y; ++iz) {
    int bz = rz.x + iz;
    if (bz >= g.nbox[2]) bz -= g.nbox[2];
    for (int iy = 0; iy < ry.y; ++iy) {
      int by = ry.x + iy;
      if (by >= g.nbox[1]) by -= g.nbox[1];
      for (int ix = 0; ix < rx.y; ++ix) {
        int bxx = rx.x + ix;
        if (bxx >= g.nbox[0]) bxx -= g.nbox[0];
        int64_t b = ((int64_t)bz * g.nbox[1] + by) * g.nbox[0] + bxx;
        int s0 = box_start[b], s1 = box_start[b + 1];
        for (int k = s0; k < s1; ++k) {
          float4 pp = pos4[k];
          uint32_t pk = __float_as_uint(pp.w);
          int ax = gx - st_of(pk, 0);
          int ay = gy - st_of(pk, 1);
          int az = gz - st_of(pk, 2);
          if (ax < 0) ax += g.N[0];
          if (ay < 0) ay += g.N[1];
          if (az < 0) az += g.N[2];
          float w = lagrange(ax, pp.x, g.p) * lagrange(ay, pp.y, g.p) * lagrange(az, pp.z, g.p);
          acc += w * q[k];
        }
      }
    }
  }
  Q[gid] = acc;
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
// interpolation + precorrection: one wavefront per row

__global__ void __launch_bounds__(256) k_interp_corr(
    GridParams g, int64_t n, const float* __restrict__ U, const float4* __restrict__ pos4,
    const int32_t* __restrict__ prp, const int32_t* __restrict__ pcol,
    const float* __restrict__ pval, const float* __restrict__ q, const float* __restrict__ uz,
    float* __restrict__ u) {
  int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (row >= n) return;
  float4 pp = pos4[row];
  uint32_t pk = __float_as_uint(pp.w);
  int sx = st_of(pk, 0), sy = st_of(pk, 1), sz = st_of(pk, 2);
  const int p1 = g.p + 1;
  const int nst = p1 * p1 * p1;
  float acc = 0.f;
  for (int l = lane; l < nst; l += 64) {
    int ax = l % p1, ay = (l / p1) % p1, az = l / (p1 * p1);
    int gx = sx + ax, gy = sy + ay, gz = sz + az;
    if (gx >= g.N[0]) gx -= g.N[0];
    if (gy >= g.N[1]) gy -= g.N[1];
    if (gz >= g.N[2]) gz -= g.N[2];
    float w = lagrange(ax, pp.x, g.p) * lagrange(ay, pp.y, g.p) * lagrange(az, pp.z, g.p);
    acc += w * U[((int64_t)gz * g.N[1] + gy) * g.N[0] + gx];
  }
  int e0 = prp[row], e1 = prp[row + 1];
  for (int e = e0 + lane; e < e1; e += 64) acc += pval[e] * q[pcol[e]];
  acc = group_sum<64>(acc);
  if (lane == 0) u[row] = acc + uz[row];
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

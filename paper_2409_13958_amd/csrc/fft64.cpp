// FP64 complex 3D FFT on the host, used once per build to take the
// spectrum of the sampled periodic Green's function. Mixed radix: each
// extent is a product of the factors 2, 3, 5 and 7; a transform of length
// n = r m splits into r interleaved transforms of length m (decimation in
// time) whose outputs are combined by r-point DFTs with twiddles.
#include <cmath>
#include <complex>
#include <vector>

#include "internal.h"

namespace pmfem {
namespace {

using cplx = std::complex<double>;

int first_factor(int n) {
  for (int r : {4, 2, 3, 5, 7})
    if (n % r == 0) return r;
  return n;  // a prime beyond 7: the direct DFT below
}

// out[k] = sum_j in[j s] w^(j k), w = exp(-2 pi i / n), k < n
void fft_rec(const cplx* in, int64_t s, cplx* out, int n, const std::vector<cplx>& w, int wstep) {
  if (n == 1) {
    out[0] = in[0];
    return;
  }
  const int r = first_factor(n), m = n / r;
  for (int q = 0; q < r; ++q) fft_rec(in + q * s, s * r, out + (int64_t)q * m, m, w, wstep * r);
  std::vector<cplx> t(r);
  for (int k = 0; k < m; ++k) {
    for (int q = 0; q < r; ++q) t[q] = out[(int64_t)q * m + k] * w[((int64_t)q * k * wstep) % ((int64_t)n * wstep)];
    for (int p = 0; p < r; ++p) {
      cplx acc = 0.0;
      for (int q = 0; q < r; ++q) acc += t[q] * w[((int64_t)q * p * m * wstep) % ((int64_t)n * wstep)];
      out[(int64_t)p * m + k] = acc;
    }
  }
}

}  // namespace

void fft3_inplace(std::vector<double>& re, std::vector<double>& im, const int M[3]) {
  const int64_t sx = 1, sy = M[0], sz = (int64_t)M[0] * M[1];
  const int64_t strides[3] = {sx, sy, sz};
  for (int ax = 0; ax < 3; ++ax) {
    const int n = M[ax];
    // w[t] = exp(-2 pi i t / n), t < n
    std::vector<cplx> w(n);
    for (int t = 0; t < n; ++t) w[t] = std::polar(1.0, -2.0 * kPi * t / n);
    int o1 = (ax + 1) % 3, o2 = (ax + 2) % 3;
    int64_t lines = (int64_t)M[o1] * M[o2];
    parallel_for(lines, [&](int64_t l) {
      int64_t i1 = l % M[o1], i2 = l / M[o1];
      int64_t base = i1 * strides[o1] + i2 * strides[o2];
      std::vector<cplx> in(n), out(n);
      for (int k = 0; k < n; ++k) in[k] = cplx(re[base + k * strides[ax]], im[base + k * strides[ax]]);
      fft_rec(in.data(), 1, out.data(), n, w, 1);
      for (int k = 0; k < n; ++k) {
        re[base + k * strides[ax]] = out[k].real();
        im[base + k * strides[ax]] = out[k].imag();
      }
    }, 16);
  }
}

}  // namespace pmfem

// FP64 complex 3D FFT on the host, used once per build to take the
// spectrum of the sampled periodic Green's function. Iterative radix-2
// decimation in time along each axis; extents are powers of two.
#include <cmath>
#include <vector>

#include "internal.h"

namespace pmfem {
namespace {

void fft1(double* re, double* im, int n, const std::vector<double>& cr,
          const std::vector<double>& ci) {
  for (int i = 1, j = 0; i < n; ++i) {  // bit reversal
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) {
      std::swap(re[i], re[j]);
      std::swap(im[i], im[j]);
    }
  }
  for (int len = 2; len <= n; len <<= 1) {
    int half = len >> 1, step = n / len;
    for (int s = 0; s < n; s += len)
      for (int k = 0; k < half; ++k) {
        double wr = cr[k * step], wi = ci[k * step];
        double xr = re[s + k + half], xi = im[s + k + half];
        double tr = xr * wr - xi * wi, ti = xr * wi + xi * wr;
        re[s + k + half] = re[s + k] - tr;
        im[s + k + half] = im[s + k] - ti;
        re[s + k] += tr;
        im[s + k] += ti;
      }
  }
}

}  // namespace

void fft3_inplace(std::vector<double>& re, std::vector<double>& im, const int M[3]) {
  const int64_t sx = 1, sy = M[0], sz = (int64_t)M[0] * M[1];
  const int64_t strides[3] = {sx, sy, sz};
  for (int ax = 0; ax < 3; ++ax) {
    int n = M[ax];
    std::vector<double> cr(n / 2 + 1), ci(n / 2 + 1);
    for (int k = 0; k <= n / 2; ++k) {
      cr[k] = std::cos(2.0 * kPi * k / n);
      ci[k] = -std::sin(2.0 * kPi * k / n);
    }
    int o1 = (ax + 1) % 3, o2 = (ax + 2) % 3;
    int64_t lines = (int64_t)M[o1] * M[o2];
    parallel_for(lines, [&](int64_t l) {
      int64_t i1 = l % M[o1], i2 = l / M[o1];
      int64_t base = i1 * strides[o1] + i2 * strides[o2];
      std::vector<double> br(n), bi(n);
      for (int k = 0; k < n; ++k) {
        br[k] = re[base + k * strides[ax]];
        bi[k] = im[base + k * strides[ax]];
      }
      fft1(br.data(), bi.data(), n, cr, ci);
      for (int k = 0; k < n; ++k) {
        re[base + k * strides[ax]] = br[k];
        im[base + k * strides[ax]] = bi[k];
      }
    }, 16);
  }
}

}  // namespace pmfem

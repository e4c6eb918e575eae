// Internal state of a pmfem context, shared by the host setup (C++) and the
// device code (HIP) of the library. Not part of the public ABI.
#pragma once

#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pmfem.h"

namespace pmfem {

constexpr double kMu0 = 4e-7 * 3.14159265358979323846;
constexpr double kPi = 3.14159265358979323846;
constexpr double kGamma0 = kMu0 * 1.76086e11;  // m/(A s)

struct Error {
  int code;
  std::string msg;
};

// Operators assembled on the host (FP64 arithmetic, stored as FP32 where
// the device reads them).
struct HostOps {
  int64_t n_nodes = 0, n_unk = 0;
  std::vector<int64_t> unk_of_node;   // [N]
  std::vector<int64_t> node_of_unk;   // [N'] LCA representative, box-sorted order
  std::vector<double> mu;             // [N'] sum_t Ms_t V_t / 4
  std::vector<double> pos;            // [N'][3] folded positions (Eq. shift_hms)
  // grid
  int N[3] = {0, 0, 0}, M[3] = {0, 0, 0}, per[3] = {0, 0, 0}, nbox[3] = {0, 0, 0};
  double delta[3] = {0, 0, 0}, origin[3] = {0, 0, 0};
  int p = 3, rb = 2;
  std::vector<float> pos4;            // [N'][4]: xi_x, xi_y, xi_z, packed box coordinates
  std::vector<int32_t> box_start;     // [nbox+1]
  // local CSR (shared pattern of exchange, charge, gradient)
  std::vector<int32_t> loc_rowptr, loc_col;
  std::vector<float> loc_val;         // [nnz][8]: L, Dx, Dy, Dz, Gx, Gy, Gz, 0
  // element-exact correction
  std::vector<int32_t> z0_rowptr, z0_col;
  std::vector<float> z0_val;          // [nnz][4]: Zx, Zy, Zz, 0
  // precorrection (already scaled by 1/(4 pi))
  std::vector<int32_t> p_rowptr, p_col;
  std::vector<float> p_val;
  // grid kernel and its spectrum
  std::vector<double> kgrid;          // [Mz][My][Mx] FP64 samples of the PGF
  std::vector<float> khat;            // [Mz][My][Mx/2+1], scaled by 1/(4 pi Mx My Mz)
  double hbar = 0.0;
};

}  // namespace pmfem

struct pmfem_dev;  // device buffers, defined in the HIP source

struct pmfem_ctx {
  int device = -1;
  void* stream = nullptr;
  // inputs
  int64_t n_nodes = 0, n_tets = 0;
  std::vector<double> xyz;
  std::vector<int32_t> tets, region;
  int32_t n_regions = 0;
  std::vector<double> Ms, Aex;
  uint32_t mask = 0;
  double L[3] = {0, 0, 0};
  double match_tol = 1e-9;
  int32_t grid[3] = {0, 0, 0};
  int32_t order_p = 3, near_boxes = 2, precision = 0;
  double z0_radius = 1.0;
  int32_t variant[4] = {0, 0, 0, 0};  // anterp, interp, fft forms, spmv lanes (0 = automatic)
  bool have_mesh = false, have_mat = false, have_aim = false;
  bool built = false;
  pmfem::HostOps ops;
  pmfem_dev* dev = nullptr;
  std::string err;
};

namespace pmfem {

// Host setup (setup.cpp). Returns PMFEM_OK or an error code; fills ctx->err.
int host_build(pmfem_ctx* ctx);
// Periodic Green's function (pgf.cpp).
double pgf_default_eta(uint32_t mask, const double L[3]);
void pgf_eval(uint32_t mask, const double L[3], double eta, int64_t n, const double* r,
              double* out);
// Element-exact correction (z0.cpp).
int build_z0(pmfem_ctx* ctx, const std::vector<uint8_t>& surface);
// FP64 complex FFT used for the kernel spectrum (fft64.cpp).
void fft3_inplace(std::vector<double>& re, std::vector<double>& im, const int M[3]);

// Thread count for host setup: OMP_NUM_THREADS if set, else the hardware.
inline unsigned host_threads() {
  unsigned hw = std::thread::hardware_concurrency();
  if (hw == 0) hw = 1;
  const char* s = std::getenv("OMP_NUM_THREADS");
  if (s) {
    long v = std::strtol(s, nullptr, 10);
    if (v > 0 && (unsigned)v < hw) hw = (unsigned)v;
  }
  return hw > 64 ? 64 : hw;
}

// Dynamic parallel loop over [0, n) in chunks of `grain`.
template <class F>
void parallel_for(int64_t n, F&& f, int64_t grain = 256) {
  if (n <= 0) return;
  unsigned nt = host_threads();
  if (nt <= 1 || n <= grain) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int64_t> next(0);
  auto work = [&]() {
    for (;;) {
      int64_t s = next.fetch_add(grain);
      if (s >= n) break;
      int64_t e = s + grain < n ? s + grain : n;
      for (int64_t i = s; i < e; ++i) f(i);
    }
  };
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nt; ++t) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
}

}  // namespace pmfem

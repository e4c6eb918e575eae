// Kernel declarations and launch parameters shared by kernels.hip and capi.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace pmfem {

struct GridParams {
  int N[3];     // grid points per axis
  int M[3];     // FFT extents (N periodic, 2N otherwise)
  int logM[3];
  int nbox[3];  // boxes per axis
  int per[3];   // periodic axes
  int p;        // Lagrange order
  int rb;       // near-region radius in boxes (<= 3)
  int gmode;    // storage of the grid charges Q and potential U between
                // kernels: 0 FP32; 1 BF16; 2 BF16 pair hi + lo (the hi part
                // in the first N_g halves of the buffer, the lo part after)
};

// anterpolation tile (grid points per workgroup) and staged-node capacity
constexpr int kAntTX = 8, kAntTY = 8, kAntTZ = 4;
constexpr int kAntCap = 2560;
constexpr int kAntHalo = (kAntTX + 6) * (kAntTY + 6) * (kAntTZ + 6) + 1;

// interpolation/precorrection by tiles of observer boxes: one workgroup per
// xs boxes along x times tz box rows along z at one y. Sizes and LDS layout
// (byte offsets into the dynamic LDS block) are chosen on the host from the
// box table so that every staged array fits.
struct IcPlan {
  int xs, tz;    // observer boxes per tile along x and z
  int nsx, nsz;  // tiles along x and z
  int sbx, szr;  // staged box columns (xs + 2 r_b) and z rows (tz + 2 r_b)
  int qcap;      // staged source charges
  int rcap;      // observer rows per tile
  int ux, uzl;   // staged potential: points per line (xs + p), z-lines (tz + p)
  int kc;        // chunks per lane in registers (2, 4, 6 or 8)
  int o_q, o_u, o_seg;  // LDS byte offsets
  int lds_bytes;
};

// anterpolation by grid lines: one workgroup per segment of `xa` points of
// one (y, z) grid line; sizes and LDS layout chosen on the host.
struct AntPlan {
  int xa;     // points per segment (= threads per workgroup)
  int nsx;    // segments per line
  int nrow;   // box rows reaching a line: ((p + 1)^2 at most)
  int sbx;    // staged boxes per box row (upper bound over segments)
  int ncap;   // staged nodes per workgroup
  int o_x, o_c, o_st, o_meta, o_off;  // LDS byte offsets
  int lds_bytes;
};

// anterpolation by scatter: one 64-lane workgroup per tile of
// tb[0] x tb[1] x tb[2] boxes, its footprint (the grid points the stencils
// of its boxes cover) fd[0] x fd[1] x fd[2] points at most
struct ScPlan {
  int tb[3];  // boxes per tile along each axis
  int nt[3];  // tiles along each axis
  int fd[3];  // footprint extent along each axis (tb + p at most)
  int fsize;  // fd[0] fd[1] fd[2]
  int lds_bytes;
};

// One unit cell of a batch: its grid and kernel plans, its own operator
// arrays, and its slices of the batch's per-unknown vectors. The multi-cell
// kernels (k_*_cells) take every workgroup's cell from a block-to-cell table
// and its workgroup index within the cell from the cell's first block.
struct CellTab {
  GridParams g;
  ScPlan sp;
  IcPlan icp;
  const float4* pos4;
  const int2* sc_list;
  const int32_t* sc_lstart;
  const int2* sc_tab[3];
  float* sc_part;
  float* grid;
  float2* spec;
  const float* khat;
  const float2 *twx, *twy, *twz;
  const float2 *twfx, *twfy, *twfz;  // full-circle tables of the mixed-radix passes
  const int32_t *ic_list, *ic_lstart, *ic_wseg;
  const uint32_t* ic_rdesc;
  const int32_t* prp;
  const float* pv;
  int lpb, by;      // per-axis FFT form: x lines per block, y columns per block
  const float* q;   // the cell's charges in the batch vector
  const float* uz;  // element correction
  float* u;         // potential
};

template <int G>
__global__ void k_rowdot3(int64_t n, const float* m, const int32_t* rp, const int4* rec,
                          float* out);
__global__ void k_anterp(GridParams g, const float* q, const float4* pos4,
                         const int32_t* box_start, const int2* brx, const int2* bry,
                         const int2* brz, float* Q);
__global__ void k_anterp_line(GridParams g, AntPlan pl, const float* q, const float4* pos4,
                              const int32_t* list, const int32_t* lstart, const int32_t* colst,
                              const int2* brx, const int2* bry, const int2* brz, float* Q);
template <int P>
__global__ void k_anterp_scatter(GridParams g, ScPlan pl, const float* q, const float4* pos4,
                                 const int2* list, const int32_t* lstart, float* part);
template <int PT>
__global__ void k_anterp_sum(GridParams g, ScPlan pl, const int2* tabx, const int2* taby,
                             const int2* tabz, const float* part, float* Q);
__global__ void k_r2c_x(GridParams g, const float* Q, float2* spec, const float2* twx,
                        int lines_per_block);
__global__ void k_fft_y(GridParams g, float2* spec, const float2* twy, int B, int inverse,
                        int n_in, int n_out);
// nsplit workgroups per z-plane (1 or 2)
__global__ void k_fft_xy_fwd(GridParams g, const float* Q, float2* spec, const float2* twx,
                             const float2* twy, int nsplit);
__global__ void k_fft_yx_inv(GridParams g, const float2* spec, float* U, const float2* twx,
                             const float2* twy, int nsplit);
__global__ void k_fft_z_mul(GridParams g, float2* spec, const float* khat, const float2* twz,
                            int B);
__global__ void k_c2r_x(GridParams g, const float2* spec, float* U, const float2* twx,
                        int lines_per_block);
// mixed-radix forms (extents that are products of 2, 3, 5, 7); twf[t] =
// exp(-2 pi i t / M) for t < M; dynamic LDS: (M + 2 lines M) complex values
__global__ void k_r2c_x_mr(GridParams g, const float* Q, float2* spec, const float2* twf,
                           int lines_per_block);
__global__ void k_fft_y_mr(GridParams g, float2* spec, const float2* twf, int B, int inverse,
                           int n_in, int n_out);
__global__ void k_fft_z_mul_mr(GridParams g, float2* spec, const float* khat, const float2* twf,
                               int B);
__global__ void k_c2r_x_mr(GridParams g, const float2* spec, float* U, const float2* twf,
                           int lines_per_block);
__global__ void k_fft_xy_fwd_mr(GridParams g, const float* Q, float2* spec, const float2* twfx,
                                const float2* twfy);
__global__ void k_fft_yx_inv_mr(GridParams g, const float2* spec, float* U, const float2* twfx,
                                const float2* twfy);
__global__ void k_fft_xy_fwd_mr_cells(const CellTab* tab, const int32_t* bcell,
                                      const int32_t* boff);
__global__ void k_fft_yx_inv_mr_cells(const CellTab* tab, const int32_t* bcell,
                                      const int32_t* boff);
__global__ void k_r2c_x_mr_cells(const CellTab* tab, const int32_t* bcell, const int32_t* boff);
__global__ void k_fft_y_mr_cells(const CellTab* tab, const int32_t* bcell, const int32_t* boff,
                                 int inverse);
__global__ void k_fft_z_mul_mr_cells(const CellTab* tab, const int32_t* bcell,
                                     const int32_t* boff, int B);
__global__ void k_c2r_x_mr_cells(const CellTab* tab, const int32_t* bcell, const int32_t* boff);

// lanes per observer row of k_interp_tile (8 x 16 B = one 128 B line per
// load; 4 and 16 measured slower)
constexpr int kIcLanes = 8;
// WT = 2 r_b + 1 runs per row; KC = 4-value chunks per lane held in registers
template <int WT, int KC>
__global__ void k_interp_tile(GridParams g, IcPlan pl, const float* U, const float4* pos4,
                              const int32_t* list, const int32_t* lstart, const int32_t* wseg,
                              const uint32_t* rdesc, const int32_t* prp, const float* pval,
                              const float* q, const float* uz, float* u);
// multi-cell forms (one launch for every cell of a batch)
template <int P>
__global__ void k_anterp_scatter_cells(const CellTab* tab, const int32_t* bcell,
                                       const int32_t* boff);
template <int PT>
__global__ void k_anterp_sum_cells(const CellTab* tab, const int32_t* bcell, const int32_t* boff);
__global__ void k_fft_xy_fwd_cells(const CellTab* tab, const int32_t* bcell, const int32_t* boff,
                                   int nsplit);
__global__ void k_fft_yx_inv_cells(const CellTab* tab, const int32_t* bcell, const int32_t* boff,
                                   int nsplit);
__global__ void k_fft_z_mul_cells(const CellTab* tab, const int32_t* bcell, const int32_t* boff,
                                  int B);
template <int WT, int KC>
__global__ void k_interp_tile_cells(const CellTab* tab, const int32_t* bcell, const int32_t* boff);
__global__ void k_r2c_x_cells(const CellTab* tab, const int32_t* bcell, const int32_t* boff);
__global__ void k_fft_y_cells(const CellTab* tab, const int32_t* bcell, const int32_t* boff,
                              int inverse);
__global__ void k_c2r_x_cells(const CellTab* tab, const int32_t* bcell, const int32_t* boff);
template <int G, typename MT>
__global__ void k_exch(int64_t n, const int32_t* rp, const int2* lrec, const MT* m, float* hex);
template <int G>
__global__ void k_gsum(int64_t n, const int32_t* rp, const int4* grec, const float* u,
                       const float* hex, float* h, float hax, float hay, float haz, int with_hex,
                       int with_ms);
__global__ void k_rk_stage(int64_t n, const double* m, const double* k, double c, double* mst,
                           float* m32);
__global__ void k_rk_rhs(int64_t n, const double* mst, const float* h, double pref,
                         double alpha, double* kout, double* acc, double weight, int first);
__global__ void k_rk_final(int64_t n, double* m, const double* acc, double dt6);
__global__ void k_mid_normalize(int64_t n, double* x);
__global__ void k_energy(int64_t n, const double* m, const double* mu, const float* hex,
                         const float* q, const float* u, double* part);
// implicit midpoint LLG (Newton-Krylov)
__global__ void k_mid_point(int64_t n3, const double* m, const double* x, double theta, double* mb,
                            float* mb32);
__global__ void k_mid_residual(int64_t n, const double* m, const double* x, const double* mb,
                               const float* H, const double* adiag, double dt, double c,
                               double alpha, double theta, double* G, double* Minv, double* part);
template <typename VT>
__global__ void k_mid_precond(int64_t n, const double* Minv, const VT* v, double* z, float* z32);
constexpr int kGsMaxVectors = 64;  // Krylov vectors one Gram-Schmidt update takes
__global__ void k_gs_dots(int64_t n3, const float* V, int64_t ldv, int nv, const double* w,
                          double* part);
__global__ void k_gs_update(int64_t n3, const float* V, int64_t ldv, int nv, const double* h,
                            double* w, double* part);
__global__ void k_gs_store(int64_t n3, const double* w, double s, float* out);
__global__ void k_gs_combine(int64_t n3, const float* V, int64_t ldv, int nv, const double* coef,
                             double* out);
__global__ void k_mid_jvp(int64_t n, const double* z, const float* Az, const double* mb,
                          const float* H, double s, double alpha, double* w);
__global__ void k_mdot(int64_t n3, const double* V, int64_t ldv, int nv, const double* w,
                       double* part);
__global__ void k_sum_parts(const double* part, int nparts, double* out);
__global__ void k_lincomb(int64_t n3, const double* V, int64_t ldv, int nv, const double* coef,
                          double aw, const double* w, double* out);

}  // namespace pmfem

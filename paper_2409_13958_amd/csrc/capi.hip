// C ABI of the library: context lifecycle, upload of the host-built
// operators, and the launch sequence of one effective-field evaluation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "surrogate.h"

using namespace pmfem;

// launch shapes (each the best of the measured alternatives on MI355X)
constexpr int kFftzB = 8;            // z columns per workgroup of the z pass
// z columns per workgroup of the mixed-radix z pass (short columns: many)
constexpr int kFftzMr = 64;
// threads of a mixed-radix plane workgroup
constexpr int kFftPlaneMrT = 512;
constexpr int kFftzT = 256;          // threads per workgroup of the z pass
constexpr int kFftSplit = 2;         // workgroups per z-plane in the plane transforms
constexpr int kIcLdsBudget = 24576;  // LDS bytes per interpolation tile
constexpr int kScTile[3] = {8, 8, 4};  // preferred boxes per scatter tile along x, y, z
constexpr int kScLdsBudget = 65536;    // LDS bytes of a scatter tile's footprint copies

// Scratch of pmfem_grid_convolve_noalloc: the half-spectrum of one grid
// convolution, at most kNoallocSpecMax complex values (16 MiB). Every device
// the library runs on holds its own copy until the process ends. Host code
// never uses the array's name as an address: the per-device address comes
// from hipGetSymbolAddress at context creation (scratch_ptr below). The host
// reference makes clang emit the array as a global symbol of the device code
// object, which the runtime looks up; an explicit `used` attribute would keep
// it local, where the lookup cannot find it.
constexpr int64_t kNoallocSpecMax = (int64_t)1 << 21;
static __device__ __align__(256) float2 scratch[kNoallocSpecMax];

struct pmfem_dev {
  int64_t n = 0;
  GridParams g{};
  float4* pos4 = nullptr;
  int32_t* box_start = nullptr;
  AntPlan ap{};            // line form of anterpolation
  int32_t *ant_list = nullptr, *ant_lstart = nullptr, *ant_col = nullptr;  // its node lists
  bool ant_ok = false, ic_ok = false, fft_ok = false;  // the plans fit
  bool ant_line = false;   // false: the tile form k_anterp
  int ant_threads = 0;
  ScPlan sp{};              // scatter form of anterpolation
  bool sc_ok = false, ant_scatter = false;
  int2* sc_list = nullptr;     // {node, stencil offset in the footprint} of every tile, box order
  int32_t* sc_lstart = nullptr;
  int2* sc_tab[3] = {};     // per axis and grid index: (tile, offset) of the covering tiles
  float* sc_part = nullptr; // footprint sums of every tile
  IcPlan icp{}, icp_small{};  // interpolation+precorrection tiles: chosen, narrow
  struct IcLists {
    int32_t *list = nullptr, *lstart = nullptr, *wseg = nullptr;
    uint32_t* rdesc = nullptr;
  } icl, icl_small;
  bool ic_small_ok = false;
  bool ic_seg = false;        // false: the narrow tiles
  bool fft_plane = false;  // x and y transforms of a whole z-plane in one kernel
  bool fft_mr = false;     // an FFT extent is not a power of two: mixed-radix passes
  float2 *twfx = nullptr, *twfy = nullptr, *twfz = nullptr;  // full-circle twiddles (mixed radix)
  size_t fft_plane_lds = 0;
  const char* kname[12] = {};  // kernel in each profiling slot
  hipStream_t side = nullptr;   // second stream: element correction beside the grid steps
  hipEvent_t fork = nullptr, join = nullptr;
  int2 *brx = nullptr, *bry = nullptr, *brz = nullptr;
  int32_t* lrp = nullptr;
  int4* drec = nullptr;   // charge operator D: {column, Dx, Dy, Dz}
  int2* lrec = nullptr;   // exchange: {column, L}
  int4* grec = nullptr;   // gradient: {column, Gx, Gy, Gz}
  int32_t* zrp = nullptr;
  int4* zrec = nullptr;   // element correction Z0: {column, Zx, Zy, Zz}
  int lanes_l = 4, lanes_z = 8;  // lanes per row on the local and element-correction patterns
  int auto_l = 4, auto_z = 8;     // chosen from the mean row lengths
  int32_t* prp = nullptr;  // device precorrection rows (runs padded to 4 values)
  float* pv = nullptr;
  int64_t nnz_p_dev = 0;
  float* khat = nullptr;
  float2 *twx = nullptr, *twy = nullptr, *twz = nullptr;
  double* mu = nullptr;
  float* hex = nullptr;  // [n][3] exchange field for pmfem_energy / heff_parts
  float *q = nullptr, *uz = nullptr, *u = nullptr, *grid = nullptr;
  float2* spec = nullptr;
  double *mst = nullptr, *kk = nullptr, *acc = nullptr;
  float *m32 = nullptr, *h32 = nullptr;
  double* part = nullptr;
  int nparts = 0;
  // implicit midpoint LLG workspace, allocated by the first pmfem_llg_implicit
  // call (again if a later call asks for a larger Krylov space)
  struct Implicit {
    int kdim = 0;
    double *x = nullptr, *mb = nullptr, *G = nullptr, *Minv = nullptr, *adiag = nullptr;
    float* V = nullptr;  // Krylov basis, FP32
    double *w = nullptr, *z = nullptr, *part = nullptr, *red = nullptr;
    double* coef = nullptr;
    float *mb32 = nullptr, *H = nullptr, *z32 = nullptr, *Az = nullptr;
    double* host = nullptr;  // pinned: coefficients out, reductions back
    double *xp = nullptr, *S = nullptr;  // adaptive steps: predictor, two slopes or states
    double* r = nullptr;                 // BDF2: the combination of past states
  } imp;
  // one captured RK4 step (pmfem_llg_step_graph) and what it was captured for
  struct StepGraph {
    hipStream_t cap = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    double* m = nullptr;
    double dt = 0.0, alpha = 0.0, happ[3] = {0.0, 0.0, 0.0};
    bool with_happ = false;
    bool net_on = false;       // captured with the surrogate in place of the FFT
    uint64_t net_version = 0;  // of that surrogate
  } sg;
  // learned surrogate of the grid convolution; net_on makes run_heff use it
  // in place of the FFT convolution. tap_q / tap_u, when set, receive copies
  // of the grid charges and potential of the next evaluation.
  Surrogate* net = nullptr;
  bool net_on = false;
  uint64_t net_version = 0;  // bumped whenever its buffers or scales may change
  float *tap_q = nullptr, *tap_u = nullptr;
  std::vector<void*> allocs;
  // profiling
  int prof_max = 0, prof_calls = 0;
  std::vector<hipEvent_t> ev;  // [calls][kernels][2]
};

namespace {

constexpr int kNumKernels = 12;
int set_err(pmfem_ctx* c, int code, const std::string& m) {
  if (c) c->err = m;
  return code;
}

int hip_err(pmfem_ctx* c, hipError_t e, const char* where) {
  return set_err(c, PMFEM_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

// Device address of `scratch` on each device, looked up once per device.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float2* g_scratch_ptr[kMaxDevices] = {};

int lookup_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return PMFEM_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return PMFEM_OK;
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) return PMFEM_EHIP;
  if (hipSetDevice(device) != hipSuccess) return PMFEM_EHIP;
  float2* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  (void)hipSetDevice(prev);
  if (e != hipSuccess || !ptr) return PMFEM_EHIP;
  g_scratch_ptr[device] = ptr;
  return PMFEM_OK;
}

float2* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}

template <class T>
int dalloc(pmfem_ctx* c, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) return set_err(c, PMFEM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  c->dev->allocs.push_back((void*)*p);
  return PMFEM_OK;
}

template <class T>
int upload(pmfem_ctx* c, T** p, const void* src, size_t count) {
  int rc = dalloc(c, p, count);
  if (rc) return rc;
  if (count) {
    hipError_t e = hipMemcpy(*p, src, count * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_err(c, e, "hipMemcpy");
  }
  return PMFEM_OK;
}

void free_dev(pmfem_ctx* c) {
  if (!c->dev) return;
  if (c->dev->side) (void)hipStreamSynchronize(c->dev->side);
  if (c->stream || c->dev->side) (void)hipStreamSynchronize((hipStream_t)c->stream);
  if (c->dev->sg.x) (void)hipGraphExecDestroy(c->dev->sg.x);
  if (c->dev->sg.g) (void)hipGraphDestroy(c->dev->sg.g);
  if (c->dev->sg.cap) (void)hipStreamDestroy(c->dev->sg.cap);
  if (c->dev->imp.host) (void)hipHostFree(c->dev->imp.host);
  if (c->dev->net) {
    sg_destroy(c->dev->net);
    delete c->dev->net;
  }
  for (void* p : c->dev->allocs) (void)hipFree(p);
  for (hipEvent_t e : c->dev->ev) (void)hipEventDestroy(e);
  if (c->dev->fork) (void)hipEventDestroy(c->dev->fork);
  if (c->dev->join) (void)hipEventDestroy(c->dev->join);
  if (c->dev->side) (void)hipStreamDestroy(c->dev->side);
  delete c->dev;
  c->dev = nullptr;
}

int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

std::vector<float2> twiddles(int n) {
  std::vector<float2> t(n / 2 > 0 ? n / 2 : 1);
  for (int k = 0; k < n / 2; ++k) {
    double a = -2.0 * kPi * k / n;
    t[k] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  return t;
}

// boxes covering each grid index along one axis: (first box, count)
std::vector<int2> box_ranges(const HostOps& o, int a) {
  int N = o.N[a], p = o.p, shift = (p - 1) / 2;
  std::vector<int2> r(N);
  for (int gi = 0; gi < N; ++gi) {
    if (o.per[a]) {
      int s0 = ((gi - p + shift) % N + N) % N;
      r[gi] = make_int2(s0, p + 1);
    } else {
      int first = -1, cnt = 0;
      for (int b = 0; b < o.nbox[a]; ++b) {
        int st = std::min(std::max(b - shift, 0), N - p - 1);
        if (st >= gi - p && st <= gi) {
          if (first < 0) first = b;
          ++cnt;
        }
      }
      r[gi] = make_int2(first < 0 ? 0 : first, cnt);
    }
  }
  return r;
}

// Kernel forms from the context's variant choice (0 automatic: the staged
// forms wherever their plans fit) and the kernel name of each profiling slot.
int select_variants(pmfem_ctx* c) {
  pmfem_dev* d = c->dev;
  const int va = c->variant[0], vi = c->variant[1], vf = c->variant[2];
  d->lanes_l = c->variant[3] == 0 ? d->auto_l : c->variant[3];
  d->lanes_z = c->variant[3] == 0 ? d->auto_z : c->variant[3];
  if ((va == 2 && !d->ant_ok) || (va == 3 && !d->sc_ok) || (vi == 2 && !d->ic_ok) ||
      (vf == 2 && !d->fft_ok) || (vi == 1 && !d->ic_small_ok))
    return set_err(c, PMFEM_EINVAL, "requested kernel form does not fit this problem");
  if (!d->ic_ok && !d->ic_small_ok)
    return set_err(c, PMFEM_EGRID, "near region too dense for the LDS staging of any tile");
  d->ant_scatter = va == 0 ? d->sc_ok : va == 3;
  d->ant_line = !d->ant_scatter && (va == 0 ? d->ant_ok : va == 2);
  d->ic_seg = vi == 0 ? d->ic_ok : vi == 2;
  d->fft_plane = vf == 0 ? d->fft_ok : vf == 2;
  const char* names_split[12] = {"k_charges", "k_anterp",    "k_r2c_x", "k_fft_y_fwd",
                                 "k_fft_z_mul", "k_fft_y_inv", "k_c2r_x", "k_interp",
                                 "k_gsum",    "k_zcorr",     "k_exch",  "-"};
  for (int k = 0; k < 12; ++k) d->kname[k] = names_split[k];
  if (d->fft_plane) {
    d->kname[2] = "k_fft_xy_fwd";
    d->kname[3] = "-";
    d->kname[5] = "-";
    d->kname[6] = "k_fft_yx_inv";
  }
  d->kname[1] = d->ant_scatter ? "k_anterp_scatter" : d->ant_line ? "k_anterp_line" : "k_anterp";
  if (d->ant_scatter) d->kname[11] = "k_anterp_sum";
  d->kname[7] = "k_interp_tile";
  return PMFEM_OK;
}

// Line plan for k_anterp_line: the longest x-segment (at most 128 points,
// a power of two) whose staged nodes fit in LDS. Returns false if none fits.
bool plan_anterp(const HostOps& o, const std::vector<int2>& bx, const std::vector<int2>& by,
                 const std::vector<int2>& bz, AntPlan& pl) {
  const int nbx = o.nbox[0], nby = o.nbox[1], nbz = o.nbox[2], p = o.p, shift = (p - 1) / 2;
  const std::vector<int32_t>& bs = o.box_start;
  int cy = 0, cz = 0;
  for (const int2& r : by) cy = std::max(cy, r.y);
  for (const int2& r : bz) cz = std::max(cz, r.y);
  const int nrow = cy * cz;
  auto cnt = [&](int x, int64_t rowbase) -> int64_t {
    if (o.per[0]) x = (x % nbx + nbx) % nbx;
    else if (x < 0 || x >= nbx) return 0;
    return bs[rowbase + x + 1] - bs[rowbase + x];
  };
  for (int xa = std::min(o.N[0], 128); xa >= 4; xa /= 2) {
    const int nsx = (o.N[0] + xa - 1) / xa;
    int sbx = 0;
    std::vector<int> fbs(nsx), nbss(nsx);
    for (int sx = 0; sx < nsx; ++sx) {
      const int x0 = sx * xa, xe = std::min(x0 + xa, o.N[0]) - 1;
      fbs[sx] = o.per[0] ? x0 - p + shift : bx[x0].x;
      nbss[sx] = o.per[0] ? (xe - x0 + 1) + p : bx[xe].x + bx[xe].y - bx[x0].x;
      sbx = std::max(sbx, nbss[sx]);
    }
    int64_t ncap = 0, colmax = 0;
    for (int gz = 0; gz < o.N[2]; ++gz)
      for (int gy = 0; gy < o.N[1]; ++gy)
        for (int sx = 0; sx < nsx; ++sx) {
          int64_t staged = 0;
          for (int k = 0; k < nbss[sx]; ++k) {
            int64_t col = 0;
            for (int iz = 0; iz < bz[gz].y; ++iz)
              for (int iy = 0; iy < by[gy].y; ++iy) {
                int b_y = by[gy].x + iy, b_z = bz[gz].x + iz;
                if (b_y >= nby) b_y -= nby;
                if (b_z >= nbz) b_z -= nbz;
                col += cnt(fbs[sx] + k, ((int64_t)b_z * nby + b_y) * nbx);
              }
            colmax = std::max(colmax, col);
            staged += col;
          }
          ncap = std::max(ncap, staged);
        }
    auto al = [](int64_t b) { return (b + 15) & ~(int64_t)15; };
    int64_t off = 0;
    pl.o_x = (int)off;
    off += al(std::max<int64_t>(ncap, 1) * 8);
    pl.o_c = pl.o_x;
    pl.o_st = pl.o_x;
    pl.o_off = (int)off;
    off += al((int64_t)(sbx + 1) * 4);
    pl.o_meta = (int)off;
    off += al((int64_t)nrow * 4);
    if (off <= 65536 && nrow <= 64 && colmax < 65536) {
      pl.xa = xa;
      pl.nsx = nsx;
      pl.nrow = nrow;
      pl.sbx = sbx;
      pl.ncap = (int)std::max<int64_t>(ncap, 1);
      pl.lds_bytes = (int)off;
      return true;
    }
  }
  return false;
}

// Node lists of k_anterp_line for plan pl, in launch order: per workgroup the
// nodes of its box columns (column-major, box row, node order), each entry
// node | row << 26, the list start of every workgroup and the column starts
// within it (stride sbx + 1).
// Node lists of k_interp_tile for plan pl, in launch order: per workgroup the
// nodes of its source block column-major (x column, z, y, node order), the
// list start of every workgroup, its observer segments (row prefix over the
// z box rows, then the first row of each; stride 2 tz + 1), and per row the
// (start | length << 16) of its 2 r_b + 1 runs in the workgroup's list.
bool build_interp_lists(const HostOps& o, const IcPlan& pl, std::vector<int32_t>& list,
                        std::vector<int32_t>& lstart, std::vector<int32_t>& wseg,
                        std::vector<uint32_t>& rdesc) {
  const int nbx = o.nbox[0], nby = o.nbox[1], nbz = o.nbox[2];
  const int rb = o.rb, W = 2 * rb + 1;
  const std::vector<int32_t>& bs = o.box_start;
  auto box = [&](int x, int y, int z) -> int64_t {
    if (o.per[0]) x = (x % nbx + nbx) % nbx;
    else if (x < 0 || x >= nbx) return -1;
    if (o.per[1]) y = (y % nby + nby) % nby;
    else if (y < 0 || y >= nby) return -1;
    if (o.per[2]) z = (z % nbz + nbz) % nbz;
    else if (z < 0 || z >= nbz) return -1;
    return ((int64_t)z * nby + y) * nbx + x;
  };
  const int64_t nwg = (int64_t)pl.nsx * nby * pl.nsz;
  const int segw = 2 * pl.tz + 1, rpc = pl.szr * W;
  lstart.assign(nwg + 1, 0);
  wseg.assign(nwg * segw, 0);
  rdesc.assign((size_t)o.n_unk * W, 0u);
  list.clear();
  std::vector<int32_t> pos((size_t)pl.sbx * (rpc + 1));
  for (int64_t w = 0; w < nwg; ++w) {
    const int sx = (int)(w % pl.nsx);
    const int64_t rest = w / pl.nsx;
    const int by = (int)(rest % nby), sz = (int)(rest / nby);
    const int x0 = sx * pl.xs, z0 = sz * pl.tz;
    const int xs = std::min(pl.xs, nbx - x0), tz = std::min(pl.tz, nbz - z0);
    const int64_t l0 = (int64_t)list.size();
    if (l0 > 2147483647LL) return false;
    lstart[w] = (int32_t)l0;
    for (int k = 0; k < pl.sbx; ++k) {
      for (int zz = 0; zz < pl.szr; ++zz)
        for (int yy = 0; yy < W; ++yy) {
          pos[(size_t)k * (rpc + 1) + zz * W + yy] = (int32_t)((int64_t)list.size() - l0);
          const int64_t b = box(x0 - rb + k, by - rb + yy, z0 - rb + zz);
          if (b < 0) continue;
          for (int32_t nd = bs[b]; nd < bs[b + 1]; ++nd) list.push_back(nd);
        }
      pos[(size_t)k * (rpc + 1) + rpc] = (int32_t)((int64_t)list.size() - l0);
    }
    if ((int64_t)list.size() - l0 >= 65536) return false;
    int32_t* sg = &wseg[w * segw];
    int32_t run = 0;
    for (int kz = 0; kz <= pl.tz; ++kz) {
      sg[kz] = run;
      if (kz >= tz) continue;
      const int64_t orow = ((int64_t)(z0 + kz) * nby + by) * nbx;
      sg[pl.tz + 1 + kz] = bs[orow + x0];
      run += bs[orow + x0 + xs] - bs[orow + x0];
      for (int kx = 0; kx < xs; ++kx) {
        const int64_t b = orow + x0 + kx;
        for (int32_t r = bs[b]; r < bs[b + 1]; ++r)
          for (int dx = 0; dx < W; ++dx) {
            const int32_t* pc = &pos[(size_t)(kx + dx) * (rpc + 1)];
            const int32_t a = pc[kz * W], e = pc[(kz + W) * W];
            rdesc[(size_t)r * W + dx] = (uint32_t)a | ((uint32_t)(e - a) << 16);
          }
      }
    }
  }
  if ((int64_t)list.size() > 2147483647LL) return false;
  lstart[nwg] = (int32_t)list.size();
  return true;
}

// Scatter plan of anterpolation: tiles of tb boxes per axis (at least p + 1,
// so that a grid point lies in the footprints of at most two tiles per axis;
// on a periodic axis at most N - p, so that a footprint does not wrap onto
// itself), the tile node lists in launch order (tiles x fastest, nodes in box
// order), and per axis and grid index the covering tiles with the point's
// offset in their footprints. Returns false if the tiles do not fit. With
// divisors, a periodic axis takes the smallest tile that divides it (a
// shorter last tile can leave a grid point in three footprints).
bool plan_scatter_with(const HostOps& o, ScPlan& pl, std::vector<int2>& list,
                       std::vector<int32_t>& lstart, std::vector<int2> tab[3], bool divisors) {
  const int p = o.p, shift = (p - 1) / 2;
  const int* want = kScTile;
  auto start = [&](int a, int b) {
    return o.per[a] ? b - shift : std::min(std::max(b - shift, 0), o.N[a] - p - 1);
  };
  // one axis: tiles of the preferred size, or (div) the size that divides a
  // periodic axis closest to the preferred one (at least p + 1, at most
  // N - p; the larger of two equally close); false if a grid index would lie
  // in three footprints or a footprint would wrap onto itself
  auto plan_axis = [&](int a, bool div) -> bool {
    int tb = std::max(want[a], p + 1);
    if (o.per[a]) tb = std::min(tb, o.N[a] - p);
    if (div) {
      if (!o.per[a]) return false;
      const int pref = std::max(want[a], p + 1);
      int best = 0;
      for (int d = p + 1; d <= o.N[a] - p; ++d)
        if (o.nbox[a] % d == 0 && (!best || std::abs(d - pref) <= std::abs(best - pref))) best = d;
      if (!best) return false;
      tb = best;
    }
    tb = std::min(tb, o.nbox[a]);
    if (tb < 1) return false;
    pl.tb[a] = tb;
    pl.nt[a] = (o.nbox[a] + tb - 1) / tb;
    int fd = 0;
    tab[a].assign((size_t)2 * o.N[a], make_int2(-1, 0));
    for (int t = 0; t < pl.nt[a]; ++t) {
      const int b0 = t * tb, b1 = std::min(b0 + tb, o.nbox[a]) - 1;
      const int f0 = start(a, b0), w = start(a, b1) + p + 1 - f0;
      fd = std::max(fd, w);
      if (o.per[a] && w > o.N[a]) return false;
      for (int i = 0; i < w; ++i) {
        int gi = f0 + i;
        if (o.per[a]) gi = ((gi % o.N[a]) + o.N[a]) % o.N[a];
        if (gi < 0 || gi >= o.N[a]) return false;
        int2* e = &tab[a][(size_t)2 * gi];
        if (e[0].x < 0) e[0] = make_int2(t, i);
        else if (e[1].x < 0) e[1] = make_int2(t, i);
        else return false;  // a third covering tile
      }
    }
    pl.fd[a] = fd;
    return true;
  };
  for (int a = 0; a < 3; ++a)
    if (!plan_axis(a, divisors) && !(!divisors && plan_axis(a, true))) return false;
  pl.fsize = pl.fd[0] * pl.fd[1] * pl.fd[2];
  const int nbx = o.nbox[0], nby = o.nbox[1];
  const std::vector<int32_t>& bs = o.box_start;
  const int64_t nt = (int64_t)pl.nt[0] * pl.nt[1] * pl.nt[2];
  lstart.assign(nt + 1, 0);
  list.clear();
  list.reserve((size_t)o.n_unk);
  for (int64_t w = 0; w < nt; ++w) {
    const int tx = (int)(w % pl.nt[0]);
    const int64_t r = w / pl.nt[0];
    const int ty = (int)(r % pl.nt[1]), tz = (int)(r / pl.nt[1]);
    lstart[w] = (int32_t)list.size();
    const int x0 = tx * pl.tb[0], x1 = std::min(x0 + pl.tb[0], nbx);
    const int y0 = ty * pl.tb[1], z0 = tz * pl.tb[2];
    for (int bz = z0; bz < std::min(z0 + pl.tb[2], o.nbox[2]); ++bz)
      for (int by = y0; by < std::min(y0 + pl.tb[1], nby); ++by) {
        const int64_t row = ((int64_t)bz * nby + by) * nbx;
        const int oz = start(2, bz) - start(2, z0), oy = start(1, by) - start(1, y0);
        for (int bx = x0; bx < x1; ++bx) {
          // offset of the box's stencil origin in the tile footprint
          const int off = (oz * pl.fd[1] + oy) * pl.fd[0] + start(0, bx) - start(0, x0);
          for (int32_t nd = bs[row + bx]; nd < bs[row + bx + 1]; ++nd) list.push_back(make_int2(nd, off));
        }
      }
  }
  lstart[nt] = (int32_t)list.size();
  // the footprint copies, one per lane group (four groups of 16 lanes for p <= 3)
  const int64_t lds = (int64_t)pl.fsize * (o.p <= 3 ? 4 : 1) * 4;
  if (lds > kScLdsBudget) return false;
  pl.lds_bytes = (int)lds;
  return (int64_t)list.size() == o.n_unk;
}

// The scatter plan: the preferred tile sizes, else tiles dividing the
// periodic axes.
bool plan_scatter(const HostOps& o, ScPlan& pl, std::vector<int2>& list,
                  std::vector<int32_t>& lstart, std::vector<int2> tab[3]) {
  return plan_scatter_with(o, pl, list, lstart, tab, false) ||
         plan_scatter_with(o, pl, list, lstart, tab, true);
}

bool build_anterp_lists(const HostOps& o, const std::vector<int2>& bx,
                        const std::vector<int2>& by, const std::vector<int2>& bz,
                        const AntPlan& pl, std::vector<int32_t>& list,
                        std::vector<int32_t>& lstart, std::vector<int32_t>& col) {
  const int nbx = o.nbox[0], nby = o.nbox[1], nbz = o.nbox[2], p = o.p, shift = (p - 1) / 2;
  const std::vector<int32_t>& bs = o.box_start;
  if (o.n_unk >= (1 << 26)) return false;
  const int64_t nwg = (int64_t)pl.nsx * o.N[1] * o.N[2];
  lstart.assign(nwg + 1, 0);
  col.assign(nwg * (pl.sbx + 1), 0);
  list.clear();
  for (int64_t w = 0; w < nwg; ++w) {
    const int sx = (int)(w % pl.nsx);
    const int64_t line = w / pl.nsx;
    const int gy = (int)(line % o.N[1]), gz = (int)(line / o.N[1]);
    const int x0 = sx * pl.xa, xe = std::min(x0 + pl.xa, o.N[0]) - 1;
    const int fb = o.per[0] ? x0 - p + shift : bx[x0].x;
    const int nbs = o.per[0] ? (xe - x0 + 1) + p : bx[xe].x + bx[xe].y - bx[x0].x;
    std::vector<int64_t> rowbase;
    for (int iz = 0; iz < bz[gz].y; ++iz)
      for (int iy = 0; iy < by[gy].y; ++iy) {
        int b_y = by[gy].x + iy, b_z = bz[gz].x + iz;
        if (b_y >= nby) b_y -= nby;
        if (b_z >= nbz) b_z -= nbz;
        rowbase.push_back(((int64_t)b_z * nby + b_y) * nbx);
      }
    const int64_t l0 = (int64_t)list.size();
    if (l0 > 2147483647LL) return false;
    lstart[w] = (int32_t)l0;
    for (int k = 0; k <= pl.sbx; ++k) {
      col[w * (pl.sbx + 1) + k] = (int32_t)((int64_t)list.size() - l0);
      if (k >= nbs) continue;
      int x = fb + k;
      if (o.per[0]) x = (x % nbx + nbx) % nbx;
      else if (x < 0 || x >= nbx) continue;
      for (size_t j = 0; j < rowbase.size(); ++j) {
        const int64_t b = rowbase[j] + x;
        for (int32_t nd = bs[b]; nd < bs[b + 1]; ++nd)
          list.push_back(nd | (int32_t)((uint32_t)j << 26));
      }
    }
  }
  if ((int64_t)list.size() > 2147483647LL) return false;
  lstart[nwg] = (int32_t)list.size();
  return true;
}

// Tile plan for k_interp_tile: the largest tile (xs boxes along x times tz
// box rows along z, both powers of two, xs <= max_xs) whose staged arrays fit
// the LDS budget; larger tiles stage each source charge fewer times.
bool plan_interp(const HostOps& o, int max_xs, IcPlan& pl) {
  const int nbx = o.nbox[0], nby = o.nbox[1], nbz = o.nbox[2];
  const int rb = o.rb, W = 2 * rb + 1, p = o.p;
  const std::vector<int32_t>& bs = o.box_start;
  auto cnt = [&](int x, int y, int z) -> int64_t {
    if (o.per[0]) x = (x % nbx + nbx) % nbx;
    else if (x < 0 || x >= nbx) return 0;
    if (o.per[1]) y = (y % nby + nby) % nby;
    else if (y < 0 || y >= nby) return 0;
    if (o.per[2]) z = (z % nbz + nbz) % nbz;
    else if (z < 0 || z >= nbz) return 0;
    const int64_t b = ((int64_t)z * nby + y) * nbx + x;
    return bs[b + 1] - bs[b];
  };
  struct Shape {
    int xs, tz;
  };
  std::vector<Shape> shapes;
  for (int xs = 1; xs <= std::min(max_xs, 128); xs *= 2)
    for (int tz = 1; tz <= 16; tz *= 2)
      if (xs * tz <= 512 && (xs <= nbx || xs == 1) && (tz <= nbz || tz == 1))
        shapes.push_back({xs, tz});
  // largest staged-to-observer ratio first: fewest staged boxes per observer box
  std::sort(shapes.begin(), shapes.end(), [&](const Shape& a, const Shape& b) {
    const double ra = (double)(a.xs + 2 * rb) * (a.tz + 2 * rb) / (a.xs * a.tz);
    const double rb2 = (double)(b.xs + 2 * rb) * (b.tz + 2 * rb) / (b.xs * b.tz);
    return ra < rb2;
  });
  for (const Shape& sh : shapes) {
    const int xs = sh.xs, tz = sh.tz;
    const int nsx = (nbx + xs - 1) / xs, nsz = (nbz + tz - 1) / tz;
    const int sbx = xs + 2 * rb, szr = tz + 2 * rb;
    int64_t qcap = 0, rcap = 0, colmax = 0;
    for (int sz = 0; sz < nsz; ++sz)
      for (int by = 0; by < nby; ++by)
        for (int sx = 0; sx < nsx; ++sx) {
          const int x0 = sx * xs, z0 = sz * tz;
          int64_t rows = 0;
          for (int kz = 0; kz < tz && z0 + kz < nbz; ++kz)
            for (int kx = 0; kx < xs && x0 + kx < nbx; ++kx) rows += cnt(x0 + kx, by, z0 + kz);
          if (rows == 0) continue;
          rcap = std::max(rcap, rows);
          int64_t staged = 0;
          for (int k = 0; k < sbx; ++k) {
            int64_t col = 0;
            for (int zz = 0; zz < szr; ++zz)
              for (int yy = 0; yy < W; ++yy)
                col += cnt(x0 - rb + k, by - rb + yy, z0 - rb + zz);
            colmax = std::max(colmax, col);
            staged += col;
          }
          qcap = std::max(qcap, staged);
        }
    auto al = [](int64_t b) { return (b + 15) & ~(int64_t)15; };
    const int ux = xs + p, uzl = tz + p;
    int64_t off = 0;
    pl.o_q = (int)off;
    off += al((qcap + 4) * 4);  // staged charges and 4 zeros
    pl.o_u = (int)off;
    off += al((int64_t)uzl * (p + 1) * ux * 4);
    pl.o_seg = (int)off;
    off += al((int64_t)(2 * tz + 1) * 4);
    (void)colmax;
    if (off <= kIcLdsBudget && qcap < 65536) {
      pl.xs = xs;
      pl.tz = tz;
      pl.nsx = nsx;
      pl.nsz = nsz;
      pl.sbx = sbx;
      pl.szr = szr;
      pl.qcap = (int)std::max<int64_t>(qcap, 1);
      pl.rcap = (int)std::max<int64_t>(rcap, 1);
      pl.ux = ux;
      pl.uzl = uzl;
      pl.lds_bytes = (int)off;
      return true;
    }
  }
  return false;
}

int upload_all(pmfem_ctx* c) {
  HostOps& o = c->ops;
  pmfem_dev* d = c->dev;
  {
    hipError_t e = hipStreamCreateWithFlags(&d->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&d->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&d->join, hipEventDisableTiming);
    if (e != hipSuccess) return hip_err(c, e, "side stream");
  }
  const int64_t n = o.n_unk;
  d->n = n;
  for (int a = 0; a < 3; ++a) {
    d->g.N[a] = o.N[a];
    d->g.M[a] = o.M[a];
    d->g.logM[a] = ilog2(o.M[a]);
    d->g.nbox[a] = o.nbox[a];
  }
  for (int a = 0; a < 3; ++a) d->g.per[a] = o.per[a];
  d->g.p = o.p;
  d->g.rb = o.rb;
  d->g.gmode = c->precision;  // grid storage between the kernels of one evaluation
  int rc;
  if ((rc = upload(c, &d->pos4, o.pos4.data(), n))) return rc;
  if ((rc = upload(c, &d->box_start, o.box_start.data(), o.box_start.size()))) return rc;
  d->ic_ok = plan_interp(o, 128, d->icp);
  d->ic_small_ok = plan_interp(o, 4, d->icp_small);
  for (int which = 0; which < 2; ++which) {
    bool& ok = which == 0 ? d->ic_ok : d->ic_small_ok;
    if (!ok) continue;
    std::vector<int32_t> list, lstart, wseg;
    std::vector<uint32_t> rdesc;
    ok = build_interp_lists(o, which == 0 ? d->icp : d->icp_small, list, lstart, wseg, rdesc);
    if (!ok) continue;
    pmfem_dev::IcLists& L = which == 0 ? d->icl : d->icl_small;
    if ((rc = upload(c, &L.list, list.data(), list.size()))) return rc;
    if ((rc = upload(c, &L.lstart, lstart.data(), lstart.size()))) return rc;
    if ((rc = upload(c, &L.wseg, wseg.data(), wseg.size()))) return rc;
    if ((rc = upload(c, &L.rdesc, rdesc.data(), rdesc.size()))) return rc;
  }

  for (int a = 0; a < 3; ++a)
    if (o.M[a] & (o.M[a] - 1)) d->fft_mr = true;
  {
    // whole-plane x/y transforms when a plane (row pairs + half-spectrum
    // columns) fits in one workgroup's LDS: radix 2 in place with half
    // twiddle tables, mixed radix with full tables and two buffers
    const int Mx = o.M[0], My = o.M[1], Hx = Mx / 2 + 1, pairs = (o.N[1] + 1) / 2;
    const size_t cap = std::max((size_t)pairs * Mx, (size_t)Hx * My);
    d->fft_plane_lds =
        d->fft_mr ? (size_t)(Mx + My + 2 * cap) * sizeof(float2)
                  : (size_t)(Mx / 2 + My / 2 + (size_t)pairs * Mx + (size_t)Hx * (My + 1)) *
                        sizeof(float2);
    int max_lds = 0;
    (void)hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device);
    d->fft_ok = d->fft_plane_lds <= (size_t)max_lds;
    if (d->fft_ok && d->fft_plane_lds > 65536) {
      const int b = (int)d->fft_plane_lds;
      const void* fwd = d->fft_mr ? (const void*)k_fft_xy_fwd_mr : (const void*)k_fft_xy_fwd;
      const void* inv = d->fft_mr ? (const void*)k_fft_yx_inv_mr : (const void*)k_fft_yx_inv;
      d->fft_ok = hipFuncSetAttribute(fwd, hipFuncAttributeMaxDynamicSharedMemorySize, b) ==
                      hipSuccess &&
                  hipFuncSetAttribute(inv, hipFuncAttributeMaxDynamicSharedMemorySize, b) ==
                      hipSuccess;
      (void)hipGetLastError();
    }
  }

  auto bx = box_ranges(o, 0), by = box_ranges(o, 1), bz = box_ranges(o, 2);
  d->ant_ok = plan_anterp(o, bx, by, bz, d->ap);
  if (d->ant_ok) {
    std::vector<int32_t> list, lstart, col;
    d->ant_ok = build_anterp_lists(o, bx, by, bz, d->ap, list, lstart, col);
    if (d->ant_ok) {
      if ((rc = upload(c, &d->ant_list, list.data(), list.size()))) return rc;
      if ((rc = upload(c, &d->ant_lstart, lstart.data(), lstart.size()))) return rc;
      if ((rc = upload(c, &d->ant_col, col.data(), col.size()))) return rc;
    }
  }
  d->ant_threads = std::max(64, std::min(128, (d->ap.xa + 63) / 64 * 64));
  {
    std::vector<int2> list;
    std::vector<int32_t> lstart;
    std::vector<int2> tab[3];
    d->sc_ok = plan_scatter(o, d->sp, list, lstart, tab);
    if (d->sc_ok) {
      if ((rc = upload(c, &d->sc_list, list.data(), list.size()))) return rc;
      if ((rc = upload(c, &d->sc_lstart, lstart.data(), lstart.size()))) return rc;
      for (int a = 0; a < 3; ++a)
        if ((rc = upload(c, &d->sc_tab[a], tab[a].data(), tab[a].size()))) return rc;
      const int64_t nt = (int64_t)d->sp.nt[0] * d->sp.nt[1] * d->sp.nt[2];
      if ((rc = dalloc(c, &d->sc_part, nt * d->sp.fsize))) return rc;
    }
  }
  if ((rc = upload(c, &d->brx, bx.data(), bx.size()))) return rc;
  if ((rc = upload(c, &d->bry, by.data(), by.size()))) return rc;
  if ((rc = upload(c, &d->brz, bz.data(), bz.size()))) return rc;
  const int64_t nnzL = o.loc_rowptr[n];
  {
    std::vector<int4> dr(nnzL), gr(nnzL);
    std::vector<int2> lr(nnzL);
    for (int64_t e = 0; e < nnzL; ++e) {
      const float* v = &o.loc_val[8 * e];  // L, Dx, Dy, Dz, Gx, Gy, Gz, 0
      int4 r, q4;
      int2 l2;
      r.x = q4.x = l2.x = o.loc_col[e];
      std::memcpy(&r.y, &v[1], 4);
      std::memcpy(&r.z, &v[2], 4);
      std::memcpy(&r.w, &v[3], 4);
      std::memcpy(&q4.y, &v[4], 4);
      std::memcpy(&q4.z, &v[5], 4);
      std::memcpy(&q4.w, &v[6], 4);
      std::memcpy(&l2.y, &v[0], 4);
      dr[e] = r;
      gr[e] = q4;
      lr[e] = l2;
    }
    if ((rc = upload(c, &d->lrp, o.loc_rowptr.data(), n + 1))) return rc;
    if ((rc = upload(c, &d->drec, dr.data(), nnzL))) return rc;
    if ((rc = upload(c, &d->lrec, lr.data(), nnzL))) return rc;
    if ((rc = upload(c, &d->grec, gr.data(), nnzL))) return rc;
  }
  const int64_t nnzZ = o.z0_rowptr[n];
  {
    // about four entries per lane
    auto pick = [](double mean) { return mean > 48.0 ? 16 : mean > 24.0 ? 8 : 4; };
    d->auto_l = pick((double)nnzL / std::max<int64_t>(n, 1));
    d->auto_z = pick((double)nnzZ / std::max<int64_t>(n, 1));
  }
  {
    std::vector<int4> zr(nnzZ);
    for (int64_t e = 0; e < nnzZ; ++e) {
      int4 r;
      r.x = o.z0_col[e];
      std::memcpy(&r.y, &o.z0_val[4 * e], 4);
      std::memcpy(&r.z, &o.z0_val[4 * e + 1], 4);
      std::memcpy(&r.w, &o.z0_val[4 * e + 2], 4);
      zr[e] = r;
    }
    if ((rc = upload(c, &d->zrp, o.z0_rowptr.data(), n + 1))) return rc;
    if ((rc = upload(c, &d->zrec, zr.data(), nnzZ))) return rc;
  }
  {
    // precorrection rows on the device: each x-offset run padded with zeros
    // to a multiple of 4 values, so every run starts 16-byte aligned
    const int nbx = o.nbox[0], nby = o.nbox[1], nbz = o.nbox[2], rb = o.rb, W = 2 * rb + 1;
    auto cnt = [&](int x, int y, int z) -> int64_t {
      if (o.per[0]) x = (x % nbx + nbx) % nbx;
      else if (x < 0 || x >= nbx) return 0;
      if (o.per[1]) y = (y % nby + nby) % nby;
      else if (y < 0 || y >= nby) return 0;
      if (o.per[2]) z = (z % nbz + nbz) % nbz;
      else if (z < 0 || z >= nbz) return 0;
      const int64_t b = ((int64_t)z * nby + y) * nbx + x;
      return o.box_start[b + 1] - o.box_start[b];
    };
    std::vector<int32_t> prp(n + 1, 0);
    std::vector<int32_t> runlen((size_t)n * W);
    int64_t tot = 0;
    for (int64_t r = 0; r < n; ++r) {
      const uint32_t bc = [&] {
        uint32_t v;
        std::memcpy(&v, &o.pos4[4 * r + 3], 4);
        return v;
      }();
      const int bx = bc & 1023, by = (bc >> 10) & 1023, bz = (bc >> 20) & 1023;
      int64_t rowlen = 0;
      prp[r] = (int32_t)tot;
      for (int dx = 0; dx < W; ++dx) {
        int64_t len = 0;
        for (int dz = -rb; dz <= rb; ++dz)
          for (int dy = -rb; dy <= rb; ++dy) len += cnt(bx + dx - rb, by + dy, bz + dz);
        runlen[(size_t)r * W + dx] = (int32_t)len;
        rowlen += len;
        tot += (len + 3) & ~(int64_t)3;
      }
      if (rowlen != o.p_rowptr[r + 1] - o.p_rowptr[r])
        return set_err(c, PMFEM_EGRID, "precorrection row does not match its near boxes");
      if (tot > 2147483647LL) return set_err(c, PMFEM_ENOMEM, "padded precorrection too large");
    }
    prp[n] = (int32_t)tot;
    // zeros after the last row: a lane's register chunks (at most 8 per lane)
    // may reach past the end of the matrix
    std::vector<float> pv((size_t)tot + 4 + 32 * kIcLanes, 0.f);
    for (int64_t r = 0; r < n; ++r) {
      int64_t src = o.p_rowptr[r], dst = prp[r];
      for (int dx = 0; dx < W; ++dx) {
        const int32_t len = runlen[(size_t)r * W + dx];
        std::memcpy(&pv[dst], &o.p_val[src], (size_t)len * sizeof(float));
        src += len;
        dst += (len + 3) & ~3;
      }
    }
    if ((rc = upload(c, &d->prp, prp.data(), n + 1))) return rc;
    if ((rc = upload(c, &d->pv, pv.data(), pv.size()))) return rc;
    d->nnz_p_dev = tot;
    // chunks per lane in registers: the mean row's share per lane, rounded up
    // to {2, 4, 6, 8} (longer rows take the rest in a loop)
    {
      const int64_t mean = n > 0 ? (tot / 4 + n - 1) / n : 0;
      const int64_t per_lane = (mean + kIcLanes - 1) / kIcLanes;
      int kc = per_lane <= 2 ? 2 : per_lane <= 4 ? 4 : per_lane <= 6 ? 6 : 8;
      d->icp.kc = kc;
      d->icp_small.kc = kc;
    }
  }
  if ((rc = upload(c, &d->khat, o.khat.data(), o.khat.size()))) return rc;
  auto tx = twiddles(o.M[0]), ty = twiddles(o.M[1]), tz = twiddles(o.M[2]);
  if ((rc = upload(c, &d->twx, tx.data(), tx.size()))) return rc;
  if ((rc = upload(c, &d->twy, ty.data(), ty.size()))) return rc;
  if ((rc = upload(c, &d->twz, tz.data(), tz.size()))) return rc;
  if (d->fft_mr) {
    auto full = [](int n) {
      std::vector<float2> t(n);
      for (int k = 0; k < n; ++k) {
        const double a = -2.0 * kPi * k / n;
        t[k] = make_float2((float)std::cos(a), (float)std::sin(a));
      }
      return t;
    };
    auto fx = full(o.M[0]), fy = full(o.M[1]), fz = full(o.M[2]);
    if ((rc = upload(c, &d->twfx, fx.data(), fx.size()))) return rc;
    if ((rc = upload(c, &d->twfy, fy.data(), fy.size()))) return rc;
    if ((rc = upload(c, &d->twfz, fz.data(), fz.size()))) return rc;
  }
  if ((rc = upload(c, &d->mu, o.mu.data(), n))) return rc;
  if ((rc = dalloc(c, &d->hex, 3 * n))) return rc;
  if ((rc = dalloc(c, &d->q, n))) return rc;
  if ((rc = dalloc(c, &d->uz, n))) return rc;
  if ((rc = dalloc(c, &d->u, n))) return rc;
  const int64_t ng = (int64_t)o.N[0] * o.N[1] * o.N[2];
  if ((rc = dalloc(c, &d->grid, ng))) return rc;
  const int64_t nspec = (int64_t)o.N[2] * o.M[1] * (o.M[0] / 2 + 1);
  if ((rc = dalloc(c, &d->spec, nspec))) return rc;
  if ((rc = dalloc(c, &d->mst, 3 * n))) return rc;
  if ((rc = dalloc(c, &d->kk, 3 * n))) return rc;
  if ((rc = dalloc(c, &d->acc, 3 * n))) return rc;
  if ((rc = dalloc(c, &d->m32, 3 * n))) return rc;
  if ((rc = dalloc(c, &d->h32, 3 * n))) return rc;
  d->nparts = 1024;
  if ((rc = dalloc(c, &d->part, 2 * d->nparts))) return rc;
  // kernel forms, now that every plan and the mean row lengths are known
  return select_variants(c);
}

hipStream_t stream_of(pmfem_ctx* c) { return (hipStream_t)c->stream; }

// Step 2 of the AIM: Ug = (1/4 pi) K * Qg on the grid (profiling slots 2-6).
// spec: the half-spectrum work buffer ([N_z][M_y][M_x/2 + 1] complex),
// written in full by the forward passes before any pass reads it.
// gmode: storage of Qg and Ug (GridParams::gmode; 0 for caller FP32 grids).
template <class Mark>
void convolve(pmfem_dev* d, hipStream_t s, const float* Qg, float* Ug, float2* spec, int gmode,
              Mark&& mark) {
  GridParams g = d->g;
  g.gmode = gmode;
  const int T = 256;
  const int Mx = g.M[0], My = g.M[1], Mz = g.M[2], Hx = Mx / 2 + 1;
  const int Bz = std::max(1, std::min(kFftzB, 4096 / Mz)), Tz = kFftzT;
  const int64_t cols = (int64_t)My * Hx;
  if (d->fft_plane && d->fft_mr) {
    // whole planes in LDS for x and y, the mixed-radix z pass between them
    const int Bzm = std::max(1, std::min(kFftzMr, 2048 / Mz));
    mark(2, 0);
    hipLaunchKernelGGL(k_fft_xy_fwd_mr, dim3((unsigned)g.N[2]), dim3(kFftPlaneMrT),
                       d->fft_plane_lds, s, g, Qg, spec, d->twfx, d->twfy);
    mark(2, 1);
    mark(4, 0);
    hipLaunchKernelGGL(k_fft_z_mul_mr, dim3((unsigned)((cols + Bzm - 1) / Bzm)), dim3(kFftzT),
                       (size_t)(Mz + 2 * Bzm * Mz) * sizeof(float2), s, g, spec, d->khat, d->twfz,
                       Bzm);
    mark(4, 1);
    mark(6, 0);
    hipLaunchKernelGGL(k_fft_yx_inv_mr, dim3((unsigned)g.N[2]), dim3(kFftPlaneMrT),
                       d->fft_plane_lds, s, g, (const float2*)spec, Ug, d->twfx, d->twfy);
    mark(6, 1);
    return;
  }
  if (d->fft_plane) {
    mark(2, 0);
    hipLaunchKernelGGL(k_fft_xy_fwd, dim3((unsigned)(g.N[2] * kFftSplit)), dim3(1024),
                       d->fft_plane_lds, s, g, Qg, spec, d->twx, d->twy, kFftSplit);
    mark(2, 1);
    mark(4, 0);
    hipLaunchKernelGGL(k_fft_z_mul, dim3((unsigned)((cols + Bz - 1) / Bz)), dim3(Tz),
                       (size_t)(Mz / 2 + Bz * Mz) * sizeof(float2), s, g, spec, d->khat,
                       d->twz, Bz);
    mark(4, 1);
    mark(6, 0);
    hipLaunchKernelGGL(k_fft_yx_inv, dim3((unsigned)(g.N[2] * kFftSplit)), dim3(1024),
                       d->fft_plane_lds, s, g, (const float2*)spec, Ug, d->twx, d->twy,
                       kFftSplit);
    mark(6, 1);
    return;
  }
  if (d->fft_mr) {
    // mixed-radix passes: twiddle table and two line buffers in LDS
    const int lpb = std::max(1, 2048 / Mx);
    const int64_t xlines = (int64_t)((g.N[1] + 1) / 2) * g.N[2];
    const int By = std::max(1, std::min(16, 2048 / My));
    const int gy = (Hx + By - 1) / By;
    const int Bzm = std::max(1, std::min(kFftzMr, 2048 / Mz));
    mark(2, 0);
    hipLaunchKernelGGL(k_r2c_x_mr, dim3((unsigned)((xlines + lpb - 1) / lpb)), dim3(T),
                       (size_t)(Mx + 2 * lpb * Mx) * sizeof(float2), s, g, Qg, spec, d->twfx, lpb);
    mark(2, 1);
    mark(3, 0);
    hipLaunchKernelGGL(k_fft_y_mr, dim3((unsigned)(g.N[2] * gy)), dim3(T),
                       (size_t)(My + 2 * By * My) * sizeof(float2), s, g, spec, d->twfy, By, 0,
                       g.N[1], My);
    mark(3, 1);
    mark(4, 0);
    hipLaunchKernelGGL(k_fft_z_mul_mr, dim3((unsigned)((cols + Bzm - 1) / Bzm)), dim3(kFftzT),
                       (size_t)(Mz + 2 * Bzm * Mz) * sizeof(float2), s, g, spec, d->khat, d->twfz,
                       Bzm);
    mark(4, 1);
    mark(5, 0);
    hipLaunchKernelGGL(k_fft_y_mr, dim3((unsigned)(g.N[2] * gy)), dim3(T),
                       (size_t)(My + 2 * By * My) * sizeof(float2), s, g, spec, d->twfy, By, 1,
                       My, g.N[1]);
    mark(5, 1);
    mark(6, 0);
    hipLaunchKernelGGL(k_c2r_x_mr, dim3((unsigned)((xlines + lpb - 1) / lpb)), dim3(T),
                       (size_t)(Mx + 2 * lpb * Mx) * sizeof(float2), s, g, spec, Ug, d->twfx, lpb);
    mark(6, 1);
    return;
  }
  const int lpb = std::max(1, 2048 / Mx);
  const int64_t xlines = (int64_t)((g.N[1] + 1) / 2) * g.N[2];
  mark(2, 0);
  hipLaunchKernelGGL(k_r2c_x, dim3((unsigned)((xlines + lpb - 1) / lpb)), dim3(T),
                     (size_t)(Mx / 2 + lpb * Mx) * sizeof(float2), s, g, Qg, spec, d->twx,
                     lpb);
  mark(2, 1);
  const int By = std::max(1, std::min(16, 4096 / My));
  const int gy = (Hx + By - 1) / By;
  mark(3, 0);
  hipLaunchKernelGGL(k_fft_y, dim3((unsigned)(g.N[2] * gy)), dim3(T),
                     (size_t)(My / 2 + By * My) * sizeof(float2), s, g, spec, d->twy, By, 0,
                     g.N[1], My);
  mark(3, 1);
  mark(4, 0);
  hipLaunchKernelGGL(k_fft_z_mul, dim3((unsigned)((cols + Bz - 1) / Bz)), dim3(Tz),
                     (size_t)(Mz / 2 + Bz * Mz) * sizeof(float2), s, g, spec, d->khat, d->twz,
                     Bz);
  mark(4, 1);
  mark(5, 0);
  hipLaunchKernelGGL(k_fft_y, dim3((unsigned)(g.N[2] * gy)), dim3(T),
                     (size_t)(My / 2 + By * My) * sizeof(float2), s, g, spec, d->twy, By, 1,
                     My, g.N[1]);
  mark(5, 1);
  mark(6, 0);
  hipLaunchKernelGGL(k_c2r_x, dim3((unsigned)((xlines + lpb - 1) / lpb)), dim3(T),
                     (size_t)(Mx / 2 + lpb * Mx) * sizeof(float2), s, g, spec, Ug, d->twx,
                     lpb);
  mark(6, 1);
}

// One evaluation. Intermediates land in the context's work buffers.
// k_interp_tile for 2 r_b + 1 = WT runs per row and the plan's chunks per lane.
template <int WT>
void launch_interp(const IcPlan& pl, dim3 grid, dim3 blk, size_t lds, hipStream_t s,
                   const GridParams& g, const pmfem_dev* d, const pmfem_dev::IcLists& L) {
#define PMFEM_IC_LAUNCH(KC)                                                                  \
  hipLaunchKernelGGL((k_interp_tile<WT, KC>), grid, blk, lds, s, g, pl, d->grid, d->pos4,    \
                     L.list, L.lstart, L.wseg, L.rdesc, d->prp, d->pv, d->q, d->uz, d->u)
  switch (pl.kc) {
    case 2:
      PMFEM_IC_LAUNCH(2);
      break;
    case 4:
      PMFEM_IC_LAUNCH(4);
      break;
    case 6:
      PMFEM_IC_LAUNCH(6);
      break;
    default:
      PMFEM_IC_LAUNCH(8);
      break;
  }
#undef PMFEM_IC_LAUNCH
}

int run_heff(pmfem_ctx* c, const float* m, float* h, uint32_t terms, const double* happ,
             const double* m64 = nullptr) {
  pmfem_dev* d = c->dev;
  hipStream_t s = stream_of(c);
  const int64_t n = d->n;
  const GridParams& g = d->g;
  const int with_ex = (terms & PMFEM_TERM_EX) ? 1 : 0;
  const int with_ms = (terms & PMFEM_TERM_MS) ? 1 : 0;
  hipEvent_t* ev = nullptr;
  if (d->prof_calls < d->prof_max) {
    ev = &d->ev[(size_t)d->prof_calls * kNumKernels * 2];
    d->prof_calls++;
  }
  auto mark = [&](int k, int which) {
    if (ev) (void)hipEventRecord(ev[2 * k + which], s);
  };
  const int T = 256;
  // the exchange reads the FP64 magnetisation where the caller has one (the
  // implicit solver's residual), else the FP32 copy
  auto exch = [&](hipStream_t st) {
    const dim3 grid((unsigned)((n * d->lanes_l + T - 1) / T));
    if (m64) {
      if (d->lanes_l == 4)
        hipLaunchKernelGGL((k_exch<4, double>), grid, dim3(T), 0, st, n, d->lrp, d->lrec, m64, d->hex);
      else if (d->lanes_l == 8)
        hipLaunchKernelGGL((k_exch<8, double>), grid, dim3(T), 0, st, n, d->lrp, d->lrec, m64, d->hex);
      else
        hipLaunchKernelGGL((k_exch<16, double>), grid, dim3(T), 0, st, n, d->lrp, d->lrec, m64, d->hex);
    } else if (d->lanes_l == 4) {
      hipLaunchKernelGGL((k_exch<4, float>), grid, dim3(T), 0, st, n, d->lrp, d->lrec, m, d->hex);
    } else if (d->lanes_l == 8) {
      hipLaunchKernelGGL((k_exch<8, float>), grid, dim3(T), 0, st, n, d->lrp, d->lrec, m, d->hex);
    } else {
      hipLaunchKernelGGL((k_exch<16, float>), grid, dim3(T), 0, st, n, d->lrp, d->lrec, m, d->hex);
    }
  };
  auto rowdot3 = [&](hipStream_t st, const int32_t* rp, const int4* rec, float* out, int lanes) {
    const dim3 grid((unsigned)((n * lanes + T - 1) / T));
    if (lanes == 4)
      hipLaunchKernelGGL(k_rowdot3<4>, grid, dim3(T), 0, st, n, m, rp, rec, out);
    else if (lanes == 8)
      hipLaunchKernelGGL(k_rowdot3<8>, grid, dim3(T), 0, st, n, m, rp, rec, out);
    else
      hipLaunchKernelGGL(k_rowdot3<16>, grid, dim3(T), 0, st, n, m, rp, rec, out);
  };
  if (with_ms) {
    mark(0, 0);
    rowdot3(s, d->lrp, d->drec, d->q, d->lanes_l);
    mark(0, 1);
    // element correction on the side stream, beside anterpolation and the
    // FFT (both bound by latency and ALU rather than HBM); joined before
    // interpolation
    (void)hipEventRecord(d->fork, s);
    (void)hipStreamWaitEvent(d->side, d->fork, 0);
    if (ev) (void)hipEventRecord(ev[2 * 9], d->side);
    rowdot3(d->side, d->zrp, d->zrec, d->uz, d->lanes_z);
    if (ev) (void)hipEventRecord(ev[2 * 9 + 1], d->side);
    if (with_ex) {
      if (ev) (void)hipEventRecord(ev[2 * 10], d->side);
      exch(d->side);
      if (ev) (void)hipEventRecord(ev[2 * 10 + 1], d->side);
    }
    (void)hipEventRecord(d->join, d->side);
  } else if (with_ex) {
    mark(10, 0);
    exch(s);
    mark(10, 1);
  }
  if (with_ms) {
    const int64_t ntiles = (int64_t)((g.N[0] + kAntTX - 1) / kAntTX) *
                           ((g.N[1] + kAntTY - 1) / kAntTY) * ((g.N[2] + kAntTZ - 1) / kAntTZ);
    mark(1, 0);
    if (d->ant_scatter) {
      const ScPlan& pl = d->sp;
      const int64_t nt = (int64_t)pl.nt[0] * pl.nt[1] * pl.nt[2];
      const size_t lds = (size_t)pl.lds_bytes;
#define PMFEM_SC_LAUNCH(P)                                                                    \
  hipLaunchKernelGGL(k_anterp_scatter<P>, dim3((unsigned)nt), dim3(64), lds, s, g, pl, d->q,   \
                     d->pos4, d->sc_list, d->sc_lstart, d->sc_part)
      switch (g.p) {
        case 1:
          PMFEM_SC_LAUNCH(1);
          break;
        case 2:
          PMFEM_SC_LAUNCH(2);
          break;
        case 3:
          PMFEM_SC_LAUNCH(3);
          break;
        case 4:
          PMFEM_SC_LAUNCH(4);
          break;
        default:
          PMFEM_SC_LAUNCH(5);
          break;
      }
#undef PMFEM_SC_LAUNCH
      mark(1, 1);
      mark(11, 0);
      const int64_t ng = (int64_t)g.N[0] * g.N[1] * g.N[2];
      if (g.N[0] % 4 == 0)
        hipLaunchKernelGGL(k_anterp_sum<4>, dim3((unsigned)((ng / 4 + T - 1) / T)), dim3(T), 0, s,
                           g, pl, d->sc_tab[0], d->sc_tab[1], d->sc_tab[2], d->sc_part, d->grid);
      else
        hipLaunchKernelGGL(k_anterp_sum<1>, dim3((unsigned)((ng + T - 1) / T)), dim3(T), 0, s, g,
                           pl, d->sc_tab[0], d->sc_tab[1], d->sc_tab[2], d->sc_part, d->grid);
      mark(11, 1);
    } else if (d->ant_line) {
      const AntPlan& pl = d->ap;
      const int64_t nwg = (int64_t)pl.nsx * g.N[1] * g.N[2];
      hipLaunchKernelGGL(k_anterp_line, dim3((unsigned)nwg), dim3(d->ant_threads),
                         (size_t)pl.lds_bytes, s, g, pl, d->q, d->pos4, d->ant_list,
                         d->ant_lstart, d->ant_col, d->brx, d->bry, d->brz, d->grid);
      mark(1, 1);
    } else {
      hipLaunchKernelGGL(k_anterp, dim3((unsigned)ntiles), dim3(T), 0, s, g, d->q, d->pos4,
                         d->box_start, d->brx, d->bry, d->brz, d->grid);
      mark(1, 1);
    }
    const size_t gbytes = (size_t)g.N[0] * g.N[1] * g.N[2] * sizeof(float);
    if (d->tap_q) (void)hipMemcpyAsync(d->tap_q, d->grid, gbytes, hipMemcpyDeviceToDevice, s);
    if (d->net_on) {
      (void)sg_apply(d->net, s, d->grid, d->grid);
    } else {
      convolve(d, s, d->grid, d->grid, d->spec, d->g.gmode, mark);
    }
    if (d->tap_u) (void)hipMemcpyAsync(d->tap_u, d->grid, gbytes, hipMemcpyDeviceToDevice, s);
    (void)hipStreamWaitEvent(s, d->join, 0);
    mark(7, 0);
    {
      const IcPlan& pl = d->ic_seg ? d->icp : d->icp_small;
      const pmfem_dev::IcLists& L = d->ic_seg ? d->icl : d->icl_small;
      const int64_t nwg = (int64_t)pl.nsx * g.nbox[1] * pl.nsz;
      const dim3 grid((unsigned)nwg), blk(T);
      const size_t lds = (size_t)pl.lds_bytes;
      switch (g.rb) {
        case 0:
          launch_interp<1>(pl, grid, blk, lds, s, g, d, L);
          break;
        case 1:
          launch_interp<3>(pl, grid, blk, lds, s, g, d, L);
          break;
        case 2:
          launch_interp<5>(pl, grid, blk, lds, s, g, d, L);
          break;
        default:
          launch_interp<7>(pl, grid, blk, lds, s, g, d, L);
          break;
      }
    }
    mark(7, 1);
  }
  float hx = 0.f, hy = 0.f, hz = 0.f;
  if (happ) {
    hx = (float)happ[0];
    hy = (float)happ[1];
    hz = (float)happ[2];
  }
  mark(8, 0);
  {
    const dim3 grid((unsigned)((n * d->lanes_l + T - 1) / T));
    if (d->lanes_l == 4)
      hipLaunchKernelGGL(k_gsum<4>, grid, dim3(T), 0, s, n, d->lrp, d->grec, d->u, d->hex, h, hx,
                         hy, hz, with_ex, with_ms);
    else if (d->lanes_l == 8)
      hipLaunchKernelGGL(k_gsum<8>, grid, dim3(T), 0, s, n, d->lrp, d->grec, d->u, d->hex, h, hx,
                         hy, hz, with_ex, with_ms);
    else
      hipLaunchKernelGGL(k_gsum<16>, grid, dim3(T), 0, s, n, d->lrp, d->grec, d->u, d->hex, h,
                         hx, hy, hz, with_ex, with_ms);
  }
  mark(8, 1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(c, e, "kernel launch");
  return PMFEM_OK;
}

// One classic RK4 step of Eq. llg on the FP64 master m (four FP32 field
// evaluations, FP64 combination, norm restored after the step), enqueued on
// the context's stream.
int enqueue_rk4(pmfem_ctx* c, double* m_dev, double dt, double alpha, const double* happ) {
  pmfem_dev* d = c->dev;
  hipStream_t s = stream_of(c);
  const int64_t n = d->n;
  const unsigned b3 = (unsigned)((3 * n + 255) / 256), b1 = (unsigned)((n + 255) / 256);
  const double pref = -kGamma0 / (1.0 + alpha * alpha);
  const uint32_t terms = PMFEM_TERM_EX | PMFEM_TERM_MS;
  int rc;
  // stage 1 at m
  hipLaunchKernelGGL(k_rk_stage, dim3(b3), dim3(256), 0, s, n, m_dev, (const double*)nullptr, 0.0,
                     (double*)nullptr, d->m32);
  if ((rc = run_heff(c, d->m32, d->h32, terms, happ))) return rc;
  hipLaunchKernelGGL(k_rk_rhs, dim3(b1), dim3(256), 0, s, n, (const double*)m_dev, d->h32, pref,
                     alpha, d->kk, d->acc, 1.0, 1);
  const double cs[3] = {0.5 * dt, 0.5 * dt, dt};
  const double ws[3] = {2.0, 2.0, 1.0};
  for (int k = 0; k < 3; ++k) {
    hipLaunchKernelGGL(k_rk_stage, dim3(b3), dim3(256), 0, s, n, (const double*)m_dev,
                       (const double*)d->kk, cs[k], d->mst, d->m32);
    if ((rc = run_heff(c, d->m32, d->h32, terms, happ))) return rc;
    hipLaunchKernelGGL(k_rk_rhs, dim3(b1), dim3(256), 0, s, n, (const double*)d->mst, d->h32, pref,
                       alpha, d->kk, d->acc, ws[k], 0);
  }
  hipLaunchKernelGGL(k_rk_final, dim3(b1), dim3(256), 0, s, n, m_dev, (const double*)d->acc,
                     dt / 6.0);
  return PMFEM_OK;
}

int ready(pmfem_ctx* c) {
  if (!c) return PMFEM_EINVAL;
  if (!c->built) return set_err(c, PMFEM_ESTATE, "pmfem_build has not succeeded");
  if (!c->dev) return set_err(c, PMFEM_ESTATE, "host-only context has no device operators");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_err(c, e, "hipSetDevice");
  return PMFEM_OK;
}

// ---------------------------------------------------------------------------
// Implicit midpoint LLG (Sec. 2.2): Newton on G(x) = x - m - dt f((m + x)/2)
// with right-preconditioned GMRES on dG/dx d = G (matrix-free, one field
// evaluation per Krylov vector) and the per-node 3x3 block inverse of dG/dx
// with the field operator replaced by its exchange diagonal as the
// preconditioner. Dot products are reduced on the device in a fixed order.

constexpr int kMaxKrylov = 60;
constexpr int kDotParts = 1024;
// device reductions: dot products at [0, 62), an updated norm at kRedNorm;
// the pinned host buffer mirrors them and carries coefficients at kHostCoef
constexpr int kRedNorm = 64;
constexpr int kHostCoef = 128;
static_assert(kMaxKrylov + 2 <= kRedNorm && kMaxKrylov + 1 <= kGsMaxVectors, "Krylov sizes");

int implicit_setup(pmfem_ctx* c, int kdim, bool adaptive) {
  pmfem_dev* d = c->dev;
  pmfem_dev::Implicit& W = d->imp;
  const int64_t n = d->n, n3 = 3 * n;
  int rc;
  if (adaptive && !W.xp &&
      ((rc = dalloc(c, &W.xp, n3)) || (rc = dalloc(c, &W.S, 2 * n3)) || (rc = dalloc(c, &W.r, n3))))
    return rc;
  if (W.kdim >= kdim) return PMFEM_OK;
  if ((rc = dalloc(c, &W.x, n3)) || (rc = dalloc(c, &W.mb, n3)) || (rc = dalloc(c, &W.G, n3)) ||
      (rc = dalloc(c, &W.Minv, 9 * n)) || (rc = dalloc(c, &W.V, (int64_t)(kdim + 1) * n3)) ||
      (rc = dalloc(c, &W.w, n3)) || (rc = dalloc(c, &W.z, n3)) ||
      (rc = dalloc(c, &W.part, (int64_t)(kMaxKrylov + 2) * kDotParts)) ||
      (rc = dalloc(c, &W.red, kRedNorm + 1)) || (rc = dalloc(c, &W.coef, kMaxKrylov + 1)) ||
      (rc = dalloc(c, &W.mb32, n3)) || (rc = dalloc(c, &W.H, n3)) || (rc = dalloc(c, &W.z32, n3)) ||
      (rc = dalloc(c, &W.Az, n3)))
    return rc;
  if (!W.adiag) {
    // the exchange operator's diagonal entry of every row (its own column)
    const HostOps& o = c->ops;
    std::vector<double> a((size_t)n, 0.0);
    for (int64_t r = 0; r < n; ++r)
      for (int32_t e = o.loc_rowptr[r]; e < o.loc_rowptr[r + 1]; ++e)
        if (o.loc_col[e] == r) a[(size_t)r] = (double)o.loc_val[8 * (size_t)e];
    if ((rc = upload(c, &W.adiag, a.data(), (size_t)n))) return rc;
  }
  if (!W.host) {
    const hipError_t e = hipHostMalloc((void**)&W.host, (kHostCoef + kMaxKrylov + 1) * sizeof(double));
    if (e != hipSuccess) return set_err(c, PMFEM_ENOMEM, "hipHostMalloc");
  }
  W.kdim = kdim;
  return PMFEM_OK;
}

// out[j] = V_j . w for j < nv (V with leading dimension ldv); synchronises
int dots(pmfem_ctx* c, hipStream_t s, const double* V, int64_t ldv, int nv, const double* w,
         double* out) {
  pmfem_dev* d = c->dev;
  pmfem_dev::Implicit& W = d->imp;
  const int64_t n3 = 3 * d->n;
  hipLaunchKernelGGL(k_mdot, dim3(kDotParts), dim3(256), 0, s, n3, V, ldv, nv, w, W.part);
  hipLaunchKernelGGL(k_sum_parts, dim3(nv), dim3(256), 0, s, (const double*)W.part, kDotParts,
                     W.red);
  hipError_t e = hipMemcpyAsync(W.host, W.red, nv * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_err(c, e, "implicit dot products");
  for (int j = 0; j < nv; ++j) out[j] = W.host[j];
  return PMFEM_OK;
}

// out = aw w + sum_j coef[j] V_j
int lincomb(pmfem_ctx* c, hipStream_t s, const double* V, int64_t ldv, int nv, const double* coef,
            double aw, const double* w, double* out) {
  pmfem_dev* d = c->dev;
  pmfem_dev::Implicit& W = d->imp;
  const int64_t n3 = 3 * d->n;
  if (nv > 0) {
    // the pinned buffer's second half carries the coefficients; the copy is
    // ordered before the kernel on the stream and the stream is drained
    // before the buffer is written again
    double* hc = W.host + kHostCoef;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_err(c, e, "implicit update");
    for (int j = 0; j < nv; ++j) hc[j] = coef[j];
    e = hipMemcpyAsync(W.coef, hc, nv * sizeof(double), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_err(c, e, "implicit update");
  }
  hipLaunchKernelGGL(k_lincomb, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, s, n3, V, ldv,
                     nv, (const double*)W.coef, aw, w, out);
  return PMFEM_OK;
}

// Newton's iteration for one implicit step x = r + dt f((1 - theta) m + theta x)
// (the midpoint rule: r = m, theta = 1/2; BDF: r from the past states, dt the
// step times the BDF coefficient, theta = 1), starting from the guess in W.x
// and leaving the solution there. Converged when the rms of
// the residual per component is <= tol after at least min_newton
// corrections (a predictor-corrector step needs one: a predictor accepted
// as it stands would make the error estimate zero and put predictor values
// into the step history); gives up after max_newton
// iterations, after three without a decrease (the residual has reached the
// rounding level of the FP32 field, above the tolerance), or when the
// residual exceeds diverge times its first value (diverge <= 0: never).
// GMRES ends a linear solve at a relative residual of 1e-6 or at half the
// Newton tolerance, whichever is reached first.
int newton_solve(pmfem_ctx* c, const double* r, const double* m, double theta, double dt,
                 double alpha, uint32_t terms, const double* happ, double tol, int kdim,
                 int min_newton, int max_newton, double diverge, bool* converged,
                 int32_t* newton_its, int32_t* krylov_its, std::string* hist) {
  pmfem_dev* d = c->dev;
  pmfem_dev::Implicit& W = d->imp;
  hipStream_t s = stream_of(c);
  const int64_t n = d->n, n3 = 3 * n;
  const unsigned b3 = (unsigned)((n3 + 255) / 256), b1 = (unsigned)((n + 255) / 256);
  const double cc = -kGamma0 / (1.0 + alpha * alpha);
  const double sj = -theta * dt * cc;  // dG/dx = I + sj D
  const double eta = 1e-6;
  const double rms = std::sqrt((double)n3);
  std::vector<double> hcol(kMaxKrylov + 2), h2(kMaxKrylov + 2), y(kMaxKrylov + 1),
      g(kMaxKrylov + 2), cs(kMaxKrylov + 1), sn(kMaxKrylov + 1);
  std::vector<double> R((size_t)(kMaxKrylov + 1) * (kMaxKrylov + 1));
  int rc;
  double best = HUGE_VAL, first = 0.0;
  int stall = 0;
  *converged = false;
  if (hist) hist->clear();
  for (int it = 0; it <= max_newton; ++it) {
    hipLaunchKernelGGL(k_mid_point, dim3(b3), dim3(256), 0, s, n3, m, (const double*)W.x, theta,
                       W.mb, W.mb32);
    if ((rc = run_heff(c, W.mb32, W.H, terms, happ, W.mb))) return rc;
    hipLaunchKernelGGL(k_mid_residual, dim3(kDotParts), dim3(256), 0, s, n, r, (const double*)W.x,
                       (const double*)W.mb, (const float*)W.H, (const double*)W.adiag, dt, cc,
                       alpha, theta, W.G, W.Minv, W.part);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, (const double*)W.part, kDotParts,
                       W.red);
    hipError_t e = hipMemcpyAsync(W.host, W.red, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_err(c, e, "implicit residual");
    const double beta = std::sqrt(W.host[0]);
    if (hist) {
      char buf[32];
      std::snprintf(buf, sizeof buf, "%s%.3e", it ? " " : "", beta / rms);
      *hist += buf;
    }
    if (it >= min_newton && beta / rms <= tol) {
      *converged = true;
      return PMFEM_OK;
    }
    if (it == 0) first = beta;
    stall = beta < best ? 0 : stall + 1;
    best = std::min(best, beta);
    if (it == max_newton || stall >= 3 || !std::isfinite(beta) ||
        (diverge > 0.0 && beta > diverge * first))
      return PMFEM_OK;
    ++*newton_its;
    // GMRES: V_0 = G / beta, Arnoldi with classical Gram-Schmidt, a second
    // pass where the first removed more than half of |w|^2 (w has lost
    // orthogonality to the basis), the basis held in FP32
    const double stop = std::max(eta * beta, 0.5 * tol * rms);
    hipLaunchKernelGGL(k_gs_store, dim3(b3), dim3(256), 0, s, n3, (const double*)W.G, 1.0 / beta,
                       W.V);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int used = 0;
    // h = V^T w and |w|^2, then w -= V h and |w|^2 again; one wait per pass
    auto gs_pass = [&](int nv, double* h, double* ww, double* w2) -> int {
      hipLaunchKernelGGL(k_gs_dots, dim3(kDotParts), dim3(256), 0, s, n3, (const float*)W.V, n3,
                         nv, (const double*)W.w, W.part);
      hipLaunchKernelGGL(k_sum_parts, dim3(nv + 1), dim3(256), 0, s, (const double*)W.part,
                         kDotParts, W.red);
      hipLaunchKernelGGL(k_gs_update, dim3(kDotParts), dim3(256), 0, s, n3, (const float*)W.V, n3,
                         nv, (const double*)W.red, W.w, W.part);
      hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, (const double*)W.part, kDotParts,
                         W.red + kRedNorm);
      hipError_t e2 = hipMemcpyAsync(W.host, W.red, (kRedNorm + 1) * sizeof(double),
                                     hipMemcpyDeviceToHost, s);
      if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
      if (e2 != hipSuccess) return hip_err(c, e2, "implicit Gram-Schmidt");
      for (int j = 0; j < nv; ++j) h[j] = W.host[j];
      *ww = W.host[nv];
      *w2 = W.host[kRedNorm];
      return PMFEM_OK;
    };
    for (int i = 0; i < kdim; ++i) {
      const float* Vi = W.V + (int64_t)i * n3;
      hipLaunchKernelGGL(k_mid_precond<float>, dim3(b1), dim3(256), 0, s, n,
                         (const double*)W.Minv, Vi, W.z, W.z32);
      if ((rc = run_heff(c, W.z32, W.Az, terms, nullptr))) return rc;
      hipLaunchKernelGGL(k_mid_jvp, dim3(b1), dim3(256), 0, s, n, (const double*)W.z,
                         (const float*)W.Az, (const double*)W.mb, (const float*)W.H, sj, alpha,
                         W.w);
      ++*krylov_its;
      double ww = 0.0, w2 = 0.0, ww2 = 0.0, w3 = 0.0;
      if ((rc = gs_pass(i + 1, hcol.data(), &ww, &w2))) return rc;
      if (w2 < 0.5 * ww) {
        if ((rc = gs_pass(i + 1, h2.data(), &ww2, &w3))) return rc;
        for (int j = 0; j <= i; ++j) hcol[j] += h2[j];
        w2 = w3;
      }
      const double hn = std::sqrt(std::max(w2, 0.0));
      // column i of the Hessenberg matrix, rotated by the previous Givens
      // rotations, then a new rotation that zeroes its subdiagonal
      for (int j = 0; j < i; ++j) {
        const double a = cs[j] * hcol[j] + sn[j] * hcol[j + 1];
        hcol[j + 1] = -sn[j] * hcol[j] + cs[j] * hcol[j + 1];
        hcol[j] = a;
      }
      const double den = std::hypot(hcol[i], hn);
      cs[i] = den > 0.0 ? hcol[i] / den : 1.0;
      sn[i] = den > 0.0 ? hn / den : 0.0;
      hcol[i] = den;
      for (int j = 0; j <= i; ++j) R[(size_t)j * (kMaxKrylov + 1) + i] = hcol[j];
      g[i + 1] = -sn[i] * g[i];
      g[i] = cs[i] * g[i];
      used = i + 1;
      if (std::fabs(g[i + 1]) <= stop || hn == 0.0 || i + 1 == kdim) break;
      hipLaunchKernelGGL(k_gs_store, dim3(b3), dim3(256), 0, s, n3, (const double*)W.w, 1.0 / hn,
                         W.V + (int64_t)(i + 1) * n3);
    }
    // y from R y = g, then x -= Minv (V y)
    for (int j = used - 1; j >= 0; --j) {
      double v = g[j];
      for (int k = j + 1; k < used; ++k) v -= R[(size_t)j * (kMaxKrylov + 1) + k] * y[k];
      const double rjj = R[(size_t)j * (kMaxKrylov + 1) + j];
      y[j] = rjj != 0.0 ? v / rjj : 0.0;
    }
    {
      hipError_t e2 = hipStreamSynchronize(s);
      double* hc = W.host + kHostCoef;
      for (int j = 0; j < used; ++j) hc[j] = y[j];
      if (e2 == hipSuccess)
        e2 = hipMemcpyAsync(W.coef, hc, used * sizeof(double), hipMemcpyHostToDevice, s);
      if (e2 != hipSuccess) return hip_err(c, e2, "implicit update");
    }
    hipLaunchKernelGGL(k_gs_combine, dim3(b3), dim3(256), 0, s, n3, (const float*)W.V, n3, used,
                       (const double*)W.coef, W.w);
    hipLaunchKernelGGL(k_mid_precond<double>, dim3(b1), dim3(256), 0, s, n,
                       (const double*)W.Minv, (const double*)W.w, W.z, (float*)nullptr);
    const double minus_one = -1.0;
    if ((rc = lincomb(c, s, W.z, n3, 1, &minus_one, 1.0, W.x, W.x))) return rc;
  }
  return PMFEM_OK;
}

int run_implicit(pmfem_ctx* c, double* m, double dt, double alpha, int32_t n_steps,
                 uint32_t terms, const double* happ, double tol, int kdim, int32_t* stats) {
  pmfem_dev::Implicit& W = c->dev->imp;
  hipStream_t s = stream_of(c);
  const int64_t n3 = 3 * c->dev->n;
  int32_t newton_total = 0, krylov_total = 0;
  int rc;
  auto report = [&]() {
    if (stats) {
      stats[0] = newton_total;
      stats[1] = krylov_total;
    }
  };
  std::string hist;  // residual rms after each Newton iteration, for the error message
  for (int32_t step = 0; step < n_steps; ++step) {
    hipError_t e = hipMemcpyAsync(W.x, m, n3 * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_err(c, e, "implicit step");
    bool converged = false;
    if ((rc = newton_solve(c, m, m, 0.5, dt, alpha, terms, happ, tol, kdim, 0, 30, 0.0,
                           &converged, &newton_total, &krylov_total, &hist)))
      return rc;
    if (!converged) {
      report();
      return set_err(c, PMFEM_ECONV,
                     "implicit midpoint: Newton did not reach the tolerance at step " +
                         std::to_string(step) + " (residual rms per iteration: " + hist + ")");
    }
    e = hipMemcpyAsync(m, W.x, n3 * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_err(c, e, "implicit step");
  }
  report();
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_err(c, e, "implicit step");
  return PMFEM_OK;
}

// Step-size-adaptive implicit stepping as a predictor-corrector pair, for
// the midpoint rule (scheme 0) and BDF2 (scheme 1). Newton corrects the
// predictor, at least once. From the third accepted step on, the local
// error is estimated from the corrector-predictor gap, and a step is
// accepted when the estimate is <= lte_tol; the next step is
// h min(2, max(0.2, 0.9 (lte_tol / E)^(1/3))), at most 0.9 h after a
// rejection; a failed Newton iteration (10 iterations, three without
// progress, or three times its first residual) halves the step; each
// accepted state is renormalised.
//
// Midpoint rule: the predictor extrapolates the midpoint slopes
// s = (m_k+1 - m_k) / h_k of the last two accepted steps linearly to the new
// step's midpoint (one slope: that slope; none: m itself), and Milne's
// device gives E = |C / (C - C_p)| rms(x_c - x_p). C = 1/12 is the rule's
// error constant for a linear right side (its local error is C h^3 times the
// third derivative of the solution); C_p is the predictor's, which counts
// the chord error of each slope (1/24), the error its own step left in the
// history (C), and the miss of the straight line through the two midpoint
// values.
//
// BDF2: the first step is backward Euler from m, the later ones variable-step
// BDF2, x = a m - b y_prev + beta h f(x) with w = h / h1, a = (1 + w)^2 /
// (1 + 2 w), b = w^2 / (1 + 2 w), beta = (1 + w) / (1 + 2 w); the predictor
// is the line through the last two states or the quadratic through the last
// three, and E = h / (h + h1 + h2) rms(x_c - x_p): the rule's own trajectory
// satisfies the scheme exactly, so it deviates from the exact flow by
// (1/6) h^2 (h + h1) y''' per step, while the quadratic misses it by
// (1/6) h (h + h1) (h + h1 + h2) y'''.
double predictor_constant(double h, double h1, double h2) {
  const double C = 1.0 / 12.0;
  const double a = 0.5 * (h + h1), b = a + 0.5 * (h1 + h2), r = (h + h1) / (h1 + h2);
  return (-0.5 * a * b + (1.0 / 24.0 + C) * ((1.0 + r) * h1 * h1 - r * h2 * h2)) / (h * h) -
         1.0 / 24.0;
}

int run_implicit_adaptive(pmfem_ctx* c, int scheme, double* m, double t_end, double* dt_io,
                          double alpha, uint32_t terms, const double* happ, double lte_tol,
                          double tol, int kdim, int32_t max_steps, int32_t* stats,
                          double* dt_log, int32_t log_cap) {
  pmfem_dev::Implicit& W = c->dev->imp;
  hipStream_t s = stream_of(c);
  const int64_t n3 = 3 * c->dev->n;
  const double rms = std::sqrt((double)n3);
  const double C = 1.0 / 12.0;
  const bool bdf = scheme == 1;
  const char* what = bdf ? "adaptive BDF2" : "adaptive midpoint";
  int32_t accepted = 0, rej_error = 0, rej_newton = 0, newton_total = 0, krylov_total = 0;
  auto report = [&]() {
    if (stats) {
      stats[0] = accepted;
      stats[1] = rej_error;
      stats[2] = rej_newton;
      stats[3] = newton_total;
      stats[4] = krylov_total;
    }
  };
  double t = 0.0, dt = *dt_io;
  int32_t attempts = 0;
  auto log_attempt = [&](double h) {
    if (dt_log && attempts < log_cap) dt_log[attempts] = h;
    ++attempts;
  };
  // history in the two slots of W.S: midpoint slopes, or BDF past states;
  // hs[slot] the step that belongs to it
  int ns = 0, newest = 0;
  double hs[2] = {0.0, 0.0};
  int rc;
  hipError_t e;
  while (t_end - t > 1e-12 * t_end) {
    if (accepted >= max_steps) {
      report();
      return set_err(c, PMFEM_ECONV,
                     std::string(what) + ": step limit reached at t = " + std::to_string(t) + " s");
    }
    const double h = std::min(dt, t_end - t);
    if (h < 1e-9 * t_end) {
      report();
      return set_err(c, PMFEM_ECONV, std::string(what) + ": time step underflow at t = " +
                                         std::to_string(t) + " s");
    }
    const double h1 = hs[newest], h2 = hs[1 - newest];
    double* y1 = W.S + (int64_t)newest * n3;
    // predictor into W.xp; for BDF2 the right side r into W.r
    double hn = h;  // the step the corrector's f is scaled with
    if (!bdf) {
      if (ns >= 2) {
        const double r = (h + h1) / (h1 + h2);
        double coef[2];
        coef[newest] = h * (1.0 + r);
        coef[1 - newest] = -h * r;
        rc = lincomb(c, s, W.S, n3, 2, coef, 1.0, m, W.xp);
      } else if (ns == 1) {
        rc = lincomb(c, s, y1, n3, 1, &h, 1.0, m, W.xp);
      } else {
        rc = lincomb(c, s, nullptr, 0, 0, nullptr, 1.0, m, W.xp);
      }
    } else {
      if (ns == 0) {
        rc = lincomb(c, s, nullptr, 0, 0, nullptr, 1.0, m, W.xp);
        if (!rc) rc = lincomb(c, s, nullptr, 0, 0, nullptr, 1.0, m, W.r);
      } else {
        const double w = h / h1, den = 1.0 + 2.0 * w;
        const double mb = -w * w / den;
        hn = h * (1.0 + w) / den;
        rc = lincomb(c, s, y1, n3, 1, &mb, (1.0 + w) * (1.0 + w) / den, m, W.r);
        if (!rc && ns >= 2) {
          double coef[2];
          coef[newest] = -h * (h + h1 + h2) / (h1 * h2);
          coef[1 - newest] = h * (h + h1) / ((h1 + h2) * h2);
          rc = lincomb(c, s, W.S, n3, 2, coef, (h + h1) * (h + h1 + h2) / (h1 * (h1 + h2)), m,
                       W.xp);
        } else if (!rc) {
          const double cl = -h / h1;
          rc = lincomb(c, s, y1, n3, 1, &cl, 1.0 + h / h1, m, W.xp);
        }
      }
    }
    if (rc) return rc;
    e = hipMemcpyAsync(W.x, W.xp, n3 * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_err(c, e, what);
    bool converged = false;
    if ((rc = newton_solve(c, bdf ? W.r : m, m, bdf ? 1.0 : 0.5, hn, alpha, terms, happ, tol,
                           kdim, 1, 10, 3.0, &converged, &newton_total, &krylov_total, nullptr)))
      return rc;
    if (!converged) {
      ++rej_newton;
      log_attempt(-h);
      dt = 0.5 * h;
      continue;
    }
    double dt_new = dt;
    if (ns >= 2) {
      const double minus_one = -1.0;
      if ((rc = lincomb(c, s, W.xp, n3, 1, &minus_one, 1.0, W.x, W.z))) return rc;
      double d2 = 0.0;
      if ((rc = dots(c, s, W.z, n3, 1, W.z, &d2))) return rc;
      const double factor =
          bdf ? h / (h + h1 + h2) : std::fabs(C / (C - predictor_constant(h, h1, h2)));
      const double est = factor * std::sqrt(d2) / rms;
      const double fac = est > 0.0 ? 0.9 * std::cbrt(lte_tol / est) : 2.0;
      if (!(est <= lte_tol)) {
        ++rej_error;
        log_attempt(-h);
        dt = h * std::max(0.2, std::min(0.9, fac));
        continue;
      }
      dt_new = h * std::min(2.0, std::max(0.2, fac));
    }
    // accept: x renormalised; the history's older slot takes the new slope
    // (x - m) / h, or for BDF2 the state m, then m = x
    hipLaunchKernelGGL(k_mid_normalize, dim3((unsigned)((n3 / 3 + 255) / 256)), dim3(256), 0, s,
                       n3 / 3, W.x);
    const int slot = ns == 0 ? 0 : 1 - newest;
    double* dst = W.S + (int64_t)slot * n3;
    if (bdf) {
      e = hipMemcpyAsync(dst, m, n3 * sizeof(double), hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return hip_err(c, e, what);
    } else {
      const double minus_inv_h = -1.0 / h;
      if ((rc = lincomb(c, s, m, n3, 1, &minus_inv_h, 1.0 / h, W.x, dst))) return rc;
    }
    newest = slot;
    hs[slot] = h;
    ns = std::min(ns + 1, 2);
    e = hipMemcpyAsync(m, W.x, n3 * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_err(c, e, what);
    log_attempt(h);
    ++accepted;
    t += h;
    dt = dt_new;
  }
  *dt_io = dt;
  report();
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_err(c, e, what);
  return PMFEM_OK;
}

// Autotuner: coordinate descent over the kernel forms of each stage, the
// objective being the mean duration of whole evaluations (the stages overlap
// on two streams, so their sum is what counts), measured with HIP events.
int autotune(pmfem_ctx* c, int trials, double* best_ms) {
  pmfem_dev* d = c->dev;
  hipStream_t s = stream_of(c);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return hip_err(c, e, "autotune events");
  // inputs of the timed evaluations: a uniform magnetisation (the kernels do
  // the same work for any values)
  e = hipMemsetAsync(d->m32, 0, 3 * d->n * sizeof(float), s);
  if (e != hipSuccess) return hip_err(c, e, "autotune");
  auto time_eval = [&](double& ms) -> int {
    int rc;
    for (int w = 0; w < 2; ++w)
      if ((rc = run_heff(c, d->m32, d->h32, PMFEM_TERM_EX | PMFEM_TERM_MS, nullptr))) return rc;
    (void)hipEventRecord(e0, s);
    for (int t = 0; t < trials; ++t)
      if ((rc = run_heff(c, d->m32, d->h32, PMFEM_TERM_EX | PMFEM_TERM_MS, nullptr))) return rc;
    (void)hipEventRecord(e1, s);
    hipError_t er = hipEventSynchronize(e1);
    float t = 0.f;
    if (er == hipSuccess) er = hipEventElapsedTime(&t, e0, e1);
    if (er != hipSuccess) return hip_err(c, er, "autotune timing");
    ms = (double)t / trials;
    return PMFEM_OK;
  };
  struct Stage {
    int k;
    std::vector<int> forms;
  };
  // SpMV lanes 0: chosen per pattern from its mean row length
  const Stage stages[4] = {{0, {3, 2, 1}}, {1, {2, 1}}, {2, {2, 1}}, {3, {0, 4, 8, 16}}};
  // start from the automatic choice, made explicit
  for (int k = 0; k < 4; ++k) c->variant[k] = 0;
  (void)select_variants(c);
  c->variant[0] = d->ant_scatter ? 3 : d->ant_line ? 2 : 1;
  c->variant[1] = d->ic_seg ? 2 : 1;
  c->variant[2] = d->fft_plane ? 2 : 1;
  c->variant[3] = 0;
  int rc = select_variants(c);
  double best = 0.0;
  if (!rc) rc = time_eval(best);
  for (int pass = 0; pass < 2 && !rc; ++pass)
    for (const Stage& st : stages) {
      const int keep = c->variant[st.k];
      int pick = keep;
      for (int v : st.forms) {
        if (v == keep) continue;
        c->variant[st.k] = v;
        if (select_variants(c) != PMFEM_OK) continue;  // the form does not fit
        double ms = 0.0;
        if ((rc = time_eval(ms))) break;
        if (ms < best) {
          best = ms;
          pick = v;
        }
      }
      c->variant[st.k] = pick;
      (void)select_variants(c);
      if (rc) break;
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best_ms) *best_ms = best;
  if (!rc) c->err.clear();  // forms that did not fit left their message
  return rc;
}

}  // namespace

// A batch of independent unit cells evaluated together: the local operators
// of all cells concatenated block-diagonally (one launch of each SpMV for all
// cells), and every grid kernel in its multi-cell form, one launch per kernel
// for all cells, each workgroup finding its cell in a block-to-cell table.
struct pmfem_batch {
  int device = 0;
  hipStream_t stream = nullptr, side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  // one captured RK4 step of the batch (pmfem_batch_llg_step_graph)
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  double* gm = nullptr;
  double gdt = 0.0, galpha = 0.0;
  std::vector<pmfem_ctx*> cells;
  std::vector<int64_t> off;  // first unknown of each cell in the batch vectors, [K + 1]
  int64_t n = 0;
  int32_t *lrp = nullptr, *zrp = nullptr;
  int4 *drec = nullptr, *grec = nullptr, *zrec = nullptr;
  int2* lrec = nullptr;
  int lanes_l = 4, lanes_z = 8;
  float *q = nullptr, *uz = nullptr, *u = nullptr, *hex = nullptr;
  float *m32 = nullptr, *h32 = nullptr;
  double *mst = nullptr, *kk = nullptr, *acc = nullptr;
  pmfem::CellTab* tab = nullptr;
  struct Launch {
    int32_t* bcell = nullptr;
    int32_t* boff = nullptr;
    unsigned blocks = 0;
  } sc, sum, xy, zm, yx, ic, r2c, fy, c2r, r2c_mr, fy_mr, zm_mr, xy_mr;
  size_t lds_sc = 0, lds_plane = 0, lds_z = 0, lds_ic = 0, lds_r2c = 0, lds_fy = 0;
  size_t lds_r2c_mr = 0, lds_fy_mr = 0, lds_z_mr = 0, lds_plane_mr = 0;
  int p = 3, W = 5, KC = 2, PT = 4, Bz = 8, Bzm = kFftzMr;
  double bytes = 0.0;
  std::vector<void*> allocs;
  std::string err;
};

namespace {

int batch_err(pmfem_batch* b, int code, const std::string& m) {
  if (b) b->err = m;
  return code;
}

template <class T>
int balloc(pmfem_batch* b, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) return batch_err(b, PMFEM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  b->allocs.push_back((void*)*p);
  return PMFEM_OK;
}

template <class T>
int bupload(pmfem_batch* b, T** p, const void* src, size_t count) {
  int rc = balloc(b, p, count);
  if (rc) return rc;
  if (count) {
    hipError_t e = hipMemcpy(*p, src, count * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return batch_err(b, PMFEM_EHIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }
  return PMFEM_OK;
}

void batch_free(pmfem_batch* b) {
  if (b->stream || b->side) (void)hipStreamSynchronize(b->stream);
  if (b->side) (void)hipStreamSynchronize(b->side);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (void* p : b->allocs) (void)hipFree(p);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->join) (void)hipEventDestroy(b->join);
  if (b->side) (void)hipStreamDestroy(b->side);
  delete b;
}

// block-to-cell table of one multi-cell launch: blocks[c] workgroups for cell c
int batch_launch_table(pmfem_batch* b, const std::vector<int64_t>& blocks, pmfem_batch::Launch& L) {
  std::vector<int32_t> boff(blocks.size() + 1, 0), bcell;
  for (size_t c = 0; c < blocks.size(); ++c) {
    if ((int64_t)boff[c] + blocks[c] > 2147483647LL)
      return batch_err(b, PMFEM_EINVAL, "batch launch too large");
    boff[c + 1] = boff[c] + (int32_t)blocks[c];
    for (int64_t k = 0; k < blocks[c]; ++k) bcell.push_back((int32_t)c);
  }
  L.blocks = (unsigned)boff.back();
  int rc = bupload(b, &L.boff, boff.data(), boff.size());
  if (!rc) rc = bupload(b, &L.bcell, bcell.data(), bcell.size());
  return rc;
}

int batch_setup(pmfem_batch* b, int32_t spmv_lanes) {
  const size_t K = b->cells.size();
  b->off.assign(K + 1, 0);
  int64_t nnzL = 0, nnzZ = 0;
  for (size_t c = 0; c < K; ++c) {
    const HostOps& o = b->cells[c]->ops;
    b->off[c + 1] = b->off[c] + o.n_unk;
    nnzL += o.loc_rowptr[o.n_unk];
    nnzZ += o.z0_rowptr[o.n_unk];
    double bpe = 0.0;
    (void)pmfem_query(b->cells[c], nullptr, nullptr, nullptr, &bpe);
    b->bytes += bpe;
  }
  const int64_t n = b->off[K];
  b->n = n;
  if (n >= 2147483647LL || nnzL >= 2147483647LL || nnzZ >= 2147483647LL)
    return batch_err(b, PMFEM_EINVAL, "batch too large for 32-bit indices");
  // concatenated local operators, columns shifted by the cell's first unknown
  {
    std::vector<int32_t> lrp(n + 1, 0), zrp(n + 1, 0);
    std::vector<int4> dr, gr, zr;
    std::vector<int2> lr;
    dr.reserve(nnzL);
    gr.reserve(nnzL);
    lr.reserve(nnzL);
    zr.reserve(nnzZ);
    for (size_t c = 0; c < K; ++c) {
      const HostOps& o = b->cells[c]->ops;
      const int32_t base = (int32_t)b->off[c];
      for (int64_t r = 0; r < o.n_unk; ++r) {
        for (int32_t e = o.loc_rowptr[r]; e < o.loc_rowptr[r + 1]; ++e) {
          const float* v = &o.loc_val[8 * (size_t)e];
          int4 d4, g4;
          int2 l2;
          d4.x = g4.x = l2.x = o.loc_col[e] + base;
          std::memcpy(&d4.y, &v[1], 4);
          std::memcpy(&d4.z, &v[2], 4);
          std::memcpy(&d4.w, &v[3], 4);
          std::memcpy(&g4.y, &v[4], 4);
          std::memcpy(&g4.z, &v[5], 4);
          std::memcpy(&g4.w, &v[6], 4);
          std::memcpy(&l2.y, &v[0], 4);
          dr.push_back(d4);
          gr.push_back(g4);
          lr.push_back(l2);
        }
        lrp[base + r + 1] = (int32_t)dr.size();
        for (int32_t e = o.z0_rowptr[r]; e < o.z0_rowptr[r + 1]; ++e) {
          int4 z4;
          z4.x = o.z0_col[e] + base;
          std::memcpy(&z4.y, &o.z0_val[4 * (size_t)e], 4);
          std::memcpy(&z4.z, &o.z0_val[4 * (size_t)e + 1], 4);
          std::memcpy(&z4.w, &o.z0_val[4 * (size_t)e + 2], 4);
          zr.push_back(z4);
        }
        zrp[base + r + 1] = (int32_t)zr.size();
      }
    }
    int rc;
    if ((rc = bupload(b, &b->lrp, lrp.data(), lrp.size())) ||
        (rc = bupload(b, &b->drec, dr.data(), dr.size())) ||
        (rc = bupload(b, &b->grec, gr.data(), gr.size())) ||
        (rc = bupload(b, &b->lrec, lr.data(), lr.size())) ||
        (rc = bupload(b, &b->zrp, zrp.data(), zrp.size())) ||
        (rc = bupload(b, &b->zrec, zr.data(), zr.size())))
      return rc;
    auto pick = [](double mean) { return mean > 48.0 ? 16 : mean > 24.0 ? 8 : 4; };
    b->lanes_l = spmv_lanes ? spmv_lanes : pick((double)nnzL / std::max<int64_t>(n, 1));
    b->lanes_z = spmv_lanes ? spmv_lanes : pick((double)nnzZ / std::max<int64_t>(n, 1));
  }
  int rc;
  if ((rc = balloc(b, &b->q, n)) || (rc = balloc(b, &b->uz, n)) || (rc = balloc(b, &b->u, n)) ||
      (rc = balloc(b, &b->hex, 3 * n)) || (rc = balloc(b, &b->m32, 3 * n)) ||
      (rc = balloc(b, &b->h32, 3 * n)) || (rc = balloc(b, &b->mst, 3 * n)) ||
      (rc = balloc(b, &b->kk, 3 * n)) || (rc = balloc(b, &b->acc, 3 * n)))
    return rc;
  // the cell table and the launch tables of the grid kernels
  std::vector<CellTab> tab(K);
  std::vector<int64_t> nsc(K), nsum(K), nxy(K), nzm(K), nic(K), nr2c(K), nfy(K), nr2c_mr(K),
      nfy_mr(K), nzm_mr(K), nxy_mr(K);
  b->p = b->cells[0]->dev->g.p;
  b->W = 2 * b->cells[0]->dev->g.rb + 1;
  b->PT = 4;
  for (size_t c = 0; c < K; ++c)
    if (b->cells[c]->dev->g.N[0] % 4 != 0) b->PT = 1;
  for (size_t c = 0; c < K; ++c) {
    const pmfem_dev* d = b->cells[c]->dev;
    if (d->g.p != b->p || 2 * d->g.rb + 1 != b->W)
      return batch_err(b, PMFEM_EINVAL, "cells of a batch must share the Lagrange order and near radius");
    if (!d->sc_ok || (!d->ic_ok && !d->ic_small_ok))
      return batch_err(b, PMFEM_EINVAL, "a cell does not fit the batched kernel forms");
    CellTab& t = tab[c];
    t.g = d->g;
    t.sp = d->sp;
    t.icp = d->icp;
    t.pos4 = d->pos4;
    t.sc_list = d->sc_list;
    t.sc_lstart = d->sc_lstart;
    for (int a = 0; a < 3; ++a) t.sc_tab[a] = d->sc_tab[a];
    t.sc_part = d->sc_part;
    t.grid = d->grid;
    t.spec = d->spec;
    t.khat = d->khat;
    t.twx = d->twx;
    t.twy = d->twy;
    t.twz = d->twz;
    t.twfx = d->twfx;
    t.twfy = d->twfy;
    t.twfz = d->twfz;
    // interpolation: the largest tiles whose staging fits, else the narrow ones
    const IcPlan& ipl = d->ic_ok ? d->icp : d->icp_small;
    const pmfem_dev::IcLists& il = d->ic_ok ? d->icl : d->icl_small;
    t.icp = ipl;
    t.ic_list = il.list;
    t.ic_lstart = il.lstart;
    t.ic_wseg = il.wseg;
    t.ic_rdesc = il.rdesc;
    t.prp = d->prp;
    t.pv = d->pv;
    t.q = b->q + b->off[c];
    t.uz = b->uz + b->off[c];
    t.u = b->u + b->off[c];
    const GridParams& g = d->g;
    const int64_t ng = (int64_t)g.N[0] * g.N[1] * g.N[2];
    const int Hx = g.M[0] / 2 + 1;
    nsc[c] = (int64_t)d->sp.nt[0] * d->sp.nt[1] * d->sp.nt[2];
    nsum[c] = (ng / b->PT + 255) / 256;
    // FFT: whole z-planes in LDS where they fit, else one axis per pass
    // (radix 2, or mixed radix where an extent is not a power of two)
    t.lpb = std::max(1, 2048 / g.M[0]);
    t.by = std::max(1, std::min(16, 4096 / g.M[1]));
    nr2c_mr[c] = nfy_mr[c] = nxy_mr[c] = 0;
    if (d->fft_mr && d->fft_ok) {
      nxy[c] = nr2c[c] = nfy[c] = 0;
      nxy_mr[c] = g.N[2];
      b->lds_plane_mr = std::max(b->lds_plane_mr, d->fft_plane_lds);
      b->Bzm = std::min(b->Bzm, std::max(1, std::min(kFftzMr, 2048 / g.M[2])));
    } else if (d->fft_mr) {
      nxy[c] = nr2c[c] = nfy[c] = 0;
      t.by = std::max(1, std::min(16, 2048 / g.M[1]));
      const int64_t xlines = (int64_t)((g.N[1] + 1) / 2) * g.N[2];
      nr2c_mr[c] = (xlines + t.lpb - 1) / t.lpb;
      nfy_mr[c] = (int64_t)g.N[2] * ((Hx + t.by - 1) / t.by);
      b->lds_r2c_mr =
          std::max(b->lds_r2c_mr, (size_t)(g.M[0] + 2 * t.lpb * g.M[0]) * sizeof(float2));
      b->lds_fy_mr = std::max(b->lds_fy_mr, (size_t)(g.M[1] + 2 * t.by * g.M[1]) * sizeof(float2));
      b->Bzm = std::min(b->Bzm, std::max(1, std::min(kFftzMr, 2048 / g.M[2])));
    } else if (d->fft_ok) {
      nxy[c] = (int64_t)g.N[2] * kFftSplit;
      nr2c[c] = nfy[c] = 0;
      b->lds_plane = std::max(b->lds_plane, d->fft_plane_lds);
    } else {
      nxy[c] = 0;
      const int64_t xlines = (int64_t)((g.N[1] + 1) / 2) * g.N[2];
      nr2c[c] = (xlines + t.lpb - 1) / t.lpb;
      nfy[c] = (int64_t)g.N[2] * ((Hx + t.by - 1) / t.by);
      b->lds_r2c = std::max(b->lds_r2c, (size_t)(g.M[0] / 2 + t.lpb * g.M[0]) * sizeof(float2));
      b->lds_fy = std::max(b->lds_fy, (size_t)(g.M[1] / 2 + t.by * g.M[1]) * sizeof(float2));
    }
    if (!d->fft_mr) b->Bz = std::min(b->Bz, std::max(1, std::min(kFftzB, 4096 / g.M[2])));
    nic[c] = (int64_t)ipl.nsx * g.nbox[1] * ipl.nsz;
    b->lds_sc = std::max(b->lds_sc, (size_t)d->sp.lds_bytes);
    b->lds_ic = std::max(b->lds_ic, (size_t)ipl.lds_bytes);
    b->KC = std::max(b->KC, ipl.kc);
  }
  for (size_t c = 0; c < K; ++c) {
    const GridParams& g = b->cells[c]->dev->g;
    const int64_t cols = (int64_t)g.M[1] * (g.M[0] / 2 + 1);
    if (b->cells[c]->dev->fft_mr) {
      nzm[c] = 0;
      nzm_mr[c] = (cols + b->Bzm - 1) / b->Bzm;
      b->lds_z_mr = std::max(b->lds_z_mr, (size_t)(g.M[2] + 2 * b->Bzm * g.M[2]) * sizeof(float2));
    } else {
      nzm_mr[c] = 0;
      nzm[c] = (cols + b->Bz - 1) / b->Bz;
      b->lds_z = std::max(b->lds_z, (size_t)(g.M[2] / 2 + b->Bz * g.M[2]) * sizeof(float2));
    }
  }
  if ((rc = bupload(b, &b->tab, tab.data(), K)) || (rc = batch_launch_table(b, nsc, b->sc)) ||
      (rc = batch_launch_table(b, nsum, b->sum)) || (rc = batch_launch_table(b, nxy, b->xy)) ||
      (rc = batch_launch_table(b, nxy, b->yx)) || (rc = batch_launch_table(b, nzm, b->zm)) ||
      (rc = batch_launch_table(b, nic, b->ic)) || (rc = batch_launch_table(b, nr2c, b->r2c)) ||
      (rc = batch_launch_table(b, nfy, b->fy)) || (rc = batch_launch_table(b, nr2c, b->c2r)) ||
      (rc = batch_launch_table(b, nr2c_mr, b->r2c_mr)) ||
      (rc = batch_launch_table(b, nfy_mr, b->fy_mr)) ||
      (rc = batch_launch_table(b, nzm_mr, b->zm_mr)) ||
      (rc = batch_launch_table(b, nxy_mr, b->xy_mr)))
    return rc;
  if (b->lds_plane_mr > 65536) {
    const int lb = (int)b->lds_plane_mr;
    if (hipFuncSetAttribute((const void*)k_fft_xy_fwd_mr_cells,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lb) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_fft_yx_inv_mr_cells,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lb) != hipSuccess)
      return batch_err(b, PMFEM_EINVAL, "FFT planes of the batch do not fit in LDS");
  }
  if (b->lds_plane > 65536) {
    const int lb = (int)b->lds_plane;
    if (hipFuncSetAttribute((const void*)k_fft_xy_fwd_cells,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lb) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_fft_yx_inv_cells,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lb) != hipSuccess)
      return batch_err(b, PMFEM_EINVAL, "FFT planes of the batch do not fit in LDS");
  }
  return PMFEM_OK;
}

template <int WT, int KC>
void launch_interp_cells(const pmfem_batch* b, hipStream_t s) {
  hipLaunchKernelGGL((k_interp_tile_cells<WT, KC>), dim3(b->ic.blocks), dim3(256), b->lds_ic, s,
                     (const CellTab*)b->tab, (const int32_t*)b->ic.bcell, (const int32_t*)b->ic.boff);
}

template <int WT>
void launch_interp_cells_kc(const pmfem_batch* b, hipStream_t s) {
  switch (b->KC) {
    case 2:
      launch_interp_cells<WT, 2>(b, s);
      break;
    case 4:
      launch_interp_cells<WT, 4>(b, s);
      break;
    case 6:
      launch_interp_cells<WT, 6>(b, s);
      break;
    default:
      launch_interp_cells<WT, 8>(b, s);
      break;
  }
}

// One evaluation of every cell: m, h [n][3] packed in cell order.
int batch_heff(pmfem_batch* b, const float* m, float* h, uint32_t terms) {
  hipStream_t s = b->stream;
  const int64_t n = b->n;
  const int T = 256;
  const int with_ex = (terms & PMFEM_TERM_EX) ? 1 : 0;
  const int with_ms = (terms & PMFEM_TERM_MS) ? 1 : 0;
  auto rowdot3 = [&](hipStream_t st, const int32_t* rp, const int4* rec, float* out, int lanes) {
    const dim3 grid((unsigned)((n * lanes + T - 1) / T));
    if (lanes == 4) hipLaunchKernelGGL(k_rowdot3<4>, grid, dim3(T), 0, st, n, m, rp, rec, out);
    else if (lanes == 8) hipLaunchKernelGGL(k_rowdot3<8>, grid, dim3(T), 0, st, n, m, rp, rec, out);
    else hipLaunchKernelGGL(k_rowdot3<16>, grid, dim3(T), 0, st, n, m, rp, rec, out);
  };
  auto exch = [&](hipStream_t st) {
    const dim3 grid((unsigned)((n * b->lanes_l + T - 1) / T));
    if (b->lanes_l == 4) hipLaunchKernelGGL((k_exch<4, float>), grid, dim3(T), 0, st, n, b->lrp, b->lrec, m, b->hex);
    else if (b->lanes_l == 8) hipLaunchKernelGGL((k_exch<8, float>), grid, dim3(T), 0, st, n, b->lrp, b->lrec, m, b->hex);
    else hipLaunchKernelGGL((k_exch<16, float>), grid, dim3(T), 0, st, n, b->lrp, b->lrec, m, b->hex);
  };
  const CellTab* tab = b->tab;
  if (with_ms) {
    rowdot3(s, b->lrp, b->drec, b->q, b->lanes_l);
    (void)hipEventRecord(b->fork, s);
    (void)hipStreamWaitEvent(b->side, b->fork, 0);
    rowdot3(b->side, b->zrp, b->zrec, b->uz, b->lanes_z);
    if (with_ex) exch(b->side);
    (void)hipEventRecord(b->join, b->side);
#define PMFEM_SCC(P)                                                                           \
  hipLaunchKernelGGL(k_anterp_scatter_cells<P>, dim3(b->sc.blocks), dim3(64), b->lds_sc, s, tab, \
                     (const int32_t*)b->sc.bcell, (const int32_t*)b->sc.boff)
    switch (b->p) {
      case 1:
        PMFEM_SCC(1);
        break;
      case 2:
        PMFEM_SCC(2);
        break;
      case 3:
        PMFEM_SCC(3);
        break;
      case 4:
        PMFEM_SCC(4);
        break;
      default:
        PMFEM_SCC(5);
        break;
    }
#undef PMFEM_SCC
    if (b->PT == 4)
      hipLaunchKernelGGL(k_anterp_sum_cells<4>, dim3(b->sum.blocks), dim3(T), 0, s, tab,
                         (const int32_t*)b->sum.bcell, (const int32_t*)b->sum.boff);
    else
      hipLaunchKernelGGL(k_anterp_sum_cells<1>, dim3(b->sum.blocks), dim3(T), 0, s, tab,
                         (const int32_t*)b->sum.bcell, (const int32_t*)b->sum.boff);
    // cells whose z-planes fit in LDS take the plane passes, the others the
    // per-axis passes; the z pass with the K multiply serves both
    if (b->xy.blocks)
      hipLaunchKernelGGL(k_fft_xy_fwd_cells, dim3(b->xy.blocks), dim3(1024), b->lds_plane, s, tab,
                         (const int32_t*)b->xy.bcell, (const int32_t*)b->xy.boff, kFftSplit);
    if (b->r2c.blocks) {
      hipLaunchKernelGGL(k_r2c_x_cells, dim3(b->r2c.blocks), dim3(T), b->lds_r2c, s, tab,
                         (const int32_t*)b->r2c.bcell, (const int32_t*)b->r2c.boff);
      hipLaunchKernelGGL(k_fft_y_cells, dim3(b->fy.blocks), dim3(T), b->lds_fy, s, tab,
                         (const int32_t*)b->fy.bcell, (const int32_t*)b->fy.boff, 0);
    }
    if (b->xy_mr.blocks)
      hipLaunchKernelGGL(k_fft_xy_fwd_mr_cells, dim3(b->xy_mr.blocks), dim3(kFftPlaneMrT),
                         b->lds_plane_mr, s, tab, (const int32_t*)b->xy_mr.bcell,
                         (const int32_t*)b->xy_mr.boff);
    if (b->r2c_mr.blocks) {
      hipLaunchKernelGGL(k_r2c_x_mr_cells, dim3(b->r2c_mr.blocks), dim3(T), b->lds_r2c_mr, s, tab,
                         (const int32_t*)b->r2c_mr.bcell, (const int32_t*)b->r2c_mr.boff);
      hipLaunchKernelGGL(k_fft_y_mr_cells, dim3(b->fy_mr.blocks), dim3(T), b->lds_fy_mr, s, tab,
                         (const int32_t*)b->fy_mr.bcell, (const int32_t*)b->fy_mr.boff, 0);
    }
    if (b->zm_mr.blocks)
      hipLaunchKernelGGL(k_fft_z_mul_mr_cells, dim3(b->zm_mr.blocks), dim3(kFftzT), b->lds_z_mr,
                         s, tab, (const int32_t*)b->zm_mr.bcell, (const int32_t*)b->zm_mr.boff,
                         b->Bzm);
    if (b->xy_mr.blocks)
      hipLaunchKernelGGL(k_fft_yx_inv_mr_cells, dim3(b->xy_mr.blocks), dim3(kFftPlaneMrT),
                         b->lds_plane_mr, s, tab, (const int32_t*)b->xy_mr.bcell,
                         (const int32_t*)b->xy_mr.boff);
    if (b->r2c_mr.blocks) {
      hipLaunchKernelGGL(k_fft_y_mr_cells, dim3(b->fy_mr.blocks), dim3(T), b->lds_fy_mr, s, tab,
                         (const int32_t*)b->fy_mr.bcell, (const int32_t*)b->fy_mr.boff, 1);
      hipLaunchKernelGGL(k_c2r_x_mr_cells, dim3(b->r2c_mr.blocks), dim3(T), b->lds_r2c_mr, s, tab,
                         (const int32_t*)b->r2c_mr.bcell, (const int32_t*)b->r2c_mr.boff);
    }
    if (b->zm.blocks)
      hipLaunchKernelGGL(k_fft_z_mul_cells, dim3(b->zm.blocks), dim3(kFftzT), b->lds_z, s, tab,
                         (const int32_t*)b->zm.bcell, (const int32_t*)b->zm.boff, b->Bz);
    if (b->yx.blocks)
      hipLaunchKernelGGL(k_fft_yx_inv_cells, dim3(b->yx.blocks), dim3(1024), b->lds_plane, s, tab,
                         (const int32_t*)b->yx.bcell, (const int32_t*)b->yx.boff, kFftSplit);
    if (b->r2c.blocks) {
      hipLaunchKernelGGL(k_fft_y_cells, dim3(b->fy.blocks), dim3(T), b->lds_fy, s, tab,
                         (const int32_t*)b->fy.bcell, (const int32_t*)b->fy.boff, 1);
      hipLaunchKernelGGL(k_c2r_x_cells, dim3(b->c2r.blocks), dim3(T), b->lds_r2c, s, tab,
                         (const int32_t*)b->c2r.bcell, (const int32_t*)b->c2r.boff);
    }
    (void)hipStreamWaitEvent(s, b->join, 0);
    switch (b->W) {
      case 1:
        launch_interp_cells_kc<1>(b, s);
        break;
      case 3:
        launch_interp_cells_kc<3>(b, s);
        break;
      case 5:
        launch_interp_cells_kc<5>(b, s);
        break;
      default:
        launch_interp_cells_kc<7>(b, s);
        break;
    }
  } else if (with_ex) {
    exch(s);
  }
  {
    const dim3 grid((unsigned)((n * b->lanes_l + T - 1) / T));
    if (b->lanes_l == 4)
      hipLaunchKernelGGL(k_gsum<4>, grid, dim3(T), 0, s, n, b->lrp, b->grec, b->u, b->hex, h, 0.f,
                         0.f, 0.f, with_ex, with_ms);
    else if (b->lanes_l == 8)
      hipLaunchKernelGGL(k_gsum<8>, grid, dim3(T), 0, s, n, b->lrp, b->grec, b->u, b->hex, h, 0.f,
                         0.f, 0.f, with_ex, with_ms);
    else
      hipLaunchKernelGGL(k_gsum<16>, grid, dim3(T), 0, s, n, b->lrp, b->grec, b->u, b->hex, h,
                         0.f, 0.f, 0.f, with_ex, with_ms);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return batch_err(b, PMFEM_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return PMFEM_OK;
}

// one RK4 step of every cell on the packed FP64 master magnetisation
int batch_rk4(pmfem_batch* b, double* m, double dt, double alpha) {
  hipStream_t s = b->stream;
  const int64_t n = b->n;
  const unsigned b3 = (unsigned)((3 * n + 255) / 256), b1 = (unsigned)((n + 255) / 256);
  const double pref = -kGamma0 / (1.0 + alpha * alpha);
  const uint32_t terms = PMFEM_TERM_EX | PMFEM_TERM_MS;
  int rc;
  hipLaunchKernelGGL(k_rk_stage, dim3(b3), dim3(256), 0, s, n, m, (const double*)nullptr, 0.0,
                     (double*)nullptr, b->m32);
  if ((rc = batch_heff(b, b->m32, b->h32, terms))) return rc;
  hipLaunchKernelGGL(k_rk_rhs, dim3(b1), dim3(256), 0, s, n, (const double*)m, b->h32, pref, alpha,
                     b->kk, b->acc, 1.0, 1);
  const double cs[3] = {0.5 * dt, 0.5 * dt, dt};
  const double ws[3] = {2.0, 2.0, 1.0};
  for (int k = 0; k < 3; ++k) {
    hipLaunchKernelGGL(k_rk_stage, dim3(b3), dim3(256), 0, s, n, (const double*)m,
                       (const double*)b->kk, cs[k], b->mst, b->m32);
    if ((rc = batch_heff(b, b->m32, b->h32, terms))) return rc;
    hipLaunchKernelGGL(k_rk_rhs, dim3(b1), dim3(256), 0, s, n, (const double*)b->mst, b->h32, pref,
                       alpha, b->kk, b->acc, ws[k], 0);
  }
  hipLaunchKernelGGL(k_rk_final, dim3(b1), dim3(256), 0, s, n, m, (const double*)b->acc, dt / 6.0);
  return PMFEM_OK;
}

}  // namespace

extern "C" {

int pmfem_create(pmfem_ctx** out, int hip_device, void* hip_stream) {
  if (!out) return PMFEM_EINVAL;
  *out = nullptr;
  if (hip_device >= 0) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || hip_device >= count) return PMFEM_EHIP;
  } else if (hip_device != -1) {
    return PMFEM_EINVAL;
  }
  // once per device, with that device current: the address of the
  // no-allocation scratch array (kept for the life of the process)
  if (hip_device >= 0) {
    const int rc = lookup_scratch(hip_device);
    if (rc) return rc;
  }
  pmfem_ctx* c = new (std::nothrow) pmfem_ctx();
  if (!c) return PMFEM_ENOMEM;
  c->device = hip_device;
  c->stream = hip_stream;
  *out = c;
  return PMFEM_OK;
}

int pmfem_set_mesh(pmfem_ctx* c, int64_t n_nodes, const double* xyz, int64_t n_tets,
                   const int32_t* tets, const int32_t* region) {
  if (!c) return PMFEM_EINVAL;
  if (n_nodes < 4 || n_tets < 1 || !xyz || !tets || !region)
    return set_err(c, PMFEM_EINVAL, "empty mesh or null array");
  if (n_nodes > 2000000000LL || n_tets > 2000000000LL) return set_err(c, PMFEM_EINVAL, "mesh too large");
  c->n_nodes = n_nodes;
  c->n_tets = n_tets;
  c->xyz.assign(xyz, xyz + 3 * n_nodes);
  c->tets.assign(tets, tets + 4 * n_tets);
  c->region.assign(region, region + n_tets);
  c->have_mesh = true;
  c->built = false;
  return PMFEM_OK;
}

int pmfem_set_materials(pmfem_ctx* c, int32_t n_regions, const double* Ms, const double* Aex) {
  if (!c) return PMFEM_EINVAL;
  if (n_regions < 1 || !Ms || !Aex) return set_err(c, PMFEM_EINVAL, "no regions");
  c->n_regions = n_regions;
  c->Ms.assign(Ms, Ms + n_regions);
  c->Aex.assign(Aex, Aex + n_regions);
  c->have_mat = true;
  c->built = false;
  return PMFEM_OK;
}

int pmfem_set_periodicity(pmfem_ctx* c, uint32_t axis_mask, const double L[3], double match_tol) {
  if (!c) return PMFEM_EINVAL;
  if (axis_mask > 7 || (axis_mask && !L)) return set_err(c, PMFEM_EINVAL, "bad periodicity");
  c->mask = axis_mask;
  for (int a = 0; a < 3; ++a) c->L[a] = L ? L[a] : 0.0;
  c->match_tol = match_tol > 0 ? match_tol : 1e-9;
  c->built = false;
  return PMFEM_OK;
}

int pmfem_set_variant(pmfem_ctx* c, const char* stage, int32_t variant) {
  if (!c) return PMFEM_EINVAL;
  if (!stage) return set_err(c, PMFEM_EINVAL, "null stage");
  int k = -1;
  if (std::strcmp(stage, "anterp") == 0) k = 0;
  if (std::strcmp(stage, "interp") == 0) k = 1;
  if (std::strcmp(stage, "fft") == 0) k = 2;
  if (std::strcmp(stage, "spmv") == 0) k = 3;
  if (k < 0) return set_err(c, PMFEM_EINVAL, "unknown stage");
  if (k == 0 && (variant < 0 || variant > 3))
    return set_err(c, PMFEM_EINVAL, "anterp variant must be 0, 1, 2 or 3");
  if ((k == 1 || k == 2) && (variant < 0 || variant > 2))
    return set_err(c, PMFEM_EINVAL, "variant must be 0, 1 or 2");
  if (k == 3 && variant != 0 && variant != 4 && variant != 8 && variant != 16)
    return set_err(c, PMFEM_EINVAL, "spmv lanes must be 0, 4, 8 or 16");
  const int old = c->variant[k];
  c->variant[k] = variant;
  if (c->dev) {
    const int rc = select_variants(c);
    if (rc) {
      c->variant[k] = old;
      (void)select_variants(c);
      return rc;
    }
  }
  return PMFEM_OK;
}

int pmfem_set_aim(pmfem_ctx* c, const int32_t grid[3], int32_t order_p, int32_t near_boxes,
                  double z0_radius_edges, int32_t precision) {
  if (!c) return PMFEM_EINVAL;
  if (!grid) return set_err(c, PMFEM_EINVAL, "null grid");
  for (int a = 0; a < 3; ++a)
    if (grid[a] < 2 || grid[a] > 1024) return set_err(c, PMFEM_EGRID, "grid size out of range");
  for (int a = 0; a < 3; ++a) c->grid[a] = grid[a];
  c->order_p = order_p;
  c->near_boxes = near_boxes;
  c->z0_radius = z0_radius_edges;
  c->precision = precision;
  c->have_aim = true;
  c->built = false;
  return PMFEM_OK;
}

int pmfem_build(pmfem_ctx* c) {
  if (!c) return PMFEM_EINVAL;
  c->built = false;
  free_dev(c);
  int rc;
  try {
    rc = host_build(c);
  } catch (const std::bad_alloc&) {
    return set_err(c, PMFEM_ENOMEM, "host allocation failed");
  }
  if (rc != PMFEM_OK) return rc;
  if (c->device >= 0) {
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_err(c, e, "hipSetDevice");
    c->dev = new (std::nothrow) pmfem_dev();
    if (!c->dev) return set_err(c, PMFEM_ENOMEM, "host allocation failed");
    try {
      rc = upload_all(c);
    } catch (const std::bad_alloc&) {
      rc = set_err(c, PMFEM_ENOMEM, "host allocation failed");
    }
    if (rc != PMFEM_OK) {
      free_dev(c);
      return rc;
    }
  }
  c->built = true;
  return PMFEM_OK;
}

int pmfem_query(pmfem_ctx* c, int64_t* n_unknowns, int64_t* unknown_of_node,
                int64_t* node_of_unknown, double* bytes_per_eval) {
  if (!c) return PMFEM_EINVAL;
  if (!c->built) return set_err(c, PMFEM_ESTATE, "pmfem_build has not succeeded");
  const HostOps& o = c->ops;
  if (n_unknowns) *n_unknowns = o.n_unk;
  if (unknown_of_node) std::memcpy(unknown_of_node, o.unk_of_node.data(), o.n_nodes * sizeof(int64_t));
  if (node_of_unknown) std::memcpy(node_of_unknown, o.node_of_unk.data(), o.n_unk * sizeof(int64_t));
  if (bytes_per_eval) {
    // algorithmic HBM bytes: every array of one evaluation touched once
    const double n = (double)o.n_unk;
    const double nL = (double)o.loc_rowptr[o.n_unk], nZ = (double)o.z0_rowptr[o.n_unk],
                 nP = (double)o.p_rowptr[o.n_unk];
    const double ng = (double)o.N[0] * o.N[1] * o.N[2];
    const double hx = o.M[0] / 2 + 1;
    const double spec = (double)o.N[2] * o.M[1] * hx * 8.0;
    const double khat = hx * o.M[1] * o.M[2] * 4.0;
    const double gb = c->precision == 1 ? 2.0 : 4.0;  // bytes per stored grid value
    double b = 0;
    b += 2 * n * (4 + 12 + 4) + nL * 16 + nZ * 16;                      // charges, u_Z
    b += n * (16 + 4) + ng * gb + (double)o.box_start.size() * 4;      // anterpolation
    b += ng * gb + spec;                                                 // x/y forward
    b += 2 * spec + khat;                                                // z, K multiply
    b += spec + ng * gb;                                                 // y/x inverse
    b += n * (16 + 4 + 4 + 4 + 4) + ng * gb + nP * 4;                    // interp+corr
    b += n * (4 + 12 + 12) + nL * 8;                                     // exchange
    b += n * (4 + 4 + 12 + 12) + nL * 16;                                // gradient sum
    *bytes_per_eval = b;
  }
  return PMFEM_OK;
}

int pmfem_heff(pmfem_ctx* c, const float* m_dev, float* h_dev, uint32_t terms,
               const double* h_applied) {
  int rc = ready(c);
  if (rc) return rc;
  if (!m_dev || !h_dev || terms > 3) return set_err(c, PMFEM_EINVAL, "bad heff arguments");
  return run_heff(c, m_dev, h_dev, terms, h_applied);
}

int pmfem_heff_parts(pmfem_ctx* c, const float* m_dev, float* h_dev, float* q_dev, float* u_dev,
                     float* hex_dev) {
  int rc = ready(c);
  if (rc) return rc;
  if (!m_dev || !h_dev) return set_err(c, PMFEM_EINVAL, "bad heff arguments");
  rc = run_heff(c, m_dev, h_dev, PMFEM_TERM_EX | PMFEM_TERM_MS, nullptr);
  if (rc) return rc;
  pmfem_dev* d = c->dev;
  hipStream_t s = stream_of(c);
  const size_t n = (size_t)d->n;
  hipError_t e = hipSuccess;
  if (q_dev) e = hipMemcpyAsync(q_dev, d->q, n * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && u_dev) e = hipMemcpyAsync(u_dev, d->u, n * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && hex_dev)
    e = hipMemcpyAsync(hex_dev, d->hex, 3 * n * 4, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_err(c, e, "copy of intermediates");
  return PMFEM_OK;
}

int pmfem_grid_convolve(pmfem_ctx* c, const float* q_grid_dev, float* u_grid_dev) {
  int rc = ready(c);
  if (rc) return rc;
  if (!q_grid_dev || !u_grid_dev) return set_err(c, PMFEM_EINVAL, "null grid buffer");
  pmfem_dev* d = c->dev;
  const GridParams& g = d->g;
  hipStream_t s = stream_of(c);
  convolve(d, s, q_grid_dev, u_grid_dev, d->spec, 0, [](int, int) {});
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(c, e, "kernel launch");
  return PMFEM_OK;
}

int pmfem_grid_convolve_noalloc(pmfem_ctx* c, const float* q_grid_dev, float* u_grid_dev) {
  int rc = ready(c);
  if (rc) return rc;
  if (!q_grid_dev || !u_grid_dev) return set_err(c, PMFEM_EINVAL, "null grid buffer");
  pmfem_dev* d = c->dev;
  const GridParams& g = d->g;
  const int64_t nspec = (int64_t)g.N[2] * g.M[1] * (g.M[0] / 2 + 1);
  if (nspec > kNoallocSpecMax)
    return set_err(c, PMFEM_EINVAL,
                   "grid too large for the no-allocation scratch: half-spectrum of " +
                       std::to_string(nspec) + " complex values, at most " +
                       std::to_string(kNoallocSpecMax));
  float2* spec = scratch_ptr(c->device);
  if (!spec) return set_err(c, PMFEM_ESTATE, "no-allocation scratch not set up on this device");
  convolve(d, stream_of(c), q_grid_dev, u_grid_dev, spec, 0, [](int, int) {});
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(c, e, "kernel launch");
  return PMFEM_OK;
}

int pmfem_llg_step(pmfem_ctx* c, double* m_dev, double dt, double alpha, int32_t n_steps,
                   const double* h_applied) {
  int rc = ready(c);
  if (rc) return rc;
  if (!m_dev || n_steps < 0 || !(dt > 0.0) || !(alpha >= 0.0))
    return set_err(c, PMFEM_EINVAL, "bad llg arguments");
  for (int32_t st = 0; st < n_steps; ++st)
    if ((rc = enqueue_rk4(c, m_dev, dt, alpha, h_applied))) return rc;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_err(c, e, "kernel launch");
  return PMFEM_OK;
}

int pmfem_llg_step_graph(pmfem_ctx* c, double* m_dev, double dt, double alpha, int32_t n_steps,
                         const double* h_applied) {
  int rc = ready(c);
  if (rc) return rc;
  if (!m_dev || n_steps < 0 || !(dt > 0.0) || !(alpha >= 0.0))
    return set_err(c, PMFEM_EINVAL, "bad llg arguments");
  if (n_steps == 0) return PMFEM_OK;
  pmfem_dev* d = c->dev;
  pmfem_dev::StepGraph& G = d->sg;
  const bool wh = h_applied != nullptr;
  bool same = G.x && G.m == m_dev && G.dt == dt && G.alpha == alpha && G.with_happ == wh &&
              G.net_on == d->net_on && (!d->net_on || G.net_version == d->net_version);
  for (int k = 0; same && wh && k < 3; ++k) same = G.happ[k] == h_applied[k];
  hipError_t e = hipSuccess;
  if (!same) {
    // capture one step on a stream of the library's own: the kernels of the
    // step and the fork to the second stream and back, nothing else
    if (G.x) {
      e = hipStreamSynchronize(stream_of(c));
      (void)hipGraphExecDestroy(G.x);
      G.x = nullptr;
    }
    if (G.g) {
      (void)hipGraphDestroy(G.g);
      G.g = nullptr;
    }
    if (e == hipSuccess && !G.cap) e = hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_err(c, e, "graph stream");
    void* saved = c->stream;
    const int prof_max = d->prof_max;
    d->prof_max = d->prof_calls;  // no profiling events inside the graph
    c->stream = G.cap;
    e = hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) rc = enqueue_rk4(c, m_dev, dt, alpha, h_applied);
    hipGraph_t g = nullptr;
    const hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(G.cap, &g) : e;
    c->stream = saved;
    d->prof_max = prof_max;
    if (rc || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return rc ? rc : hip_err(c, e2, "graph capture");
    }
    e = hipGraphInstantiate(&G.x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      G.x = nullptr;
      return hip_err(c, e, "graph instantiate");
    }
    G.g = g;
    G.m = m_dev;
    G.dt = dt;
    G.alpha = alpha;
    G.with_happ = wh;
    G.net_on = d->net_on;
    G.net_version = d->net_version;
    for (int k = 0; k < 3; ++k) G.happ[k] = wh ? h_applied[k] : 0.0;
  }
  for (int32_t i = 0; i < n_steps && e == hipSuccess; ++i) e = hipGraphLaunch(G.x, stream_of(c));
  if (e != hipSuccess) return hip_err(c, e, "graph launch");
  return PMFEM_OK;
}

int pmfem_llg_implicit(pmfem_ctx* c, double* m_dev, double dt, double alpha, int32_t n_steps,
                       uint32_t terms, const double* h_applied, double newton_tol,
                       int32_t krylov_dim, int32_t* iterations) {
  int rc = ready(c);
  if (rc) return rc;
  if (!m_dev || n_steps < 0 || !(dt > 0.0) || !(alpha >= 0.0) || terms < 1 || terms > 3)
    return set_err(c, PMFEM_EINVAL, "bad implicit llg arguments");
  const int kdim = krylov_dim <= 0 ? 30 : krylov_dim;
  if (kdim > kMaxKrylov) return set_err(c, PMFEM_EINVAL, "krylov_dim above 60");
  const double tol = newton_tol > 0.0 ? newton_tol : 1e-8;
  if ((rc = implicit_setup(c, kdim, false))) return rc;
  return run_implicit(c, m_dev, dt, alpha, n_steps, terms, h_applied, tol, kdim, iterations);
}

int pmfem_llg_implicit_adaptive(pmfem_ctx* c, double* m_dev, double t_end, double* dt,
                                double alpha, uint32_t terms, const double* h_applied,
                                double lte_tol, double newton_tol, int32_t krylov_dim,
                                int32_t max_steps, int32_t* stats, double* dt_log,
                                int32_t dt_log_cap) {
  int rc = ready(c);
  if (rc) return rc;
  if (!m_dev || !dt || !(t_end > 0.0) || !(*dt > 0.0) || !(alpha >= 0.0) || terms < 1 ||
      terms > 3 || !(lte_tol > 0.0) || max_steps < 0 || dt_log_cap < 0 ||
      (dt_log_cap > 0 && !dt_log))
    return set_err(c, PMFEM_EINVAL, "bad adaptive llg arguments");
  const int kdim = krylov_dim <= 0 ? 30 : krylov_dim;
  if (kdim > kMaxKrylov) return set_err(c, PMFEM_EINVAL, "krylov_dim above 60");
  const double tol = newton_tol > 0.0 ? newton_tol : 0.1 * lte_tol;
  if ((rc = implicit_setup(c, kdim, true))) return rc;
  return run_implicit_adaptive(c, 0, m_dev, t_end, dt, alpha, terms, h_applied, lte_tol, tol,
                               kdim, max_steps > 0 ? max_steps : 1000000, stats, dt_log,
                               dt_log_cap);
}

int pmfem_llg_bdf2_adaptive(pmfem_ctx* c, double* m_dev, double t_end, double* dt, double alpha,
                            uint32_t terms, const double* h_applied, double lte_tol,
                            double newton_tol, int32_t krylov_dim, int32_t max_steps,
                            int32_t* stats, double* dt_log, int32_t dt_log_cap) {
  int rc = ready(c);
  if (rc) return rc;
  if (!m_dev || !dt || !(t_end > 0.0) || !(*dt > 0.0) || !(alpha >= 0.0) || terms < 1 ||
      terms > 3 || !(lte_tol > 0.0) || max_steps < 0 || dt_log_cap < 0 ||
      (dt_log_cap > 0 && !dt_log))
    return set_err(c, PMFEM_EINVAL, "bad adaptive llg arguments");
  const int kdim = krylov_dim <= 0 ? 30 : krylov_dim;
  if (kdim > kMaxKrylov) return set_err(c, PMFEM_EINVAL, "krylov_dim above 60");
  const double tol = newton_tol > 0.0 ? newton_tol : 0.1 * lte_tol;
  if ((rc = implicit_setup(c, kdim, true))) return rc;
  return run_implicit_adaptive(c, 1, m_dev, t_end, dt, alpha, terms, h_applied, lte_tol, tol,
                               kdim, max_steps > 0 ? max_steps : 1000000, stats, dt_log,
                               dt_log_cap);
}

int pmfem_energy(pmfem_ctx* c, const double* m_dev, double* e_ex, double* e_ms) {
  int rc = ready(c);
  if (rc) return rc;
  if (!m_dev || !e_ex || !e_ms) return set_err(c, PMFEM_EINVAL, "bad energy arguments");
  pmfem_dev* d = c->dev;
  hipStream_t s = stream_of(c);
  const int64_t n = d->n;
  hipLaunchKernelGGL(k_rk_stage, dim3((unsigned)((3 * n + 255) / 256)), dim3(256), 0, s, n, m_dev,
                     (const double*)nullptr, 0.0, (double*)nullptr, d->m32);
  // the both-terms evaluation leaves H_ex in d->hex and q, u in their buffers
  if ((rc = run_heff(c, d->m32, d->h32, PMFEM_TERM_EX | PMFEM_TERM_MS, nullptr))) return rc;
  hipLaunchKernelGGL(k_energy, dim3(d->nparts), dim3(256), 0, s, n, m_dev, (const double*)d->mu,
                     (const float*)d->hex, (const float*)d->q, (const float*)d->u, d->part);
  std::vector<double> part(2 * d->nparts);
  hipError_t e = hipMemcpyAsync(part.data(), d->part, part.size() * sizeof(double),
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_err(c, e, "energy");
  double a = 0.0, b = 0.0;
  for (int i = 0; i < d->nparts; ++i) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  *e_ex = -0.5 * kMu0 * a;
  *e_ms = 0.5 * kMu0 * b;
  return PMFEM_OK;
}

int pmfem_profile_begin(pmfem_ctx* c, int32_t max_calls) {
  int rc = ready(c);
  if (rc) return rc;
  if (max_calls < 1 || max_calls > 100000) return set_err(c, PMFEM_EINVAL, "bad max_calls");
  pmfem_dev* d = c->dev;
  for (hipEvent_t e : d->ev) (void)hipEventDestroy(e);
  d->ev.assign((size_t)max_calls * kNumKernels * 2, nullptr);
  for (auto& e : d->ev) {
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return hip_err(c, r, "hipEventCreate");
  }
  d->prof_max = max_calls;
  d->prof_calls = 0;
  return PMFEM_OK;
}

int pmfem_profile_end(pmfem_ctx* c, int32_t* n_kernels, double* ms, int32_t* count,
                      char (*names)[32]) {
  int rc = ready(c);
  if (rc) return rc;
  pmfem_dev* d = c->dev;
  hipError_t e = hipStreamSynchronize(stream_of(c));
  if (e != hipSuccess) return hip_err(c, e, "hipStreamSynchronize");
  int out = 0;
  for (int k = 0; k < kNumKernels; ++k) {
    double tot = 0.0;
    int cnt = 0;
    for (int call = 0; call < d->prof_calls; ++call) {
      hipEvent_t a = d->ev[((size_t)call * kNumKernels + k) * 2];
      hipEvent_t b = d->ev[((size_t)call * kNumKernels + k) * 2 + 1];
      float t = 0.f;
      if (hipEventElapsedTime(&t, a, b) == hipSuccess) {
        tot += t;
        ++cnt;
      }
    }
    if (cnt == 0) continue;  // slot not used by this context's launch sequence
    if (ms) ms[out] = tot;
    if (count) count[out] = cnt;
    if (names) {
      std::strncpy(names[out], d->kname[k] ? d->kname[k] : "?", 31);
      names[out][31] = 0;
    }
    ++out;
  }
  if (n_kernels) *n_kernels = out;
  (void)hipGetLastError();  // events of kernels that did not run report errors
  d->prof_max = 0;
  d->prof_calls = 0;
  return PMFEM_OK;
}

int pmfem_export(pmfem_ctx* c, const char* name, void* out, int64_t* count, int32_t* elem_bytes) {
  if (!c || !name || !count) return PMFEM_EINVAL;
  if (!c->built) return set_err(c, PMFEM_ESTATE, "pmfem_build has not succeeded");
  const HostOps& o = c->ops;
  const void* src = nullptr;
  int64_t cnt = 0;
  int32_t eb = 0;
  std::vector<double> info;
  std::vector<int32_t> ivec;
  std::string nm(name);
  if (nm == "mu") { src = o.mu.data(); cnt = (int64_t)o.mu.size(); eb = 8; }
  else if (nm == "pos") { src = o.pos.data(); cnt = (int64_t)o.pos.size(); eb = 8; }
  else if (nm == "pos4") { src = o.pos4.data(); cnt = (int64_t)o.pos4.size(); eb = 4; }
  else if (nm == "box_start") { src = o.box_start.data(); cnt = (int64_t)o.box_start.size(); eb = 4; }
  else if (nm == "loc_rowptr") { src = o.loc_rowptr.data(); cnt = (int64_t)o.loc_rowptr.size(); eb = 4; }
  else if (nm == "loc_col") { src = o.loc_col.data(); cnt = (int64_t)o.loc_col.size(); eb = 4; }
  else if (nm == "loc_val") { src = o.loc_val.data(); cnt = (int64_t)o.loc_val.size(); eb = 4; }
  else if (nm == "z0_rowptr") { src = o.z0_rowptr.data(); cnt = (int64_t)o.z0_rowptr.size(); eb = 4; }
  else if (nm == "z0_col") { src = o.z0_col.data(); cnt = (int64_t)o.z0_col.size(); eb = 4; }
  else if (nm == "z0_val") { src = o.z0_val.data(); cnt = (int64_t)o.z0_val.size(); eb = 4; }
  else if (nm == "p_rowptr") { src = o.p_rowptr.data(); cnt = (int64_t)o.p_rowptr.size(); eb = 4; }
  else if (nm == "p_col") { src = o.p_col.data(); cnt = (int64_t)o.p_col.size(); eb = 4; }
  else if (nm == "p_val") { src = o.p_val.data(); cnt = (int64_t)o.p_val.size(); eb = 4; }
  else if (nm == "khat") { src = o.khat.data(); cnt = (int64_t)o.khat.size(); eb = 4; }
  else if (nm == "kgrid") { src = o.kgrid.data(); cnt = (int64_t)o.kgrid.size(); eb = 8; }
  else if (nm == "unk_of_node") { src = o.unk_of_node.data(); cnt = (int64_t)o.unk_of_node.size(); eb = 8; }
  else if (nm == "node_of_unk") { src = o.node_of_unk.data(); cnt = (int64_t)o.node_of_unk.size(); eb = 8; }
  else if (nm == "grid_info") {
    // N[3], M[3], delta[3], origin[3], hbar, p, r_b, periodic[3]
    for (int a = 0; a < 3; ++a) info.push_back(o.N[a]);
    for (int a = 0; a < 3; ++a) info.push_back(o.M[a]);
    for (int a = 0; a < 3; ++a) info.push_back(o.delta[a]);
    for (int a = 0; a < 3; ++a) info.push_back(o.origin[a]);
    info.push_back(o.hbar);
    info.push_back(o.p);
    info.push_back(o.rb);
    for (int a = 0; a < 3; ++a) info.push_back(o.per[a]);
    src = info.data();
    cnt = (int64_t)info.size();
    eb = 8;
  } else if (nm == "sc_plan" || nm == "sc_list" || nm == "sc_lstart" || nm == "sc_tab") {
    // the scatter anterpolation's tiles (built here from the box table)
    ScPlan pl{};
    std::vector<int2> list, tab[3];
    std::vector<int32_t> lstart;
    if (!plan_scatter(o, pl, list, lstart, tab))
      return set_err(c, PMFEM_EGRID, "scatter tiles do not fit this problem");
    if (nm == "sc_plan") {
      ivec = {pl.tb[0], pl.tb[1], pl.tb[2], pl.nt[0], pl.nt[1], pl.nt[2],
              pl.fd[0], pl.fd[1], pl.fd[2], pl.fsize};
    } else if (nm == "sc_list") {
      for (const int2& e : list) ivec.insert(ivec.end(), {e.x, e.y});
    } else if (nm == "sc_lstart") {
      ivec = lstart;
    } else {
      for (int a = 0; a < 3; ++a)
        for (const int2& e : tab[a]) ivec.insert(ivec.end(), {e.x, e.y});
    }
    src = ivec.data();
    cnt = (int64_t)ivec.size();
    eb = 4;
  } else {
    return set_err(c, PMFEM_EINVAL, "unknown export name: " + nm);
  }
  *count = cnt;
  if (elem_bytes) *elem_bytes = eb;
  if (out && cnt) std::memcpy(out, src, (size_t)cnt * eb);
  return PMFEM_OK;
}

int pmfem_autotune(pmfem_ctx* c, int32_t trials, int32_t* chosen, double* best_ms) {
  int rc = ready(c);
  if (rc) return rc;
  if (trials < 1 || trials > 10000) return set_err(c, PMFEM_EINVAL, "trials must be in [1, 10000]");
  if (c->dev->prof_max > 0) return set_err(c, PMFEM_ESTATE, "autotune while profiling");
  // the forms are timed on the plain path (the FFT convolution among them)
  const bool net_on = c->dev->net_on;
  c->dev->net_on = false;
  rc = autotune(c, trials, best_ms);
  c->dev->net_on = net_on;
  if (rc) return rc;
  if (chosen)
    for (int k = 0; k < 4; ++k) chosen[k] = c->variant[k];
  return PMFEM_OK;
}

int pmfem_batch_create(pmfem_batch** out, int32_t n_cells, pmfem_ctx* const* cells,
                       void* hip_stream, int32_t spmv_lanes) {
  if (!out) return PMFEM_EINVAL;
  *out = nullptr;
  if (n_cells < 1 || !cells) return PMFEM_EINVAL;
  if (spmv_lanes != 0 && spmv_lanes != 4 && spmv_lanes != 8 && spmv_lanes != 16) return PMFEM_EINVAL;
  for (int32_t k = 0; k < n_cells; ++k) {
    if (!cells[k] || !cells[k]->built || !cells[k]->dev) return PMFEM_ESTATE;
    if (cells[k]->device != cells[0]->device) return PMFEM_EINVAL;
    for (int32_t j = 0; j < k; ++j)
      if (cells[j] == cells[k]) return PMFEM_EINVAL;
  }
  pmfem_batch* b = new (std::nothrow) pmfem_batch();
  if (!b) return PMFEM_ENOMEM;
  b->device = cells[0]->device;
  b->stream = (hipStream_t)hip_stream;
  b->cells.assign(cells, cells + n_cells);
  hipError_t e = hipSetDevice(b->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join, hipEventDisableTiming);
  if (e != hipSuccess) {
    batch_free(b);
    return PMFEM_EHIP;
  }
  int rc;
  try {
    rc = batch_setup(b, spmv_lanes);
  } catch (const std::bad_alloc&) {
    rc = PMFEM_ENOMEM;
  }
  if (rc) {
    // the caller gets the batch back to read the message, unless it could not be made
    *out = b;
    return rc;
  }
  *out = b;
  return PMFEM_OK;
}

int pmfem_batch_query(pmfem_batch* b, int64_t* n_unknowns, int64_t* cell_offsets,
                      double* bytes_per_eval) {
  if (!b) return PMFEM_EINVAL;
  if (n_unknowns) *n_unknowns = b->n;
  if (cell_offsets)
    for (size_t c = 0; c < b->off.size(); ++c) cell_offsets[c] = b->off[c];
  if (bytes_per_eval) *bytes_per_eval = b->bytes;
  return PMFEM_OK;
}

int pmfem_batch_heff(pmfem_batch* b, const float* m_dev, float* h_dev, uint32_t terms) {
  if (!b) return PMFEM_EINVAL;
  if (!b->tab) return batch_err(b, PMFEM_ESTATE, "batch set-up failed");
  if (!m_dev || !h_dev || terms < 1 || terms > 3)
    return batch_err(b, PMFEM_EINVAL, "bad batch heff arguments");
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return batch_err(b, PMFEM_EHIP, "hipSetDevice");
  return batch_heff(b, m_dev, h_dev, terms);
}

int pmfem_batch_llg_step(pmfem_batch* b, double* m_dev, double dt, double alpha, int32_t n_steps) {
  if (!b) return PMFEM_EINVAL;
  if (!b->tab) return batch_err(b, PMFEM_ESTATE, "batch set-up failed");
  if (!m_dev || n_steps < 0 || !(dt > 0.0) || !(alpha >= 0.0))
    return batch_err(b, PMFEM_EINVAL, "bad batch llg arguments");
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return batch_err(b, PMFEM_EHIP, "hipSetDevice");
  for (int32_t st = 0; st < n_steps; ++st) {
    const int rc = batch_rk4(b, m_dev, dt, alpha);
    if (rc) return rc;
  }
  e = hipGetLastError();
  if (e != hipSuccess) return batch_err(b, PMFEM_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return PMFEM_OK;
}

int pmfem_batch_llg_step_graph(pmfem_batch* b, double* m_dev, double dt, double alpha,
                               int32_t n_steps) {
  if (!b) return PMFEM_EINVAL;
  if (!b->tab) return batch_err(b, PMFEM_ESTATE, "batch set-up failed");
  if (!m_dev || n_steps < 0 || !(dt > 0.0) || !(alpha >= 0.0))
    return batch_err(b, PMFEM_EINVAL, "bad batch llg arguments");
  hipError_t e = hipSetDevice(b->device);
  if (e != hipSuccess) return batch_err(b, PMFEM_EHIP, "hipSetDevice");
  if (n_steps == 0) return PMFEM_OK;
  if (!(b->gexec && b->gm == m_dev && b->gdt == dt && b->galpha == alpha)) {
    // capture one step on a stream of the batch's own: its kernels and the
    // fork to the second stream and back
    if (b->gexec) {
      e = hipStreamSynchronize(b->stream);
      (void)hipGraphExecDestroy(b->gexec);
      b->gexec = nullptr;
    }
    if (b->graph) {
      (void)hipGraphDestroy(b->graph);
      b->graph = nullptr;
    }
    if (e == hipSuccess && !b->cap) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return batch_err(b, PMFEM_EHIP, "graph stream");
    hipStream_t saved = b->stream;
    b->stream = b->cap;
    int rc = PMFEM_OK;
    e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) rc = batch_rk4(b, m_dev, dt, alpha);
    hipGraph_t g = nullptr;
    const hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(b->cap, &g) : e;
    b->stream = saved;
    if (rc || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return rc ? rc : batch_err(b, PMFEM_EHIP, std::string("graph capture: ") + hipGetErrorString(e2));
    }
    e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      b->gexec = nullptr;
      return batch_err(b, PMFEM_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    b->graph = g;
    b->gm = m_dev;
    b->gdt = dt;
    b->galpha = alpha;
  }
  for (int32_t i = 0; i < n_steps && e == hipSuccess; ++i) e = hipGraphLaunch(b->gexec, b->stream);
  if (e != hipSuccess) return batch_err(b, PMFEM_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
  return PMFEM_OK;
}

const char* pmfem_batch_last_error(const pmfem_batch* b) { return b ? b->err.c_str() : "null batch"; }

void pmfem_batch_destroy(pmfem_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  batch_free(b);
}

const char* pmfem_last_error(const pmfem_ctx* c) { return c ? c->err.c_str() : "null context"; }

void pmfem_destroy(pmfem_ctx* c) {
  if (!c) return;
  if (c->dev && c->device >= 0) (void)hipSetDevice(c->device);
  free_dev(c);
  delete c;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Learned surrogate of the grid convolution (layers, layout and precision in
// surrogate.h).

namespace {

int net_ready(pmfem_ctx* c, bool need_scales) {
  int rc = ready(c);
  if (rc) return rc;
  if (!c->dev->net) return set_err(c, PMFEM_ESTATE, "pmfem_surrogate_init has not been called");
  if (need_scales && !(c->dev->net->s_in > 0.f && c->dev->net->s_out > 0.f))
    return set_err(c, PMFEM_ESTATE, "surrogate scales not set (train it or set its parameters)");
  return PMFEM_OK;
}

// host RNG for the texture parameters: the same SplitMix64 finaliser
struct HostRng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uni() { return ((double)(next() >> 11) + 0.5) * 0x1p-53; }
};

SgTexture draw_texture(const pmfem_ctx* c, int kind, uint64_t seed) {
  HostRng r{seed * 0x2545F4914F6CDD1Dull + 0x1234567ull};
  SgTexture t{};
  t.kind = kind;
  t.seed = (uint32_t)(r.next() & 0xffffffffu);
  t.Lx = c->L[0];
  t.Ly = c->L[1];
  const double lmin = std::min(t.Lx, t.Ly);
  if (kind == 1) {
    t.cx = r.uni() * t.Lx;
    t.cy = r.uni() * t.Ly;
    t.rc = lmin * (0.03 + 0.12 * r.uni());
    t.chir = r.uni() < 0.5 ? -1.0 : 1.0;
    t.pol = r.uni() < 0.5 ? -1.0 : 1.0;
  } else if (kind == 2) {
    const bool along_x = r.uni() < 0.5;
    t.nx = along_x ? 1.0 : 0.0;
    t.ny = along_x ? 0.0 : 1.0;
    const double L = along_x ? t.Lx : t.Ly;
    t.cx = r.uni() * L;
    t.rc = L * (0.01 + 0.05 * r.uni());
    // domain direction uniform on the sphere, the turning direction uniform
    // on the circle perpendicular to it
    const double z = 2.0 * r.uni() - 1.0, ph = 2.0 * kPi * r.uni(), rr = std::sqrt(1.0 - z * z);
    const double ed[3] = {rr * std::cos(ph), rr * std::sin(ph), z};
    double a[3] = {std::fabs(ed[0]) < 0.9 ? 1.0 : 0.0, std::fabs(ed[0]) < 0.9 ? 0.0 : 1.0, 0.0};
    double u[3] = {ed[1] * a[2] - ed[2] * a[1], ed[2] * a[0] - ed[0] * a[2], ed[0] * a[1] - ed[1] * a[0]};
    const double un = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (double& x : u) x /= un;
    const double v[3] = {ed[1] * u[2] - ed[2] * u[1], ed[2] * u[0] - ed[0] * u[2], ed[0] * u[1] - ed[1] * u[0]};
    const double ps = 2.0 * kPi * r.uni();
    for (int k = 0; k < 3; ++k) {
      t.ed[k] = ed[k];
      t.er[k] = std::cos(ps) * u[k] + std::sin(ps) * v[k];
    }
  }
  return t;
}

}  // namespace

extern "C" {

int pmfem_surrogate_init(pmfem_ctx* c, int32_t depth, uint64_t seed, int32_t bf16_activations) {
  int rc = ready(c);
  if (rc) return rc;
  pmfem_dev* d = c->dev;
  if (depth < 2 || depth > kSgMaxDepth)
    return set_err(c, PMFEM_EINVAL, "surrogate depth must be in [2, " + std::to_string(kSgMaxDepth) + "]");
  if (!(d->g.per[0] && d->g.per[1] && !d->g.per[2]))
    return set_err(c, PMFEM_EINVAL, "the surrogate needs a film: periodic along x and y only");
  if (d->g.gmode != 0)
    return set_err(c, PMFEM_EINVAL, "the surrogate needs the FP32 grid (precision 0)");
  if (d->net) {
    sg_destroy(d->net);
    delete d->net;
    d->net = nullptr;
    d->net_on = false;
  }
  Surrogate* net = new Surrogate();
  const SgGrid gd{d->g.N[0], d->g.N[1], d->g.N[2]};
  hipError_t e = sg_create(net, depth, gd, d->n, c->ops.pos.data(), bf16_activations == 0);
  if (e != hipSuccess) {
    sg_destroy(net);
    delete net;
    return e == hipErrorOutOfMemory ? set_err(c, PMFEM_ENOMEM, "surrogate buffers")
                                    : hip_err(c, e, "surrogate allocation");
  }
  d->net = net;
  d->net_version++;
  std::vector<float> p;
  sg_default_params(net, seed, p);
  if ((e = sg_set_params(net, p.data(), stream_of(c))) != hipSuccess)
    return hip_err(c, e, "surrogate parameters");
  if ((e = hipStreamSynchronize(stream_of(c))) != hipSuccess) return hip_err(c, e, "surrogate init");
  return PMFEM_OK;
}

int pmfem_surrogate_param_count(pmfem_ctx* c, int64_t* count) {
  int rc = net_ready(c, false);
  if (rc) return rc;
  if (!count) return set_err(c, PMFEM_EINVAL, "null count");
  *count = c->dev->net->nparam;
  return PMFEM_OK;
}

int pmfem_surrogate_set_params(pmfem_ctx* c, const float* params, int64_t count,
                               const double* scales) {
  int rc = net_ready(c, false);
  if (rc) return rc;
  Surrogate* net = c->dev->net;
  if (!params || count != net->nparam)
    return set_err(c, PMFEM_EINVAL, "parameter vector must hold " + std::to_string(net->nparam) + " values");
  if (scales && !(scales[0] > 0.0 && scales[1] > 0.0))
    return set_err(c, PMFEM_EINVAL, "surrogate scales must be positive");
  hipError_t e = sg_set_params(net, params, stream_of(c));
  if (e == hipSuccess) e = hipStreamSynchronize(stream_of(c));
  if (e != hipSuccess) return hip_err(c, e, "surrogate parameters");
  if (scales) {
    net->s_in = (float)scales[0];
    net->s_out = (float)scales[1];
  }
  c->dev->net_version++;
  return PMFEM_OK;
}

int pmfem_surrogate_get_params(pmfem_ctx* c, float* params, int64_t count, double* scales) {
  int rc = net_ready(c, false);
  if (rc) return rc;
  Surrogate* net = c->dev->net;
  if (params) {
    if (count != net->nparam)
      return set_err(c, PMFEM_EINVAL, "parameter vector must hold " + std::to_string(net->nparam) + " values");
    hipError_t e = sg_get_params(net, params, stream_of(c));
    if (e != hipSuccess) return hip_err(c, e, "surrogate parameters");
  }
  if (scales) {
    scales[0] = net->s_in;
    scales[1] = net->s_out;
  }
  return PMFEM_OK;
}

int pmfem_surrogate_apply(pmfem_ctx* c, const float* q_grid_dev, float* u_grid_dev) {
  int rc = net_ready(c, true);
  if (rc) return rc;
  if (!q_grid_dev || !u_grid_dev) return set_err(c, PMFEM_EINVAL, "null grid buffer");
  hipError_t e = sg_apply(c->dev->net, stream_of(c), q_grid_dev, u_grid_dev);
  if (e != hipSuccess) return hip_err(c, e, "surrogate launch");
  return PMFEM_OK;
}

int pmfem_surrogate_profile(pmfem_ctx* c, const float* q_grid_dev, float* u_grid_dev, int32_t reps,
                            double* ms_per_layer) {
  int rc = net_ready(c, true);
  if (rc) return rc;
  if (!q_grid_dev || !u_grid_dev || !ms_per_layer || reps < 1)
    return set_err(c, PMFEM_EINVAL, "bad profile arguments");
  hipError_t e = sg_profile(c->dev->net, stream_of(c), q_grid_dev, u_grid_dev, reps, ms_per_layer);
  if (e != hipSuccess) return hip_err(c, e, "surrogate profile");
  return PMFEM_OK;
}

int pmfem_surrogate_loss_grad(pmfem_ctx* c, const float* q_grid_dev, const float* t_grid_dev,
                              double* loss, float* grad, int64_t count) {
  int rc = net_ready(c, true);
  if (rc) return rc;
  Surrogate* net = c->dev->net;
  if (!q_grid_dev || !t_grid_dev) return set_err(c, PMFEM_EINVAL, "null grid buffer");
  if (grad && count != net->nparam)
    return set_err(c, PMFEM_EINVAL, "gradient vector must hold " + std::to_string(net->nparam) + " values");
  hipStream_t s = stream_of(c);
  c->dev->net_version++;  // the activation buffers may be reallocated
  hipError_t e = sg_ensure_training(net, 1);
  if (e != hipSuccess) return set_err(c, PMFEM_ENOMEM, "surrogate training buffers");
  if ((e = sg_loss_grad(net, s, q_grid_dev, t_grid_dev, 1.f, 0)) != hipSuccess)
    return hip_err(c, e, "surrogate launch");
  if (loss && (e = hipMemcpyAsync(loss, net->loss, sizeof(double), hipMemcpyDeviceToHost, s)))
    return hip_err(c, e, "loss copy");
  if (grad && (e = hipMemcpyAsync(grad, net->grad, (size_t)count * 4, hipMemcpyDeviceToHost, s)))
    return hip_err(c, e, "gradient copy");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_err(c, e, "surrogate gradient");
  return PMFEM_OK;
}

int pmfem_surrogate_texture(pmfem_ctx* c, int32_t kind, uint64_t seed, double* m_dev) {
  int rc = net_ready(c, false);
  if (rc) return rc;
  if (!m_dev || kind < 0 || kind > 2) return set_err(c, PMFEM_EINVAL, "bad texture arguments");
  hipError_t e = sg_texture(c->dev->net, stream_of(c), draw_texture(c, kind, seed), m_dev);
  if (e != hipSuccess) return hip_err(c, e, "texture launch");
  return PMFEM_OK;
}

int pmfem_surrogate_train(pmfem_ctx* c, int32_t n_pairs, double lr, uint64_t seed, uint32_t kinds,
                          double* loss_log) {
  int rc = net_ready(c, false);
  if (rc) return rc;
  if (n_pairs < 0 || !(lr > 0.0) || (kinds & 7u) == 0)
    return set_err(c, PMFEM_EINVAL, "bad training arguments");
  pmfem_dev* d = c->dev;
  Surrogate* net = d->net;
  hipStream_t s = stream_of(c);
  d->net_version++;  // the scales may be set below
  hipError_t e = sg_ensure_training(net, std::max(1, n_pairs));
  if (e != hipSuccess) return set_err(c, PMFEM_ENOMEM, "surrogate training buffers");
  int list[3], nk = 0;
  for (int k = 0; k < 3; ++k)
    if (kinds & (1u << k)) list[nk++] = k;
  const bool was_on = d->net_on;
  for (int32_t it = 0; it < n_pairs; ++it) {
    // one AIM pair: texture -> charges -> grid charges Q -> grid potential U
    const SgTexture tx = draw_texture(c, list[it % nk], seed * 1000003ull + (uint64_t)it);
    if ((e = sg_texture(net, s, tx, net->m64)) || (e = sg_to_f32(net, s, net->m64, net->m32)))
      return hip_err(c, e, "texture launch");
    d->net_on = false;
    d->tap_q = net->qbuf;
    d->tap_u = net->ubuf;
    rc = run_heff(c, net->m32, net->ha, PMFEM_TERM_MS, nullptr);
    d->tap_q = d->tap_u = nullptr;
    d->net_on = was_on;
    if (rc) return rc;
    if (!(net->s_in > 0.f && net->s_out > 0.f)) {
      // scales from the first pair: unit mean square at the input and output
      double sq = 0.0, su = 0.0;
      if ((e = sg_sumsq(net, s, net->qbuf, net->nvox, &sq)) ||
          (e = sg_sumsq(net, s, net->ubuf, net->nvox, &su)))
        return hip_err(c, e, "scale reduction");
      if (!(sq > 0.0 && su > 0.0)) return set_err(c, PMFEM_ECONV, "training pair with zero charges");
      net->s_in = (float)(1.0 / std::sqrt(sq / (double)net->nvox));
      net->s_out = (float)std::sqrt(su / (double)net->nvox);
    }
    if ((e = sg_loss_grad(net, s, net->qbuf, net->ubuf, 1.f / net->s_out, it)) ||
        (e = sg_adam(net, s, lr)))
      return hip_err(c, e, "surrogate training launch");
  }
  if (loss_log && n_pairs > 0 &&
      (e = hipMemcpyAsync(loss_log, net->loss, (size_t)n_pairs * sizeof(double),
                          hipMemcpyDeviceToHost, s)))
    return hip_err(c, e, "loss copy");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_err(c, e, "surrogate training");
  return PMFEM_OK;
}

int pmfem_surrogate_enable(pmfem_ctx* c, int32_t on) {
  int rc = on ? net_ready(c, true) : ready(c);
  if (rc) return rc;
  c->dev->net_on = on != 0;
  return PMFEM_OK;
}

int pmfem_llg_step_judged(pmfem_ctx* c, double* m_dev, double dt, double alpha, int32_t n_steps,
                          const double* h_applied, int32_t check_every, double tol,
                          double* report) {
  int rc = net_ready(c, true);
  if (rc) return rc;
  if (!m_dev || n_steps < 0 || !(dt > 0.0) || !(alpha >= 0.0) || check_every < 1 || !(tol >= 0.0))
    return set_err(c, PMFEM_EINVAL, "bad llg arguments");
  pmfem_dev* d = c->dev;
  Surrogate* net = d->net;
  hipStream_t s = stream_of(c);
  const bool was_on = d->net_on;
  bool use = true;
  double checks = 0.0, emax = 0.0, elast = -1.0, fallback = -1.0;
  hipError_t e;
  for (int32_t st = 0; st < n_steps; ++st) {
    if (use && st % check_every == 0) {
      // the plain AIM judges the surrogate on the magnetostatic field
      if ((e = sg_to_f32(net, s, m_dev, net->m32))) return hip_err(c, e, "conversion launch");
      d->net_on = false;
      if ((rc = run_heff(c, net->m32, net->ha, PMFEM_TERM_MS, nullptr))) break;
      d->net_on = true;
      if ((rc = run_heff(c, net->m32, net->hs, PMFEM_TERM_MS, nullptr))) break;
      double e2[2];
      if ((e = sg_field_error(net, s, net->hs, net->ha, e2))) {
        rc = hip_err(c, e, "field error");
        break;
      }
      const double err = e2[1] > 0.0 ? std::sqrt(e2[0] / e2[1]) : std::sqrt(e2[0]);
      checks += 1.0;
      emax = std::max(emax, err);
      elast = err;
      if (!(err <= tol)) {
        use = false;
        fallback = st;
      }
    }
    d->net_on = use;
    if ((rc = enqueue_rk4(c, m_dev, dt, alpha, h_applied))) break;
  }
  d->net_on = was_on;
  if (rc) return rc;
  if (report) {
    report[0] = checks;
    report[1] = emax;
    report[2] = elast;
    report[3] = fallback;
  }
  return PMFEM_OK;
}

}  // extern "C"

// Internal declarations of the gfx950 DEAM library (plan layout, kernel
// parameter blocks, launchers).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "../../include/deam.h"

namespace deam {

// In-plane description of the ray of one (view, channel), in grid units
// (voxel index coordinates).  The ray is walked along its driving axis a
// (y if |dy| >= |dx| in grid units, else x) and its lateral coordinate is
// b(a) = ib + b0 + a*mb.  The integer origin ib is the lateral pixel at the
// middle of the grid's driving range, so that b0 + a*mb stays small along
// the ray: its rounding (and with it the error of every lateral crossing,
// that rounding divided by |mb|) is then set by the lateral distance
// travelled, not by the grid size, which matters for rays nearly parallel
// to a grid axis in FP32.  Computed once per plan in FP64, stored in the
// plan precision; shared by all detector rows of a helical channel.
template <typename T>
struct RayXY {
  T b0, mb, imb;  // lateral line relative to ib, and 1/mb (huge when mb == 0)
  T sa, ida;      // driving coordinate of the source, 1/da (da = in-plane run in grid units)
  T iadb;         // 1/|db| (huge when db == 0)
  T yd;           // 1 when a = y (rows), 0 when a = x
  T ib;           // integer lateral origin (exact in the plan precision)
};

// Geometry as the kernels see it.
struct GeomDev {
  int is3d;
  int nx, ny, nz;
  int n_views, n_rows, n_cols;
  // views walked by the projectors and the backprojector: v = voff + vsub * i,
  // i < nvl (all views: 0, 1, n_views; an ordered subset otherwise)
  int voff, vsub, nvl;
  double dx, dy, dz;
  double x0, y0, z0;            // grid corner (mm)
  double sid, sdd, dgamma, kc;  // kc = (n_cols-1)/2 + col_offset
  double dzeta, rc;             // row pitch at the detector (mm), (n_rows-1)/2
  const double* view;           // [n_views][4]: cos b, sin b, z_s (mm), w_s (grid units)
  const double* row;            // [n_rows][4]: zeta_r/dz (grid units), 3D ray length L_r (mm), dz/zeta_r (0 if zeta_r = 0), 0
  const void* rays;             // RayXY<T> [n_views][n_cols] in the plan precision
  const RayXY<double>* rays64;  // FP64 copy (metal trace, FP64 plans)
  const void* bowtie;           // [2][n_cols] filter path in the basis (plan precision) or NULL
  const uint32_t* mbits;        // bit-packed trace read instead of the byte mask, or NULL
  int64_t R, V;
};

// Energy table, one record per kept bin (both spectra zero -> dropped).
template <typename T>
struct EBin {
  T mu1, mu2;      // basis attenuation (1/mm)
  T i0l, i0h;      // photons per ray, low / high spectrum
  T m1l, m2l;      // mu1*i0l, mu2*i0l
  T m1h, m2h;      // mu1*i0h, mu2*i0h
};

// Back-projection tile: tx*ty columns x tz slices owned by one workgroup.
struct Tiling {
  int tx, ty, tz;
  int ntx, nty, ntz;
};

// Tile shape of the backprojector for NCH channels: 32 x 32 pixels in 2D,
// or 16 x 16 (SM) for images with fewer 32 x 32 tiles than compute units; in
// 3D flat 32 x 32 x tz slabs (rays are close to the slice planes, so a wide,
// thin slab gives long in-tile paths).  PK: two channels share one 64-bit LDS
// word (non-negative weights, see the kernel).  At most 80 KiB of LDS, so
// two tiles share a CU.
// Threads per tile: 1024 in 2D (a whole CU, 16 waves), 256 for SM tiles (four
// per CU); 512 in 3D (two tiles per CU).
#ifndef DEAM_BP3_PK_TZ
#define DEAM_BP3_PK_TZ 1
#endif
#ifndef DEAM_BP3_PK_BLOCK
#define DEAM_BP3_PK_BLOCK 512
#endif
template <bool Z3, bool SM, bool PK = false>
constexpr int bp_block() { return Z3 ? (PK ? DEAM_BP3_PK_BLOCK : 512) : (SM ? 256 : 1024); }

template <bool Z3, int NCH, bool PK, bool SM>
struct BpTile {
  static_assert(!(Z3 && SM), "small tiles are 2D only");
  static constexpr int block = bp_block<Z3, SM, PK>();
  static constexpr int wpv = PK ? NCH / 2 : NCH;   // 64-bit LDS words per voxel
  static constexpr int tx = SM ? 16 : 32;
  static constexpr int ty = SM ? 16 : 32;
  static constexpr int tz = Z3 ? (PK ? DEAM_BP3_PK_TZ : 8 / NCH) : 1;
  static constexpr size_t lds_bytes = (size_t)(tx + 1) * ty * tz * wpv * 8;
  static_assert(lds_bytes <= 81920, "backprojection tile exceeds 80 KiB");
};

enum PolyMode { PM_L = 0, PM_AM = 1, PM_GRAD = 2, PM_VJP = 3, PM_TRACE = 4, PM_STEP = 5 };

constexpr int kFpBlock = 256;

// 3D projector: detector rows walked together by one lane (see k_fp3), and
// its grid: (view, row group, channel padded to whole waves)
template <typename T>
constexpr int fp3_rows() { return sizeof(T) == 4 ? 4 : 2; }
constexpr int kFp3Views = 4;   // consecutive views per block (one wave each)
inline int64_t fp3_blocks(int n_views, int n_rows, int n_cols, int rg) {
  const int64_t nkb = (n_cols + 63) / 64;                       // channel blocks of 64
  const int64_t nvb = (n_views + kFp3Views - 1) / kFp3Views;    // view blocks
  const int64_t ng = (n_rows + rg - 1) / rg;
  return nvb * nkb * ng;
}
// Views per backprojector batch: each batch ends in a barrier that waits for
// the tile's slowest wave (in 2D a tile holds a whole CU), so a batch should
// give every thread several items; the packed accumulation's resolution
// shrinks in proportion to it
constexpr int kViewBatch = 128;
constexpr int kMaxFbpCols = 4096;   // FBP filter: one detector row of p and g in LDS (64 KiB)

// Device scratch of deam_poly_mean_noalloc (a file-scope array of the kernel
// library, one copy per GPU): the FP64 per-block partial sums of the
// objective, from byte kNoAllocPartialOffset.
constexpr size_t kNoAllocScratchBytes = (size_t)2 << 20;
constexpr size_t kNoAllocPartialOffset = 256;

// Elements of the zeroed tail that follows the two packed image copies.  The
// lanes of a forward-projector wave walk a common range of plane rows q <
// max(nx, ny), so a lane whose row lies outside the slices (3D) reads the
// tail at in-plane element q * nb + A <= max(nx, ny) * nb - 1 (nb, the
// lateral extent, is nx or ny), and float plans fetch the pixel after that
// one too (one 16-byte load per pixel pair): at most max(nx, ny)^2 + 1
// elements, rounded up to keep 16-byte multiples.
inline size_t packed_tail_elems(int nx, int ny) {
  const size_t mx = (size_t)(nx > ny ? nx : ny);
  return mx * mx + 2;
}

// Coarse map of the weight maxima: max |w_c| over the rays of one view,
// one group of kMapRows detector rows and one block of kMapCols channels,
// per channel c < 4, as float bits (non-negative, so atomicMax on the bits
// is the float maximum).  Written by the kernels that produce weights, read
// by the backprojector's tile pre-pass, which takes each tile's maximum over
// the entries of the rays that can meet it: the fixed-point scale of a tile
// then follows the weights of its own rays, not the largest weight of the
// scan.
constexpr int kMapRows = 4;
constexpr int kMapCols = 64;
struct WMapDev {
  uint32_t* map;        // [n_views][ngm][nkb][4], or NULL (no map)
  int n_rows, n_cols;
  int ngm, nkb;         // row groups, channel blocks
};
inline WMapDev wmap_dev(const GeomDev& G, void* map) {
  return WMapDev{(uint32_t*)map, G.n_rows, G.n_cols, (G.n_rows + kMapRows - 1) / kMapRows,
                 (G.n_cols + kMapCols - 1) / kMapCols};
}
inline int64_t wmap_words(const GeomDev& G) {
  const WMapDev M = wmap_dev(G, nullptr);
  return (int64_t)G.n_views * M.ngm * M.nkb * 4;
}
// An upper bound of the backprojector's tile count over its tile shapes
// (per-tile maxima, 4 floats each).
inline int64_t max_tiles(const GeomDev& G) {
  return (int64_t)((G.nx + 15) / 16) * ((G.ny + 15) / 16) * (G.is3d ? G.nz : 1);
}

// Workspace pieces (byte offsets, 256-aligned).
struct WsLayout {
  size_t cp_y, cp_x;     // packed projection images (natural and transposed)
  size_t w;              // per-ray weights
  size_t b;              // back-projections
  size_t partial;        // per-block FP64 partial sums
  size_t wmap, tmax;     // weight-maxima map and per-tile maxima (backprojection)
  size_t scratch;        // small FP64 scratch
  size_t l, u, ab, lam, bl;   // iteration VJP: line integrals, upstream images, their
                              // projections, lambda, its backprojection
  size_t c_prev;              // penalised iteration: the iterate entering the update
  size_t p, q, mu0, prior, pp, pc, mu1;   // MAR initialisation: line integrals, filtered
                                          // copy, FBP images, prior, its projection,
                                          // corrected line integrals, corrected FBP
  size_t total;
};

}  // namespace deam

struct deam_plan {
  deam_geometry g;
  int precision;
  int device;
  deam::GeomDev gd;
  int nE;                        // kept energy bins (padded to a multiple of 8)
  void* d_tables;                // view/row tables (FP64)
  void* d_rays;                  // RayXY<float> (MIXED only)
  void* d_rays64;                // RayXY<double>
  void* d_energy;                // EBin<float> or EBin<double> [nE]
  double h1_bound;               // upper bound of max_x sum_y h(x,y)
  double hmax;                   // upper bound of one h(x,y): the voxel diagonal
  int64_t fp_blocks;             // blocks of the fused projector kernel (its FP64 partials)
  int64_t ray_blocks;            // blocks of one-thread-per-ray kernels
  int n_cu;                      // compute units of the plan's device
  void* d_bowtie;                // bowtie offsets [2][n_cols] (plan precision) or NULL
  // MAR initialisation (2D fan-beam full scans): ramp kernel g(0..n-1) and
  // pre-weights sid cos(gamma_k) in d_tables (NULL when not supported),
  // photons per ray of each spectrum, and the inverse of the spectrum-weighted
  // attenuation matrix Mt[j][i] = sum_E I0_j mu_i / sum_E I0_j
  const double* d_fbp;
  double i0sum[2];
  double mu_eff[2][2];
  double mu_eff_inv[2][2];
  void* noalloc;                 // device address of the no-allocation scratch (NULL if unavailable)
  // MIXED plans: per backprojector tile, a bound of max_x sum_y h(x,y) over
  // the rays of one view batch, measured by the packed backprojector itself
  // at plan creation ([max_tiles] float, device), or NULL
  void* d_hbt;
  double bp_rays_per_voxel;      // rays of one view that can pass through one voxel (a bound)
};

namespace deam {

// Launchers (deam_kernels.hip).  All asynchronous on `st`.
hipError_t launch_pack(const deam_plan* p, const void* c, int n_ch, bool from_u8, bool dbl,
                       void* cp_y, void* cp_x, hipStream_t st);
hipError_t launch_zero_tail(const deam_plan* p, void* cp_x, bool dbl, hipStream_t st);
hipError_t launch_forward(const deam_plan* p, const void* cp_y, const void* cp_x, void* l,
                          int n_out, hipStream_t st);
hipError_t launch_metal_trace(const deam_plan* p, const void* cp_y, const void* cp_x, double t,
                              uint8_t* mask, double* T, hipStream_t st);
// wmap (or NULL): the weight-maxima map, which must hold zeros before
hipError_t launch_fp_poly(const deam_plan* p, const void* cp_y, const void* cp_x, const float* d,
                          const uint8_t* mask, int mode, void* w, double* partial,
                          hipStream_t st, uint32_t* wmap = nullptr);
hipError_t launch_poly(const deam_plan* p, const void* l, const float* d, const uint8_t* mask,
                       int mode, const void* v, void* w, void* g, double* partial,
                       hipStream_t st, uint32_t* wmap = nullptr);
hipError_t launch_reduce(const double* partial, int64_t n, double* out, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st);
// the weight-maxima map of w (zeroed here first)
hipError_t launch_absmax(const deam_plan* p, const void* w, int n_ch, uint32_t* wmap, hipStream_t st);
// nonneg: every weight is >= 0 (the AM weights), which allows a cheaper rounding.
// wmap: the weights' map (from the kernel that wrote them or launch_absmax);
// The bound pass of the packed backprojector: every weight 1, the plan's own
// view set; writes per tile a bound of the largest sum of h(x,y) over one
// view batch into hbt_out [max_tiles] (MIXED plans).
hipError_t launch_bp_bound(const deam_plan* p, float* hbt_out, hipStream_t st);
// tmax: per-tile maxima, max_tiles(G) x 4 floats of scratch
hipError_t launch_backproject(const deam_plan* p, const void* w, int n_ch, bool nonneg,
                              const uint32_t* wmap, float* tmax, void* b, hipStream_t st);
// iteration VJP: u = (-G_i/(Z_i b~_i), ..., G_i/(Z_i b^_i)) planar [4][V]
hipError_t launch_step_u(const deam_plan* p, const double* G, const void* b, double z1, double z2,
                         void* u, hipStream_t st);
// out = G + bl (double [2][V])
hipError_t launch_add_g(const deam_plan* p, const double* G, const void* bl, double* out,
                        hipStream_t st);
// b2 (or NULL) is added to b: the backprojections of a second scan
hipError_t launch_update(const deam_plan* p, double* c64, const void* b, double z1, double z2,
                         void* c_proj, void* cp_y, void* cp_x, hipStream_t st,
                         const void* b2 = nullptr);
// penalised update (Eqs. 6-7): c64 <- argmin of the decoupled per-voxel
// surrogate around c_prev (distinct from c64), same outputs as launch_update
hipError_t launch_update_pen(const deam_plan* p, const double* c_prev, double* c64, const void* b,
                             double z1, double z2, double lambda, double delta, void* c_proj,
                             void* cp_y, void* cp_x, hipStream_t st);
// R(c) of Eq. 6: one FP64 partial per block into partial[0, pen_blocks(p))
hipError_t launch_penalty(const deam_plan* p, const double* c, double lambda, double delta,
                          double* partial, hipStream_t st);
int64_t pen_blocks(const deam_plan* p);
// MAR initialisation: line integrals [2][R]; FBP of n_ch sinograms through
// the filtered copy q [n_ch][R]; NMAR; metal and prior images; Eq. 4
hipError_t launch_line_integrals(const deam_plan* p, const float* d, void* out, hipStream_t st);
hipError_t launch_fbp(const deam_plan* p, const void* sino, int n_ch, void* q, void* img,
                      hipStream_t st);
hipError_t launch_nmar(const deam_plan* p, const void* sino, const uint8_t* mask, const void* pp,
                       double eps, void* out, hipStream_t st);
hipError_t launch_mar_classes(const deam_plan* p, const void* mu0, const double water[2],
                              double fa, double fb, double fm, uint8_t* M, void* prior,
                              hipStream_t st);
hipError_t launch_dilate(const deam_plan* p, const uint8_t* mask, int radius, uint8_t* out,
                         hipStream_t st);
hipError_t launch_pack_mask(const deam_plan* p, const uint8_t* mask, uint32_t* bits,
                            hipStream_t st);
hipError_t launch_decompose(const deam_plan* p, const void* mu, double* c64, hipStream_t st);
// input check: cnt[0] += non-finite entries of c64 [2][V], cnt[1] += entries
// of d [2][R] that are negative or non-finite (either pointer may be NULL)
hipError_t launch_validate(const deam_plan* p, const double* c64, const float* d,
                           unsigned long long* cnt, hipStream_t st);

WsLayout workspace_layout(const deam_plan* p, int op);

// Device address of the no-allocation scratch on the current device, looked
// up once per device (hipGetSymbolAddress) and cached; the host-side name of
// the array is not a device address.
hipError_t noalloc_scratch(void** ptr);

}  // namespace deam

// C ABI of the gfx950 DEAM library: argument checks, plan tables, workspace
// layout and the order of kernel launches.  No C++ exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "deam_internal.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int ok() {
  g_err.clear();
  return DEAM_OK;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(DEAM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t real_size(const deam_plan* p) { return p->precision == DEAM_PREC_FP64 ? 8 : 4; }

int check_plan(const deam_plan* p) {
  if (!p) return fail(DEAM_ERR_NULL, "plan is NULL");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(DEAM_ERR_HIP, "hipGetDevice failed");
  if (dev != p->device)
    return fail(DEAM_ERR_VALUE, "current device %d differs from the plan's device %d", dev,
                p->device);
  return DEAM_OK;
}

// Upper bound of max_x sum_y h(x,y): per view at most nk channels and nr rows
// pass through one voxel, each with a chord no longer than the voxel diagonal.
// rays (optional): nk * nr, the bound of the rays of one view through a voxel.
double h1_bound(const deam_geometry& g, double* rays = nullptr) {
  const bool is3d = g.kind == DEAM_HELICAL3D;
  const double rc = 0.5 * std::hypot(g.nx * g.dx, g.ny * g.dy);
  const double dmin = g.sid - rc;
  const double rho = 0.5 * std::hypot(g.dx, g.dy);
  const double w = 2.0 * std::asin(std::min(1.0, rho / dmin));
  const double nk = std::floor(w / g.dgamma) + 2.0;
  double nr = 1.0, diag = std::hypot(g.dx, g.dy);
  if (is3d) {
    const double dzeta = g.drow_iso * g.sdd / g.sid;
    const double zmax = 0.5 * (g.n_rows - 1) * dzeta;
    const double width = (g.dz * g.sdd + 2.0 * rho * zmax) / dmin;
    nr = std::min<double>(std::floor(width / dzeta) + 2.0, g.n_rows);
    diag = std::sqrt(g.dx * g.dx + g.dy * g.dy + g.dz * g.dz);
  }
  if (rays) *rays = std::min<double>(nk, g.n_cols) * nr;
  return (double)g.n_views * std::min<double>(nk, g.n_cols) * nr * diag;
}

int validate_geometry(const deam_geometry* g) {
  if (!g) return fail(DEAM_ERR_NULL, "geometry is NULL");
  if (g->kind != DEAM_FAN2D && g->kind != DEAM_HELICAL3D)
    return fail(DEAM_ERR_GEOMETRY, "unknown geometry kind %d", g->kind);
  const bool is3d = g->kind == DEAM_HELICAL3D;
  if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0 || g->n_views <= 0 || g->n_rows <= 0 ||
      g->n_cols <= 0)
    return fail(DEAM_ERR_SHAPE, "grid and detector sizes must be positive");
  if (!is3d && (g->nz != 1 || g->n_rows != 1))
    return fail(DEAM_ERR_SHAPE, "a fan-beam geometry needs nz = 1 and n_rows = 1");
  const double V = (double)g->nx * g->ny * g->nz;
  const double R = (double)g->n_views * g->n_rows * g->n_cols;
  if (V >= 2147483647.0 || R >= 2147483647.0)
    return fail(DEAM_ERR_SHAPE, "more than 2^31 voxels or rays");
  if (!(g->dx > 0 && g->dy > 0 && g->dz > 0 && std::isfinite(g->dx * g->dy * g->dz)))
    return fail(DEAM_ERR_GEOMETRY, "voxel sizes must be positive and finite");
  if (!(g->dgamma > 0 && std::isfinite(g->dgamma)))
    return fail(DEAM_ERR_GEOMETRY, "dgamma must be positive");
  if (!(g->views_per_rot > 0 && std::isfinite(g->views_per_rot)))
    return fail(DEAM_ERR_GEOMETRY, "views_per_rot must be positive");
  if (!(std::isfinite(g->beta0) && std::isfinite(g->col_offset) && std::isfinite(g->feed_per_rot)))
    return fail(DEAM_ERR_GEOMETRY, "non-finite geometry parameter");
  if (is3d && !(g->drow_iso > 0 && std::isfinite(g->drow_iso)))
    return fail(DEAM_ERR_GEOMETRY, "drow_iso must be positive");
  const double rc = 0.5 * std::hypot(g->nx * g->dx, g->ny * g->dy);
  if (!(g->sid > rc))
    return fail(DEAM_ERR_GEOMETRY, "the source circle (sid=%g) must lie outside the grid (radius %g)",
                g->sid, rc);
  if (!(g->sdd > g->sid + rc))
    return fail(DEAM_ERR_GEOMETRY, "the detector must lie beyond the grid (sdd > sid + grid radius)");
  const double half_fan = 0.5 * g->n_cols * g->dgamma + std::fabs(g->col_offset) * g->dgamma;
  if (!(half_fan < 1.5))
    return fail(DEAM_ERR_GEOMETRY, "the fan must be narrower than about 170 degrees");
  return DEAM_OK;
}

template <typename T>
void fill_energy(std::vector<unsigned char>& out, int& nE, int n_energy, const double* I0,
                 const double* mu) {
  std::vector<deam::EBin<T>> bins;
  for (int e = 0; e < n_energy; ++e) {
    const double il = I0[e], ih = I0[n_energy + e];
    if (il == 0.0 && ih == 0.0) continue;
    const double m1 = mu[e], m2 = mu[n_energy + e];
    deam::EBin<T> b;
    b.mu1 = (T)m1;
    b.mu2 = (T)m2;
    b.i0l = (T)il;
    b.i0h = (T)ih;
    b.m1l = (T)(m1 * il);
    b.m2l = (T)(m2 * il);
    b.m1h = (T)(m1 * ih);
    b.m2h = (T)(m2 * ih);
    bins.push_back(b);
  }
  while (bins.size() % 8 != 0 || bins.empty()) bins.push_back(deam::EBin<T>{});  // zero records
  nE = (int)bins.size();
  out.resize(bins.size() * sizeof(deam::EBin<T>));
  std::memcpy(out.data(), bins.data(), out.size());
}

// The size fields of a plan (grid, detector, ray and block counts): all that
// the workspace layout depends on, computed from the geometry alone.
void fill_plan_sizes(deam_plan* p, const deam_geometry& g, int precision) {
  const bool is3d = g.kind == DEAM_HELICAL3D;
  p->g = g;
  p->precision = precision;
  deam::GeomDev& G = p->gd;
  G.is3d = is3d ? 1 : 0;
  G.nx = g.nx;
  G.ny = g.ny;
  G.nz = is3d ? g.nz : 1;
  G.n_views = g.n_views;
  G.n_rows = g.n_rows;
  G.n_cols = g.n_cols;
  G.voff = 0;
  G.vsub = 1;
  G.nvl = g.n_views;
  G.R = (int64_t)g.n_views * g.n_rows * g.n_cols;
  G.V = (int64_t)g.nx * g.ny * G.nz;
  p->ray_blocks = (G.R + deam::kFpBlock - 1) / deam::kFpBlock;
  if (is3d) {
    const int rg = precision == DEAM_PREC_FP64 ? deam::fp3_rows<double>() : deam::fp3_rows<float>();
    p->fp_blocks = deam::fp3_blocks(g.n_views, g.n_rows, g.n_cols, rg);
  } else {
    p->fp_blocks = p->ray_blocks;
  }
}

}  // namespace

namespace deam {

WsLayout workspace_layout(const deam_plan* p, int op) {
  WsLayout L{};
  const size_t rs = p->precision == DEAM_PREC_FP64 ? 8 : 4;
  const size_t V = (size_t)p->gd.V, R = (size_t)p->gd.R;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t nblk = (size_t)p->fp_blocks;
  // The packed image copies: natural order, then (with no gap) x-major order,
  // then packed_tail_elems zeroed elements.  The forward projector's lanes
  // walk a common range of plane rows; a lane outside its own range reads,
  // with zero weight, rows up to max(nx, ny) of its copy, and a row outside
  // the slices reads the tail; every such read stays inside this region and
  // finds finite values.
  const size_t tail = packed_tail_elems(p->gd.nx, p->gd.ny);
  auto take_packed = [&](size_t es) {
    L.cp_y = take((2 * V + tail) * es);
    L.cp_x = L.cp_y + V * es;
  };
  // the weight-maxima map and the per-tile maxima of the backprojector
  auto take_bp_maps = [&]() {
    L.wmap = take((size_t)wmap_words(p->gd) * 4);
    L.tmax = take((size_t)max_tiles(p->gd) * 4 * sizeof(float));
  };
  switch (op) {
    case DEAM_OP_FORWARD:
      take_packed(2 * rs);
      break;
    case DEAM_OP_METAL_TRACE:
      take_packed(2 * 8);
      break;
    case DEAM_OP_POLY_MEAN:
      L.partial = take((size_t)p->ray_blocks * 8);
      L.scratch = take(64);
      break;
    case DEAM_OP_BACKPROJECT:
      take_bp_maps();
      break;
    case DEAM_OP_ITERATE_VJP:
      take_packed(2 * rs);
      L.l = take(R * 2 * rs);
      L.w = take(R * 4 * rs);
      L.b = take(V * 4 * rs);
      L.u = take(V * 4 * rs);
      L.ab = take(R * 4 * rs);
      L.lam = take(R * 2 * rs);
      L.bl = take(V * 2 * rs);
      L.partial = take((size_t)p->ray_blocks * 8);
      take_bp_maps();
      break;
    case DEAM_OP_PENALTY:
      L.partial = take((size_t)pen_blocks(p) * 8);
      break;
    case DEAM_OP_ITERATE_PENALIZED:
      take_packed(2 * rs);
      L.w = take(R * 4 * rs);
      L.b = take(V * 4 * rs);
      L.c_prev = take(V * 2 * 8);
      // projector partials, then (contiguous) penalty partials: one reduction
      L.partial = take((nblk + (size_t)pen_blocks(p)) * 8);
      L.scratch = take(64);
      take_bp_maps();
      break;
    case DEAM_OP_FBP:
      L.q = take(R * 2 * rs);
      break;
    case DEAM_OP_MAR_INIT:
      take_packed(2 * 8);  // FP64 copies of M for the trace; then the prior's copies
      L.p = take(R * 2 * rs);
      L.q = take(R * 2 * rs);
      L.mu0 = take(V * 2 * rs);
      L.prior = take(V * 2 * rs);
      L.pp = take(R * 2 * rs);
      L.pc = take(R * 2 * rs);
      L.mu1 = take(V * 2 * rs);
      break;
    case DEAM_OP_ITERATE:
    default:
      take_packed(2 * rs);
      L.w = take(R * 4 * rs);
      L.b = take(V * 4 * rs);
      L.partial = take(nblk * 8);
      L.scratch = take(64);
      take_bp_maps();
      break;
  }
  L.total = off;
  return L;
}

}  // namespace deam

extern "C" {

const char* deam_last_error(void) { return g_err.c_str(); }

int deam_plan_create(const deam_geometry* geom, int32_t n_energy, const double* I0,
                     const double* mu, int32_t precision, deam_plan** out) {
  if (!out) return fail(DEAM_ERR_NULL, "out is NULL");
  *out = nullptr;
  if (int rc = validate_geometry(geom)) return rc;
  if (!I0 || !mu) return fail(DEAM_ERR_NULL, "I0 or mu is NULL");
  if (n_energy <= 0 || n_energy > 100000) return fail(DEAM_ERR_SHAPE, "n_energy out of range");
  if (precision != DEAM_PREC_MIXED && precision != DEAM_PREC_FP64)
    return fail(DEAM_ERR_VALUE, "unknown precision %d", precision);
  {
    // the projector addresses both packed image copies (and the padding after
    // the second) with 32-bit byte offsets; the metal trace packs in FP64 on
    // every plan
    const double V = (double)geom->nx * geom->ny * (geom->kind == DEAM_HELICAL3D ? geom->nz : 1);
    const double tail = (double)deam::packed_tail_elems(geom->nx, geom->ny);
    const double bytes = (2.0 * V + tail) * 2.0 * 8.0 + 512.0;
    if (bytes >= 4294967296.0)
      return fail(DEAM_ERR_UNSUPPORTED, "volume too large for this library (packed images >= 4 GiB)");
  }
  for (int i = 0; i < 2 * n_energy; ++i) {
    if (!(std::isfinite(I0[i]) && I0[i] >= 0.0))
      return fail(DEAM_ERR_VALUE, "I0 must be finite and non-negative");
    if (!(std::isfinite(mu[i]) && mu[i] >= 0.0))
      return fail(DEAM_ERR_VALUE, "mu must be finite and non-negative");
  }
  const deam_geometry& g = *geom;
  const bool is3d = g.kind == DEAM_HELICAL3D;

  deam_plan* p = new (std::nothrow) deam_plan();
  if (!p) return fail(DEAM_ERR_VALUE, "out of host memory");
  fill_plan_sizes(p, g, precision);
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return fail(DEAM_ERR_HIP, "hipGetDevice failed");
  }
  if (hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device) !=
          hipSuccess ||
      p->n_cu < 1) {
    delete p;
    return fail(DEAM_ERR_HIP, "hipDeviceGetAttribute(multiprocessor count) failed");
  }

  // geometry tables (FP64): per view [cos b, sin b, z_s, w_s], per row [zeta_r/dz, L_r, dz/zeta_r, 0]
  const double x0 = -0.5 * g.nx * g.dx, y0 = -0.5 * g.ny * g.dy;
  const int nzv = is3d ? g.nz : 1;
  const double z0 = -0.5 * nzv * g.dz;
  // 2D fan-beam full scans also get the FBP tables of the MAR initialisation
  const bool fbp_ok = !is3d && g.n_rows == 1 && g.n_cols <= deam::kMaxFbpCols &&
                      std::fabs(g.n_views * 2.0 * M_PI / g.views_per_rot - 2.0 * M_PI) <= 1e-9;
  std::vector<double> tab((size_t)g.n_views * 4 + (size_t)g.n_rows * 4 +
                          (fbp_ok ? (size_t)2 * g.n_cols : 0));
  double* tv = tab.data();
  double* tr = tv + (size_t)g.n_views * 4;
  for (int v = 0; v < g.n_views; ++v) {
    const double beta = g.beta0 + 2.0 * M_PI * (double)v / g.views_per_rot;
    const double zs = is3d ? ((double)v - 0.5 * (g.n_views - 1)) * g.feed_per_rot / g.views_per_rot : 0.0;
    tv[4 * v] = std::cos(beta);
    tv[4 * v + 1] = std::sin(beta);
    tv[4 * v + 2] = zs;
    tv[4 * v + 3] = (zs - z0) / g.dz;
  }
  const double dzeta = is3d ? g.drow_iso * g.sdd / g.sid : 1.0;
  for (int r = 0; r < g.n_rows; ++r) {
    const double zeta = is3d ? ((double)r - 0.5 * (g.n_rows - 1)) * dzeta : 0.0;
    tr[4 * r] = zeta / g.dz;
    tr[4 * r + 1] = std::sqrt(g.sdd * g.sdd + zeta * zeta);
    tr[4 * r + 2] = zeta != 0.0 ? g.dz / zeta : 0.0;
    tr[4 * r + 3] = 0.0;
  }
  if (fbp_ok) {
    // equiangular ramp kernel g(j), j = 0..n-1, and pre-weights sid cos(gamma_k)
    double* tg = tr + (size_t)g.n_rows * 4;
    for (int j = 0; j < g.n_cols; ++j) {
      const double sj = std::sin(j * g.dgamma);
      tg[j] = j == 0 ? 1.0 / (8.0 * g.dgamma * g.dgamma)
                     : (j % 2 ? -1.0 / (2.0 * M_PI * M_PI * sj * sj) : 0.0);
    }
    for (int k = 0; k < g.n_cols; ++k)
      tg[g.n_cols + k] = g.sid * std::cos(((double)k - 0.5 * (g.n_cols - 1) - g.col_offset) * g.dgamma);
  }
  // in-plane ray of every (view, channel), walked along its driving axis
  const size_t nvk = (size_t)g.n_views * g.n_cols;
  std::vector<deam::RayXY<double>> rays64(nvk);
  std::vector<deam::RayXY<float>> rays32(precision == DEAM_PREC_MIXED ? nvk : 0);
  for (int v = 0; v < g.n_views; ++v) {
    const double cb = tv[4 * v], sb = tv[4 * v + 1];
    for (int k = 0; k < g.n_cols; ++k) {
      const double gam = ((double)k - 0.5 * (g.n_cols - 1) - g.col_offset) * g.dgamma;
      const double cg = std::cos(gam), sg = std::sin(gam);
      const double ex = -(cg * cb - sg * sb), ey = -(sg * cb + cg * sb);  // R(gamma) u
      const double su = (g.sid * cb - x0) / g.dx, sv = (g.sid * sb - y0) / g.dy;
      const double du = g.sdd * ex / g.dx, dv = g.sdd * ey / g.dy;
      const bool yd = std::fabs(dv) >= std::fabs(du);
      const double sa = yd ? sv : su, da = yd ? dv : du;
      const double sbb = yd ? su : sv, db = yd ? du : dv;
      const double mb = db / da;
      deam::RayXY<double> t;
      const double b0 = sbb - sa * mb;            // lateral coordinate at a = 0
      const double na = yd ? g.ny : g.nx;         // extent of the driving axis
      const double ib = std::floor(std::fmin(std::fmax(b0 + 0.5 * na * mb, -1e6), 1e6));
      t.b0 = b0 - ib;
      t.mb = mb;
      t.imb = mb != 0.0 ? 1.0 / mb : 1e30;
      t.sa = sa;
      t.ida = 1.0 / da;
      t.iadb = db != 0.0 ? 1.0 / std::fabs(db) : 1e30;
      t.yd = yd ? 1.0 : 0.0;
      t.ib = ib;
      const size_t i = (size_t)v * g.n_cols + k;
      rays64[i] = t;
      if (!rays32.empty()) {
        deam::RayXY<float>& f = rays32[i];
        f.b0 = (float)t.b0;
        f.mb = (float)t.mb;
        f.imb = (float)t.imb;
        f.sa = (float)t.sa;
        f.ida = (float)t.ida;
        f.iadb = (float)t.iadb;
        f.yd = (float)t.yd;
        f.ib = (float)t.ib;
      }
    }
  }

  std::vector<unsigned char> etab;
  if (precision == DEAM_PREC_FP64) fill_energy<double>(etab, p->nE, n_energy, I0, mu);
  else fill_energy<float>(etab, p->nE, n_energy, I0, mu);

  auto release = [&]() {
    if (p->d_tables) (void)hipFree(p->d_tables);
    if (p->d_energy) (void)hipFree(p->d_energy);
    if (p->d_rays) (void)hipFree(p->d_rays);
    if (p->d_rays64) (void)hipFree(p->d_rays64);
    if (p->d_hbt) (void)hipFree(p->d_hbt);
    delete p;
  };
  if (hipMalloc(&p->d_tables, tab.size() * sizeof(double)) != hipSuccess ||
      hipMalloc(&p->d_energy, etab.size()) != hipSuccess ||
      hipMalloc(&p->d_rays64, nvk * sizeof(deam::RayXY<double>)) != hipSuccess ||
      (!rays32.empty() && hipMalloc(&p->d_rays, nvk * sizeof(deam::RayXY<float>)) != hipSuccess)) {
    release();
    return fail(DEAM_ERR_HIP, "hipMalloc of plan tables failed");
  }
  if (hipMemcpy(p->d_tables, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(p->d_energy, etab.data(), etab.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->d_rays64, rays64.data(), nvk * sizeof(deam::RayXY<double>),
                hipMemcpyHostToDevice) != hipSuccess ||
      (!rays32.empty() && hipMemcpy(p->d_rays, rays32.data(), nvk * sizeof(deam::RayXY<float>),
                                    hipMemcpyHostToDevice) != hipSuccess)) {
    release();
    return fail(DEAM_ERR_HIP, "hipMemcpy of plan tables failed");
  }

  deam::GeomDev& G = p->gd;
  G.dx = g.dx;
  G.dy = g.dy;
  G.dz = g.dz;
  G.x0 = x0;
  G.y0 = y0;
  G.z0 = z0;
  G.sid = g.sid;
  G.sdd = g.sdd;
  G.dgamma = g.dgamma;
  G.kc = 0.5 * (g.n_cols - 1) + g.col_offset;
  G.dzeta = dzeta;
  G.rc = 0.5 * (g.n_rows - 1);
  G.view = (const double*)p->d_tables;
  G.row = G.view + (size_t)g.n_views * 4;
  G.rays = precision == DEAM_PREC_MIXED ? p->d_rays : p->d_rays64;
  G.rays64 = (const deam::RayXY<double>*)p->d_rays64;
  G.bowtie = nullptr;
  G.mbits = nullptr;

  p->d_fbp = fbp_ok ? G.row + (size_t)g.n_rows * 4 : nullptr;
  // photons per ray and spectrum-weighted attenuation (Eq. 4's weights)
  for (int j = 0; j < 2; ++j) {
    double t = 0.0, m1 = 0.0, m2 = 0.0;
    for (int e = 0; e < n_energy; ++e) {
      const double i0 = I0[(size_t)j * n_energy + e];
      t += i0;
      m1 += i0 * mu[e];
      m2 += i0 * mu[(size_t)n_energy + e];
    }
    p->i0sum[j] = t;
    p->mu_eff[j][0] = t > 0.0 ? m1 / t : 0.0;
    p->mu_eff[j][1] = t > 0.0 ? m2 / t : 0.0;
  }
  {
    const double a = p->mu_eff[0][0], b = p->mu_eff[0][1], c = p->mu_eff[1][0], d = p->mu_eff[1][1];
    const double det = a * d - b * c;
    const double id = det != 0.0 ? 1.0 / det : 0.0;
    p->mu_eff_inv[0][0] = d * id;
    p->mu_eff_inv[0][1] = -b * id;
    p->mu_eff_inv[1][0] = -c * id;
    p->mu_eff_inv[1][1] = a * id;
  }
  // the no-allocation scratch of this device (looked up once per device)
  if (deam::noalloc_scratch(&p->noalloc) != hipSuccess) p->noalloc = nullptr;
  p->h1_bound = h1_bound(g, &p->bp_rays_per_voxel);
  p->hmax = is3d ? std::sqrt(g.dx * g.dx + g.dy * g.dy + g.dz * g.dz) : std::hypot(g.dx, g.dy);
  // MIXED plans: the packed backprojector's per-tile batch bound, measured
  // once by the backprojector itself with every weight 1 (synchronous)
  if (precision == DEAM_PREC_MIXED) {
    if (hipMalloc(&p->d_hbt, (size_t)deam::max_tiles(G) * sizeof(float)) != hipSuccess) {
      release();
      return fail(DEAM_ERR_HIP, "hipMalloc of the backprojector bounds failed");
    }
    if (deam::launch_bp_bound(p, (float*)p->d_hbt, nullptr) != hipSuccess ||
        hipStreamSynchronize(nullptr) != hipSuccess) {
      release();
      return fail(DEAM_ERR_HIP, "the backprojector bound pass failed");
    }
  }
  *out = p;
  return ok();
}

int deam_plan_destroy(deam_plan* plan) {
  if (!plan) return fail(DEAM_ERR_NULL, "plan is NULL");
  (void)hipFree(plan->d_tables);
  (void)hipFree(plan->d_energy);
  if (plan->d_rays) (void)hipFree(plan->d_rays);
  (void)hipFree(plan->d_rays64);
  if (plan->d_bowtie) (void)hipFree(plan->d_bowtie);
  if (plan->d_hbt) (void)hipFree(plan->d_hbt);
  delete plan;
  return ok();
}

int deam_plan_set_bowtie(deam_plan* plan, const double* bt) {
  if (int rc = check_plan(plan)) return rc;
  if (!bt) {
    if (plan->d_bowtie) (void)hipFree(plan->d_bowtie);
    plan->d_bowtie = nullptr;
    plan->gd.bowtie = nullptr;
    return ok();
  }
  const int n = plan->gd.n_cols;
  for (int i = 0; i < 2 * n; ++i)
    if (!(std::isfinite(bt[i]) && bt[i] >= 0.0))
      return fail(DEAM_ERR_VALUE, "bowtie path lengths must be finite and non-negative");
  const bool dbl = plan->precision == DEAM_PREC_FP64;
  std::vector<double> b64(bt, bt + 2 * n);
  std::vector<float> b32(dbl ? 0 : 2 * n);
  for (int i = 0; i < (int)b32.size(); ++i) b32[i] = (float)bt[i];
  const size_t bytes = (size_t)2 * n * (dbl ? sizeof(double) : sizeof(float));
  if (!plan->d_bowtie && hipMalloc(&plan->d_bowtie, bytes) != hipSuccess) {
    plan->d_bowtie = nullptr;
    return fail(DEAM_ERR_HIP, "hipMalloc of the bowtie table failed");
  }
  const void* src = dbl ? (const void*)b64.data() : (const void*)b32.data();
  if (hipMemcpy(plan->d_bowtie, src, bytes, hipMemcpyHostToDevice) != hipSuccess)
    return fail(DEAM_ERR_HIP, "hipMemcpy of the bowtie table failed");
  plan->gd.bowtie = plan->d_bowtie;
  return ok();
}

int deam_plan_sizes(const deam_plan* plan, int64_t* n_rays, int64_t* n_voxels) {
  if (!plan || !n_rays || !n_voxels) return fail(DEAM_ERR_NULL, "NULL argument");
  *n_rays = plan->gd.R;
  *n_voxels = plan->gd.V;
  return ok();
}

int deam_workspace_size(const deam_plan* plan, int32_t op, size_t* bytes) {
  if (!plan || !bytes) return fail(DEAM_ERR_NULL, "NULL argument");
  if (op < DEAM_OP_FORWARD || op > DEAM_OP_MAR_INIT)
    return fail(DEAM_ERR_VALUE, "unknown op %d", op);
  *bytes = deam::workspace_layout(plan, op).total;
  return ok();
}

int deam_workspace_size_for(const deam_geometry* geom, int32_t precision, int32_t op,
                            size_t* bytes) {
  if (!bytes) return fail(DEAM_ERR_NULL, "bytes is NULL");
  if (int rc = validate_geometry(geom)) return rc;
  if (precision != DEAM_PREC_MIXED && precision != DEAM_PREC_FP64)
    return fail(DEAM_ERR_VALUE, "unknown precision %d", precision);
  if (op < DEAM_OP_FORWARD || op > DEAM_OP_MAR_INIT)
    return fail(DEAM_ERR_VALUE, "unknown op %d", op);
  deam_plan q{};
  fill_plan_sizes(&q, *geom, precision);
  *bytes = deam::workspace_layout(&q, op).total;
  return ok();
}

static int check_ws(const deam_plan* p, int op, const void* ws, size_t ws_bytes,
                    deam::WsLayout& L) {
  L = deam::workspace_layout(p, op);
  if (L.total > 0 && !ws) return fail(DEAM_ERR_NULL, "workspace is NULL");
  if (ws_bytes < L.total)
    return fail(DEAM_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
  if (((uintptr_t)ws & 255) != 0) return fail(DEAM_ERR_VALUE, "workspace must be 256-byte aligned");
  return DEAM_OK;
}

int deam_metal_trace(const deam_plan* plan, const uint8_t* M, double t, uint8_t* mask, double* T,
                     void* ws, size_t ws_bytes, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!M || !mask) return fail(DEAM_ERR_NULL, "M or mask is NULL");
  if (!std::isfinite(t)) return fail(DEAM_ERR_VALUE, "threshold must be finite");
  deam::WsLayout L;
  if (int rc = check_ws(plan, DEAM_OP_METAL_TRACE, ws, ws_bytes, L)) return rc;
  char* w = (char*)ws;
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(deam::launch_pack(plan, M, 1, true, true, w + L.cp_y, w + L.cp_x, st));
  HIP_TRY(deam::launch_metal_trace(plan, w + L.cp_y, w + L.cp_x, t, mask, T, st));
  return ok();
}

int deam_forward(const deam_plan* plan, const void* c, int32_t n_ch, void* l, void* ws,
                 size_t ws_bytes, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!c || !l) return fail(DEAM_ERR_NULL, "c or l is NULL");
  if (n_ch != 1 && n_ch != 2) return fail(DEAM_ERR_SHAPE, "n_ch must be 1 or 2 (got %d)", n_ch);
  deam::WsLayout L;
  if (int rc = check_ws(plan, DEAM_OP_FORWARD, ws, ws_bytes, L)) return rc;
  char* w = (char*)ws;
  hipStream_t st = (hipStream_t)stream;
  const bool dbl = plan->precision == DEAM_PREC_FP64;
  HIP_TRY(deam::launch_pack(plan, c, n_ch, false, dbl, w + L.cp_y, w + L.cp_x, st));
  HIP_TRY(deam::launch_forward(plan, w + L.cp_y, w + L.cp_x, l, n_ch, st));
  return ok();
}

int deam_poly_mean(const deam_plan* plan, const void* l, const float* d, const uint8_t* mask,
                   int32_t mode, const void* v, void* w, void* g, double* obj, void* ws,
                   size_t ws_bytes, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!l || !w) return fail(DEAM_ERR_NULL, "l or w is NULL");
  if (mode != DEAM_W_AM && mode != DEAM_W_GRAD && mode != DEAM_W_VJP && mode != DEAM_W_STEP_VJP)
    return fail(DEAM_ERR_VALUE, "unknown weight mode %d", mode);
  if ((mode == DEAM_W_VJP || mode == DEAM_W_STEP_VJP) && !v)
    return fail(DEAM_ERR_NULL, "v is NULL in VJP mode");
  if (mode != DEAM_W_VJP && !d) return fail(DEAM_ERR_NULL, "d is NULL");
  deam::WsLayout L;
  if (int rc = check_ws(plan, DEAM_OP_POLY_MEAN, ws, ws_bytes, L)) return rc;
  char* wsb = (char*)ws;
  hipStream_t st = (hipStream_t)stream;
  const int pm = mode == DEAM_W_AM     ? deam::PM_AM
                 : mode == DEAM_W_GRAD ? deam::PM_GRAD
                 : mode == DEAM_W_VJP  ? deam::PM_VJP
                                       : deam::PM_STEP;
  double* partial = (double*)(wsb + L.partial);
  HIP_TRY(deam::launch_poly(plan, l, d, mask, pm, v, w, g, partial, st));
  if (obj) HIP_TRY(deam::launch_reduce(partial, plan->ray_blocks, obj, st));
  return ok();
}

int deam_poly_mean_noalloc(const deam_plan* plan, const void* l, const float* d,
                           const uint8_t* mask, int32_t mode, const void* v, void* w, void* g,
                           double* obj, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!l || !w) return fail(DEAM_ERR_NULL, "l or w is NULL");
  if (mode != DEAM_W_AM && mode != DEAM_W_GRAD && mode != DEAM_W_VJP && mode != DEAM_W_STEP_VJP)
    return fail(DEAM_ERR_VALUE, "unknown weight mode %d", mode);
  if ((mode == DEAM_W_VJP || mode == DEAM_W_STEP_VJP) && !v)
    return fail(DEAM_ERR_NULL, "v is NULL in VJP mode");
  if (mode != DEAM_W_VJP && !d) return fail(DEAM_ERR_NULL, "d is NULL");
  const size_t need = deam::kNoAllocPartialOffset + (size_t)plan->ray_blocks * sizeof(double);
  if (need > deam::kNoAllocScratchBytes)
    return fail(DEAM_ERR_UNSUPPORTED,
                "%lld rays need %zu bytes of scratch, more than the %zu of deam_poly_mean_noalloc "
                "(at most %lld rays); use deam_poly_mean with a workspace",
                (long long)plan->gd.R, need, deam::kNoAllocScratchBytes,
                (long long)((deam::kNoAllocScratchBytes - deam::kNoAllocPartialOffset) /
                            sizeof(double) * deam::kFpBlock));
  if (!plan->noalloc)
    return fail(DEAM_ERR_HIP, "the device scratch of deam_poly_mean_noalloc is not available");
  hipStream_t st = (hipStream_t)stream;
  const int pm = mode == DEAM_W_AM     ? deam::PM_AM
                 : mode == DEAM_W_GRAD ? deam::PM_GRAD
                 : mode == DEAM_W_VJP  ? deam::PM_VJP
                                       : deam::PM_STEP;
  char* s = (char*)plan->noalloc;
  double* partial = (double*)(s + deam::kNoAllocPartialOffset);
  // the kernel writes every partial it reduces (nothing to clear)
  HIP_TRY(deam::launch_poly(plan, l, d, mask, pm, v, w, g, partial, st));
  if (obj) HIP_TRY(deam::launch_reduce(partial, plan->ray_blocks, obj, st));
  return ok();
}

int deam_backproject(const deam_plan* plan, const void* w, int32_t n_ch, int32_t flags, void* b,
                     void* ws, size_t ws_bytes, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!w || !b) return fail(DEAM_ERR_NULL, "w or b is NULL");
  if (n_ch != 1 && n_ch != 2 && n_ch != 4)
    return fail(DEAM_ERR_SHAPE, "n_ch must be 1, 2 or 4 (got %d)", n_ch);
  if (flags & ~DEAM_BP_NONNEG) return fail(DEAM_ERR_VALUE, "unknown flags 0x%x", (unsigned)flags);
  deam::WsLayout L;
  if (int rc = check_ws(plan, DEAM_OP_BACKPROJECT, ws, ws_bytes, L)) return rc;
  hipStream_t st = (hipStream_t)stream;
  uint32_t* wmap = (uint32_t*)((char*)ws + L.wmap);
  float* tmax = (float*)((char*)ws + L.tmax);
  HIP_TRY(deam::launch_absmax(plan, w, n_ch, wmap, st));
  HIP_TRY(deam::launch_backproject(plan, w, n_ch, (flags & DEAM_BP_NONNEG) != 0, wmap, tmax, b,
                                   st));
  return ok();
}

int deam_update(const deam_plan* plan, double* c64, void* c_proj, const void* b, const double* Z,
                void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!c64 || !b || !Z) return fail(DEAM_ERR_NULL, "c64, b or Z is NULL");
  if (!(Z[0] > 0.0 && Z[1] > 0.0 && std::isfinite(Z[0]) && std::isfinite(Z[1])))
    return fail(DEAM_ERR_VALUE, "Z must be positive and finite");
  HIP_TRY(deam::launch_update(plan, c64, b, Z[0], Z[1], c_proj, nullptr, nullptr,
                              (hipStream_t)stream));
  return ok();
}

static int check_penalty(double lambda, double delta) {
  if (!(lambda >= 0.0 && std::isfinite(lambda)))
    return fail(DEAM_ERR_VALUE, "lambda must be >= 0 and finite");
  if (!(delta > 0.0 && std::isfinite(delta)))
    return fail(DEAM_ERR_VALUE, "delta must be > 0 and finite");
  return DEAM_OK;
}

int deam_update_penalized(const deam_plan* plan, const double* c_prev, double* c64, void* c_proj,
                          const void* b, const double* Z, double lambda, double delta,
                          void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!c_prev || !c64 || !b || !Z) return fail(DEAM_ERR_NULL, "c_prev, c64, b or Z is NULL");
  if (!(Z[0] > 0.0 && Z[1] > 0.0 && std::isfinite(Z[0]) && std::isfinite(Z[1])))
    return fail(DEAM_ERR_VALUE, "Z must be positive and finite");
  if (int rc = check_penalty(lambda, delta)) return rc;
  const size_t nb = (size_t)plan->gd.V * 2 * sizeof(double);
  const char *a0 = (const char*)c_prev, *b0 = (const char*)c64;
  if (a0 < b0 + nb && b0 < a0 + nb) return fail(DEAM_ERR_VALUE, "c64 overlaps c_prev");
  HIP_TRY(deam::launch_update_pen(plan, c_prev, c64, b, Z[0], Z[1], lambda, delta, c_proj,
                                  nullptr, nullptr, (hipStream_t)stream));
  return ok();
}

int deam_penalty(const deam_plan* plan, const double* c64, double lambda, double delta,
                 double* out, void* ws, size_t ws_bytes, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!c64 || !out) return fail(DEAM_ERR_NULL, "c64 or out is NULL");
  if (int rc = check_penalty(lambda, delta)) return rc;
  deam::WsLayout L;
  if (int rc = check_ws(plan, DEAM_OP_PENALTY, ws, ws_bytes, L)) return rc;
  hipStream_t st = (hipStream_t)stream;
  double* partial = (double*)((char*)ws + L.partial);
  HIP_TRY(deam::launch_penalty(plan, c64, lambda, delta, partial, st));
  HIP_TRY(deam::launch_reduce(partial, deam::pen_blocks(plan), out, st));
  return ok();
}

struct PenSpec {
  double lambda, delta;
};

static int iterate_impl(const deam_plan* plan, double* c64, void* c_proj, const float* d,
                        const uint8_t* mask, const double* Z, int32_t n_iter, double* obj_hist,
                        void* ws, size_t ws_bytes, void* stream, float* kernel_ms,
                        const PenSpec* pen = nullptr) {
  if (int rc = check_plan(plan)) return rc;
  if (!c64 || !d || !Z) return fail(DEAM_ERR_NULL, "c64, d or Z is NULL");
  if (n_iter < 0) return fail(DEAM_ERR_VALUE, "n_iter must be >= 0");
  if (!(Z[0] > 0.0 && Z[1] > 0.0 && std::isfinite(Z[0]) && std::isfinite(Z[1])))
    return fail(DEAM_ERR_VALUE, "Z must be positive and finite");
  if (pen)
    if (int rc = check_penalty(pen->lambda, pen->delta)) return rc;
  deam::WsLayout L;
  if (int rc = check_ws(plan, pen ? DEAM_OP_ITERATE_PENALIZED : DEAM_OP_ITERATE, ws, ws_bytes, L))
    return rc;
  char* w = (char*)ws;
  hipStream_t st = (hipStream_t)stream;
  void* cpy = w + L.cp_y;
  void* cpx = w + L.cp_x;
  uint32_t* wmap = (uint32_t*)(w + L.wmap);
  float* tmax = (float*)(w + L.tmax);
  const int64_t nmap = deam::wmap_words(plan->gd);
  double* partial = (double*)(w + L.partial);
  // events: per iteration, before/after the ray kernel, before/after the
  // backprojection, after the update
  std::vector<hipEvent_t> ev;
  auto cleanup = [&]() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  };
  if (kernel_ms) {
    ev.resize((size_t)5 * std::max(n_iter, 1), nullptr);
    for (auto& e : ev)
      if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
        cleanup();
        return fail(DEAM_ERR_HIP, "hipEventCreate failed");
      }
  }
  auto mark = [&](int k, int j) -> hipError_t {
    return kernel_ms ? hipEventRecord(ev[(size_t)5 * k + j], st) : hipSuccess;
  };
#define STEP(expr)                                                                         \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) {                                                                \
      cleanup();                                                                           \
      return fail(DEAM_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));                   \
    }                                                                                      \
  } while (0)
  // projection copies of the starting image, and the zeroed tail after them
  // (with no iteration, c_proj is the starting image's copy)
  STEP(deam::launch_update(plan, c64, nullptr, Z[0], Z[1], n_iter == 0 ? c_proj : nullptr, cpy,
                           cpx, st));
  STEP(deam::launch_zero_tail(plan, cpx, plan->precision == DEAM_PREC_FP64, st));
  for (int k = 0; k < n_iter; ++k) {
    STEP(deam::launch_fill_u32(wmap, 0u, nmap, st));
    STEP(mark(k, 0));
    STEP(deam::launch_fp_poly(plan, cpy, cpx, d, mask, deam::PM_AM, w + L.w, partial, st,
                              wmap));
    STEP(mark(k, 1));
    if (obj_hist) {
      int64_t np = plan->fp_blocks;
      if (pen) {
        STEP(deam::launch_penalty(plan, c64, pen->lambda, pen->delta, partial + np, st));
        np += deam::pen_blocks(plan);
      }
      STEP(deam::launch_reduce(partial, np, obj_hist + k, st));
    }
    STEP(mark(k, 2));
    STEP(deam::launch_backproject(plan, w + L.w, 4, true, wmap, tmax, w + L.b, st));
    STEP(mark(k, 3));
    void* cp_out = k == n_iter - 1 ? c_proj : nullptr;   // the final iterate's copy
    if (pen) {
      double* cprev = (double*)(w + L.c_prev);
      STEP(hipMemcpyAsync(cprev, c64, (size_t)plan->gd.V * 2 * sizeof(double),
                          hipMemcpyDeviceToDevice, st));
      STEP(deam::launch_update_pen(plan, cprev, c64, w + L.b, Z[0], Z[1], pen->lambda,
                                   pen->delta, cp_out, cpy, cpx, st));
    } else {
      STEP(deam::launch_update(plan, c64, w + L.b, Z[0], Z[1], cp_out, cpy, cpx, st));
    }
    STEP(mark(k, 4));
  }
  if (kernel_ms) {
    STEP(hipStreamSynchronize(st));
    float acc_ms[3] = {0.f, 0.f, 0.f};
    for (int k = 0; k < n_iter; ++k) {
      float a = 0.f, b = 0.f, c = 0.f;
      STEP(hipEventElapsedTime(&a, ev[(size_t)5 * k], ev[(size_t)5 * k + 1]));
      STEP(hipEventElapsedTime(&b, ev[(size_t)5 * k + 2], ev[(size_t)5 * k + 3]));
      STEP(hipEventElapsedTime(&c, ev[(size_t)5 * k + 3], ev[(size_t)5 * k + 4]));
      acc_ms[0] += a;
      acc_ms[1] += b;
      acc_ms[2] += c;
    }
    kernel_ms[0] = acc_ms[0];
    kernel_ms[1] = acc_ms[1];
    kernel_ms[2] = acc_ms[2];
    kernel_ms[3] = 0.f;
    if (n_iter > 0)
      STEP(hipEventElapsedTime(&kernel_ms[3], ev[0], ev[(size_t)5 * (n_iter - 1) + 4]));
  }
#undef STEP
  cleanup();
  return ok();
}

int deam_iterate(const deam_plan* plan, double* c64, void* c_proj, const float* d,
                 const uint8_t* mask, const double* Z, int32_t n_iter, double* obj_hist,
                 void* ws, size_t ws_bytes, void* stream) {
  return iterate_impl(plan, c64, c_proj, d, mask, Z, n_iter, obj_hist, ws, ws_bytes, stream,
                      nullptr);
}

int deam_iterate_sync(const deam_plan* plan, double* c64, void* c_proj, const float* d,
                      const uint8_t* mask, const double* Z, int32_t n_iter, double* obj_hist,
                      void* ws, size_t ws_bytes, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (n_iter < 0) return fail(DEAM_ERR_VALUE, "n_iter must be >= 0");
  hipStream_t st = (hipStream_t)stream;
  double* dev_hist = nullptr;
  if (obj_hist && n_iter > 0) {
    // the history is reduced on the device and copied out at the end
    if (hipMalloc(&dev_hist, (size_t)n_iter * sizeof(double)) != hipSuccess)
      return fail(DEAM_ERR_HIP, "hipMalloc of the objective history failed");
  }
  int rc = iterate_impl(plan, c64, c_proj, d, mask, Z, n_iter, dev_hist, ws, ws_bytes, stream,
                        nullptr);
  if (rc == DEAM_OK && dev_hist) {
    const hipError_t e = hipMemcpyAsync(obj_hist, dev_hist, (size_t)n_iter * sizeof(double),
                                        hipMemcpyDeviceToHost, st);
    if (e != hipSuccess)
      rc = fail(DEAM_ERR_HIP, "copy of the objective history: %s", hipGetErrorString(e));
  }
  const std::string enqueue_err = rc == DEAM_OK ? std::string() : g_err;
  // wait for the iterations, also after an enqueue error (earlier launches
  // may be in flight), and report a device fault
  const hipError_t es = hipStreamSynchronize(st);
  if (dev_hist) (void)hipFree(dev_hist);
  if (rc != DEAM_OK) {
    g_err = enqueue_err;
    return rc;
  }
  if (es != hipSuccess)
    return fail(DEAM_ERR_HIP, "device fault during the iterations: %s", hipGetErrorString(es));
  return ok();
}

int deam_validate_inputs(const deam_plan* plan, const double* c64, const float* d,
                         int64_t* n_bad, void* ws, size_t ws_bytes, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!ws) return fail(DEAM_ERR_NULL, "workspace is NULL");
  if (ws_bytes < 16) return fail(DEAM_ERR_WORKSPACE, "workspace too small: %zu < 16 bytes", ws_bytes);
  if (((uintptr_t)ws & 7) != 0) return fail(DEAM_ERR_VALUE, "workspace must be 8-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  unsigned long long* cnt = (unsigned long long*)ws;
  HIP_TRY(deam::launch_fill_u32((uint32_t*)cnt, 0u, 4, st));
  HIP_TRY(deam::launch_validate(plan, c64, d, cnt, st));
  unsigned long long h[2] = {0ull, 0ull};
  HIP_TRY(hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (n_bad) {
    n_bad[0] = (int64_t)h[0];
    n_bad[1] = (int64_t)h[1];
  }
  if (h[0] || h[1])
    return fail(DEAM_ERR_VALUE, "%llu non-finite image values, %llu counts negative or non-finite",
                h[0], h[1]);
  return ok();
}

int deam_iterate_penalized(const deam_plan* plan, double* c64, const float* d,
                           const uint8_t* mask, const double* Z, double lambda, double delta,
                           int32_t n_iter, double* obj_hist, void* ws, size_t ws_bytes,
                           void* stream) {
  const PenSpec pen{lambda, delta};
  return iterate_impl(plan, c64, nullptr, d, mask, Z, n_iter, obj_hist, ws, ws_bytes, stream,
                      nullptr, &pen);
}

static int check_fbp(const deam_plan* plan) {
  if (!plan->d_fbp)
    return fail(DEAM_ERR_UNSUPPORTED,
                "the MAR initialisation needs a 2D fan-beam plan over one full rotation with at "
                "most %d channels",
                deam::kMaxFbpCols);
  return DEAM_OK;
}

int deam_dilate_mask(const deam_plan* plan, const uint8_t* mask, int32_t radius, uint8_t* out,
                     void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!mask || !out) return fail(DEAM_ERR_NULL, "mask or out is NULL");
  if (radius < 0 || radius > plan->gd.n_cols) return fail(DEAM_ERR_VALUE, "radius out of range");
  const size_t nb = (size_t)plan->gd.R;
  if ((const char*)mask < (const char*)out + nb && (const char*)out < (const char*)mask + nb)
    return fail(DEAM_ERR_VALUE, "out overlaps mask");
  HIP_TRY(deam::launch_dilate(plan, mask, radius, out, (hipStream_t)stream));
  return ok();
}

int deam_fbp(const deam_plan* plan, const void* p, int32_t n_ch, void* img, void* ws,
             size_t ws_bytes, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!p || !img) return fail(DEAM_ERR_NULL, "p or img is NULL");
  if (n_ch != 1 && n_ch != 2) return fail(DEAM_ERR_SHAPE, "n_ch must be 1 or 2 (got %d)", n_ch);
  if (int rc = check_fbp(plan)) return rc;
  deam::WsLayout L;
  if (int rc = check_ws(plan, DEAM_OP_FBP, ws, ws_bytes, L)) return rc;
  HIP_TRY(deam::launch_fbp(plan, p, n_ch, (char*)ws + L.q, img, (hipStream_t)stream));
  return ok();
}

int deam_nmar(const deam_plan* plan, const void* p, const uint8_t* mask, const void* p_prior,
              double eps, void* out, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!p || !mask || !p_prior || !out) return fail(DEAM_ERR_NULL, "p, mask, p_prior or out is NULL");
  if (int rc = check_fbp(plan)) return rc;
  if (!(eps > 0.0 && std::isfinite(eps))) return fail(DEAM_ERR_VALUE, "eps must be > 0 and finite");
  const size_t nb = (size_t)plan->gd.R * 2 * real_size(plan);
  const char *a0 = (const char*)p, *b0 = (const char*)out;
  if (a0 < b0 + nb && b0 < a0 + nb) return fail(DEAM_ERR_VALUE, "out overlaps p");
  HIP_TRY(deam::launch_nmar(plan, p, mask, p_prior, eps, out, (hipStream_t)stream));
  return ok();
}

int deam_mar_init(const deam_plan* plan, const float* d, const deam_mar_params* prm, double* c64,
                  uint8_t* M, uint8_t* mask, void* ws, size_t ws_bytes, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!d || !prm || !c64 || !M || !mask) return fail(DEAM_ERR_NULL, "d, prm, c64, M or mask is NULL");
  if (int rc = check_fbp(plan)) return rc;
  if (plan->gd.bowtie)
    return fail(DEAM_ERR_UNSUPPORTED, "the MAR initialisation does not model a bowtie filter");
  const double vals[] = {prm->t, prm->water[0], prm->water[1], prm->air_frac, prm->bone_frac,
                         prm->metal_frac, prm->eps};
  for (double v : vals)
    if (!std::isfinite(v)) return fail(DEAM_ERR_VALUE, "MAR parameters must be finite");
  if (!(prm->water[0] > 0.0 && prm->water[1] > 0.0 && prm->eps > 0.0))
    return fail(DEAM_ERR_VALUE, "water attenuations and eps must be > 0");
  if (!(plan->i0sum[0] > 0.0 && plan->i0sum[1] > 0.0))
    return fail(DEAM_ERR_VALUE, "both spectra must have photons");
  deam::WsLayout L;
  if (int rc = check_ws(plan, DEAM_OP_MAR_INIT, ws, ws_bytes, L)) return rc;
  char* w = (char*)ws;
  hipStream_t st = (hipStream_t)stream;
  const bool dbl = plan->precision == DEAM_PREC_FP64;
  // line integrals and their FBP
  HIP_TRY(deam::launch_line_integrals(plan, d, w + L.p, st));
  HIP_TRY(deam::launch_fbp(plan, w + L.p, 2, w + L.q, w + L.mu0, st));
  // metal image, its trace, the prior images and their projections
  HIP_TRY(deam::launch_mar_classes(plan, w + L.mu0, prm->water, prm->air_frac, prm->bone_frac,
                                   prm->metal_frac, M, w + L.prior, st));
  HIP_TRY(deam::launch_pack(plan, M, 1, true, true, w + L.cp_y, w + L.cp_x, st));
  HIP_TRY(deam::launch_metal_trace(plan, w + L.cp_y, w + L.cp_x, prm->t, mask, nullptr, st));
  HIP_TRY(deam::launch_pack(plan, w + L.prior, 2, false, dbl, w + L.cp_y,
                            w + L.cp_y + (size_t)plan->gd.V * 2 * real_size(plan), st));
  HIP_TRY(deam::launch_forward(plan, w + L.cp_y, w + L.cp_y + (size_t)plan->gd.V * 2 * real_size(plan),
                               w + L.pp, 2, st));
  // NMAR, FBP of the corrected sinograms, Eq. 4
  HIP_TRY(deam::launch_nmar(plan, w + L.p, mask, w + L.pp, prm->eps, w + L.pc, st));
  HIP_TRY(deam::launch_fbp(plan, w + L.pc, 2, w + L.q, w + L.mu1, st));
  HIP_TRY(deam::launch_decompose(plan, w + L.mu1, c64, st));
  return ok();
}

// A view of the plan restricted to the ordered subset s of n_sub: views
// s, s + n_sub, s + 2 n_sub, ...  (same tables and buffers; only the walked
// views and the grid sizes change).
static deam_plan subset_plan(const deam_plan* p, int n_sub, int s) {
  deam_plan q = *p;
  q.gd.voff = s;
  q.gd.vsub = n_sub;
  q.gd.nvl = (p->gd.n_views - s + n_sub - 1) / n_sub;
  const int64_t rl = (int64_t)q.gd.nvl * p->gd.n_rows * p->gd.n_cols;
  q.ray_blocks = (rl + deam::kFpBlock - 1) / deam::kFpBlock;
  if (p->gd.is3d) {
    const int rg = p->precision == DEAM_PREC_FP64 ? deam::fp3_rows<double>() : deam::fp3_rows<float>();
    q.fp_blocks = deam::fp3_blocks(q.gd.nvl, p->gd.n_rows, p->gd.n_cols, rg);
  } else {
    q.fp_blocks = q.ray_blocks;
  }
  return q;
}

int deam_iterate_os(const deam_plan* plan, double* c64, const float* d, const uint8_t* mask,
                    const double* Z, int32_t n_sub, int32_t n_iter, double* obj_hist, void* ws,
                    size_t ws_bytes, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!c64 || !d || !Z) return fail(DEAM_ERR_NULL, "c64, d or Z is NULL");
  if (n_iter < 0) return fail(DEAM_ERR_VALUE, "n_iter must be >= 0");
  if (n_sub < 1 || n_sub > plan->gd.n_views)
    return fail(DEAM_ERR_VALUE, "n_sub must be in [1, n_views] (got %d)", n_sub);
  if (!(Z[0] > 0.0 && Z[1] > 0.0 && std::isfinite(Z[0]) && std::isfinite(Z[1])))
    return fail(DEAM_ERR_VALUE, "Z must be positive and finite");
  deam::WsLayout L;
  if (int rc = check_ws(plan, DEAM_OP_ITERATE, ws, ws_bytes, L)) return rc;
  char* w = (char*)ws;
  hipStream_t st = (hipStream_t)stream;
  void* cpy = w + L.cp_y;
  void* cpx = w + L.cp_x;
  uint32_t* wmap = (uint32_t*)(w + L.wmap);
  float* tmax = (float*)(w + L.tmax);
  const int64_t nmap = deam::wmap_words(plan->gd);
  double* partial = (double*)(w + L.partial);
  HIP_TRY(deam::launch_update(plan, c64, nullptr, Z[0], Z[1], nullptr, cpy, cpx, st));
  HIP_TRY(deam::launch_zero_tail(plan, cpx, plan->precision == DEAM_PREC_FP64, st));
  for (int k = 0; k < n_iter; ++k) {
    if (obj_hist) {  // the objective needs every view at the epoch's iterate
          HIP_TRY(deam::launch_fp_poly(plan, cpy, cpx, d, mask, deam::PM_AM, w + L.w, partial, st));
      HIP_TRY(deam::launch_reduce(partial, plan->fp_blocks, obj_hist + k, st));
    }
    for (int s = 0; s < n_sub; ++s) {
      const deam_plan sub = subset_plan(plan, n_sub, s);
          HIP_TRY(deam::launch_fill_u32(wmap, 0u, nmap, st));
      HIP_TRY(deam::launch_fp_poly(&sub, cpy, cpx, d, mask, deam::PM_AM, w + L.w, partial, st,
                                   wmap));
      HIP_TRY(deam::launch_backproject(&sub, w + L.w, 4, true, wmap, tmax, w + L.b, st));
      HIP_TRY(deam::launch_update(plan, c64, w + L.b, Z[0], Z[1], nullptr, cpy, cpx, st));
    }
  }
  return ok();
}

static int check_dual(const deam_plan* lo, const deam_plan* hi) {
  if (int rc = check_plan(lo)) return rc;
  if (int rc = check_plan(hi)) return rc;
  if (lo->precision != hi->precision) return fail(DEAM_ERR_VALUE, "the two plans differ in precision");
  const deam_geometry &a = lo->g, &b = hi->g;
  if (a.kind != b.kind || lo->gd.nx != hi->gd.nx || lo->gd.ny != hi->gd.ny ||
      lo->gd.nz != hi->gd.nz || a.dx != b.dx || a.dy != b.dy || (a.kind == DEAM_HELICAL3D && a.dz != b.dz))
    return fail(DEAM_ERR_VALUE, "the two plans must share the image grid");
  if (!(lo->i0sum[0] > 0.0 && lo->i0sum[1] == 0.0 && hi->i0sum[0] == 0.0 && hi->i0sum[1] > 0.0))
    return fail(DEAM_ERR_VALUE,
                "plan_lo must carry only the low spectrum and plan_hi only the high spectrum");
  return DEAM_OK;
}

int deam_dual_workspace_size(const deam_plan* plan_lo, const deam_plan* plan_hi, size_t* bytes) {
  if (!bytes) return fail(DEAM_ERR_NULL, "bytes is NULL");
  if (int rc = check_dual(plan_lo, plan_hi)) return rc;
  *bytes = align256(deam::workspace_layout(plan_lo, DEAM_OP_ITERATE).total) +
           deam::workspace_layout(plan_hi, DEAM_OP_ITERATE).total;
  return ok();
}

int deam_iterate_dual(const deam_plan* plan_lo, const deam_plan* plan_hi, double* c64,
                      const float* d_lo, const uint8_t* mask_lo, const float* d_hi,
                      const uint8_t* mask_hi, const double* Z, int32_t n_iter, double* obj_hist,
                      void* ws, size_t ws_bytes, void* stream) {
  if (int rc = check_dual(plan_lo, plan_hi)) return rc;
  if (!c64 || !d_lo || !d_hi || !Z) return fail(DEAM_ERR_NULL, "c64, d_lo, d_hi or Z is NULL");
  if (n_iter < 0) return fail(DEAM_ERR_VALUE, "n_iter must be >= 0");
  if (!(Z[0] > 0.0 && Z[1] > 0.0 && std::isfinite(Z[0]) && std::isfinite(Z[1])))
    return fail(DEAM_ERR_VALUE, "Z must be positive and finite");
  const deam::WsLayout LA = deam::workspace_layout(plan_lo, DEAM_OP_ITERATE);
  const deam::WsLayout LB = deam::workspace_layout(plan_hi, DEAM_OP_ITERATE);
  const size_t offb = align256(LA.total);
  if (!ws) return fail(DEAM_ERR_NULL, "workspace is NULL");
  if (ws_bytes < offb + LB.total)
    return fail(DEAM_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, offb + LB.total);
  if (((uintptr_t)ws & 255) != 0) return fail(DEAM_ERR_VALUE, "workspace must be 256-byte aligned");
  char* wa = (char*)ws;
  char* wb = wa + offb;
  hipStream_t st = (hipStream_t)stream;
  // one packed copy of c serves both scans (same image grid)
  void* cpy = wa + LA.cp_y;
  void* cpx = wa + LA.cp_x;
  uint32_t* wmap_a = (uint32_t*)(wa + LA.wmap);
  uint32_t* wmap_b = (uint32_t*)(wb + LB.wmap);
  float* tmax_a = (float*)(wa + LA.tmax);
  float* tmax_b = (float*)(wb + LB.tmax);
  double* part_a = (double*)(wa + LA.partial);
  double* part_b = (double*)(wb + LB.partial);
  double* two = (double*)(wa + LA.scratch);
  HIP_TRY(deam::launch_update(plan_lo, c64, nullptr, Z[0], Z[1], nullptr, cpy, cpx, st));
  HIP_TRY(deam::launch_zero_tail(plan_lo, cpx, plan_lo->precision == DEAM_PREC_FP64, st));
  for (int k = 0; k < n_iter; ++k) {
    HIP_TRY(deam::launch_fill_u32(wmap_a, 0u, deam::wmap_words(plan_lo->gd), st));
    HIP_TRY(deam::launch_fill_u32(wmap_b, 0u, deam::wmap_words(plan_hi->gd), st));
    HIP_TRY(deam::launch_fp_poly(plan_lo, cpy, cpx, d_lo, mask_lo, deam::PM_AM, wa + LA.w, part_a,
                                 st, wmap_a));
    HIP_TRY(deam::launch_fp_poly(plan_hi, cpy, cpx, d_hi, mask_hi, deam::PM_AM, wb + LB.w, part_b,
                                 st, wmap_b));
    if (obj_hist) {
      HIP_TRY(deam::launch_reduce(part_a, plan_lo->fp_blocks, two, st));
      HIP_TRY(deam::launch_reduce(part_b, plan_hi->fp_blocks, two + 1, st));
      HIP_TRY(deam::launch_reduce(two, 2, obj_hist + k, st));
    }
    HIP_TRY(deam::launch_backproject(plan_lo, wa + LA.w, 4, true, wmap_a, tmax_a, wa + LA.b, st));
    HIP_TRY(deam::launch_backproject(plan_hi, wb + LB.w, 4, true, wmap_b, tmax_b, wb + LB.b, st));
    HIP_TRY(deam::launch_update(plan_lo, c64, wa + LA.b, Z[0], Z[1], nullptr, cpy, cpx, st,
                                wb + LB.b));
  }
  return ok();
}

int deam_iterate_vjp(const deam_plan* plan, const double* c64, const float* d,
                     const uint8_t* mask, const double* Z, const double* G, double* out,
                     void* ws, size_t ws_bytes, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!c64 || !d || !Z || !G || !out) return fail(DEAM_ERR_NULL, "c64, d, Z, G or out is NULL");
  if (!(Z[0] > 0.0 && Z[1] > 0.0 && std::isfinite(Z[0]) && std::isfinite(Z[1])))
    return fail(DEAM_ERR_VALUE, "Z must be positive and finite");
  if (out == G || out == c64) return fail(DEAM_ERR_VALUE, "out may not alias G or c64");
  deam::WsLayout L;
  if (int rc = check_ws(plan, DEAM_OP_ITERATE_VJP, ws, ws_bytes, L)) return rc;
  char* w = (char*)ws;
  hipStream_t st = (hipStream_t)stream;
  const bool dbl = plan->precision == DEAM_PREC_FP64;
  const size_t rs = real_size(plan);
  const size_t V = (size_t)plan->gd.V, R = (size_t)plan->gd.R;
  void* cpy = w + L.cp_y;
  void* cpx = w + L.cp_x;
  uint32_t* wmap = (uint32_t*)(w + L.wmap);
  float* tmax = (float*)(w + L.tmax);
  double* partial = (double*)(w + L.partial);
  // forward pass of the iteration, recomputed: l = H c, weights, b = H^T w
  HIP_TRY(deam::launch_update(plan, const_cast<double*>(c64), nullptr, Z[0], Z[1], nullptr, cpy,
                              cpx, st));
  HIP_TRY(deam::launch_zero_tail(plan, cpx, dbl, st));
  HIP_TRY(deam::launch_forward(plan, cpy, cpx, w + L.l, 2, st));
  HIP_TRY(deam::launch_fill_u32(wmap, 0u, deam::wmap_words(plan->gd), st));
  HIP_TRY(deam::launch_poly(plan, w + L.l, d, mask, deam::PM_AM, nullptr, w + L.w, nullptr,
                            partial, st, wmap));
  HIP_TRY(deam::launch_backproject(plan, w + L.w, 4, true, wmap, tmax, w + L.b, st));
  // upstream images for b~ and b^, and their projections alpha = H u~, beta = H u^
  HIP_TRY(deam::launch_step_u(plan, G, w + L.b, Z[0], Z[1], w + L.u, st));
  for (int p = 0; p < 2; ++p) {
    HIP_TRY(deam::launch_pack(plan, w + L.u + (size_t)p * 2 * V * rs, 2, false, dbl, cpy, cpx, st));
    HIP_TRY(deam::launch_forward(plan, cpy, cpx, w + L.ab + (size_t)p * 2 * R * rs, 2, st));
  }
  // lambda per ray, then out = G + H^T lambda
  HIP_TRY(deam::launch_poly(plan, w + L.l, d, mask, deam::PM_STEP, w + L.ab, w + L.lam, nullptr,
                            partial, st));
  HIP_TRY(deam::launch_absmax(plan, w + L.lam, 2, wmap, st));
  HIP_TRY(deam::launch_backproject(plan, w + L.lam, 2, false, wmap, tmax, w + L.bl, st));
  HIP_TRY(deam::launch_add_g(plan, G, w + L.bl, out, st));
  return ok();
}

int deam_pack_mask(const deam_plan* plan, const uint8_t* mask, uint32_t* bits, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!mask || !bits) return fail(DEAM_ERR_NULL, "mask or bits is NULL");
  HIP_TRY(deam::launch_pack_mask(plan, mask, bits, (hipStream_t)stream));
  return ok();
}

int deam_iterate_packed(const deam_plan* plan, double* c64, const float* d,
                        const uint32_t* mask_bits, const double* Z, int32_t n_iter,
                        double* obj_hist, void* ws, size_t ws_bytes, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!mask_bits) return fail(DEAM_ERR_NULL, "mask_bits is NULL");
  deam_plan q = *plan;   // the same plan reading the bit-packed trace
  q.gd.mbits = mask_bits;
  return iterate_impl(&q, c64, nullptr, d, nullptr, Z, n_iter, obj_hist, ws, ws_bytes, stream,
                      nullptr);
}

int deam_iterate_timed(const deam_plan* plan, double* c64, void* c_proj, const float* d,
                       const uint8_t* mask, const double* Z, int32_t n_iter, double* obj_hist,
                       void* ws, size_t ws_bytes, void* stream, float* kernel_ms) {
  if (!kernel_ms) return fail(DEAM_ERR_NULL, "kernel_ms is NULL");
  return iterate_impl(plan, c64, c_proj, d, mask, Z, n_iter, obj_hist, ws, ws_bytes, stream,
                      kernel_ms);
}

}  // extern "C"

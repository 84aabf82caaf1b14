/*
 * FP64 CPU oracle for the DEAM hot path with metal-trace data substitution.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it; the product path never
 * does.  It shares no source, header or table with the GPU library.
 *
 * What it computes (paper: Ge et al., "A Metal Artifact Reduction Scheme For
 * Accurate Iterative Dual-Energy CT Algorithms"):
 *   - system operator h(x,y): exact intersection length of ray y with voxel x
 *     (Section 2.3, the operator inside Eq. 8), by Siddon's method: all
 *     crossings of the ray with the grid planes, merged in order, each
 *     consecutive pair giving one voxel (found from the midpoint) and one
 *     length;
 *   - metal trace T(y) = sum_x h(x,y) M(x) and the corrupt-ray test
 *     T(y) >= t (Section 2.1, Eqs. 2-3);
 *   - forward model g_j(y) = sum_E I0_j(E) exp(-sum_i mu_i(E) l_i(y)) with
 *     l_i = H c_i (Section 2.3, Eq. 8);
 *   - the linear-family split of the I-divergence (Section 2.3, Eqs. 9-10)
 *     with p_j = q_j on the metal trace (Section 2.3, Eq. 11 and the sentence
 *     that follows it) and p_j = q_j d_j / g_j elsewhere;
 *   - the alternating-minimisation component update
 *     c_i <- c_i - ln(b~_i / b^_i) / Z_i, where b~_i and b^_i back-project the
 *     energy sums of mu_i p_j and mu_i q_j (the DEAM step the paper cites to
 *     O'Sullivan and Benac; derived from Eqs. 5, 8, 9-10);
 *   - the masked I-divergence of Eq. 5 and the Poisson negative
 *     log-likelihood with its gradient b~ - b^;
 *   - the penalised iteration: the roughness penalty of Eq. 6 with the
 *     potential of Eq. 7 (read as the convex "fair" potential), and the
 *     c-step as one convex problem per voxel (De Pierro's decoupling),
 *     solved by bisection.
 * Everything is FP64; ray sums and energy sums use Neumaier compensation.
 */
#include "deam_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* ----------------------------------------------------------------------- */
/* Geometry: the scanner convention of the workloads.                       */
/* ----------------------------------------------------------------------- */

int orc_num_threads(void) { return omp_get_max_threads(); }
void orc_set_num_threads(int n) { if (n > 0) omp_set_num_threads(n); }

long orc_n_rays(const orc_geom* g) { return (long)g->n_views * g->n_rows * g->n_cols; }
long orc_n_voxels(const orc_geom* g) { return (long)g->nx * g->ny * (g->kind == ORC_HELICAL3D ? g->nz : 1); }

void orc_ray(const orc_geom* g, long ray, double S[3], double P[3]) {
  long k = ray % g->n_cols;
  long r = (ray / g->n_cols) % g->n_rows;
  long v = ray / ((long)g->n_cols * g->n_rows);
  double beta = g->beta0 + 2.0 * M_PI * (double)v / g->views_per_rot;
  double cb = cos(beta), sb = sin(beta);
  double gam = ((double)k - 0.5 * (g->n_cols - 1) - g->col_offset) * g->dgamma;
  double cg = cos(gam), sg = sin(gam);
  double ux = -cb, uy = -sb;
  double dirx = cg * ux - sg * uy, diry = sg * ux + cg * uy;
  double zs = 0.0, zeta = 0.0;
  if (g->kind == ORC_HELICAL3D) {
    zs = ((double)v - 0.5 * (g->n_views - 1)) * g->feed_per_rot / g->views_per_rot;
    zeta = ((double)r - 0.5 * (g->n_rows - 1)) * g->drow_iso * g->sdd / g->sid;
  }
  S[0] = g->sid * cb; S[1] = g->sid * sb; S[2] = zs;
  P[0] = S[0] + g->sdd * dirx; P[1] = S[1] + g->sdd * diry; P[2] = zs + zeta;
}

/* ----------------------------------------------------------------------- */
/* Siddon's method on the grid, restricted to the voxel sub-box [lo, hi).   */
/* ----------------------------------------------------------------------- */

/* Merge the ascending runs run[0..nrun) (run r is src[beg[r]..end[r])) into
 * dst, behind dst[0], in ascending order (Siddon's merge of the parametric
 * crossing sets of the three axes). */
static int merge_runs(const double* src, const int* beg, const int* end, int nrun,
                      double* dst, int m) {
  int pos[3] = {0, 0, 0};
  for (int r = 0; r < nrun; ++r) pos[r] = beg[r];
  for (;;) {
    int best = -1;
    for (int r = 0; r < nrun; ++r)
      if (pos[r] < end[r] && (best < 0 || src[pos[r]] < src[pos[best]])) best = r;
    if (best < 0) return m;
    dst[m++] = src[pos[best]++];
  }
}

int orc_siddon(const orc_geom* g, const double S[3], const double P[3],
               const int lo[3], const int hi[3], long* idx, double* len, int cap,
               double* scratch) {
  int is3d = (g->kind == ORC_HELICAL3D);
  int naxes = is3d ? 3 : 2;
  int n[3] = {g->nx, g->ny, is3d ? g->nz : 1};
  double dlt[3] = {g->dx, g->dy, g->dz};
  double org[3];
  for (int a = 0; a < 3; ++a) org[a] = -0.5 * n[a] * dlt[a];
  double D[3] = {P[0] - S[0], P[1] - S[1], is3d ? P[2] - S[2] : 0.0};
  double L = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);

  /* ray parameter range inside the sub-box (and on the segment S..P) */
  double amin = 0.0, amax = 1.0;
  for (int a = 0; a < naxes; ++a) {
    double p0 = org[a] + lo[a] * dlt[a], p1 = org[a] + hi[a] * dlt[a];
    double s = (a < 2 || is3d) ? S[a] : 0.0;
    if (D[a] == 0.0) {
      if (!(s >= p0 && s < p1)) return 0;
      continue;
    }
    double t0 = (p0 - s) / D[a], t1 = (p1 - s) / D[a];
    if (t0 > t1) { double t = t0; t0 = t1; t1 = t; }
    if (t0 > amin) amin = t0;
    if (t1 < amax) amax = t1;
  }
  if (!(amax > amin)) return 0;

  /* all plane crossings strictly inside (amin, amax), one ascending run per
     axis (alpha grows with the plane index when D > 0 and falls when D < 0,
     and the rounded values keep that order), merged into the sorted list
     amin, crossings..., amax in the second half of scratch */
  int n_in = 0, nrun = 0;
  int beg[3], end[3];
  for (int a = 0; a < naxes; ++a) {
    if (D[a] == 0.0) continue;
    double s = S[a];
    /* planes whose coordinate lies between the ray's coordinates at amin and
       amax (widened by one plane; the strict test below decides) */
    double xa = s + amin * D[a], xb = s + amax * D[a];
    if (xa > xb) { double t = xa; xa = xb; xb = t; }
    int i0 = (int)floor((xa - org[a]) / dlt[a]) - 1;
    int i1 = (int)ceil((xb - org[a]) / dlt[a]) + 1;
    if (i0 < lo[a] + 1) i0 = lo[a] + 1;
    if (i1 > hi[a] - 1) i1 = hi[a] - 1;
    beg[nrun] = n_in;
    for (int k = 0; k <= i1 - i0; ++k) {
      int i = D[a] > 0.0 ? i0 + k : i1 - k;
      double al = (org[a] + i * dlt[a] - s) / D[a];
      if (al > amin && al < amax) scratch[n_in++] = al;
    }
    end[nrun++] = n_in;
  }
  double* list = scratch + n_in;
  int m = 0;
  list[m++] = amin;
  m = merge_runs(scratch, beg, end, nrun, list, m);
  list[m++] = amax;

  int cnt = 0;
  for (int q = 0; q + 1 < m; ++q) {
    double a0 = list[q], a1 = list[q + 1];
    if (!(a1 > a0)) continue;                       /* coincident crossings */
    double am = 0.5 * (a0 + a1);
    int iv[3] = {0, 0, 0};
    int ok = 1;
    for (int a = 0; a < naxes; ++a) {
      double x = S[a] + am * D[a];
      iv[a] = (int)floor((x - org[a]) / dlt[a]);
      if (iv[a] < lo[a]) iv[a] = lo[a];
      if (iv[a] >= hi[a]) iv[a] = hi[a] - 1;
      if (iv[a] < 0 || iv[a] >= n[a]) ok = 0;
    }
    if (!ok) continue;
    if (cnt >= cap) return -1;
    idx[cnt] = ((long)iv[2] * n[1] + iv[1]) * n[0] + iv[0];
    len[cnt] = (a1 - a0) * L;
    ++cnt;
  }
  return cnt;
}

static int max_segments(const orc_geom* g) {
  int is3d = (g->kind == ORC_HELICAL3D);
  return g->nx + g->ny + (is3d ? g->nz : 1) + 8;
}

int orc_siddon_ray(const orc_geom* g, const double S[3], const double P[3],
                   long* idx, double* len, int cap) {
  int lo[3] = {0, 0, 0};
  int hi[3] = {g->nx, g->ny, g->kind == ORC_HELICAL3D ? g->nz : 1};
  double* scratch = (double*)malloc(sizeof(double) * (size_t)(2 * (max_segments(g) + 4)));
  int c = orc_siddon(g, S, P, lo, hi, idx, len, cap, scratch);
  free(scratch);
  return c;
}

/* Neumaier compensated accumulation */
typedef struct { double s, c; } nsum;
static inline void nadd(nsum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static inline double nval(const nsum* a) { return a->s + a->c; }

/* ----------------------------------------------------------------------- */
/* Forward projection l_k(y) = sum_x h(x,y) img_k(x)                        */
/* ----------------------------------------------------------------------- */

void orc_forward(const orc_geom* g, int nch, const double* img, double* sino) {
  long R = orc_n_rays(g), V = orc_n_voxels(g);
  int cap = max_segments(g);
  int lo[3] = {0, 0, 0};
  int hi[3] = {g->nx, g->ny, g->kind == ORC_HELICAL3D ? g->nz : 1};
#pragma omp parallel
  {
    long* idx = (long*)malloc(sizeof(long) * (size_t)cap);
    double* len = (double*)malloc(sizeof(double) * (size_t)cap);
    double* scratch = (double*)malloc(sizeof(double) * (size_t)(2 * (cap + 4)));
#pragma omp for schedule(dynamic, 256)
    for (long y = 0; y < R; ++y) {
      double S[3], P[3];
      orc_ray(g, y, S, P);
      int n = orc_siddon(g, S, P, lo, hi, idx, len, cap, scratch);
      for (int k = 0; k < nch; ++k) {
        nsum acc = {0.0, 0.0};
        for (int q = 0; q < n; ++q) nadd(&acc, len[q] * img[(long)k * V + idx[q]]);
        sino[(long)k * R + y] = nval(&acc);
      }
    }
    free(idx); free(len); free(scratch);
  }
}

/* Forward projection of a subset of rays (for sampled checks at full size). */
void orc_forward_rays(const orc_geom* g, int nch, const double* img, long n_sel,
                      const long* rays, double* out /*[nch][n_sel]*/) {
  long V = orc_n_voxels(g);
  int cap = max_segments(g);
  int lo[3] = {0, 0, 0};
  int hi[3] = {g->nx, g->ny, g->kind == ORC_HELICAL3D ? g->nz : 1};
#pragma omp parallel
  {
    long* idx = (long*)malloc(sizeof(long) * (size_t)cap);
    double* len = (double*)malloc(sizeof(double) * (size_t)cap);
    double* scratch = (double*)malloc(sizeof(double) * (size_t)(2 * (cap + 4)));
#pragma omp for schedule(dynamic, 64)
    for (long s = 0; s < n_sel; ++s) {
      double S[3], P[3];
      orc_ray(g, rays[s], S, P);
      int n = orc_siddon(g, S, P, lo, hi, idx, len, cap, scratch);
      for (int k = 0; k < nch; ++k) {
        nsum acc = {0.0, 0.0};
        for (int q = 0; q < n; ++q) nadd(&acc, len[q] * img[(long)k * V + idx[q]]);
        out[(long)k * n_sel + s] = nval(&acc);
      }
    }
    free(idx); free(len); free(scratch);
  }
}

/* ----------------------------------------------------------------------- */
/* Backprojection img_k(x) = sum_y h(x,y) sino_k(y): the transpose of the   */
/* forward projection.  Each task owns a band of rows iy (3D: one slice iz) */
/* and walks every ray clipped to that band, so the sums are deterministic  */
/* without atomics.  The band's bounding planes are crossings of the whole  */
/* ray, computed with the same expression, so a ray's segments inside the   */
/* band are those of the whole ray, and each voxel adds its rays in the     */
/* order of the ray index in either band shape.                             */
/* ----------------------------------------------------------------------- */

/* 3D: the task of slice iz walks only the detector rows whose segment S->P
 * reaches that slice (S and P bound the segment's z, and rows that cannot
 * reach it would be clipped away by orc_siddon anyway); every other ray is
 * walked exactly as in 2D, so the sums do not depend on the band shape. */
static void backproject_slabs(const orc_geom* g, int nch, const double* sino, double* img) {
  long R = orc_n_rays(g), V = orc_n_voxels(g);
  int cap = max_segments(g);
  double z0 = -0.5 * g->nz * g->dz;
#pragma omp parallel
  {
    long* idx = (long*)malloc(sizeof(long) * (size_t)cap);
    double* len = (double*)malloc(sizeof(double) * (size_t)cap);
    double* scratch = (double*)malloc(sizeof(double) * (size_t)(2 * (cap + 4)));
#pragma omp for schedule(dynamic, 1)
    for (int iz = 0; iz < g->nz; ++iz) {
      int lo[3] = {0, 0, iz};
      int hi[3] = {g->nx, g->ny, iz + 1};
      /* the slab with a margin far above rounding: the test only skips rows */
      double zlo = z0 + iz * g->dz - 1e-6 * g->dz, zhi = z0 + (iz + 1) * g->dz + 1e-6 * g->dz;
      for (long v = 0; v < g->n_views; ++v) {
        for (long r = 0; r < g->n_rows; ++r) {
          /* S and P of every channel of (v, r) share their z */
          double S0[3], P0[3];
          orc_ray(g, (v * g->n_rows + r) * g->n_cols, S0, P0);
          if ((S0[2] < zlo && P0[2] < zlo) || (S0[2] > zhi && P0[2] > zhi)) continue;
          for (long k = 0; k < g->n_cols; ++k) {
            long y = (v * g->n_rows + r) * g->n_cols + k;
            double S[3], P[3];
            orc_ray(g, y, S, P);
            int n = orc_siddon(g, S, P, lo, hi, idx, len, cap, scratch);
            for (int c = 0; c < nch; ++c) {
              double w = sino[(long)c * R + y];
              if (w == 0.0) continue;
              for (int q = 0; q < n; ++q) img[(long)c * V + idx[q]] += len[q] * w;
            }
          }
        }
      }
    }
    free(idx); free(len); free(scratch);
  }
}

void orc_backproject(const orc_geom* g, int nch, const double* sino, double* img) {
  long R = orc_n_rays(g), V = orc_n_voxels(g);
  int cap = max_segments(g);
  int band = 4;
  int nbands = (g->ny + band - 1) / band;
  memset(img, 0, sizeof(double) * (size_t)(nch * V));
  if (g->kind == ORC_HELICAL3D && g->nz >= 8) {
    backproject_slabs(g, nch, sino, img);
    return;
  }
#pragma omp parallel
  {
    long* idx = (long*)malloc(sizeof(long) * (size_t)cap);
    double* len = (double*)malloc(sizeof(double) * (size_t)cap);
    double* scratch = (double*)malloc(sizeof(double) * (size_t)(2 * (cap + 4)));
#pragma omp for schedule(dynamic, 1)
    for (int b = 0; b < nbands; ++b) {
      int lo[3] = {0, b * band, 0};
      int hi[3] = {g->nx, (b + 1) * band < g->ny ? (b + 1) * band : g->ny,
                   g->kind == ORC_HELICAL3D ? g->nz : 1};
      for (long y = 0; y < R; ++y) {
        double S[3], P[3];
        orc_ray(g, y, S, P);
        int n = orc_siddon(g, S, P, lo, hi, idx, len, cap, scratch);
        for (int k = 0; k < nch; ++k) {
          double w = sino[(long)k * R + y];
          if (w == 0.0) continue;
          for (int q = 0; q < n; ++q) img[(long)k * V + idx[q]] += len[q] * w;
        }
      }
    }
    free(idx); free(len); free(scratch);
  }
}

/* ----------------------------------------------------------------------- */
/* Per-ray polyenergetic mean with metal-trace substitution.                */
/* ----------------------------------------------------------------------- */

/* bt (or NULL): a bowtie filter, given as its path lengths (mm) in the two
 * basis materials per detector channel, bt[i * n_cols + k]: ray y of channel
 * k = y mod n_cols then sees the spectra I0_j(E) exp(-mu_1(E) bt_1k -
 * mu_2(E) bt_2k) (energy and channel dependent I0_j(y,E) of Eq. 8). */
static void poly_mean_impl(long R, int nE, const double* I0, const double* mu,
                           const double* bt, int n_cols,
                           const double* l, const double* d, const unsigned char* mask,
                           int mode, const double* v, double* w, double* gout, double* obj) {
#pragma omp parallel for schedule(static)
  for (long y = 0; y < R; ++y) {
    double l1 = l[y], l2 = l[R + y];
    long kb = bt ? y % n_cols : 0;
    nsum gs[2] = {{0, 0}, {0, 0}};
    nsum as[2][2] = {{{0, 0}, {0, 0}}, {{0, 0}, {0, 0}}};   /* as[i][j] */
    nsum ms[2][3] = {{{0, 0}, {0, 0}, {0, 0}}, {{0, 0}, {0, 0}, {0, 0}}};  /* m_11, m_12, m_22 */
    for (int e = 0; e < nE; ++e) {
      double mu1 = mu[e], mu2 = mu[nE + e];
      double ex = exp(-(mu1 * l1 + mu2 * l2));
      double fb = bt ? exp(-(mu1 * bt[kb] + mu2 * bt[n_cols + kb])) : 1.0;
      for (int j = 0; j < 2; ++j) {
        double q = I0[j * nE + e] * ex;                     /* q_j(y,E) */
        if (bt) q = (I0[j * nE + e] * fb) * ex;             /* the ray's own spectrum */
        nadd(&gs[j], q);
        nadd(&as[0][j], mu1 * q);
        nadd(&as[1][j], mu2 * q);
        if (mode == ORC_W_STEP_VJP) {                       /* sum_E mu_i mu_k q_j */
          nadd(&ms[j][0], mu1 * mu1 * q);
          nadd(&ms[j][1], mu1 * mu2 * q);
          nadd(&ms[j][2], mu2 * mu2 * q);
        }
      }
    }
    double gj[2] = {nval(&gs[0]), nval(&gs[1])};
    double a[2][2] = {{nval(&as[0][0]), nval(&as[0][1])}, {nval(&as[1][0]), nval(&as[1][1])}};
    int metal = mask ? (mask[y] != 0) : 0;
    /* r_j = d_j/g_j off the trace, 1 on it (p = q there); r_j*a_ij := 0 if g_j == 0 */
    double ra[2][2];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        double dj = d[(long)j * R + y];
        if (metal) ra[i][j] = a[i][j];
        else ra[i][j] = gj[j] > 0.0 ? (dj / gj[j]) * a[i][j] : 0.0;
      }
    double term = 0.0;
    if (mode == ORC_W_AM) {
      for (int i = 0; i < 2; ++i) {
        w[(long)i * R + y] = ra[i][0] + ra[i][1];            /* w~_i */
        w[(long)(2 + i) * R + y] = a[i][0] + a[i][1];        /* w^_i */
      }
      if (!metal)
        for (int j = 0; j < 2; ++j) {
          double dj = d[(long)j * R + y], g = gj[j];
          if (!(g > 0.0)) continue;
          term += (dj > 0.0 ? dj * log(dj / g) : 0.0) - dj + g;
        }
    } else if (mode == ORC_W_GRAD) {
      for (int i = 0; i < 2; ++i)
        w[(long)i * R + y] = (ra[i][0] - a[i][0]) + (ra[i][1] - a[i][1]);
      if (!metal)
        for (int j = 0; j < 2; ++j) {
          double dj = d[(long)j * R + y], g = gj[j];
          if (!(g > 0.0)) continue;
          term += g - (dj > 0.0 ? dj * log(g) : 0.0);
        }
    } else if (mode == ORC_W_VJP) { /* u_i = -sum_j v_j a_ij, with v_j = dloss/dg_j */
      for (int i = 0; i < 2; ++i)
        w[(long)i * R + y] = -(v[y] * a[i][0] + v[R + y] * a[i][1]);
    } else { /* ORC_W_STEP_VJP */
      /* Upstream gradients alpha_i = dloss/dw~_i and beta_i = dloss/dw^_i (v =
       * [alpha_1, alpha_2, beta_1, beta_2]); output lambda_k = dloss/dl_k.
       * With dq_j/dl_k = -mu_k q_j: dg_j/dl_k = -a_kj, da_ij/dl_k = -m_ik^j,
       * d(d_j/g_j)/dl_k = (d_j/g_j^2) a_kj off the trace (r_j = 1 and
       * constant on it; r_j a_ij := 0 when g_j = 0), so
       *   dw~_i/dl_k = sum_j [ (d_j/g_j^2) a_kj a_ij - r_j m_ik^j ]
       *   dw^_i/dl_k = -sum_j m_ik^j.                                        */
      double m[2][2][2];   /* m[j][i][k] */
      for (int j = 0; j < 2; ++j) {
        m[j][0][0] = nval(&ms[j][0]);
        m[j][0][1] = m[j][1][0] = nval(&ms[j][1]);
        m[j][1][1] = nval(&ms[j][2]);
      }
      for (int k = 0; k < 2; ++k) {
        double lam = 0.0;
        for (int i = 0; i < 2; ++i) {
          double al = v[(long)i * R + y], be = v[(long)(2 + i) * R + y];
          double dwt = 0.0, dwh = 0.0;
          for (int j = 0; j < 2; ++j) {
            double dj = d[(long)j * R + y], g = gj[j];
            double r;
            if (metal) r = 1.0;
            else r = g > 0.0 ? dj / g : 0.0;
            if (!metal && g > 0.0) dwt += dj / (g * g) * a[k][j] * a[i][j];
            if (metal || g > 0.0) dwt -= r * m[j][i][k];
            dwh -= m[j][i][k];
          }
          lam += al * dwt + be * dwh;
        }
        w[(long)k * R + y] = lam;
      }
    }
    if (gout) { gout[y] = gj[0]; gout[R + y] = gj[1]; }
    if (obj) obj[y] = term;
  }
}

void orc_poly_mean(long R, int nE, const double* I0, const double* mu,
                   const double* l, const double* d, const unsigned char* mask,
                   int mode, const double* v, double* w, double* gout, double* obj) {
  poly_mean_impl(R, nE, I0, mu, NULL, 0, l, d, mask, mode, v, w, gout, obj);
}

void orc_poly_mean_bt(long R, int nE, const double* I0, const double* mu, const double* bt,
                      int n_cols, const double* l, const double* d, const unsigned char* mask,
                      int mode, const double* v, double* w, double* gout, double* obj) {
  poly_mean_impl(R, nE, I0, mu, bt, n_cols, l, d, mask, mode, v, w, gout, obj);
}

double orc_sum(long n, const double* x) {
  nsum s = {0.0, 0.0};
  for (long i = 0; i < n; ++i) nadd(&s, x[i]);
  return nval(&s);
}

/* ----------------------------------------------------------------------- */
/* Component update c_i <- c_i - ln(b~_i / b^_i) / Z_i where both are > 0.  */
/* ----------------------------------------------------------------------- */

void orc_update(long V, const double* b, const double Z[2], double* c) {
#pragma omp parallel for schedule(static)
  for (long x = 0; x < V; ++x)
    for (int i = 0; i < 2; ++i) {
      double bt = b[(long)i * V + x], bh = b[(long)(2 + i) * V + x];
      if (bt > 0.0 && bh > 0.0) c[(long)i * V + x] -= log(bt / bh) / Z[i];
    }
}

/* ----------------------------------------------------------------------- */
/* Metal trace and corrupt-ray mask                                          */
/* ----------------------------------------------------------------------- */

void orc_metal_trace(const orc_geom* g, const unsigned char* M, double t,
                     unsigned char* mask, double* T) {
  long R = orc_n_rays(g), V = orc_n_voxels(g);
  double* img = (double*)malloc(sizeof(double) * (size_t)V);
  for (long x = 0; x < V; ++x) img[x] = M[x] ? 1.0 : 0.0;
  double* tr = T ? T : (double*)malloc(sizeof(double) * (size_t)R);
  orc_forward(g, 1, img, tr);
  for (long y = 0; y < R; ++y) mask[y] = tr[y] >= t ? 1 : 0;
  if (!T) free(tr);
  free(img);
}

/* ----------------------------------------------------------------------- */
/* DEAM iterations                                                           */
/* ----------------------------------------------------------------------- */

int orc_iterate(const orc_geom* g, int nE, const double* I0, const double* mu,
                const double* d, const unsigned char* mask, const double Z[2],
                int n_iter, double* c, double* obj_hist) {
  return orc_iterate_b(g, nE, I0, mu, d, mask, Z, n_iter, c, obj_hist, NULL);
}

/* orc_iterate that also returns the backprojections b~_1, b~_2, b^_1, b^_2
 * ([4][V]) of the last iteration in b_last (may be NULL). */
int orc_iterate_b(const orc_geom* g, int nE, const double* I0, const double* mu,
                  const double* d, const unsigned char* mask, const double Z[2],
                  int n_iter, double* c, double* obj_hist, double* b_last) {
  long R = orc_n_rays(g), V = orc_n_voxels(g);
  double* l = (double*)malloc(sizeof(double) * (size_t)(2 * R));
  double* w = (double*)malloc(sizeof(double) * (size_t)(4 * R));
  double* obj = (double*)malloc(sizeof(double) * (size_t)R);
  double* b = (double*)malloc(sizeof(double) * (size_t)(4 * V));
  if (!l || !w || !obj || !b) { free(l); free(w); free(obj); free(b); return -1; }
  for (int k = 0; k < n_iter; ++k) {
    orc_forward(g, 2, c, l);
    orc_poly_mean(R, nE, I0, mu, l, d, mask, ORC_W_AM, NULL, w, NULL, obj);
    if (obj_hist) obj_hist[k] = orc_sum(R, obj);
    orc_backproject(g, 4, w, b);
    orc_update(V, b, Z, c);
    if (b_last && k == n_iter - 1) memcpy(b_last, b, sizeof(double) * (size_t)(4 * V));
  }
  free(l); free(w); free(obj); free(b);
  return 0;
}

/* Vector-Jacobian product of one DEAM iteration Phi(c) = c - ln(b~/b^)/Z
 * (componentwise, c unchanged where b~ <= 0 or b^ <= 0): out = G + H^T lambda
 * for the upstream gradient G = dloss/dPhi (both [2][V]), with
 *   u~_i = -G_i / (Z_i b~_i), u^_i = G_i / (Z_i b^_i)    (0 where skipped)
 *   alpha = H u~, beta = H u^, lambda from the STEP_VJP poly-mean mode.     */
int orc_step_vjp(const orc_geom* g, int nE, const double* I0, const double* mu,
                 const double* d, const unsigned char* mask, const double Z[2],
                 const double* c, const double* G, double* out) {
  long R = orc_n_rays(g), V = orc_n_voxels(g);
  double* l = (double*)malloc(sizeof(double) * (size_t)(2 * R));
  double* w = (double*)malloc(sizeof(double) * (size_t)(4 * R));
  double* b = (double*)malloc(sizeof(double) * (size_t)(4 * V));
  double* u = (double*)malloc(sizeof(double) * (size_t)(4 * V));
  double* ab = (double*)malloc(sizeof(double) * (size_t)(4 * R));
  double* lam = (double*)malloc(sizeof(double) * (size_t)(2 * R));
  if (!l || !w || !b || !u || !ab || !lam) {
    free(l); free(w); free(b); free(u); free(ab); free(lam);
    return -1;
  }
  orc_forward(g, 2, c, l);
  orc_poly_mean(R, nE, I0, mu, l, d, mask, ORC_W_AM, NULL, w, NULL, NULL);
  orc_backproject(g, 4, w, b);
  for (int i = 0; i < 2; ++i)
    for (long x = 0; x < V; ++x) {
      double bt = b[(long)i * V + x], bh = b[(long)(2 + i) * V + x];
      double gi = G[(long)i * V + x];
      int act = bt > 0.0 && bh > 0.0;
      u[(long)i * V + x] = act ? -gi / (Z[i] * bt) : 0.0;       /* dloss/db~_i */
      u[(long)(2 + i) * V + x] = act ? gi / (Z[i] * bh) : 0.0;  /* dloss/db^_i */
    }
  orc_forward(g, 4, u, ab);
  orc_poly_mean(R, nE, I0, mu, l, d, mask, ORC_W_STEP_VJP, ab, lam, NULL, NULL);
  orc_backproject(g, 2, lam, out);
  for (long x = 0; x < 2 * V; ++x) out[x] += G[x];
  free(l); free(w); free(b); free(u); free(ab); free(lam);
  return 0;
}

/* Objective only: masked I-divergence (mode AM) or NLL (mode GRAD) at c. */
double orc_objective(const orc_geom* g, int nE, const double* I0, const double* mu,
                     const double* d, const unsigned char* mask, const double* c, int mode) {
  long R = orc_n_rays(g);
  double* l = (double*)malloc(sizeof(double) * (size_t)(2 * R));
  double* w = (double*)malloc(sizeof(double) * (size_t)(4 * R));
  double* obj = (double*)malloc(sizeof(double) * (size_t)R);
  orc_forward(g, 2, c, l);
  orc_poly_mean(R, nE, I0, mu, l, d, mask, mode, NULL, w, NULL, obj);
  double s = orc_sum(R, obj);
  free(l); free(w); free(obj);
  return s;
}

/* Negative log-likelihood L(c) and its gradient H^T u (u from GRAD mode). */
double orc_nll_grad(const orc_geom* g, int nE, const double* I0, const double* mu,
                    const double* d, const unsigned char* mask, const double* c,
                    double* grad) {
  long R = orc_n_rays(g);
  double* l = (double*)malloc(sizeof(double) * (size_t)(2 * R));
  double* u = (double*)malloc(sizeof(double) * (size_t)(2 * R));
  double* obj = (double*)malloc(sizeof(double) * (size_t)R);
  orc_forward(g, 2, c, l);
  orc_poly_mean(R, nE, I0, mu, l, d, mask, ORC_W_GRAD, NULL, u, NULL, obj);
  double s = orc_sum(R, obj);
  if (grad) orc_backproject(g, 2, u, grad);
  free(l); free(u); free(obj);
  return s;
}

/* ----------------------------------------------------------------------- */
/* Penalised DEAM (Section 2.3, Eqs. 6-7)                                   */
/* ----------------------------------------------------------------------- */

/* Edge-preserving potential of Eq. 7.  As printed, the sign inside the
 * logarithm makes phi concave and undefined for |t| >= delta; the reading
 * used here is the convex "fair" potential of Lange,
 *   phi(t) = delta^2 (|t|/delta - ln(1 + |t|/delta)),
 * even, ~ t^2/2 for |t| << delta and ~ delta |t| for |t| >> delta. */
double orc_fair(double t, double delta) {
  double a = fabs(t) / delta;
  return delta * delta * (a - log1p(a));
}

/* Its derivative phi'(t) = t / (1 + |t|/delta). */
double orc_fair_d1(double t, double delta) { return t / (1.0 + fabs(t) / delta); }

/* Neighbourhood N_x of Eq. 6: the voxels that differ from x by at most one
 * step along every axis and lie inside the grid (8 in 2D, 26 in 3D away from
 * the border), with w(x, x~) = 1 / (physical distance between the centres). */
static int neighbours(const orc_geom* g, long x, long nb[26], double w[26]) {
  long nx = g->nx, ny = g->ny, nz = g->nz;
  long ix = x % nx, iy = (x / nx) % ny, iz = x / (nx * ny);
  int n = 0;
  for (int oz = -1; oz <= 1; ++oz)
    for (int oy = -1; oy <= 1; ++oy)
      for (int ox = -1; ox <= 1; ++ox) {
        if (!ox && !oy && !oz) continue;
        long jx = ix + ox, jy = iy + oy, jz = iz + oz;
        if (jx < 0 || jx >= nx || jy < 0 || jy >= ny || jz < 0 || jz >= nz) continue;
        double ddx = ox * g->dx, ddy = oy * g->dy, ddz = oz * g->dz;
        nb[n] = (jz * ny + jy) * nx + jx;
        w[n] = 1.0 / sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
        ++n;
      }
  return n;
}

/* R(c) of Eq. 6 for c [2][V]: lambda sum_i sum_x sum_{x~ in N_x} w phi(c_i(x) - c_i(x~))
 * (every neighbouring pair enters twice, once from each side). */
double orc_penalty(const orc_geom* g, const double* c, double lambda, double delta) {
  long V = orc_n_voxels(g);
  double total = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : total)
  for (long x = 0; x < V; ++x) {
    long nb[26];
    double w[26];
    int n = neighbours(g, x, nb, w);
    double s = 0.0;
    for (int i = 0; i < 2; ++i)
      for (int k = 0; k < n; ++k) s += w[k] * orc_fair(c[(long)i * V + x] - c[(long)i * V + nb[k]], delta);
    total += s;
  }
  return lambda * total;
}

/* Penalised component update.  With the data surrogate of the DEAM step
 * (convexity of exp, weights h mu_i / Z_i) and De Pierro's decoupling of the
 * penalty (convexity of phi: c(x) - c(x~) is the mean of 2c(x) - c^k(x) -
 * c^k(x~) and -(2c(x~) - c^k(x) - c^k(x~))), the c-step separates into one
 * convex problem per voxel and component:
 *   minimise  b~ c + (b^/Z) exp(-Z (c - c^k)) + lambda sum_{x~} w phi(2c - c^k(x) - c^k(x~)),
 * whose derivative
 *   f'(c) = b~ - b^ exp(-Z (c - c^k)) + 2 lambda sum_{x~} w phi'(2c - c^k(x) - c^k(x~))
 * increases with c.  Its root lies between the data-only minimiser
 * c^k - ln(b~/b^)/Z and the penalty-only one, which is inside
 * [min, max] of (c^k(x) + c^k(x~))/2; it is found by bisection.  Voxels with
 * b~ <= 0 or b^ <= 0 keep c^k, as in the unpenalised update (lambda = 0 gives
 * the same update up to rounding).  c_prev and c_next are [2][V], distinct. */
/* The c-step of component i at voxel x (see orc_update_pen). */
static double pen_voxel(const orc_geom* g, const double* b, const double Z[2], double lambda,
                        double delta, const double* c_prev, long x, int i) {
  long V = orc_n_voxels(g);
  long nb[26];
  double w[26];
  int n = neighbours(g, x, nb, w);
  const double* ci = c_prev + (long)i * V;
  double ck = ci[x];
  double bt = b[(long)i * V + x], bh = b[(long)(2 + i) * V + x];
  if (!(bt > 0.0 && bh > 0.0)) return ck;
  double cu = ck - log(bt / bh) / Z[i];
  double lo = cu, hi = cu;
  for (int k = 0; k < n; ++k) {
    double m = 0.5 * (ck + ci[nb[k]]);
    if (m < lo) lo = m;
    if (m > hi) hi = m;
  }
  /* f'(lo) <= 0 <= f'(hi); halve until the bracket is below 1e-17 absolute
   * or cannot be split */
  for (;;) {
    double mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi) || hi - lo <= 1e-17) break;
    double f = bt - bh * exp(-Z[i] * (mid - ck));
    double p = 0.0;
    for (int k = 0; k < n; ++k) p += w[k] * orc_fair_d1(2.0 * mid - ck - ci[nb[k]], delta);
    f += 2.0 * lambda * p;
    if (f > 0.0) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

void orc_update_pen(const orc_geom* g, const double* b, const double Z[2], double lambda,
                    double delta, const double* c_prev, double* c_next) {
  long V = orc_n_voxels(g);
#pragma omp parallel for schedule(dynamic, 64)
  for (long x = 0; x < V; ++x)
    for (int i = 0; i < 2; ++i)
      c_next[(long)i * V + x] = pen_voxel(g, b, Z, lambda, delta, c_prev, x, i);
}

/* The penalised c-step at n_sel chosen voxels only: out [2][n_sel]. */
void orc_update_pen_voxels(const orc_geom* g, const double* b, const double Z[2], double lambda,
                           double delta, const double* c_prev, long n_sel, const long* voxels,
                           double* out) {
#pragma omp parallel for schedule(dynamic, 16)
  for (long k = 0; k < n_sel; ++k)
    for (int i = 0; i < 2; ++i)
      out[(long)i * n_sel + k] = pen_voxel(g, b, Z, lambda, delta, c_prev, voxels[k], i);
}

/* n_iter penalised DEAM iterations from c (in place); obj_hist[k] (or NULL)
 * = masked I-divergence + R(c^k) at the iterate entering iteration k. */
int orc_iterate_pen(const orc_geom* g, int nE, const double* I0, const double* mu,
                    const double* d, const unsigned char* mask, const double Z[2],
                    double lambda, double delta, int n_iter, double* c, double* obj_hist) {
  long R = orc_n_rays(g), V = orc_n_voxels(g);
  double* l = (double*)malloc(sizeof(double) * (size_t)(2 * R));
  double* w = (double*)malloc(sizeof(double) * (size_t)(4 * R));
  double* obj = (double*)malloc(sizeof(double) * (size_t)R);
  double* b = (double*)malloc(sizeof(double) * (size_t)(4 * V));
  double* cp = (double*)malloc(sizeof(double) * (size_t)(2 * V));
  if (!l || !w || !obj || !b || !cp) {
    free(l); free(w); free(obj); free(b); free(cp);
    return -1;
  }
  for (int k = 0; k < n_iter; ++k) {
    orc_forward(g, 2, c, l);
    orc_poly_mean(R, nE, I0, mu, l, d, mask, ORC_W_AM, NULL, w, NULL, obj);
    if (obj_hist) obj_hist[k] = orc_sum(R, obj) + orc_penalty(g, c, lambda, delta);
    orc_backproject(g, 4, w, b);
    memcpy(cp, c, sizeof(double) * (size_t)(2 * V));
    orc_update_pen(g, b, Z, lambda, delta, cp, c);
  }
  free(l); free(w); free(obj); free(b); free(cp);
  return 0;
}

/* ----------------------------------------------------------------------- */
/* Ordered subsets of views                                                  */
/* ----------------------------------------------------------------------- */

/* n_iter epochs of ordered-subset DEAM: the views are split into n_sub
 * interleaved subsets (view v belongs to subset v mod n_sub), and each epoch
 * runs one DEAM step per subset s = 0, 1, ..., n_sub - 1 in which only the rays
 * of subset s are backprojected (their weights are kept, all others are set
 * to zero).  obj_hist[k] (or NULL) = masked I-divergence at the iterate
 * entering epoch k.  n_sub = 1 is the DEAM iteration. */
int orc_iterate_os(const orc_geom* g, int nE, const double* I0, const double* mu,
                   const double* d, const unsigned char* mask, const double Z[2], int n_sub,
                   int n_iter, double* c, double* obj_hist) {
  long R = orc_n_rays(g), V = orc_n_voxels(g);
  long per_view = (long)g->n_rows * g->n_cols;
  double* l = (double*)malloc(sizeof(double) * (size_t)(2 * R));
  double* w = (double*)malloc(sizeof(double) * (size_t)(4 * R));
  double* obj = (double*)malloc(sizeof(double) * (size_t)R);
  double* b = (double*)malloc(sizeof(double) * (size_t)(4 * V));
  if (!l || !w || !obj || !b || n_sub < 1) {
    free(l); free(w); free(obj); free(b);
    return -1;
  }
  for (int k = 0; k < n_iter; ++k) {
    for (int s = 0; s < n_sub; ++s) {
      orc_forward(g, 2, c, l);
      orc_poly_mean(R, nE, I0, mu, l, d, mask, ORC_W_AM, NULL, w, NULL, obj);
      if (s == 0 && obj_hist) obj_hist[k] = orc_sum(R, obj);
      for (long y = 0; y < R; ++y)
        if ((y / per_view) % n_sub != s)
          for (int ch = 0; ch < 4; ++ch) w[(long)ch * R + y] = 0.0;
      orc_backproject(g, 4, w, b);
      orc_update(V, b, Z, c);
    }
  }
  free(l); free(w); free(obj); free(b);
  return 0;
}

/* ----------------------------------------------------------------------- */
/* Separate low- and high-energy scans                                       */
/* ----------------------------------------------------------------------- */

/* DEAM with a system operator and a metal trace per scan (the general case
 * of Section 2.1, where h and T differ between the two spectra): scan j has
 * geometry g[j] (same image grid), counts d[j] [R_j] and mask[j] [R_j] (or
 * NULL).  Each scan's energy sums use its own spectrum only, so its weights
 * are those of Eqs. 9-11 for that spectrum; b~ and b^ are the sums of the
 * two scans' backprojections, and the update is the DEAM update.
 * obj_hist[k] (or NULL) = the two scans' masked I-divergences at c^k. */
int orc_iterate_dual(const orc_geom* const g[2], int nE, const double* I0, const double* mu,
                     const double* const d[2], const unsigned char* const mask[2],
                     const double Z[2], int n_iter, double* c, double* obj_hist) {
  long V = orc_n_voxels(g[0]);
  long R[2] = {orc_n_rays(g[0]), orc_n_rays(g[1])};
  long Rm = R[0] > R[1] ? R[0] : R[1];
  double* l = (double*)malloc(sizeof(double) * (size_t)(2 * Rm));
  double* w = (double*)malloc(sizeof(double) * (size_t)(4 * Rm));
  double* obj = (double*)malloc(sizeof(double) * (size_t)Rm);
  double* dd = (double*)malloc(sizeof(double) * (size_t)(2 * Rm));
  double* b = (double*)malloc(sizeof(double) * (size_t)(4 * V));
  double* bs = (double*)malloc(sizeof(double) * (size_t)(4 * V));
  double* I0j = (double*)malloc(sizeof(double) * (size_t)(2 * nE));
  if (!l || !w || !obj || !dd || !b || !bs || !I0j || orc_n_voxels(g[1]) != V) {
    free(l); free(w); free(obj); free(dd); free(b); free(bs); free(I0j);
    return -1;
  }
  for (int k = 0; k < n_iter; ++k) {
    double f = 0.0;
    memset(b, 0, sizeof(double) * (size_t)(4 * V));
    for (int j = 0; j < 2; ++j) {
      /* spectrum j alone, and its counts in its own slot */
      for (int e = 0; e < nE; ++e) {
        I0j[e] = j == 0 ? I0[e] : 0.0;
        I0j[nE + e] = j == 1 ? I0[nE + e] : 0.0;
      }
      memset(dd, 0, sizeof(double) * (size_t)(2 * R[j]));
      memcpy(dd + (long)j * R[j], d[j], sizeof(double) * (size_t)R[j]);
      orc_forward(g[j], 2, c, l);
      orc_poly_mean(R[j], nE, I0j, mu, l, dd, mask[j], ORC_W_AM, NULL, w, NULL, obj);
      f += orc_sum(R[j], obj);
      orc_backproject(g[j], 4, w, bs);
      for (long x = 0; x < 4 * V; ++x) b[x] += bs[x];
    }
    if (obj_hist) obj_hist[k] = f;
    orc_update(V, b, Z, c);
  }
  free(l); free(w); free(obj); free(dd); free(b); free(bs); free(I0j);
  return 0;
}

/* Dilation of a trace mask along the detector channels: out[y] = 1 when any
 * ray of the same view and row within `radius` channels of y is in mask. */
void orc_dilate_mask(const orc_geom* g, const unsigned char* mask, int radius, unsigned char* out) {
  long R = orc_n_rays(g);
  for (long y = 0; y < R; ++y) {
    long k = y % g->n_cols, row0 = y - k;
    unsigned char m = 0;
    for (long q = k - radius; q <= k + radius; ++q)
      if (q >= 0 && q < g->n_cols && mask[row0 + q]) m = 1;
    out[y] = m;
  }
}

/* DEAM with a bowtie filter (see poly_mean_impl): n_iter iterations from c
 * (in place); obj_hist[k] (or NULL) = masked I-divergence at c^k. */
int orc_iterate_bt(const orc_geom* g, int nE, const double* I0, const double* mu,
                   const double* bt, const double* d, const unsigned char* mask,
                   const double Z[2], int n_iter, double* c, double* obj_hist) {
  long R = orc_n_rays(g), V = orc_n_voxels(g);
  double* l = (double*)malloc(sizeof(double) * (size_t)(2 * R));
  double* w = (double*)malloc(sizeof(double) * (size_t)(4 * R));
  double* obj = (double*)malloc(sizeof(double) * (size_t)R);
  double* b = (double*)malloc(sizeof(double) * (size_t)(4 * V));
  if (!l || !w || !obj || !b) { free(l); free(w); free(obj); free(b); return -1; }
  for (int k = 0; k < n_iter; ++k) {
    orc_forward(g, 2, c, l);
    orc_poly_mean_bt(R, nE, I0, mu, bt, g->n_cols, l, d, mask, ORC_W_AM, NULL, w, NULL, obj);
    if (obj_hist) obj_hist[k] = orc_sum(R, obj);
    orc_backproject(g, 4, w, b);
    orc_update(V, b, Z, c);
  }
  free(l); free(w); free(obj); free(b);
  return 0;
}

/*
 * FP64 CPU oracle for the DEAM hot path (test infrastructure only; see
 * deam_oracle.c).  Plain C, no dependency on the GPU library.
 */
#ifndef DEAM_ORACLE_H
#define DEAM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_FAN2D = 0, ORC_HELICAL3D = 1 };
enum { ORC_W_AM = 0, ORC_W_GRAD = 1, ORC_W_VJP = 2, ORC_W_STEP_VJP = 3 };

typedef struct {
  int kind, nx, ny, nz;
  double dx, dy, dz;
  int n_views, n_rows, n_cols;
  double sid, sdd, dgamma, col_offset, drow_iso, beta0, views_per_rot, feed_per_rot;
} orc_geom;

int orc_num_threads(void);
/* threads of the parallel loops that follow (a timing control: only the rounding of the
 * penalty's parallel sum depends on it) */
void orc_set_num_threads(int n);
long orc_n_rays(const orc_geom* g);
long orc_n_voxels(const orc_geom* g);
void orc_ray(const orc_geom* g, long ray, double S[3], double P[3]);
/* scratch: 2 * (nx + ny + nz + 12) doubles */
int orc_siddon(const orc_geom* g, const double S[3], const double P[3],
               const int lo[3], const int hi[3], long* idx, double* len, int cap,
               double* scratch);
int orc_siddon_ray(const orc_geom* g, const double S[3], const double P[3],
                   long* idx, double* len, int cap);
void orc_forward(const orc_geom* g, int nch, const double* img, double* sino);
void orc_forward_rays(const orc_geom* g, int nch, const double* img, long n_sel,
                      const long* rays, double* out);
void orc_backproject(const orc_geom* g, int nch, const double* sino, double* img);
void orc_poly_mean(long R, int nE, const double* I0, const double* mu,
                   const double* l, const double* d, const unsigned char* mask,
                   int mode, const double* v, double* w, double* gout, double* obj);
void orc_poly_mean_bt(long R, int nE, const double* I0, const double* mu, const double* bt,
                      int n_cols, const double* l, const double* d, const unsigned char* mask,
                      int mode, const double* v, double* w, double* gout, double* obj);
int orc_iterate_bt(const orc_geom* g, int nE, const double* I0, const double* mu,
                   const double* bt, const double* d, const unsigned char* mask,
                   const double Z[2], int n_iter, double* c, double* obj_hist);
double orc_sum(long n, const double* x);
int orc_step_vjp(const orc_geom* g, int nE, const double* I0, const double* mu,
                 const double* d, const unsigned char* mask, const double Z[2],
                 const double* c, const double* G, double* out);
void orc_update(long V, const double* b, const double Z[2], double* c);
void orc_metal_trace(const orc_geom* g, const unsigned char* M, double t,
                     unsigned char* mask, double* T);
int orc_iterate(const orc_geom* g, int nE, const double* I0, const double* mu,
                const double* d, const unsigned char* mask, const double Z[2],
                int n_iter, double* c, double* obj_hist);
int orc_iterate_b(const orc_geom* g, int nE, const double* I0, const double* mu,
                  const double* d, const unsigned char* mask, const double Z[2],
                  int n_iter, double* c, double* obj_hist, double* b_last);
double orc_objective(const orc_geom* g, int nE, const double* I0, const double* mu,
                     const double* d, const unsigned char* mask, const double* c, int mode);
double orc_fair(double t, double delta);
double orc_fair_d1(double t, double delta);
double orc_penalty(const orc_geom* g, const double* c, double lambda, double delta);
void orc_update_pen(const orc_geom* g, const double* b, const double Z[2], double lambda,
                    double delta, const double* c_prev, double* c_next);
void orc_update_pen_voxels(const orc_geom* g, const double* b, const double Z[2], double lambda,
                           double delta, const double* c_prev, long n_sel, const long* voxels,
                           double* out);
int orc_iterate_pen(const orc_geom* g, int nE, const double* I0, const double* mu,
                    const double* d, const unsigned char* mask, const double Z[2],
                    double lambda, double delta, int n_iter, double* c, double* obj_hist);
int orc_iterate_os(const orc_geom* g, int nE, const double* I0, const double* mu,
                   const double* d, const unsigned char* mask, const double Z[2], int n_sub,
                   int n_iter, double* c, double* obj_hist);
int orc_iterate_dual(const orc_geom* const g[2], int nE, const double* I0, const double* mu,
                     const double* const d[2], const unsigned char* const mask[2],
                     const double Z[2], int n_iter, double* c, double* obj_hist);
void orc_dilate_mask(const orc_geom* g, const unsigned char* mask, int radius, unsigned char* out);
double orc_nll_grad(const orc_geom* g, int nE, const double* I0, const double* mu,
                    const double* d, const unsigned char* mask, const double* c,
                    double* grad);

#ifdef __cplusplus
}
#endif
#endif

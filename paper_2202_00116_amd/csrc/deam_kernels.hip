// gfx950 kernels of the DEAM hot path (Ge et al., Section 2.3, Eqs. 5-11).
//
// Projector.  h(x,y) is the exact intersection length of ray y with voxel x
// (the system operator of Eq. 8).  Rays are walked along their driving axis
// (the in-plane axis along which the ray advances fastest, so the lateral
// and axial slopes are at most 1 in grid units): each step crosses one grid
// plane of that axis, and inside the step the ray is split at the lateral
// (and, in 3D, axial) plane it crosses.  This yields exactly the segments of
// Siddon's method, grouped per plane step, so that the 64 lanes of a
// wavefront (64 neighbouring channels of one view) move through the same
// image row at the same time and read neighbouring pixels.  Rays driven
// along x read a transposed copy of the image so those reads stay
// contiguous too.
//
// Backprojection.  Floating-point atomics are slow on this part (both in LDS
// and in L2), while LDS integer atomics run at full rate.  Each workgroup
// owns a tile of voxels in LDS, loops over all views, walks every ray that
// crosses its tile (clipped to the tile) and accumulates h*w in 64-bit
// fixed point with integer LDS atomics.  Integer addition is associative,
// so the result is bitwise reproducible, and the tile is written once with
// plain stores: no global atomics, no partial images.
//
// Ray set-up.  The in-plane part of every (view, channel) ray is computed
// once per plan in FP64 and stored in the plan precision (RayXY); the
// forward projector and the backprojector both start from it, so their
// segment lengths agree bit for bit away from tile edges.
#include "deam_internal.hpp"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <mutex>
#include <type_traits>

// Scratch of deam_poly_mean_noalloc: every call on a GPU uses that GPU's
// copy, so calls that overlap on one GPU race.
static __device__ __align__(256) unsigned char scratch[deam::kNoAllocScratchBytes];


namespace deam {
namespace {

template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };
// two packed float pixels read by one 16-byte load at an 8-byte boundary
typedef float Pix2f __attribute__((ext_vector_type(4), aligned(8)));

// clamp to [lo, hi] in one v_med3_i32 (the compiler emits min + max)
__device__ __forceinline__ int clampi(int v, int lo, int hi) {
  int r;
  asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(v), "v"(lo), "v"(hi));
  return r;
}
// floor and convert in one v_cvt_flr_i32_f32 (the compiler emits floor + cvt)
__device__ __forceinline__ int ifloor(float x) {
  int r;
  asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}
__device__ __forceinline__ int ifloor(double x) { return __double2int_rd(x); }
// clamp to [0, hi] (v_med3_f32 for float)
__device__ __forceinline__ float clamp0(float x, float hi) { return __builtin_amdgcn_fmed3f(x, 0.f, hi); }
__device__ __forceinline__ double clamp0(double x, double hi) { return fmin(fmax(x, 0.0), hi); }
// clamp to [lo, hi] (lo <= hi; v_med3_f32 for float)
__device__ __forceinline__ float clampf(float x, float lo, float hi) {
  return __builtin_amdgcn_fmed3f(x, lo, hi);
}
__device__ __forceinline__ double clampf(double x, double lo, double hi) {
  return fmin(fmax(x, lo), hi);
}
// min(x, hi) for finite operands, as the median of (x, hi, -3e38)
// (v_med3_f32 for float: no canonicalisation of the loop-invariant bound
// inside the loop)
__device__ __forceinline__ float min_fin(float x, float hi) {
  return __builtin_amdgcn_fmed3f(x, hi, -3.0e38f);
}
__device__ __forceinline__ double min_fin(double x, double hi) { return fmin(x, hi); }
// Attenuation exp(-(mu1 l1 + mu2 l2)) of one energy bin, given the ray's
// line integrals as prepared by bin_args: FP32 plans scale them by log2(e)
// once per ray and use the hardware 2^x (one instruction per bin; the
// argument is rounded once, as it is for exp); FP64 plans use exp.
template <typename T>
__device__ __forceinline__ void bin_args(T l1, T l2, T& k1, T& k2) {
  if constexpr (sizeof(T) == 4) {
    k1 = l1 * 1.44269504088896340736f;
    k2 = l2 * 1.44269504088896340736f;
  } else {
    k1 = l1;
    k2 = l2;
  }
}
template <typename T>
__device__ __forceinline__ T bin_att(T mu1, T mu2, T k1, T k2) {
  if constexpr (sizeof(T) == 4)
    return __builtin_amdgcn_exp2f(-fma(mu1, k1, mu2 * k2));
  else
    return exp(-fma(mu1, k1, mu2 * k2));
}

template <bool PK> struct QType { using type = unsigned long long; };
template <> struct QType<true> { using type = uint32_t; };

// Minimum / maximum over the lanes of the wave, as a wave-uniform value.
// Must be reached by all 64 lanes (the reduction reads lanes 0 and 32).
__device__ __forceinline__ int wave_min(int x) {
  return __builtin_amdgcn_readfirstlane(__ockl_wfred_min_i32(x));
}
__device__ __forceinline__ int wave_max(int x) {
  return __builtin_amdgcn_readfirstlane(__ockl_wfred_max_i32(x));
}

// Logical block index that gives each XCD a contiguous range of blocks
// (blocks are dispatched round-robin over the 8 XCDs).
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int per = nb >> 3, rem = nb & 7, x = b & 7, i = b >> 3;
  return x * per + (x < rem ? x : rem) + i;
}

// ---------------------------------------------------------------------------
// Ray set-up (FP64) and the plane-by-plane walk (plan precision)
// ---------------------------------------------------------------------------
template <typename T>
struct Ray {
  T b0, mb;       // lateral grid coordinate b(a) = ib + b0 + a*mb: the walk
                  // counts lateral pixels from the ray's origin ib
  T imb;          // 1/mb (huge when mb = 0)
  T w0, mw, imw;  // axial grid coordinate w(a) = iw + w0 + a*mw, imw = 1/|mw|: the
                  // walk counts slices from the ray's origin iw
  T La, Lb;       // mm of ray per unit of a, per unit of b
  T alo, ahi;     // range of a inside the clip box
  int ydrive;     // 1: a = y (rows) and b = x; 0: a = x and b = y
  int ib;         // lateral origin: lateral pixel indices of the walk are relative to it
  int iw;         // axial origin (3D): slice indices of the walk are relative to it
};

// Ray (v, r, k) clipped to the voxel box [lo, hi) (grid units, axes x, y, z).
// Returns false if the ray misses the box.  Lateral pixel indices of the
// walk (and the lateral bounds given to walk_row) are relative to ry.ib, and
// in 3D slice indices (and the axial bounds) relative to ry.iw, the slice at
// the middle of the ray's driving range, so that the rounding of the axial
// coordinate, and with it the error of a slice crossing (that rounding
// divided by |mw|, which is small for rays close to the slice planes), is
// set by the axial distance travelled and not by the volume's height.
template <typename T>
__device__ __forceinline__ bool make_ray(const GeomDev& G, const RayXY<T>* __restrict__ rays,
                                         int v, int r, int k, int lox, int loy, int loz, int hix,
                                         int hiy, int hiz, Ray<T>& ry) {
  const RayXY<T> t = rays[(int64_t)v * G.n_cols + k];
  const bool yd = t.yd != (T)0;
  const int ib = (int)t.ib;
  const T Lr = (T)G.row[4 * r + 1];
  T mw = 0, w0 = (T)0.5, rmw = 0;
  int iw = 0;
  if (G.is3d) {
    // w(a) = w_s + (a - s_a) mw: w_s (the source's slice coordinate) enters
    // relative to iw through one FP64 subtraction, so no rounding of a
    // coordinate as large as the volume is left
    const T zr = (T)G.row[4 * r];
    mw = zr * t.ida;
    const double ws = G.view[4 * v + 3];
    const T pz = zr * (t.sa * t.ida);                  // w_s - w(0)
    const T amid = (T)(0.5 * (yd ? G.ny : G.nx));
    iw = ifloor(clampf(fma(amid, mw, (T)ws - pz), (T)-1e6, (T)1e6));
    w0 = (T)(ws - (double)iw) - pz;
    rmw = mw != (T)0 ? (T)1 / mw : (T)0;
  }
  const T alo_box = (T)(yd ? loy : lox), ahi_box = (T)(yd ? hiy : hix);
  const T blo = (T)((yd ? lox : loy) - ib), bhi = (T)((yd ? hix : hiy) - ib);
  T alo = alo_box, ahi = ahi_box;
  if (t.mb != (T)0) {
    const T t0 = (blo - t.b0) * t.imb, t1 = (bhi - t.b0) * t.imb;
    alo = fmax(alo, fmin(t0, t1));
    ahi = fmin(ahi, fmax(t0, t1));
  } else if (!(t.b0 >= blo && t.b0 < bhi)) {
    return false;
  }
  if (G.is3d) {
    const T wlo = (T)(loz - iw), whi = (T)(hiz - iw);
    if (mw != (T)0) {
      const T t0 = (wlo - w0) * rmw, t1 = (whi - w0) * rmw;
      alo = fmax(alo, fmin(t0, t1));
      ahi = fmin(ahi, fmax(t0, t1));
    } else if (!(w0 >= wlo && w0 < whi)) {
      return false;
    }
  }
  if (!(ahi > alo)) return false;
  ry.b0 = t.b0;
  ry.mb = t.mb;
  ry.imb = t.imb;
  ry.w0 = w0;
  ry.mw = mw;
  ry.imw = fabs(rmw);
  ry.La = Lr * fabs(t.ida);
  ry.Lb = Lr * t.iadb;
  ry.alo = alo;
  ry.ahi = ahi;
  ry.ydrive = yd ? 1 : 0;
  ry.ib = ib;
  ry.iw = iw;
  return true;
}

// One piece [va, vb] of a plane step at axial index iw: split at the
// lateral plane it crosses (at most one, since |mb| <= 1).
template <typename T, bool SKIP, typename F>
__device__ __forceinline__ void walk_piece(const Ray<T>& ry, int ia, T va, T vb, int iw, int blo,
                                           int bhi, F& visit) {
  const T ba = fma(va, ry.mb, ry.b0), bb = fma(vb, ry.mb, ry.b0);
  const int A = clampi(ifloor(ba), blo, bhi - 1);
  int B = clampi(ifloor(bb), blo, bhi - 1);
  B = clampi(B, A - 1, A + 1);
  const T seg = (vb - va) * ry.La;
  T hA = seg;
  if (A != B) hA = fmin(fabs((T)(A > B ? A : B) - ba) * ry.Lb, seg);
  visit(ia, A, iw, hA);
  if (!SKIP || B != A) visit(ia, B, iw, seg - hA);
}

// One plane step ia of the driving axis (clipped to [alo, ahi]), restricted
// to lateral indices [blo, bhi) and axial indices [wlo, whi).  visit(ia, ib,
// iw, h) receives every segment (with SKIP = false also a zero-length second
// visit per piece, which keeps the loads of the forward projector uniform).
template <typename T, bool Z3, bool SKIP, typename F>
__device__ __forceinline__ void walk_row(const Ray<T>& ry, int ia, int blo, int bhi, int wlo,
                                         int whi, F& visit) {
  const T va = fmax((T)ia, ry.alo), vb = fmin((T)(ia + 1), ry.ahi);
  if (!(vb > va)) return;
  if constexpr (Z3) {
    const T wa = fma(va, ry.mw, ry.w0), wb = fma(vb, ry.mw, ry.w0);
    int C = clampi(ifloor(wa), wlo, whi - 1);
    const int D = clampi(ifloor(wb), wlo, whi - 1);
    T vcur = va, wcur = wa;
    while (C != D) {  // axial plane crossings inside this step (rare)
      const int dir = D > C ? 1 : -1;
      const T wz = (T)(dir > 0 ? C + 1 : C);
      const T vz = fmin(fmax(vcur + fabs(wz - wcur) * ry.imw, vcur), vb);
      walk_piece<T, SKIP>(ry, ia, vcur, vz, C, blo, bhi, visit);
      vcur = vz;
      wcur = wz;
      C += dir;
    }
    walk_piece<T, SKIP>(ry, ia, vcur, vb, C, blo, bhi, visit);
  } else {
    walk_piece<T, SKIP>(ry, ia, va, vb, 0, blo, bhi, visit);
  }
}

// All plane steps of the ray inside [alo_i, ahi_i) (driving-axis indices).
template <typename T, bool Z3, bool SKIP, typename F>
__device__ __forceinline__ void walk(const Ray<T>& ry, int alo_i, int ahi_i, int blo, int bhi,
                                     int wlo, int whi, F& visit) {
  const int ia0 = max(ifloor(ry.alo), alo_i);
  const int ia1 = min((int)ceil(ry.ahi) - 1, ahi_i - 1);
  for (int ia = ia0; ia <= ia1; ++ia) walk_row<T, Z3, SKIP>(ry, ia, blo, bhi, wlo, whi, visit);
}

template <typename T>
__device__ __forceinline__ void neumaier(T& s, T& c, T x) {
  const T t = s + x;
  c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
  s = t;
}

// Line integrals of the two packed components along one ray (compensated).
// cp holds the packed image twice: natural order at element 0 and x-major at
// element xoff; rays driven along y read the first copy, rays driven along
// x the second, so neighbouring lanes gather neighbouring addresses.
// The walk carries the lateral pixel and coordinate from one plane step to
// the next (one lateral floor per step) and keeps lengths in units of the
// driving axis; the sums are scaled by the mm per unit at the end.  Steps go
// four at a time with all gathers issued before the accumulation.  In 3D a
// step that crosses an axial plane is left out of the fast walk and recorded
// in a 64-bit mask; every 16 groups (a point common to all lanes still
// walking) and at the end, the recorded steps are summed through the general
// walk_row.
// Called by all lanes of the wave (valid = false: no ray, result 0); the
// ray index runs fastest over the lanes.
template <typename T, bool Z3>
__device__ void project_ray(const GeomDev& G, const RayXY<T>* __restrict__ rays,
                            const typename Vec2<T>::type* __restrict__ cp, uint32_t xoff, int v,
                            int r, int k, bool valid, T& l1, T& l2) {
  using T2 = typename Vec2<T>::type;
  constexpr uint32_t E = sizeof(T2);
  l1 = 0;
  l2 = 0;
  Ray<T> ry{};
  const int nzz = G.is3d ? G.nz : 1;
  const bool hit = valid && make_ray<T>(G, rays, v, r, k, 0, 0, 0, G.nx, G.ny, nzz, ry);
  const uint32_t base = ry.ydrive ? 0u : xoff;
  const int nb = ry.ydrive ? G.nx : G.ny;
  // lateral pixel range [blo, bhi] relative to the ray's origin ry.ib (0 for
  // a lane without a ray); addresses add the origin back
  const int blo = -ry.ib, bhi = nb - 1 - ry.ib;
  const uint32_t plane = (uint32_t)G.nx * (uint32_t)G.ny;
  const uint32_t rstep = (uint32_t)nb * E;
  const char* __restrict__ cpb = (const char*)cp;
  T s1 = 0, c1 = 0, s2 = 0, c2 = 0, p1 = 0, p2 = 0;
  auto flush = [&]() {
    neumaier(s1, c1, p1);
    neumaier(s2, c2, p2);
    p1 = 0;
    p2 = 0;
  };
  // plane steps [q0, q1); empty for a lane without a ray
  const int q0 = hit ? ifloor(ry.alo) : (1 << 30);
  const int q1 = hit ? -ifloor(-ry.ahi) : -(1 << 30);
  T tp = ry.alo;                                         // start of the current step
  T bp = fma(tp, ry.mb, ry.b0);                          // lateral coordinate there
  int A = clampi(ifloor(bp), blo, bhi);
  // slices relative to the ray's axial origin ry.iw (0 in 2D)
  const int wlo = -ry.iw, whi = nzz - 1 - ry.iw;
  int C = 0;
  if constexpr (Z3) C = clampi(ifloor(fma(tp, ry.mw, ry.w0)), wlo, whi);
  uint64_t rest = 0;   // 3D: deferred steps, bit = step - qw
  int qw = 0;
  T fa = 0;
  uint32_t row = 0;   // byte offset of lateral index 0 in the current plane row and slice
  // one plane step: gather offsets and lengths (zero when deferred)
  auto step = [&](int q, uint32_t& oA, uint32_t& oB, T& dA, T& dB) {
    fa += (T)1;
    const T tn = clampf(fa, ry.alo, ry.ahi);
    const T bn = fma(tn, ry.mb, ry.b0);
    const int B = clampi(ifloor(bn), blo, bhi);
    T ds = tn - tp;
    const uint32_t rq = row;
    row += rstep;
    if constexpr (Z3) {
      // (clamped: a step that reaches a face of the volume stays in the edge
      // slice up to the ray's end)
      const int D = clampi(ifloor(fma(tn, ry.mw, ry.w0)), wlo, whi);
      if (D != C) {
        rest |= 1ull << (q - qw);
        ds = (T)0;
        row += (uint32_t)((D - C) * (int)plane) * E;
        C = D;
      }
    }
    const T a = (B == A) ? ds : clamp0(((T)max(A, B) - bp) * ry.imb, ds);
    dA = a;
    dB = ds - a;
    oA = rq + (uint32_t)A * E;
    oB = rq + (uint32_t)B * E;
    A = B;
    bp = bn;
    tp = tn;
  };
  const T iLa = (T)1 / ry.La;
  auto visit = [&](int ia, int ib, int iw, T h) {
    const T2 cv = cp[base + (uint32_t)(iw + ry.iw) * plane + (uint32_t)ia * (uint32_t)nb +
                     (uint32_t)(ib + ry.ib)];
    p1 = fma(h * iLa, cv.x, p1);
    p2 = fma(h * iLa, cv.y, p2);
  };
  auto fixup = [&]() {
    while (rest != 0ull) {
      const int bit = __ffsll((unsigned long long)rest) - 1;
      rest &= rest - 1ull;
      walk_row<T, true, false>(ry, qw + bit, blo, bhi + 1, wlo, whi + 1, visit);
    }
  };
  // the lanes of a wave walk the same plane rows together (a common range),
  // so that their gathers share cache lines; outside its own range a lane's
  // steps have zero length (the step ends are clamped to [alo, ahi]) and its
  // pixel state does not move
  const int qlo = wave_min(q0), qhi = wave_max(q1);
  if (qlo >= qhi) return;
  qw = qlo;
  fa = (T)qlo;
  // (the unsigned offsets wrap for a negative relative pixel; sums with the
  // origin's offset are the true, in-range offsets)
  row = (base + (uint32_t)qlo * (uint32_t)nb + (uint32_t)(C + ry.iw) * plane + (uint32_t)ry.ib) * E;
  int q = qlo;
  int groups = 0;
  // gathers and sums of four steps: all gathers before the sums.  2D float
  // plans: the two pixels of a step are neighbours in one row (|A - B| <= 1),
  // so one 16-byte load at the lower offset fetches both, and the step's two
  // lengths are matched to the lower and upper pixel instead (when A = B
  // the upper length is 0; the element after a copy's last pixel lies in the
  // next copy or the zeroed tail, so it is finite)
  constexpr bool PAIR = !Z3 && sizeof(T) == 4;
  auto accumulate4 = [&](const uint32_t* oA, const uint32_t* oB, const T* dA, const T* dB) {
    if constexpr (PAIR) {
      Pix2f v[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) v[s] = *(const Pix2f*)(cpb + min(oA[s], oB[s]));
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const bool al = oA[s] <= oB[s];
        const T dl = al ? dA[s] : dB[s], dh = al ? dB[s] : dA[s];
        p1 = fma(dl, v[s].x, p1);
        p2 = fma(dl, v[s].y, p2);
        p1 = fma(dh, v[s].z, p1);
        p2 = fma(dh, v[s].w, p2);
      }
    } else {
      T2 vA[4], vB[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        vA[s] = *(const T2*)(cpb + oA[s]);
        vB[s] = *(const T2*)(cpb + oB[s]);
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        p1 = fma(dA[s], vA[s].x, p1);
        p2 = fma(dA[s], vA[s].y, p2);
        p1 = fma(dB[s], vB[s].x, p1);
        p2 = fma(dB[s], vB[s].y, p2);
      }
    }
  };
  auto accumulate1 = [&](uint32_t oA, uint32_t oB, T dA, T dB) {
    if constexpr (PAIR) {
      const Pix2f v = *(const Pix2f*)(cpb + min(oA, oB));
      const bool al = oA <= oB;
      const T dl = al ? dA : dB, dh = al ? dB : dA;
      p1 = fma(dl, v.x, p1);
      p2 = fma(dl, v.y, p2);
      p1 = fma(dh, v.z, p1);
      p2 = fma(dh, v.w, p2);
    } else {
      const T2 vA = *(const T2*)(cpb + oA), vB = *(const T2*)(cpb + oB);
      p1 = fma(dA, vA.x, p1);
      p2 = fma(dA, vA.y, p2);
      p1 = fma(dB, vB.x, p1);
      p2 = fma(dB, vB.y, p2);
    }
  };
  // plane steps [q, qe) through the general step
  auto general = [&](int qe) {
    for (; q + 4 <= qe; q += 4) {
      uint32_t oA[4], oB[4];
      T dA[4], dB[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) step(q + s, oA[s], oB[s], dA[s], dB[s]);
      accumulate4(oA, oB, dA, dB);
      ++groups;
      if ((groups & 3) == 0) flush();
      if constexpr (Z3) {
        if ((groups & 15) == 0) {
          fixup();
          qw = q + 4;
        }
      }
    }
    for (; q < qe; ++q) {
      uint32_t oA, oB;
      T dA, dB;
      step(q, oA, oB, dA, dB);
      accumulate1(oA, oB, dA, dB);
    }
  };
  if constexpr (Z3) {
    general(qhi);
    fixup();
  } else {
    // 2D: plane steps [qa, qb) lie inside the chord of every lane that has a
    // ray, so each is a whole plane spacing.  There the walk is Siddon's
    // incremental form: e is the distance (in plane spacings) from the start
    // of the step to the next lateral plane, and a step with e < 1 splits
    // there and moves one pixel in the direction sg.  e is recomputed from the
    // ray's line every 16 steps, which bounds its rounding drift.  Lanes
    // without a ray (zero ray: sg = 0) stay on pixel 0 of the rows walked.
    const int qa = max(wave_max(hit ? -ifloor(-ry.alo) : qlo), qlo);
    const int qb = min(wave_min(hit ? ifloor(ry.ahi) : qhi), qhi);
    if (qa >= qb) {
      general(qhi);
    } else {
      general(qa);
      flush();
      const int sg = ry.mb > (T)0 ? 1 : (ry.mb < (T)0 ? -1 : 0);
      const T iab = fabs(ry.imb), iab1 = iab - (T)1;
      T e = 0;
      auto sync = [&]() {
        bp = fma((T)q, ry.mb, ry.b0);
        A = clampi(ifloor(bp), blo, bhi);
        e = sg > 0 ? ((T)(A + 1) - bp) * iab : (sg < 0 ? (bp - (T)A) * iab : (T)1e30);
      };
      auto istep = [&](uint32_t& oA, uint32_t& oB, T& dA, T& dB) {
        const bool cr = e < (T)1;
        dA = clampf(e, (T)0, (T)1);
        dB = (T)1 - dA;
        const int B = clampi(A + (cr ? sg : 0), blo, bhi);
        oA = row + (uint32_t)A * E;
        oB = row + (uint32_t)B * E;
        row += rstep;
        e += cr ? iab1 : (T)-1;
        A = B;
      };
      sync();
      for (; q + 4 <= qb; q += 4) {
        if (q != qa && ((q - qa) & 15) == 0) {
          flush();
          sync();
        }
        uint32_t oA[4], oB[4];
        T dA[4], dB[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) istep(oA[s], oB[s], dA[s], dB[s]);
        accumulate4(oA, oB, dA, dB);
      }
      for (; q < qb; ++q) {
        uint32_t oA, oB;
        T dA, dB;
        istep(oA, oB, dA, dB);
        accumulate1(oA, oB, dA, dB);
      }
      flush();
      // back to the general step at plane qb
      fa = (T)qb;
      tp = (T)qb;
      sync();
      general(qhi);
    }
  }
  flush();
  if (hit) {
    l1 = (s1 + c1) * ry.La;
    l2 = (s2 + c2) * ry.La;
  }
}

// ---------------------------------------------------------------------------
// Per-ray polyenergetic mean and weights
// ---------------------------------------------------------------------------
template <typename T>
__device__ void energy_sums(const EBin<T>* __restrict__ eb, int nE, T l1, T l2, T g[2],
                            T a[2][2]) {
  T S[6] = {0, 0, 0, 0, 0, 0}, C[6] = {0, 0, 0, 0, 0, 0};
  T k1, k2;
  bin_args(l1, l2, k1, k2);
  for (int e0 = 0; e0 < nE; e0 += 8) {  // nE is padded to a multiple of 8
    T p[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const EBin<T> B = eb[e0 + e];
      const T ex = bin_att(B.mu1, B.mu2, k1, k2);
      p[0] = fma(B.i0l, ex, p[0]);
      p[1] = fma(B.i0h, ex, p[1]);
      p[2] = fma(B.m1l, ex, p[2]);
      p[3] = fma(B.m2l, ex, p[3]);
      p[4] = fma(B.m1h, ex, p[4]);
      p[5] = fma(B.m2h, ex, p[5]);
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) neumaier(S[i], C[i], p[i]);
  }
  g[0] = S[0] + C[0];
  g[1] = S[1] + C[1];
  a[0][0] = S[2] + C[2];  // sum_E mu1 q_L
  a[1][0] = S[3] + C[3];  // sum_E mu2 q_L
  a[0][1] = S[4] + C[4];  // sum_E mu1 q_H
  a[1][1] = S[5] + C[5];  // sum_E mu2 q_H
}

// energy_sums plus the second moments m[j] = (sum_E mu1^2 q_j, sum_E mu1 mu2 q_j,
// sum_E mu2^2 q_j) of both spectra
template <typename T>
__device__ void energy_sums2(const EBin<T>* __restrict__ eb, int nE, T l1, T l2, T g[2],
                             T a[2][2], T m[2][3]) {
  T S[12], C[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) S[i] = C[i] = 0;
  T k1, k2;
  bin_args(l1, l2, k1, k2);
  for (int e0 = 0; e0 < nE; e0 += 8) {
    T p[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) p[i] = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const EBin<T> B = eb[e0 + e];
      const T ex = bin_att(B.mu1, B.mu2, k1, k2);
      p[0] = fma(B.i0l, ex, p[0]);
      p[1] = fma(B.i0h, ex, p[1]);
      p[2] = fma(B.m1l, ex, p[2]);
      p[3] = fma(B.m2l, ex, p[3]);
      p[4] = fma(B.m1h, ex, p[4]);
      p[5] = fma(B.m2h, ex, p[5]);
      p[6] = fma(B.mu1 * B.m1l, ex, p[6]);
      p[7] = fma(B.mu1 * B.m2l, ex, p[7]);
      p[8] = fma(B.mu2 * B.m2l, ex, p[8]);
      p[9] = fma(B.mu1 * B.m1h, ex, p[9]);
      p[10] = fma(B.mu1 * B.m2h, ex, p[10]);
      p[11] = fma(B.mu2 * B.m2h, ex, p[11]);
    }
#pragma unroll
    for (int i = 0; i < 12; ++i) neumaier(S[i], C[i], p[i]);
  }
  g[0] = S[0] + C[0];
  g[1] = S[1] + C[1];
  a[0][0] = S[2] + C[2];
  a[1][0] = S[3] + C[3];
  a[0][1] = S[4] + C[4];
  a[1][1] = S[5] + C[5];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    m[0][i] = S[6 + i] + C[6 + i];
    m[1][i] = S[9 + i] + C[9 + i];
  }
}

// I-divergence term d ln(d/g) - d + g, written as g((1+rho) ln(1+rho) - rho)
// with rho = (d - g)/g so that it does not cancel when d is close to g.
__device__ __forceinline__ double idiv_term(double d, double g) {
  if (!(g > 0.0)) return 0.0;
  if (d <= 0.0) return g;
  const double rho = (d - g) / g;
  return g * ((1.0 + rho) * log1p(rho) - rho);
}

__device__ __forceinline__ double nll_term(double d, double g) {
  if (!(g > 0.0)) return 0.0;
  return d > 0.0 ? g - d * log(g) : g;
}

// Weights and objective term of one ray.  Returns |w| per channel in wabs.
template <typename T, int MODE>
__device__ void poly_epilogue(const EBin<T>* __restrict__ eb, int nE, T l1, T l2, int64_t ray,
                              int64_t R, const float* __restrict__ d,
                              const uint8_t* __restrict__ mask, const T* __restrict__ v,
                              T* __restrict__ w, T* __restrict__ gout, double& term, T wabs[4],
                              const uint32_t* __restrict__ mbits = nullptr) {
  T g[2], a[2][2];
  [[maybe_unused]] T m[2][3];
  if constexpr (MODE == PM_STEP)
    energy_sums2<T>(eb, nE, l1, l2, g, a, m);
  else
    energy_sums<T>(eb, nE, l1, l2, g, a);
  // the trace: one byte per ray, or (mbits) one bit per ray, bit (ray % 32) of word ray / 32
  const bool metal = mbits ? ((mbits[ray >> 5] >> (ray & 31)) & 1u) != 0
                           : (mask != nullptr && mask[ray] != 0);
  if (gout) {
    gout[ray] = g[0];
    gout[R + ray] = g[1];
  }
  if constexpr (MODE == PM_STEP) {
    // lambda_k = sum_i alpha_i dw~_i/dl_k + beta_i dw^_i/dl_k with
    //   dw~_i/dl_k = sum_j (d_j/g_j^2) a_kj a_ij [off the trace] - r_j m_ik^j
    //   dw^_i/dl_k = -sum_j m_ik^j      (m_ik^j = m[j][i + k])
    const T dj[2] = {(T)d[ray], (T)d[R + ray]};
    const T al[2] = {v[ray], v[R + ray]}, be[2] = {v[2 * R + ray], v[3 * R + ray]};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      T lam = 0;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        T dwt = 0, dwh = 0;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const T gj = g[j], mm = m[j][i + k];
          const T r = metal ? (T)1 : (gj > (T)0 ? dj[j] / gj : (T)0);
          if (!metal && gj > (T)0) dwt += dj[j] / (gj * gj) * a[k][j] * a[i][j];
          if (metal || gj > (T)0) dwt -= r * mm;
          dwh -= mm;
        }
        lam = fma(al[i], dwt, fma(be[i], dwh, lam));
      }
      w[(int64_t)k * R + ray] = lam;
      wabs[k] = fabs(lam);
    }
    term = 0.0;
    return;
  } else if constexpr (MODE == PM_VJP) {
    const T vl = v[ray], vh = v[R + ray];
    const T u1 = -(vl * a[0][0] + vh * a[0][1]);
    const T u2 = -(vl * a[1][0] + vh * a[1][1]);
    w[ray] = u1;
    w[R + ray] = u2;
    wabs[0] = fabs(u1);
    wabs[1] = fabs(u2);
    term = 0.0;
    return;
  } else {
    const float dl = d[ray], dh = d[R + ray];
    // r_j = d_j / g_j off the trace, 1 on it (p = q); r_j a_ij := 0 when g_j = 0
    T rl = 1, rh = 1;
    if (!metal) {
      rl = g[0] > (T)0 ? (T)dl / g[0] : (T)0;
      rh = g[1] > (T)0 ? (T)dh / g[1] : (T)0;
    }
    if constexpr (MODE == PM_AM) {
      const T wt1 = fma(rl, a[0][0], rh * a[0][1]);
      const T wt2 = fma(rl, a[1][0], rh * a[1][1]);
      const T wh1 = a[0][0] + a[0][1];
      const T wh2 = a[1][0] + a[1][1];
      w[ray] = metal ? wh1 : wt1;
      w[R + ray] = metal ? wh2 : wt2;
      w[2 * R + ray] = wh1;
      w[3 * R + ray] = wh2;
      wabs[0] = metal ? wh1 : wt1;
      wabs[1] = metal ? wh2 : wt2;
      wabs[2] = wh1;
      wabs[3] = wh2;
      term = metal ? 0.0 : idiv_term(dl, (double)g[0]) + idiv_term(dh, (double)g[1]);
    } else {  // PM_GRAD: u_i = sum_j (r_j - 1) a_ij
      const T u1 = metal ? (T)0 : fma(rl - 1, a[0][0], (rh - 1) * a[0][1]);
      const T u2 = metal ? (T)0 : fma(rl - 1, a[1][0], (rh - 1) * a[1][1]);
      w[ray] = u1;
      w[R + ray] = u2;
      wabs[0] = fabs(u1);
      wabs[1] = fabs(u2);
      term = metal ? 0.0 : nll_term(dl, (double)g[0]) + nll_term(dh, (double)g[1]);
    }
  }
}

// Weight-maxima map: the lanes of the wave with the same entry (a view, a
// group of rows, a block of channels) take the maximum of their |w_c| and one
// of them raises the entry with atomicMax on the float bits (non-negative).
// A wave's lanes map to at most a few entries; all 64 lanes must call this.
__device__ __forceinline__ void map_update(const WMapDev& M, int64_t entry, const float m[4],
                                           int nch, bool valid) {
  if (!M.map) return;
  const int lane = threadIdx.x & 63;
  unsigned long long todo = __ballot(valid);
  while (todo) {
    const int src = __ffsll(todo) - 1;
    const int lo = __shfl((int)(entry & 0xffffffff), src), hi = __shfl((int)(entry >> 32), src);
    const int64_t e0 = ((int64_t)hi << 32) | (uint32_t)lo;
    const bool sel = valid && entry == e0;
    float mx[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      mx[c] = sel ? m[c] : 0.f;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) mx[c] = fmaxf(mx[c], __shfl_xor(mx[c], o));
    }
    if (lane == src)
      for (int c = 0; c < nch; ++c) atomicMax(&M.map[e0 * 4 + c], __float_as_uint(mx[c]));
    todo &= ~__ballot(sel);
  }
}

__device__ __forceinline__ int64_t map_entry(const WMapDev& M, int v, int r, int k) {
  return ((int64_t)v * M.ngm + r / kMapRows) * M.nkb + k / kMapCols;
}

// Block reduction of the FP64 objective terms into partial[lb] (a fixed
// order), and the map entry of each lane's ray.
template <int NW, int NT = kFpBlock>
__device__ void block_reduce(double term, const float wabs[4], int nch, double* partial, int lb,
                             const WMapDev& M = WMapDev{}, int64_t entry = 0, bool valid = false) {
  map_update(M, entry, wabs, nch, valid);
  __shared__ double s_sum[NT / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) term += __shfl_xor(term, o);
  if (lane == 0) s_sum[wv] = term;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int i = 0; i < NT / 64; ++i) sum += s_sum[i];
    if (partial) partial[lb] = sum;
  }
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
// 2D float plans: eight waves per SIMD (64 VGPRs, no spills)
template <typename T, bool Z3, int MODE>
__global__ __launch_bounds__(kFpBlock) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && !Z3 ? 8 : 1))) void k_fp(
    GeomDev G, const typename Vec2<T>::type* __restrict__ cp, uint32_t xoff,
    const EBin<T>* __restrict__ eb, int nE,
    const float* __restrict__ d, const uint8_t* __restrict__ mask, T* __restrict__ out,
    double* __restrict__ partial, double tthr,
    uint8_t* __restrict__ mask_out, double* __restrict__ Tout, int nout, WMapDev M) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  // rays of the walked views, channel fastest; `ray` is the index in the
  // full sinogram
  const int64_t lray = (int64_t)lb * kFpBlock + threadIdx.x;
  const bool active = lray < (int64_t)G.nvl * G.n_rows * G.n_cols;
  double term = 0.0;
  T wabs[4] = {0, 0, 0, 0};
  int64_t entry = 0;
  {
    const int64_t ra = active ? lray : 0;
    const int k = (int)(ra % G.n_cols);
    const int rv = (int)(ra / G.n_cols);
    const int r = rv % G.n_rows, v = G.voff + G.vsub * (rv / G.n_rows);
    entry = map_entry(M, v, r, k);
    const int64_t ray = ((int64_t)v * G.n_rows + r) * G.n_cols + k;
    T l1, l2;
    const RayXY<T>* rays = (sizeof(T) == 8) ? (const RayXY<T>*)G.rays64 : (const RayXY<T>*)G.rays;
    // all lanes of the wave take part in the walk (lanes past the last ray idle)
    project_ray<T, Z3>(G, rays, cp, xoff, v, r, k, active, l1, l2);
    if (!active) {
    } else if constexpr (MODE == PM_L) {
      out[ray] = l1;
      if (nout > 1) out[G.R + ray] = l2;
    } else if constexpr (MODE == PM_TRACE) {
      if (Tout) Tout[ray] = (double)l1;
      mask_out[ray] = (double)l1 >= tthr ? 1 : 0;
    } else {
      if (G.bowtie) {  // the filter's path in the basis, in front of the energy sums
        const T* bt = (const T*)G.bowtie;
        l1 += bt[k];
        l2 += bt[G.n_cols + k];
      }
      poly_epilogue<T, MODE>(eb, nE, l1, l2, ray, G.R, d, mask, nullptr, out, nullptr, term, wabs,
                             G.mbits);
    }
  }
  if constexpr (MODE == PM_AM || MODE == PM_GRAD) {
    const float wf[4] = {(float)wabs[0], (float)wabs[1], (float)wabs[2], (float)wabs[3]};
    block_reduce<4>(term, wf, MODE == PM_AM ? 4 : 2, partial, lb, M, entry, active);
  }
}

// 3D projector.  The detector rows of one (view, channel) share the in-plane
// path of their rays and differ only in z, so one lane walks the in-plane
// path of a (view, channel) once and gathers RG rows at every plane step:
// the lateral geometry of a step (pixels, split, lengths, gather offsets) is
// computed once for RG line integrals, and each row only finds its slice.
// A wave holds 64 neighbouring channels of one (view, row group), so the
// rows' axial slopes are wave-uniform; the waves of a block take
// consecutive views of the same channels and rows, whose rays lie within
// about a pixel of each other, so that they gather through the same cache
// lines.  Blocks run over the views, then the channel blocks, then the row
// groups.  The lanes of a wave walk the same plane rows together, as in
// project_ray.
// Row j's axial grid coordinate is w_j(a) = w_s + (a - s_a) / d_a * zr_j
// (zr_j = zeta_j / dz); its slice for a step is that of the step's end.  A
// row outside the slices gathers from the zeroed tail of the packed images.
// A step in which a row changes slice is gathered from the new slice by the
// fast walk, recorded in a mask, and corrected later: the exact pieces are
// summed through the general walker and the fast walk's value (recomputed
// with identical arithmetic) is taken away.
template <typename T, int MODE, int RG>
__global__ __launch_bounds__(64 * kFp3Views) void k_fp3(
    GeomDev G, const typename Vec2<T>::type* __restrict__ cp, uint32_t xoff,
    const EBin<T>* __restrict__ eb, int nE,
    const float* __restrict__ d, const uint8_t* __restrict__ mask, T* __restrict__ out,
    double* __restrict__ partial, double tthr,
    uint8_t* __restrict__ mask_out, double* __restrict__ Tout, int nout, WMapDev M) {
  using T2 = typename Vec2<T>::type;
  constexpr uint32_t E = sizeof(T2);
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int NKB = (G.n_cols + 63) >> 6;                           // channel blocks of 64
  const int NVB = (G.nvl + kFp3Views - 1) / kFp3Views;            // view blocks
  const int vb = lb % NVB, kb = (lb / NVB) % NKB, g = lb / (NVB * NKB);
  const int vi = vb * kFp3Views + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int k = kb * 64 + (int)(threadIdx.x & 63);
  const bool valid = vi < G.nvl && k < G.n_cols;
  const int v = G.voff + G.vsub * min(vi, G.nvl - 1);           // a walked view
  const int r0 = g * RG;
  const RayXY<T>* __restrict__ rays =
      (sizeof(T) == 8) ? (const RayXY<T>*)G.rays64 : (const RayXY<T>*)G.rays;
  RayXY<T> t{};
  if (valid) t = rays[(int64_t)v * G.n_cols + k];
  const bool yd = t.yd != (T)0;
  const int nb = yd ? G.nx : G.ny, na = yd ? G.ny : G.nx;
  // lateral pixels are counted from the ray's origin t.ib (see RayXY):
  // [blo, bhi] is the grid's lateral range in that frame
  const int ib = (int)t.ib;
  const int blo = -ib, bhi = nb - 1 - ib;
  const uint32_t base = yd ? 0u : xoff;
  const uint32_t plane = (uint32_t)G.nx * (uint32_t)G.ny;
  const uint32_t pstep = plane * E, rstep = (uint32_t)nb * E;
  // offset from a lane's in-plane address to the zeroed tail after both copies
  const uint32_t zoff0 = (2u * (uint32_t)G.V - base) * E;
  const int vs = min(v, G.n_views - 1);
  const T sw = (T)G.view[4 * vs + 3];
  T zr[RG], Lr[RG];
#pragma unroll
  for (int j = 0; j < RG; ++j) {
    const int r = min(r0 + j, G.n_rows - 1);
    zr[j] = (T)G.row[4 * r];
    Lr[j] = (T)G.row[4 * r + 1];
  }
  // in-plane clip to the x-y extent of the grid
  T alo = 0, ahi = (T)na;
  bool hit = valid;
  if (t.mb != (T)0) {
    const T t0 = ((T)blo - t.b0) * t.imb, t1 = ((T)(bhi + 1) - t.b0) * t.imb;
    alo = fmax(alo, fmin(t0, t1));
    ahi = fmin(ahi, fmax(t0, t1));
  } else if (!(t.b0 >= (T)blo && t.b0 < (T)(bhi + 1))) {
    hit = false;
  }
  hit = hit && ahi > alo;
  if (!hit) {
    alo = 0;
    ahi = 0;
  }
  const int nzz = G.nz;
  auto slice_off = [&](int D) -> uint32_t {
    return (D >= 0 && D < nzz) ? (uint32_t)D * pstep : zoff0;
  };
  const char* __restrict__ cpb = (const char*)cp;
  T s1[RG], c1[RG], s2[RG], c2[RG], p1[RG], p2[RG];
  int C[RG];
  uint32_t zo[RG], rest[RG];
  T tp = alo;
  T bp = fma(tp, t.mb, t.b0);
  int A = clampi(ifloor(bp), blo, bhi);
  {
    const T u = (tp - t.sa) * t.ida;
#pragma unroll
    for (int j = 0; j < RG; ++j) {
      s1[j] = c1[j] = s2[j] = c2[j] = p1[j] = p2[j] = 0;
      C[j] = ifloor(fma(u, zr[j], sw));
      zo[j] = slice_off(C[j]);
      rest[j] = 0u;
    }
  }
  const int q0 = hit ? ifloor(alo) : (1 << 30);
  const int q1 = hit ? -ifloor(-ahi) : -(1 << 30);
  const int qlo = wave_min(q0), qhi = wave_max(q1);
  T iLa[RG];
#pragma unroll
  for (int j = 0; j < RG; ++j) iLa[j] = (T)1 / (Lr[j] * fabs(t.ida));

  if (qlo < qhi) {
    T fa = (T)qlo;
    // byte offset of lateral pixel 0 of the ray's frame (the unsigned sums
    // with a negative relative pixel wrap to the true offsets)
    uint32_t row = (base + (uint32_t)qlo * (uint32_t)nb + (uint32_t)ib) * E;
    int qw = qlo;
    // the fast walk's lengths and offsets of plane step q (identical
    // arithmetic to the walk itself)
    auto step_geom = [&](int q, T& dA, T& dB, uint32_t& oA, uint32_t& oB, T& tn) {
      const T ta = clampf((T)q, alo, ahi);
      tn = clampf((T)(q + 1), alo, ahi);
      const T ba = fma(ta, t.mb, t.b0), bn = fma(tn, t.mb, t.b0);
      const int Aq = clampi(ifloor(ba), blo, bhi), Bq = clampi(ifloor(bn), blo, bhi);
      const T ds = tn - ta;
      dA = (Bq == Aq) ? ds : clamp0(((T)max(Aq, Bq) - ba) * t.imb, ds);
      dB = ds - dA;
      const uint32_t rq = (base + (uint32_t)q * (uint32_t)nb + (uint32_t)ib) * E;
      oA = rq + (uint32_t)Aq * E;
      oB = rq + (uint32_t)Bq * E;
    };
    auto fixup = [&]() {
#pragma unroll
      for (int j = 0; j < RG; ++j) {
        if (rest[j] == 0u) continue;
        // row j's ray clipped to the whole grid
        Ray<T> ry{};
        ry.b0 = t.b0;
        ry.mb = t.mb;
        ry.imb = t.imb;
        ry.mw = zr[j] * t.ida;
        ry.w0 = sw - t.sa * ry.mw;
        const T rmw = ry.mw != (T)0 ? (T)1 / ry.mw : (T)0;
        ry.imw = fabs(rmw);
        ry.La = Lr[j] * fabs(t.ida);
        ry.Lb = Lr[j] * t.iadb;
        ry.alo = alo;
        ry.ahi = ahi;
        ry.ydrive = yd ? 1 : 0;
        ry.ib = ib;
        if (ry.mw != (T)0) {
          const T z0 = ((T)0 - ry.w0) * rmw, z1 = ((T)nzz - ry.w0) * rmw;
          ry.alo = fmax(ry.alo, fmin(z0, z1));
          ry.ahi = fmin(ry.ahi, fmax(z0, z1));
        } else if (!(ry.w0 >= (T)0 && ry.w0 < (T)nzz)) {
          ry.ahi = ry.alo;
        }
        T e1 = 0, e2 = 0;
        auto visit = [&](int ia, int jb, int iw, T h) {
          const T2 cv = cp[base + (uint32_t)iw * plane + (uint32_t)ia * (uint32_t)nb +
                           (uint32_t)(jb + ib)];
          e1 = fma(h * iLa[j], cv.x, e1);
          e2 = fma(h * iLa[j], cv.y, e2);
        };
        while (rest[j] != 0u) {
          const int bit = __ffs(rest[j]) - 1;
          rest[j] &= rest[j] - 1u;
          const int q = qw + bit;
          T dA, dB, tn;
          uint32_t oA, oB;
          step_geom(q, dA, dB, oA, oB, tn);
          const uint32_t z = slice_off(ifloor(fma((tn - t.sa) * t.ida, zr[j], sw)));
          const T2 vA = *(const T2*)(cpb + (uint32_t)(oA + z));
          const T2 vB = *(const T2*)(cpb + (uint32_t)(oB + z));
          e1 -= fma(dA, vA.x, dB * vB.x);
          e2 -= fma(dA, vA.y, dB * vB.y);
          walk_row<T, true, false>(ry, q, blo, bhi + 1, 0, nzz, visit);
        }
        p1[j] += e1;
        p2[j] += e2;
      }
    };
    int nstep = 0;
    for (int q = qlo; q < qhi; ++q) {
      fa += (T)1;
      const T tn = clampf(fa, alo, ahi);
      const T bn = fma(tn, t.mb, t.b0);
      const int B = clampi(ifloor(bn), blo, bhi);
      const T ds = tn - tp;
      const T dA = (B == A) ? ds : clamp0(((T)max(A, B) - bp) * t.imb, ds);
      const T dB = ds - dA;
      const uint32_t oA = row + (uint32_t)A * E, oB = row + (uint32_t)B * E;
      row += rstep;
      const T un = (tn - t.sa) * t.ida;
#pragma unroll
      for (int j = 0; j < RG; ++j) {
        const int D = ifloor(fma(un, zr[j], sw));
        if (D != C[j]) {
          rest[j] |= 1u << (q - qw);
          C[j] = D;
          zo[j] = slice_off(D);
        }
      }
      // one 32-bit offset from the uniform base (SGPR-based addressing).
      // Float plans: the two pixels are neighbours in one row, so one 16-byte
      // load at the lower offset fetches both, and the two lengths are matched
      // to the lower and upper pixel once for all rows (when A = B the upper
      // length is 0).  The element after the lower pixel is the next one in
      // its row, the first of the next row or copy, or, for a row outside the
      // slices, an element of the zeroed tail, which is sized for the pixel
      // after the last one a lane can address (packed_tail_elems): finite
      // and in bounds)
      if constexpr (sizeof(T) == 4) {
        const uint32_t om = min(oA, oB);
        const bool al = oA <= oB;
        const T dl = al ? dA : dB, dh = al ? dB : dA;
        Pix2f v2[RG];
#pragma unroll
        for (int j = 0; j < RG; ++j) v2[j] = *(const Pix2f*)(cpb + (uint32_t)(om + zo[j]));
#pragma unroll
        for (int j = 0; j < RG; ++j) {
          p1[j] = fma(dl, v2[j].x, fma(dh, v2[j].z, p1[j]));
          p2[j] = fma(dl, v2[j].y, fma(dh, v2[j].w, p2[j]));
        }
      } else {
        T2 vA[RG], vB[RG];
#pragma unroll
        for (int j = 0; j < RG; ++j) {
          vA[j] = *(const T2*)(cpb + (uint32_t)(oA + zo[j]));
          vB[j] = *(const T2*)(cpb + (uint32_t)(oB + zo[j]));
        }
#pragma unroll
        for (int j = 0; j < RG; ++j) {
          p1[j] = fma(dA, vA[j].x, fma(dB, vB[j].x, p1[j]));
          p2[j] = fma(dA, vA[j].y, fma(dB, vB[j].y, p2[j]));
        }
      }
      A = B;
      bp = bn;
      tp = tn;
      ++nstep;
      if ((nstep & 15) == 0) {
#pragma unroll
        for (int j = 0; j < RG; ++j) {
          neumaier(s1[j], c1[j], p1[j]);
          neumaier(s2[j], c2[j], p2[j]);
          p1[j] = 0;
          p2[j] = 0;
        }
      }
      if ((nstep & 31) == 0) {
        fixup();
        qw = q + 1;
      }
    }
    fixup();
  }

  double term = 0.0;
  T wabs[4] = {0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < RG; ++j) {
    neumaier(s1[j], c1[j], p1[j]);
    neumaier(s2[j], c2[j], p2[j]);
    const int r = r0 + j;
    if (!valid || r >= G.n_rows) continue;
    const T La = Lr[j] * fabs(t.ida);
    const T l1 = hit ? (s1[j] + c1[j]) * La : (T)0;
    const T l2 = hit ? (s2[j] + c2[j]) * La : (T)0;
    const int64_t ray = ((int64_t)v * G.n_rows + r) * G.n_cols + k;
    if constexpr (MODE == PM_L) {
      out[ray] = l1;
      if (nout > 1) out[G.R + ray] = l2;
    } else if constexpr (MODE == PM_TRACE) {
      if (Tout) Tout[ray] = (double)l1;
      mask_out[ray] = (double)l1 >= tthr ? 1 : 0;
    } else {
      double tj = 0.0;
      T wj[4] = {0, 0, 0, 0};
      T o1 = 0, o2 = 0;
      if (G.bowtie) {  // the filter's path in the basis, in front of the energy sums
        const T* bt = (const T*)G.bowtie;
        o1 = bt[k];
        o2 = bt[G.n_cols + k];
      }
      poly_epilogue<T, MODE>(eb, nE, l1 + o1, l2 + o2, ray, G.R, d, mask, nullptr, out, nullptr,
                             tj, wj, G.mbits);
      term += tj;
#pragma unroll
      for (int c = 0; c < 4; ++c) wabs[c] = fmax(wabs[c], wj[c]);
    }
  }
  if constexpr (MODE == PM_AM || MODE == PM_GRAD) {
    const float wf[4] = {(float)wabs[0], (float)wabs[1], (float)wabs[2], (float)wabs[3]};
    // the lane's rows r0 .. r0 + RG - 1 lie in one group of the map (RG divides it)
    static_assert(kMapRows % RG == 0, "row groups of the map hold whole row groups of the walk");
    block_reduce<4, 64 * kFp3Views>(term, wf, MODE == PM_AM ? 4 : 2, partial, lb, M,
                                     map_entry(M, v, r0, k), valid);
  }
}

template <typename T, int MODE>
__global__ __launch_bounds__(kFpBlock) void k_poly(
    int64_t R, const EBin<T>* __restrict__ eb, int nE, const T* __restrict__ l,
    const float* __restrict__ d, const uint8_t* __restrict__ mask, const T* __restrict__ v,
    T* __restrict__ w, T* __restrict__ gout, double* __restrict__ partial,
    int n_cols, const T* __restrict__ bt, WMapDev M) {
  const int64_t ray = (int64_t)blockIdx.x * kFpBlock + threadIdx.x;
  double term = 0.0;
  T wabs[4] = {0, 0, 0, 0};
  if (ray < R) {
    T l1 = l[ray], l2 = l[R + ray];
    if (bt) {  // bowtie: the filter's path in the basis, per channel
      const int k = (int)(ray % n_cols);
      l1 += bt[k];
      l2 += bt[n_cols + k];
    }
    poly_epilogue<T, MODE>(eb, nE, l1, l2, ray, R, d, mask, v, w, gout, term, wabs);
  }
  const float wf[4] = {(float)wabs[0], (float)wabs[1], (float)wabs[2], (float)wabs[3]};
  const int64_t rr = ray < R ? ray : 0;
  const int64_t vr = rr / M.n_cols;
  const int64_t entry =
      map_entry(M, (int)(vr / M.n_rows), (int)(vr % M.n_rows), (int)(rr % M.n_cols));
  block_reduce<4>(term, wf, MODE == PM_AM ? 4 : 2, partial, blockIdx.x, M, entry, ray < R);
}

// max |w_c| over rays, per channel (for the fixed-point scale of a
// backprojection of arbitrary weights).
template <typename T>
__global__ __launch_bounds__(kFpBlock) void k_absmax(int64_t R, int nch, const T* __restrict__ w,
                                                     WMapDev M) {
  const int64_t ray = (int64_t)blockIdx.x * kFpBlock + threadIdx.x;
  float m[4] = {0.f, 0.f, 0.f, 0.f};
  const int64_t rr = ray < R ? ray : 0;
  if (ray < R)
    for (int c = 0; c < nch; ++c) m[c] = (float)fabs(w[c * R + ray]);
  const int64_t vr = rr / M.n_cols;
  map_update(M, map_entry(M, (int)(vr / M.n_rows), (int)(vr % M.n_rows), (int)(rr % M.n_cols)),
             m, nch, ray < R);
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Deterministic FP64 sum of n partials into out[0] (one block of 1024).
__global__ __launch_bounds__(1024) void k_reduce(const double* __restrict__ p, int64_t n,
                                                 double* __restrict__ out) {
  __shared__ double s[1024];
  double acc = 0.0, cmp = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) neumaier(acc, cmp, p[i]);
  s[threadIdx.x] = acc + cmp;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0];
}

// ---------------------------------------------------------------------------
// Backprojection: tile-owned, fixed point in LDS
// ---------------------------------------------------------------------------
// Fixed point: one signed 64-bit word per voxel and channel holding the sum
// of round(h * w_c * s_c).  max|w_c| below is the tile's own bound: the
// largest |w_c| of the rays that can meet the tile (k_tile_max).
//  * FP32 plans: s_c = (2^31 - 2^11) / (hmax * max|w_c|), hmax = the voxel
//    diagonal (no segment is longer), so every term fits a signed 32-bit
//    integer and converts with one instruction: the FP32 roundings of s_c,
//    of w_c s_c L_a and of the final product (at most 4 units of 2^-24)
//    raise the largest term by at most 2^31 * 2^-22 = 512 < 2^11.  The
//    resolution is 2^-31 of the largest possible term, below the FP32
//    rounding of the product for all but terms 2^8 times smaller than the
//    largest, and sums of up to 2^32 terms cannot overflow 64 bits.
//  * FP64 plans: s_c = 2^61 / (h1 * max|w_c|), h1 >= max_x sum_y h(x,y), so
//    every partial sum stays below 2^61 + (number of additions)/2 < 2^63; a
//    term (< 2^52) is split exactly into two 32-bit halves.
// Integer sums are exact, so the result does not depend on the order of the
// additions.
__device__ __forceinline__ unsigned long long to_fixed(float x) {
  const int q = (int)rintf(x);          // |x| < 2^31 by the choice of the scale
  return (unsigned long long)(long long)q;
}

// Non-negative terms (the AM weights): round half up with one FMA.
__device__ __forceinline__ unsigned long long to_fixed_nonneg(float h, float ws) {
  return (unsigned long long)(uint32_t)fmaf(h, ws, 0.5f);
}

__device__ __forceinline__ unsigned long long to_fixed(double x) {
  const double ax = fabs(x) + 0.5;                        // round half away from zero
  const double hi = floor(ax * 2.3283064365386963e-10);   // 2^-32, exact scaling
  const double lo = fma(-hi, 4294967296.0, ax);           // ax - hi*2^32, exact
  unsigned long long q = ((unsigned long long)(uint32_t)hi << 32) | (unsigned long long)(uint32_t)lo;
  return x < 0.0 ? (unsigned long long)(-(long long)q) : q;
}

// Non-negative FP64 terms (the AM weights), kept below 2^51 by their scale:
// x + 2^52 lies in [2^52, 2^53), where the doubles are the integers, so the
// addition rounds x to the nearest integer (ties to even) and leaves it in
// the low 52 bits of the result.
__device__ __forceinline__ unsigned long long to_fixed_nonneg(double x) {
  return (unsigned long long)__double_as_longlong(x + 4503599627370496.0) & 0x000FFFFFFFFFFFFFull;
}

// View set-up of a tile for one batch of VB views (all threads of
// the block take part; three barriers).  For every view of the batch: the
// channels [kl, kl + nk) whose rays can meet the tile, from the channel
// coordinates of the tile's corners, and the detector rows [rl, rl + nr)
// whose rays can meet its slices, from its z-range and its distance to the
// source; s_off receives the exclusive prefix sum of the work items per view,
// nk * ceil(nr / RG).
// Channel coordinate (fractional channel index) of the ray of view v through
// the point (px, py) (mm).
__device__ __forceinline__ float channel_coord(const GeomDev& G, int v, double px, double py) {
  const double cb = G.view[4 * v], sb = G.view[4 * v + 1];
  const double qx = px - G.sid * cb, qy = py - G.sid * sb;
  const float cr = (float)(-cb * qy + sb * qx), dt = (float)(-cb * qx - sb * qy);
  return atan2f(cr, dt) / (float)G.dgamma + (float)G.kc;
}

// Detector rows [rl, rh] of view v whose rays can meet the slab [Z0, Z1] of
// the box [X0, X1] x [Y0, Y1] (3D; from its distance to the source).
__device__ __forceinline__ void slab_rows(const GeomDev& G, int v, double X0, double X1, double Y0,
                                          double Y1, double Z0, double Z1, int& rl, int& rh) {
  const double sx = G.sid * G.view[4 * v], sy = G.sid * G.view[4 * v + 1];
  const double zs = G.view[4 * v + 2];
  const double cx = fmin(fmax(sx, X0), X1), cy = fmin(fmax(sy, Y0), Y1);
  const double dmin = fmax(sqrt((sx - cx) * (sx - cx) + (sy - cy) * (sy - cy)), 1e-6);
  const double fx = fmax(fabs(sx - X0), fabs(sx - X1)), fy = fmax(fabs(sy - Y0), fabs(sy - Y1));
  const double dmax = sqrt(fx * fx + fy * fy);
  const double za = (Z0 - zs) * G.sdd, zb = (Z1 - zs) * G.sdd;
  const double q0 = za / dmin, q1 = za / dmax, q2 = zb / dmin, q3 = zb / dmax;
  const double zmn = fmin(fmin(q0, q1), fmin(q2, q3)), zmx = fmax(fmax(q0, q1), fmax(q2, q3));
  rl = max((int)ceil(zmn / G.dzeta + G.rc - 1e-3), 0);
  rh = min(ifloor(zmx / G.dzeta + G.rc + 1e-3), G.n_rows - 1);
}

template <int RG, int VB>
__device__ __forceinline__ void cull_views(const GeomDev& G, int vb0, double X0, double X1,
                                           double Y0, double Y1, double Z0, double Z1,
                                           float (*s_kap)[4], int* s_kl, int* s_nk, int* s_rl,
                                           int* s_nr, int* s_off) {
  static_assert(VB % 64 == 0, "the prefix sum runs over whole waves of views");
  for (int i = threadIdx.x; i < 4 * VB; i += blockDim.x) {
    const int j = i >> 2, cn = i & 3;
    const int v = G.voff + G.vsub * (vb0 + j);
    float kap = 0.f;
    if (vb0 + j < G.nvl) kap = channel_coord(G, v, (cn & 1) ? X1 : X0, (cn & 2) ? Y1 : Y0);
    s_kap[j][cn] = kap;
  }
  __syncthreads();
  // channel and row ranges of each view
  for (int j = threadIdx.x; j < VB; j += blockDim.x) {
    const int v = G.voff + G.vsub * (vb0 + j);
    int kl = 0, nk = 0, rl = 0, nr = 0;
    if (vb0 + j < G.nvl) {
      const float kmn = fminf(fminf(s_kap[j][0], s_kap[j][1]), fminf(s_kap[j][2], s_kap[j][3]));
      const float kmx = fmaxf(fmaxf(s_kap[j][0], s_kap[j][1]), fmaxf(s_kap[j][2], s_kap[j][3]));
      kl = max((int)ceilf(kmn - 0.01f), 0);
      const int kh = min((int)floorf(kmx + 0.01f), G.n_cols - 1);
      nk = max(kh - kl + 1, 0);
      if (G.is3d) {
        int rh;
        slab_rows(G, v, X0, X1, Y0, Y1, Z0, Z1, rl, rh);
        nr = max(rh - rl + 1, 0);
      } else {
        nr = 1;
      }
    }
    s_kl[j] = kl;
    s_nk[j] = nk;
    s_rl[j] = rl;
    s_nr[j] = nr;
  }
  __syncthreads();
  // exclusive prefix sum of the item counts (one wave, 64 views at a time)
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    int carry = 0;
    if (lane == 0) s_off[0] = 0;
#pragma unroll
    for (int c = 0; c < VB; c += 64) {
      int run = s_nk[c + lane] * ((s_nr[c + lane] + RG - 1) / RG);
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(run, d);
        if (lane >= d) run += u;
      }
      run += carry;
      s_off[c + lane + 1] = run;
      carry = __shfl(run, 63);
    }
  }
  __syncthreads();
}

// Weight bound of every backprojector tile: the largest |w_c| (c < nch) over
// the map entries of the rays that can meet the tile, one block per tile
// (the tile index is the backprojector's logical one).  The channel and row
// ranges are those of cull_views widened by one, so they hold every ray the
// tile walks.
__global__ __launch_bounds__(256) void k_tile_max(GeomDev G, Tiling TL, WMapDev M, int nch,
                                                  float* __restrict__ tmax) {
  const int t = blockIdx.x;
  const int tix = t % TL.ntx, tiy = (t / TL.ntx) % TL.nty, tiz = t / (TL.ntx * TL.nty);
  const int tx0 = tix * TL.tx, ty0 = tiy * TL.ty, tz0 = tiz * TL.tz;
  const int tx1 = min(tx0 + TL.tx, G.nx), ty1 = min(ty0 + TL.ty, G.ny);
  const int tz1 = min(tz0 + TL.tz, G.is3d ? G.nz : 1);
  const double X0 = G.x0 + tx0 * G.dx, X1 = G.x0 + tx1 * G.dx;
  const double Y0 = G.y0 + ty0 * G.dy, Y1 = G.y0 + ty1 * G.dy;
  const double Z0 = G.z0 + tz0 * G.dz, Z1 = G.z0 + tz1 * G.dz;
  uint32_t m[4] = {0u, 0u, 0u, 0u};
  for (int i = threadIdx.x; i < G.nvl; i += 256) {
    const int v = G.voff + G.vsub * i;
    float kmn = 1e30f, kmx = -1e30f;
#pragma unroll
    for (int cn = 0; cn < 4; ++cn) {
      const float kap = channel_coord(G, v, (cn & 1) ? X1 : X0, (cn & 2) ? Y1 : Y0);
      kmn = fminf(kmn, kap);
      kmx = fmaxf(kmx, kap);
    }
    const int kl = max((int)ceilf(kmn - 0.01f) - 1, 0);
    const int kh = min((int)floorf(kmx + 0.01f) + 1, G.n_cols - 1);
    int rl = 0, rh = 0;
    if (G.is3d) {
      slab_rows(G, v, X0, X1, Y0, Y1, Z0, Z1, rl, rh);
      rl = max(rl - 1, 0);
      rh = min(rh + 1, G.n_rows - 1);
    }
    if (kl > kh || rl > rh) continue;
    for (int gr = rl / kMapRows; gr <= rh / kMapRows; ++gr)
      for (int kb = kl / kMapCols; kb <= kh / kMapCols; ++kb) {
        const uint32_t* e = M.map + (((int64_t)v * M.ngm + gr) * M.nkb + kb) * 4;
        for (int c = 0; c < nch; ++c) m[c] = max(m[c], e[c]);
      }
  }
  // block maximum (bit patterns of non-negative floats order as the floats)
  __shared__ uint32_t s_m[4][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m[c] = max(m[c], (uint32_t)__shfl_xor((int)m[c], o));
    if (lane == 0) s_m[wv][c] = m[c];
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int c = threadIdx.x;
    const uint32_t x = max(max(s_m[0][c], s_m[1][c]), max(s_m[2][c], s_m[3][c]));
    tmax[(int64_t)t * 4 + c] = __uint_as_float(x);
  }
}

// One backprojector for both geometries.  A workgroup owns a tile of
// BpTile<Z3, NCH, PK, SM> voxels in LDS and scatters every ray that meets it, view
// batch by view batch; work items are (view, detector row, channel) with the
// channel fastest, so neighbouring lanes walk neighbouring rays.
//
// Each lane walks its ray through the tile one plane step of the driving
// axis at a time, carrying the lateral pixel and coordinate from the end of
// the previous step: a step costs one lateral floor, and splits into at most
// two segments (pixel A, then pixel B after the lateral plane crossing).
// Lengths are kept in units of the driving axis; the weights carry the mm per
// unit.  In 3D the rare steps that cross an axial plane (or leave the tile's
// slices) are only flagged in a bit mask during the walk and scattered
// afterwards through the general walk_row, so that the lanes of a wave stay
// on the common path.
template <typename T, bool Z3, int NCH, bool NONNEG, bool SM>
__global__ __launch_bounds__((bp_block<Z3, SM, NONNEG && sizeof(T) == 4 && NCH == 4>())) __attribute__((amdgpu_waves_per_eu(4))) void k_bp(GeomDev G, Tiling TL, const T* __restrict__ w,
                                                 const float* __restrict__ tmax, double h1,
                                                 double hmax, T* __restrict__ b,
                                                 const float* __restrict__ hbt,
                                                 float* __restrict__ hbt_out, double nterm) {
  // Packed accumulation (float plans, the 4 non-negative AM channels): the
  // LDS word of a voxel holds two channels as 32-bit halves, so one atomic
  // adds two terms.  The scale is chosen so that the sum over one view batch
  // stays below 2^32 in each half (no carry into the upper half); after every
  // batch each thread moves the words it owns into 64-bit register totals.
  constexpr bool PK = NONNEG && sizeof(T) == 4 && NCH == 4;
  using BT = BpTile<Z3, NCH, PK, SM>;
  constexpr int RS = BT::tx + 1;       // padded row stride (words)
  constexpr int TXY = RS * BT::ty;     // words per slice
  constexpr int NVOX = TXY * BT::tz;   // words per channel (pair of channels when PK)
  constexpr int NW = NVOX * BT::wpv;   // LDS words
  constexpr int NT = BT::block;         // threads per tile
  constexpr int NOWN = PK ? (NW + NT - 1) / NT : 1;
  static_assert(BT::tx <= 32 && BT::ty <= 32, "deferred steps live in a 32-bit mask");
  extern __shared__ unsigned long long acc[];
  constexpr int VB = kViewBatch;
  __shared__ float s_kap[VB][4];
  __shared__ int s_kl[VB], s_nk[VB], s_rl[VB], s_nr[VB];
  __shared__ int s_off[VB + 1];
  const RayXY<T>* __restrict__ rays =
      (sizeof(T) == 8) ? (const RayXY<T>*)G.rays64 : (const RayXY<T>*)G.rays;

  // tiles in row-major order; each XCD gets a contiguous band of them, so the
  // rays a tile reads are mostly read by other tiles of the same L2
  const int t = xcd_block(blockIdx.x, gridDim.x);
  const int tix = t % TL.ntx, tiy = (t / TL.ntx) % TL.nty, tiz = t / (TL.ntx * TL.nty);
  const int tx0 = tix * BT::tx, ty0 = tiy * BT::ty, tz0 = tiz * BT::tz;
  const int tx1 = min(tx0 + BT::tx, G.nx), ty1 = min(ty0 + BT::ty, G.ny);
  const int tz1 = min(tz0 + BT::tz, G.is3d ? G.nz : 1);
  // LDS layout acc[c][z][y][x], row stride tx + 1 words: lanes walking
  // neighbouring rays of one view (neighbouring x for rays driven along y,
  // neighbouring y for rays driven along x) hit distinct banks; the channel
  // stride is a compile-time constant, so it folds into the instruction offset
  for (int i = threadIdx.x; i < NW; i += NT) acc[i] = 0ull;
  unsigned long long tot[2 * NOWN];   // PK: 64-bit totals of the owned words
#pragma unroll
  for (int o = 0; o < 2 * NOWN; ++o) tot[o] = 0ull;
  uint32_t bmx = 0u;   // bound pass: the largest sum of one batch in an owned word

  // h1 bounds max_x sum_y h(x,y) over all views (n_views times a per-view
  // bound); a batch of VB views contributes at most VB / n_views of it.
  // Packed plans have a tighter bound of their own per tile when the views
  // are the plan's (hbt, measured when the plan was made).  The weight bound
  // m is the tile's own (k_tile_max): the largest |w_c| of the rays that can
  // meet the tile.  In the bound pass (hbt_out) every weight is 1.
  const bool bnd = PK && hbt_out != nullptr;
  double hb = h1 * (double)min(VB, G.nvl) / (double)G.n_views;
  if (PK && hbt && !bnd) hb = fmin(hb, (double)hbt[t]);
  T scl[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    const float m = bnd ? 1.f : tmax[(int64_t)t * 4 + c];
    double s;
    if (PK)   // 2^32 - 2^20: room for the +1/2 of every term's rounding and for the FP32
              // roundings of the scaled weights (at most 2^-22 of the bound, 1024)
      s = (m > 0.f && hb > 0.0) ? 4293918720.0 / (hb * (double)m) : 0.0;
    else if (sizeof(T) == 4)
      s = (m > 0.f && hmax > 0.0) ? 2147481600.0 / (hmax * (double)m) : 0.0;
    else
      s = (m > 0.f && h1 > 0.0) ? 2305843009213693952.0 / (h1 * (double)m) : 0.0;
    // FP64, non-negative: every term (at most hmax * max|w| * s) below 2^51
    // for the conversion by addition; h1 >= n_views * hmax, so this binds
    // only for scans of fewer than 1024 views
    if (sizeof(T) == 8 && NONNEG && m > 0.f && hmax > 0.0)
      s = fmin(s, 2251799813685248.0 / (hmax * (double)m));
    scl[c] = (T)fmin(s, 1e30);
  }

  // tile rectangle (mm) and axial range
  const double X0 = G.x0 + tx0 * G.dx, X1 = G.x0 + tx1 * G.dx;
  const double Y0 = G.y0 + ty0 * G.dy, Y1 = G.y0 + ty1 * G.dy;
  const double Z0 = G.z0 + tz0 * G.dz, Z1 = G.z0 + tz1 * G.dz;
  __syncthreads();

  for (int vb0 = 0; vb0 < G.nvl; vb0 += VB) {
    cull_views<1, VB>(G, vb0, X0, X1, Y0, Y1, Z0, Z1, s_kap, s_kl, s_nk, s_rl, s_nr, s_off);
    const int total = s_off[VB];
    for (int it0 = threadIdx.x; it0 < total; it0 += NT) {
      // 3D: within each whole block of 64 items (one wave), even items go to
      // the first 32 lanes and odd ones to the rest, so that neighbouring
      // lanes walk rays two channels apart (fewer same-address LDS atomics)
      // while the wave keeps its items and their similar chord lengths
      int it = it0;
      if constexpr (Z3) {
        const int blk = it0 & ~63;
        if (blk + 64 <= total) {
          const int l = it0 & 63;
          it = blk + (l < 32 ? 2 * l : 2 * (l - 32) + 1);
        }
      }
      // view of the item: the last j with s_off[j] <= it (binary search)
      int j = 0;
#pragma unroll
      for (int step = VB / 2; step > 0; step >>= 1)
        if (s_off[j + step] <= it) j += step;
      const int loc = it - s_off[j];
      const int nk = s_nk[j];
      const int rr = loc / nk;
      // 2D: the view's even channels first, then its odd ones, so that
      // neighbouring lanes walk rays two channels apart, which rarely meet the
      // same voxel in the same step (neighbouring channels are about a pixel
      // apart and often do, and LDS atomics on one address serialise).  In 3D
      // a wave spans the channels of several (view, row) pairs, and the
      // contiguous order keeps their chord lengths alike.
      const int kk = loc - rr * nk, nh = (nk + 1) >> 1;
      const int k = s_kl[j] + ((Z3 || kk < nh) ? (Z3 ? kk : 2 * kk) : 2 * (kk - nh) + 1);
      const int r = s_rl[j] + rr;
      const int v = G.voff + G.vsub * (vb0 + j);
      // the weights are loaded before the ray set-up, which does not need
      // them, so that the two loads' latencies overlap
      const int64_t ray = ((int64_t)v * G.n_rows + r) * G.n_cols + k;
      T wa[NCH];   // weight x scale x mm per unit of the driving axis
#pragma unroll
      for (int c = 0; c < NCH; ++c) wa[c] = bnd ? (T)1 : w[c * G.R + ray];
      Ray<T> ry;
      if (!make_ray<T>(G, rays, v, r, k, tx0, ty0, tz0, tx1, ty1, tz1, ry)) continue;
#pragma unroll
      for (int c = 0; c < NCH; ++c) wa[c] = wa[c] * scl[c] * ry.La;
      const bool yd = ry.ydrive != 0;
      const int la = yd ? ty0 : tx0;
      // the tile's lateral range in the ray's frame (pixels relative to ry.ib)
      const int lbb = (yd ? tx0 : ty0) - ry.ib, hb = (yd ? tx1 : ty1) - ry.ib;
      const int sa = yd ? RS : 1, sbs = yd ? 1 : RS;
      // lb: byte offset of the voxel in channel 0; da: length in units of
      // the driving axis; quantised terms are 32-bit halves when packed,
      // 64-bit words otherwise
      using QT = typename QType<PK>::type;
      char* const accb = reinterpret_cast<char*>(acc);
      auto quant = [&](T da, QT* qv) {
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          if constexpr (PK)
            qv[c] = (uint32_t)fmaf((float)da, (float)wa[c], 0.5f);
          else if constexpr (NONNEG && sizeof(T) == 4)
            qv[c] = to_fixed_nonneg((float)da, (float)wa[c]);
          else if constexpr (NONNEG)
            qv[c] = to_fixed_nonneg((double)(da * wa[c]));
          else
            qv[c] = to_fixed(da * wa[c]);
        }
      };
      auto add = [&](int lb, const QT* qv) {
        if constexpr (PK) {
#pragma unroll
          for (int p = 0; p < 2; ++p)
            atomicAdd(reinterpret_cast<unsigned long long*>(accb + (uint32_t)lb + p * NVOX * 8),
                      ((unsigned long long)qv[2 * p + 1] << 32) | qv[2 * p]);
        } else {
#pragma unroll
          for (int c = 0; c < NCH; ++c)
            atomicAdd(reinterpret_cast<unsigned long long*>(accb + (uint32_t)lb + c * NVOX * 8),
                      (unsigned long long)qv[c]);
        }
      };
      auto deposit = [&](int lb, T da) {
        QT qv[NCH];
        quant(da, qv);
        add(lb, qv);
      };
      // a whole plane step inside one pixel, quantised once per ray: in a
      // full step split between two pixels the second one receives this
      // minus the first one's share (an exact integer split of the step)
      QT LQ[NCH];
      quant((T)1, LQ);
      const int q0 = ifloor(ry.alo) - la;        // first plane step (tile-relative)
      const int q1 = -ifloor(-ry.ahi) - la;      // one past the last
      T tp = ry.alo;                             // start of the current step
      T bp = fma(tp, ry.mb, ry.b0);              // lateral coordinate there
      T fa = (T)(la + q0);
      int A = clampi(ifloor(bp), lbb, hb - 1);
      const int sb8 = 8 * sbs;
      // byte offset of lateral index 0 in the current plane row and slice
      int row8 = 8 * (q0 * sa - lbb * sbs);
      // the tile's slices in the ray's axial frame (relative to ry.iw)
      const int tzl = tz0 - ry.iw, tzh = tz1 - ry.iw;
      int C = 0, cs = 0;
      if constexpr (Z3) {
        C = clampi(ifloor(fma(tp, ry.mw, ry.w0)), tzl, tzh - 1);
        row8 += 8 * (C - tzl) * TXY;
        cs = ry.mw > (T)0 ? 1 : -1;
      }
      // 3D: the step that holds the next crossing of a slice plane inside the
      // tile (the chord is clipped to the tile's slices, so a tile face ends
      // it): the plane w = wb is met at a = (wb - w0)/mw, and step q, which
      // ends on plane la + q + 1, holds it when it lies in (start, end].
      // Predicted once per crossing, not tested at every step; at least
      // `lo`, the step being walked (a crossing is never skipped).
      auto next_cross = [&](int lo) -> int {
        const int wb = cs > 0 ? C + 1 : C;
        if (ry.mw == (T)0 || wb <= tzl || wb >= tzh) return 0x7fffffff;
        const T qf = ceil(fabs((T)wb - ry.w0) * ry.imw) - (T)(la + 1);   // (wb - w0)/mw
        return max((int)fmin(qf, (T)1e9), lo);
      };
      int qc = 0x7fffffff;
      if constexpr (Z3) qc = next_cross(q0);
      uint32_t rest = 0;   // 3D: steps left to the general walk
      // 3D: a step that crosses a slice plane is recorded for the general
      // walk, and the walk moves on in the new slice.
      auto cross = [&](int q) {
        rest |= 1u << q;
        do {
          C += cs;
          row8 += 8 * cs * TXY;
          qc = next_cross(q);
        } while (qc == q);
      };
      auto flat_step = [&](int q, T) {
        if constexpr (Z3) {
          if (q == qc) {
            cross(q);
            return false;
          }
        }
        return true;
      };
      // a step that may be partial (the ray's first and last)
      auto gstep = [&](int q) {
        fa += (T)1;
        const T tn = min_fin(fa, ry.ahi);
        const T bn = fma(tn, ry.mb, ry.b0);
        const int B = clampi(ifloor(bn), lbb, hb - 1);
        if (flat_step(q, tn)) {
          const T ds = tn - tp;
          // the part of the step before the lateral crossing (all of it when
          // the step stays in one pixel)
          const T dA = (B == A) ? ds : clamp0(((T)max(A, B) - bp) * ry.imb, ds);
          deposit(__mul24(A, sb8) + row8, dA);
          if (B != A) deposit(__mul24(B, sb8) + row8, ds - dA);
        }
        row8 += 8 * sa;
        A = B;
        tp = tn;
        bp = bn;
      };
      // a full step [fa, fa + 1] inside one slice (DEP), or one that crosses
      // a slice plane and only advances the in-plane state (!DEP), in
      // Siddon's incremental form: e is the distance (in plane
      // spacings) from the start of the step to the next lateral plane.  A
      // step with e < 1 splits there and moves one pixel in the direction sg,
      // and e grows by 1/|mb| - 1, otherwise it falls by 1 (exact).  Only the
      // crossings round, so over the at most 32 steps of a chord in the tile
      // e stays within a few ulp of the line's value.  (The clamp keeps a
      // split at the tile's lateral face, within rounding of the chord's end,
      // in the tile.)
      const int sg = ry.mb > (T)0 ? 1 : (ry.mb < (T)0 ? -1 : 0);
      const T iab = fabs(ry.imb), iab1 = iab - (T)1;
      T e = (T)0;
      auto fstep = [&](auto dep) {
        fa += (T)1;
        const bool cr = e < (T)1;
        const int B = clampi(A + (cr ? sg : 0), lbb, hb - 1);
        if constexpr (decltype(dep)::value) {
          const T dA = clamp0(e, (T)1);
          QT qa[NCH];
          quant(dA, qa);
          add(__mul24(A, sb8) + row8, qa);
          if (cr) {
#pragma unroll
            for (int c = 0; c < NCH; ++c) qa[c] = LQ[c] - qa[c];
            add(__mul24(B, sb8) + row8, qa);
          }
        }
        e += cr ? iab1 : (T)-1;
        row8 += 8 * sa;
        A = B;
      };
      if (q0 < q1) {
        gstep(q0);
        const int ql = q1 - 1;     // the last step (partial) is gstep's
        int q = q0 + 1;
        // the distance to the next lateral plane from the line at the start
        // of the first full step
        e = sg > 0 ? ((T)(A + 1) - bp) * iab : (sg < 0 ? (bp - (T)A) * iab : (T)1e30);
        while (q < ql) {
          // full steps up to the next slice crossing, then the crossing step
          const int qe = min(qc, ql);
          for (; q < qe; ++q) fstep(std::true_type{});
          if (q < ql) {
            cross(q);
            fstep(std::false_type{});
            ++q;
          }
        }
        tp = fa;   // the last step starts on a plane
        // back to the line for the last (partial) step
        bp = fma(fa, ry.mb, ry.b0);
        A = clampi(ifloor(bp), lbb, hb - 1);
        if (ql > q0) gstep(ql);
      }
      if constexpr (Z3) {
        const T iLa = (T)1 / ry.La;
        auto visit3 = [&](int ia, int ib, int iw, T h) {
          deposit(8 * ((iw - tzl) * TXY + (ia - la) * sa + (ib - lbb) * sbs), h * iLa);
        };
        while (rest != 0u) {
          const int q = __ffs(rest) - 1;
          rest &= rest - 1u;
          walk_row<T, true, true>(ry, la + q, lbb, hb, tzl, tzh, visit3);
        }
      }
    }
    __syncthreads();
    if constexpr (PK) {
      // move the batch into the 64-bit totals; the next batch deposits only
      // after the barrier that follows its view set-up
#pragma unroll
      for (int o = 0; o < NOWN; ++o) {
        const int i = threadIdx.x + o * NT;
        if (i < NW) {
          const unsigned long long x = acc[i];
          acc[i] = 0ull;
          tot[2 * o] += (uint32_t)x;
          tot[2 * o + 1] += x >> 32;
          if (bnd) bmx = max(bmx, max((uint32_t)x, (uint32_t)(x >> 32)));
        }
      }
    }
  }

  if (bnd) {
    // the tile's largest sum of one batch, in mm: every term was rounded half
    // up (at most nterm terms per voxel and batch, each at most 1/2 low) and
    // carries FP32 roundings of at most 2^-22 of its value; the margin
    // covers both, and the bound never exceeds the geometric one
    __shared__ uint32_t s_bm[NT / 64];
    uint32_t m = bmx;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o));
    if ((threadIdx.x & 63) == 0) s_bm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int i = 1; i < NT / 64; ++i) m = max(m, s_bm[i]);
      const double q = (double)m * (1.0 + 1.0 / 1048576.0) + 0.5 * nterm + 64.0;
      const double hbx = fmin(q / (double)scl[0] * (1.0 + 1.0 / 1048576.0), hb);
      hbt_out[t] = (float)hbx;
    }
    return;
  }
  if constexpr (PK) {
#pragma unroll
    for (int o = 0; o < NOWN; ++o) {
      const int i = threadIdx.x + o * NT;
      if (i >= NW) continue;
      const int p = i >= NVOX ? 1 : 0;
      const int vi = i - p * NVOX;
      const int lx = vi % RS, ly = (vi / RS) % BT::ty, lz = vi / TXY;
      const int gx = tx0 + lx, gy = ty0 + ly, gz = tz0 + lz;
      if (lx >= BT::tx || gx >= tx1 || gy >= ty1 || gz >= tz1) continue;
      const int64_t gi = ((int64_t)gz * G.ny + gy) * G.nx + gx;
      const T slo = p ? scl[2] : scl[0], shi = p ? scl[3] : scl[1];
      b[(2 * p) * G.V + gi] = slo > (T)0 ? (T)((double)tot[2 * o] / (double)slo) : (T)0;
      b[(2 * p + 1) * G.V + gi] = shi > (T)0 ? (T)((double)tot[2 * o + 1] / (double)shi) : (T)0;
    }
    return;
  }

  // write the tile
  for (int i = threadIdx.x; i < NVOX; i += NT) {
    const int lx = i % RS, ly = (i / RS) % BT::ty, lz = i / TXY;
    const int gx = tx0 + lx, gy = ty0 + ly, gz = tz0 + lz;
    if (lx >= BT::tx || gx >= tx1 || gy >= ty1 || gz >= tz1) continue;
    const int64_t gi = ((int64_t)gz * G.ny + gy) * G.nx + gx;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const double val = (double)(long long)acc[c * NVOX + i];
      b[c * G.V + gi] = scl[c] > (T)0 ? (T)(val / (double)scl[c]) : (T)0;
    }
  }
}

// ---------------------------------------------------------------------------
// Iteration VJP helpers (voxel-wise)
// ---------------------------------------------------------------------------
// u = (dloss/db~_1, dloss/db~_2, dloss/db^_1, dloss/db^_2) for the update
// c_i - ln(b~_i/b^_i)/Z_i: -G_i/(Z_i b~_i) and G_i/(Z_i b^_i) where the update
// applies (both > 0), else 0.  FP64 arithmetic, stored in the plan precision.
template <typename T>
__global__ __launch_bounds__(256) void k_step_u(int64_t V, const double* __restrict__ G,
                                                const T* __restrict__ b, double iz1, double iz2,
                                                T* __restrict__ u) {
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (x >= V) return;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double bt = (double)b[i * V + x], bh = (double)b[(2 + i) * V + x];
    const double g = G[i * V + x] * (i == 0 ? iz1 : iz2);
    const bool act = bt > 0.0 && bh > 0.0;
    u[i * V + x] = act ? (T)(-g / bt) : (T)0;
    u[(2 + i) * V + x] = act ? (T)(g / bh) : (T)0;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_add_g(int64_t n, const double* __restrict__ G,
                                               const T* __restrict__ bl, double* __restrict__ out) {
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (x < n) out[x] = G[x] + (double)bl[x];
}

// ---------------------------------------------------------------------------
// Update and packing (32x32 tiles, LDS transpose for the x-major copy)
// ---------------------------------------------------------------------------
// b2 (or NULL): a second set of backprojections added to b (two scans).
template <typename T>
__global__ __launch_bounds__(256) void k_update(GeomDev G, double* __restrict__ c64,
                                                const T* __restrict__ b, const T* __restrict__ b2,
                                                double iz1, double iz2,
                                                T* __restrict__ c_proj,
                                                typename Vec2<T>::type* __restrict__ cpy,
                                                typename Vec2<T>::type* __restrict__ cpx) {
  using T2 = typename Vec2<T>::type;
  __shared__ T2 tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int bx = blockIdx.x, by = blockIdx.y, z = blockIdx.z;
  const int64_t V = G.V;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int ix = bx * 32 + tx, iy = by * 32 + ty + 8 * j;
    if (ix < G.nx && iy < G.ny) {
      const int64_t idx = ((int64_t)z * G.ny + iy) * G.nx + ix;
      double c1 = c64[idx], c2 = c64[V + idx];
      if (b) {
        double bt1 = (double)b[idx], bt2 = (double)b[V + idx];
        double bh1 = (double)b[2 * V + idx], bh2 = (double)b[3 * V + idx];
        if (b2) {
          bt1 += (double)b2[idx];
          bt2 += (double)b2[V + idx];
          bh1 += (double)b2[2 * V + idx];
          bh2 += (double)b2[3 * V + idx];
        }
        if (bt1 > 0.0 && bh1 > 0.0) c1 -= log(bt1 / bh1) * iz1;
        if (bt2 > 0.0 && bh2 > 0.0) c2 -= log(bt2 / bh2) * iz2;
        c64[idx] = c1;
        c64[V + idx] = c2;
      }
      T2 p;
      p.x = (T)c1;
      p.y = (T)c2;
      if (c_proj) {
        c_proj[idx] = p.x;
        c_proj[V + idx] = p.y;
      }
      if (cpy) cpy[idx] = p;
      tile[ty + 8 * j][tx] = p;
    }
  }
  if (!cpx) return;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int ix = bx * 32 + ty + 8 * j, iy = by * 32 + tx;
    if (ix < G.nx && iy < G.ny) cpx[((int64_t)z * G.nx + ix) * G.ny + iy] = tile[tx][ty + 8 * j];
  }
}

// planar [n_ch][V] (T, or uint8 when U8) -> packed natural and transposed copies
template <typename T, typename S>
__global__ __launch_bounds__(256) void k_pack(GeomDev G, const S* __restrict__ c, int n_ch,
                                              typename Vec2<T>::type* __restrict__ cpy,
                                              typename Vec2<T>::type* __restrict__ cpx) {
  using T2 = typename Vec2<T>::type;
  __shared__ T2 tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int bx = blockIdx.x, by = blockIdx.y, z = blockIdx.z;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int ix = bx * 32 + tx, iy = by * 32 + ty + 8 * j;
    if (ix < G.nx && iy < G.ny) {
      const int64_t idx = ((int64_t)z * G.ny + iy) * G.nx + ix;
      T2 p;
      p.x = (T)c[idx];
      p.y = n_ch > 1 ? (T)c[G.V + idx] : (T)0;
      cpy[idx] = p;
      tile[ty + 8 * j][tx] = p;
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int ix = bx * 32 + ty + 8 * j, iy = by * 32 + tx;
    if (ix < G.nx && iy < G.ny) cpx[((int64_t)z * G.nx + ix) * G.ny + iy] = tile[tx][ty + 8 * j];
  }
}

// ---------------------------------------------------------------------------
// Penalised update (Eqs. 6-7)
// ---------------------------------------------------------------------------
// The roughness penalty lambda sum_i sum_x sum_{x~ in N_x} w(x,x~) phi(c_i(x) -
// c_i(x~)) with the convex "fair" potential phi(t) = delta^2 (|t|/delta -
// ln(1 + |t|/delta)), N_x the voxels one step away along every axis (8 in 2D,
// 26 in 3D) and w = 1 / distance.  De Pierro's decoupling (convexity of phi)
// and the DEAM data surrogate split the c-step into one convex problem per
// voxel and component:
//   minimise b~ c + (b^/Z) exp(-Z (c - c^k)) + lambda sum_n w_n phi(2c - s_n),
//   s_n = c^k(x) + c^k(x~_n).
// Its derivative increases with c; the root lies between the data-only
// minimiser c^k - ln(b~/b^)/Z and [min, max] of s_n / 2 and is found by
// Newton's method from the data-only minimiser, falling back to bisection
// whenever a step leaves the bracket.  Everything is FP64.
struct PenArgs {
  const double* c_prev;  // [2][V] iterate c^k (all neighbours are read from here)
  double z1, z2;         // Z_1, Z_2
  double lam2, lam4;     // 2 lambda, 4 lambda
  double idelta;         // 1 / delta
  double delta2;         // delta^2 (penalty value)
  double w[7];           // 1 / distance by offset class |ox| + 2|oy| + 4|oz| - 1
};

constexpr int kPenMaxIter = 60;

// 1 / a for a >= 1: hardware reciprocal refined by two Newton-Raphson steps
// (each squares the relative error), to about one ulp.
__device__ __forceinline__ double recip_ge1(double a) {
  double r = __builtin_amdgcn_rcp(a);
  r = fma(r, fma(-a, r, 1.0), r);
  return fma(r, fma(-a, r, 1.0), r);
}

// Root of f'(c) = b~ - b^ exp(-Z (c - c^k)) + 2 lambda sum_n w_n phi'(2c - s_n)
// inside [lo, hi].  Newton steps from the data-only minimiser; a step that
// leaves the bracket is replaced by bisection.  A step below
// 1e-13 (|c| + 1e-3) is taken and ends the iteration (near the root the step
// falls below one ulp and would otherwise land on a bracket end).
// Neighbour n has weight P.w[cls_n] when bit n of `in` is set, else 0.
// ALL: every neighbour is inside the grid (the weights are then uniform).
template <int NB, bool ALL>
__device__ __forceinline__ double pen_solve(double ck, double bt, double bh, double Z,
                                            const double* s, uint32_t in, double lo, double hi,
                                            const PenArgs& P) {
  double c = ck - log(bt / bh) / Z;  // data-only minimiser, inside [lo, hi]
  for (int it = 0; it < kPenMaxIter; ++it) {
    const double e = bh * exp(-Z * (c - ck));
    double pf = 0.0, pfp = 0.0;
    int n = 0;
#pragma unroll
    for (int oz = (NB == 26 ? -1 : 0); oz <= (NB == 26 ? 1 : 0); ++oz)
#pragma unroll
      for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
        for (int ox = -1; ox <= 1; ++ox) {
          if (ox == 0 && oy == 0 && oz == 0) continue;
          const double wc = P.w[(ox != 0) + 2 * (oy != 0) + 4 * (oz != 0) - 1];
          const double wn = (ALL || ((in >> n) & 1u)) ? wc : 0.0;
          const double t = 2.0 * c - s[n];
          const double r = recip_ge1(1.0 + fabs(t) * P.idelta);  // phi'(t) = t r, phi''(t) = r^2
          pf = fma(wn, t * r, pf);
          pfp = fma(wn, r * r, pfp);
          ++n;
        }
    const double f = (bt - e) + P.lam2 * pf;
    const double fp = Z * e + P.lam4 * pfp;
    if (f > 0.0) hi = c;
    else if (f < 0.0) lo = c;
    else break;
    const double step = f / fp;
    if (fabs(step) <= 1e-13 * (fabs(c) + 1e-3)) {
      c -= step;
      break;
    }
    const double cn = c - step;
    c = (cn > lo && cn < hi) ? cn : 0.5 * (lo + hi);
  }
  return c;
}

// One voxel, both components: gathers the neighbours of c_prev (clamped
// indices, so every load is in bounds; bit n of `in` marks the neighbours
// inside the grid) and solves each component.  Voxels with b~ <= 0 or
// b^ <= 0 keep c^k, as in the unpenalised update.
template <bool Z3>
__device__ __forceinline__ void pen_voxel(const GeomDev& G, int ix, int iy, int iz, int64_t idx,
                                          double bt1, double bt2, double bh1, double bh2,
                                          const PenArgs& P, double& c1, double& c2) {
  constexpr int NB = Z3 ? 26 : 8;
  const int64_t V = G.V;
#pragma unroll 1
  for (int i = 0; i < 2; ++i) {
    const double* cp = P.c_prev + (i ? V : 0);
    const double ck = cp[idx];
    double s[NB];
    double lo = ck, hi = ck;
    uint32_t in = 0;
    int n = 0;
#pragma unroll
    for (int oz = (Z3 ? -1 : 0); oz <= (Z3 ? 1 : 0); ++oz)
#pragma unroll
      for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
        for (int ox = -1; ox <= 1; ++ox) {
          if (ox == 0 && oy == 0 && oz == 0) continue;
          const int jx = min(max(ix + ox, 0), G.nx - 1);
          const int jy = min(max(iy + oy, 0), G.ny - 1);
          const int jz = Z3 ? min(max(iz + oz, 0), G.nz - 1) : iz;
          if (jx == ix + ox && jy == iy + oy && jz == iz + oz) in |= 1u << n;
          s[n] = ck + cp[((int64_t)jz * G.ny + jy) * G.nx + jx];
          // the bracket may include clamped (outside) neighbours: it only widens
          lo = fmin(lo, 0.5 * s[n]);
          hi = fmax(hi, 0.5 * s[n]);
          ++n;
        }
    const double bt = i ? bt2 : bt1, bh = i ? bh2 : bh1, Z = i ? P.z2 : P.z1;
    double c = ck;
    if (bt > 0.0 && bh > 0.0) {
      const double cu = ck - log(bt / bh) / Z;
      if (in == (1u << NB) - 1u)
        c = pen_solve<NB, true>(ck, bt, bh, Z, s, in, fmin(lo, cu), fmax(hi, cu), P);
      else
        c = pen_solve<NB, false>(ck, bt, bh, Z, s, in, fmin(lo, cu), fmax(hi, cu), P);
    }
    if (i) c2 = c;
    else c1 = c;
  }
}

// One voxel per thread, 32 x 8 tiles; the x-major copy goes through LDS.
template <typename T, bool Z3>
__global__ __launch_bounds__(256) void k_update_pen(GeomDev G, PenArgs P, double* __restrict__ c64,
                                                    const T* __restrict__ b,
                                                    T* __restrict__ c_proj,
                                                    typename Vec2<T>::type* __restrict__ cpy,
                                                    typename Vec2<T>::type* __restrict__ cpx) {
  using T2 = typename Vec2<T>::type;
  __shared__ T2 tile[8][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int z = blockIdx.z;
  const int64_t V = G.V;
  const int ix = blockIdx.x * 32 + tx, iy = blockIdx.y * 8 + ty;
  if (ix < G.nx && iy < G.ny) {
    const int64_t idx = ((int64_t)z * G.ny + iy) * G.nx + ix;
    double c1, c2;
    pen_voxel<Z3>(G, ix, iy, z, idx, (double)b[idx], (double)b[V + idx], (double)b[2 * V + idx],
                  (double)b[3 * V + idx], P, c1, c2);
    c64[idx] = c1;
    c64[V + idx] = c2;
    T2 p;
    p.x = (T)c1;
    p.y = (T)c2;
    if (c_proj) {
      c_proj[idx] = p.x;
      c_proj[V + idx] = p.y;
    }
    if (cpy) cpy[idx] = p;
    tile[ty][tx] = p;
  }
  if (!cpx) return;
  __syncthreads();
  // thread t writes the x-major element (ix = 32 bx + t/8, iy = 8 by + t%8)
  const int jx = blockIdx.x * 32 + (threadIdx.x >> 3), jy = blockIdx.y * 8 + (threadIdx.x & 7);
  if (jx < G.nx && jy < G.ny)
    cpx[((int64_t)z * G.nx + jx) * G.ny + jy] = tile[threadIdx.x & 7][threadIdx.x >> 3];
}

// R(c): per voxel sum_i sum_n w_n phi(c_i(x) - c_i(x~_n)) (each pair is met
// from both sides, as in Eq. 6), times lambda; one FP64 partial per block.
template <bool Z3>
__global__ __launch_bounds__(256) void k_penalty(GeomDev G, PenArgs P, double lambda,
                                                 const double* __restrict__ c,
                                                 double* __restrict__ partial) {
  __shared__ double red[256];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int bx = blockIdx.x, by = blockIdx.y, z = blockIdx.z;
  const int64_t V = G.V;
  double acc = 0.0;
  for (int j = 0; j < 4; ++j) {
    const int ix = bx * 32 + tx, iy = by * 32 + ty + 8 * j;
    if (ix >= G.nx || iy >= G.ny) continue;
    const int64_t idx = ((int64_t)z * G.ny + iy) * G.nx + ix;
    const double a1 = c[idx], a2 = c[V + idx];
#pragma unroll
    for (int oz = (Z3 ? -1 : 0); oz <= (Z3 ? 1 : 0); ++oz)
#pragma unroll
      for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
        for (int ox = -1; ox <= 1; ++ox) {
          if (ox == 0 && oy == 0 && oz == 0) continue;
          const int jx = ix + ox, jy = iy + oy, jz = z + oz;
          if (jx < 0 || jx >= G.nx || jy < 0 || jy >= G.ny || jz < 0 || jz >= (Z3 ? G.nz : 1))
            continue;
          const int64_t jn = ((int64_t)jz * G.ny + jy) * G.nx + jx;
          const double u1 = fabs(a1 - c[jn]) * P.idelta, u2 = fabs(a2 - c[V + jn]) * P.idelta;
          acc += P.w[(ox != 0) + 2 * (oy != 0) + 4 * (oz != 0) - 1] *
                 ((u1 - log1p(u1)) + (u2 - log1p(u2)));
        }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    partial[((int64_t)z * gridDim.y + by) * gridDim.x + bx] = lambda * P.delta2 * red[0];
}

// ---------------------------------------------------------------------------
// MAR initialisation (Section 2.2, Fig. 1, Eq. 4), 2D fan-beam full scans
// ---------------------------------------------------------------------------
// p_j = ln(sum_E I0_j) - ln(max(d_j, 1)): counts below one photon count as one.
template <typename T>
__global__ __launch_bounds__(256) void k_line_integrals(int64_t R, const float* __restrict__ d,
                                                        double lt1, double lt2, T* __restrict__ p) {
  const int64_t y = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (y >= R) return;
  p[y] = (T)(lt1 - log(fmax((double)d[y], 1.0)));
  p[R + y] = (T)(lt2 - log(fmax((double)d[R + y], 1.0)));
}

// Ramp filtering of one view of one sinogram per block (equiangular fan beam):
//   Q_v[k] = a sum_m p_v[m] w[m] g(|k - m|),  w[m] = sid cos(gamma_m),
//   g(0) = 1/(8 a^2), g(j odd) = -1/(2 pi^2 sin^2(j a)), g(j even) = 0,
// a = dgamma.  tab = [g(0..n-1), w(0..n-1)] (FP64, from the plan).  The
// weighted row and the kernel sit in LDS; sums are FP64.
template <typename T>
__global__ __launch_bounds__(256) void k_fbp_filter(int n_cols, int64_t R, const T* __restrict__ p,
                                                    const double* __restrict__ tab, double a,
                                                    T* __restrict__ Q) {
  extern __shared__ double sh_fbp[];
  double* rw = sh_fbp;
  double* gk = sh_fbp + n_cols;
  const int v = blockIdx.x, c = blockIdx.y;
  const int64_t base = (int64_t)c * R + (int64_t)v * n_cols;
  for (int k = threadIdx.x; k < n_cols; k += 256) {
    rw[k] = (double)p[base + k] * tab[n_cols + k];
    gk[k] = tab[k];
  }
  __syncthreads();
  for (int k = threadIdx.x; k < n_cols; k += 256) {
    double acc = rw[k] * gk[0];
    for (int j = 1; j < n_cols; j += 2) {
      const int lo = k - j, hi = k + j;
      const double s = (lo >= 0 ? rw[lo] : 0.0) + (hi < n_cols ? rw[hi] : 0.0);
      acc = fma(s, gk[j], acc);
    }
    Q[base + k] = (T)(a * acc);
  }
}

// Distance-weighted backprojection of n_ch filtered sinograms, one thread per
// pixel: f(x) = (2 pi / n_views) sum_v Q_v(gamma') / L^2, where gamma' and L are
// the fan angle and the distance of the pixel centre seen from the source of
// view v, and Q_v is interpolated linearly between channels (zero outside the
// detector).  Geometry, interpolation and sums in FP64 in both precisions: the
// channel coordinate is a few hundred channels, so in FP32 its rounding alone
// (up to 6e-5 channel) would move the interpolation by that fraction of the
// jump between neighbouring channels, which next to metal is most of the
// image's range.
template <typename T>
__global__ __launch_bounds__(256) void k_fbp_bp(GeomDev G, int n_ch, const T* __restrict__ Q,
                                                double scale, T* __restrict__ img) {
  const int64_t V = (int64_t)G.nx * G.ny;
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (x >= V) return;
  const int ix = (int)(x % G.nx), iy = (int)(x / G.nx);
  const double px = G.x0 + (ix + 0.5) * G.dx, py = G.y0 + (iy + 0.5) * G.dy;
  const double ida = 1.0 / G.dgamma;
  const int n = G.n_cols;
  const int64_t R = G.R;
  double acc0 = 0.0, acc1 = 0.0;
  for (int v = 0; v < G.n_views; ++v) {
    const double cb = G.view[4 * v], sb = G.view[4 * v + 1];
    const double vx = px - G.sid * cb, vy = py - G.sid * sb;
    // central ray u = -(cos b, sin b): cross(u, v) and dot(u, v)
    const double gam = atan2(sb * vx - cb * vy, -(cb * vx + sb * vy));
    const double L2 = vx * vx + vy * vy;
    const double kf = gam * ida + G.kc;
    const double fk = floor(kf);
    const int k0 = (int)fk;
    if (k0 < -1 || k0 > n - 1) continue;
    const double fr = kf - fk;
    const int64_t r0 = (int64_t)v * n + k0;
    const double q00 = k0 >= 0 ? (double)Q[r0] : 0.0, q01 = k0 + 1 < n ? (double)Q[r0 + 1] : 0.0;
    acc0 += ((1.0 - fr) * q00 + fr * q01) / L2;
    if (n_ch > 1) {
      const double q10 = k0 >= 0 ? (double)Q[R + r0] : 0.0;
      const double q11 = k0 + 1 < n ? (double)Q[R + r0 + 1] : 0.0;
      acc1 += ((1.0 - fr) * q10 + fr * q11) / L2;
    }
  }
  img[x] = (T)(scale * acc0);
  if (n_ch > 1) img[V + x] = (T)(scale * acc1);
}

// NMAR (normalised interpolation across the trace), one view per block: on a
// trace channel k the value p/(pp + eps) is interpolated linearly between the
// nearest non-trace channels on either side (the nearest one beyond a detector
// end) and multiplied back by pp + eps; other channels are copied.
template <typename T>
__global__ __launch_bounds__(256) void k_nmar(int n_cols, int64_t R, const T* __restrict__ p,
                                              const uint8_t* __restrict__ mask,
                                              const T* __restrict__ pp, double eps,
                                              T* __restrict__ out) {
  const int64_t row = (int64_t)blockIdx.x * n_cols;
  for (int k = threadIdx.x; k < n_cols; k += 256) {
    const int64_t y = row + k;
    if (!mask[y]) {
      out[y] = p[y];
      out[R + y] = p[R + y];
      continue;
    }
    int kl = k - 1, kr = k + 1;
    while (kl >= 0 && mask[row + kl]) --kl;
    while (kr < n_cols && mask[row + kr]) ++kr;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int64_t o = (int64_t)c * R;
      if (kl < 0 && kr >= n_cols) {
        out[o + y] = p[o + y];
        continue;
      }
      double val;
      if (kl < 0) {
        val = (double)p[o + row + kr] / ((double)pp[o + row + kr] + eps);
      } else if (kr >= n_cols) {
        val = (double)p[o + row + kl] / ((double)pp[o + row + kl] + eps);
      } else {
        const double fl = (double)p[o + row + kl] / ((double)pp[o + row + kl] + eps);
        const double fh = (double)p[o + row + kr] / ((double)pp[o + row + kr] + eps);
        val = (fh - fl) / (double)(kr - kl) * (double)(k - kl) + fl;
      }
      out[o + y] = (T)(val * ((double)pp[o + y] + eps));
    }
  }
}

// Metal image and prior images from the uncorrected FBP images mu0 (L, H):
// M = [mu_H >= thr_m]; prior_j = 0 below thr_air_j, water_j below thr_bone_j
// or on M, mu_j above.  Thresholds are compared in the plan precision.
template <typename T>
__global__ __launch_bounds__(256) void k_mar_classes(int64_t V, const T* __restrict__ mu0,
                                                     double wl, double wh, double fa, double fb,
                                                     double fm, uint8_t* __restrict__ M,
                                                     T* __restrict__ prior) {
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (x >= V) return;
  const T ml = mu0[x], mh = mu0[V + x];
  const bool metal = mh >= (T)(fm * wh);
  M[x] = metal ? 1 : 0;
  const T w[2] = {(T)wl, (T)wh};
  const T m[2] = {ml, mh};
  const double wd[2] = {wl, wh};
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    T q = m[j] < (T)(fa * wd[j]) ? (T)0 : (m[j] < (T)(fb * wd[j]) ? w[j] : m[j]);
    prior[j * V + x] = metal ? w[j] : q;
  }
}

// Eq. 4: c = Mt^-1 (mu_L, mu_H) per voxel (inverse from the plan, FP64).
template <typename T>
__global__ __launch_bounds__(256) void k_decompose(int64_t V, const T* __restrict__ mu,
                                                   double a00, double a01, double a10, double a11,
                                                   double* __restrict__ c) {
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (x >= V) return;
  const double ml = (double)mu[x], mh = (double)mu[V + x];
  c[x] = a00 * ml + a01 * mh;
  c[V + x] = a10 * ml + a11 * mh;
}

// Trace dilation along the channels: out[y] = 1 when a ray of the same view
// and row within `radius` channels of y is in mask.
__global__ __launch_bounds__(256) void k_dilate(int64_t R, int n_cols, int radius,
                                                const uint8_t* __restrict__ mask,
                                                uint8_t* __restrict__ out) {
  const int64_t y = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (y >= R) return;
  const int k = (int)(y % n_cols);
  const int64_t row = y - k;
  const int lo = max(k - radius, 0), hi = min(k + radius, n_cols - 1);
  uint8_t m = 0;
  for (int q = lo; q <= hi; ++q) m |= mask[row + q];
  out[y] = m ? 1 : 0;
}

// Bit-packed trace: bit b of word i is mask[32 i + b] != 0 (one wave per
// 64 words; rays past R give 0 bits).
__global__ __launch_bounds__(256) void k_pack_mask(int64_t R, const uint8_t* __restrict__ mask,
                                                   uint32_t* __restrict__ bits) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;   // word
  const int64_t nw = (R + 31) / 32;
  if (i >= nw) return;
  uint32_t wv = 0;
  const int64_t y0 = i * 32;
  for (int b = 0; b < 32; ++b)
    if (y0 + b < R && mask[y0 + b]) wv |= 1u << b;
  bits[i] = wv;
}

// Input check (a debug call, off the hot path): counts of non-finite image
// values and of counts that are negative or non-finite.  Grid-stride loop,
// one atomic per wave.
__global__ __launch_bounds__(256) void k_validate(const double* __restrict__ c, int64_t nc,
                                                  const float* __restrict__ d, int64_t nd,
                                                  unsigned long long* __restrict__ cnt) {
  unsigned long long bc = 0, bd = 0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nc; i += stride)
    bc += isfinite(c[i]) ? 0 : 1;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nd; i += stride)
    bd += (isfinite(d[i]) && d[i] >= 0.f) ? 0 : 1;
  for (int o = 32; o > 0; o >>= 1) {
    bc += __shfl_down(bc, o);
    bd += __shfl_down(bd, o);
  }
  if ((threadIdx.x & 63) == 0) {
    if (bc) atomicAdd(&cnt[0], bc);
    if (bd) atomicAdd(&cnt[1], bd);
  }
}

inline dim3 image_grid(const deam_plan* p) {
  return dim3((p->gd.nx + 31) / 32, (p->gd.ny + 31) / 32, p->gd.is3d ? p->gd.nz : 1);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t launch_pack(const deam_plan* p, const void* c, int n_ch, bool from_u8, bool dbl,
                       void* cp_y, void* cp_x, hipStream_t st) {
  if (dbl) {
    if (from_u8)
      hipLaunchKernelGGL((k_pack<double, uint8_t>), image_grid(p), dim3(256), 0, st, p->gd,
                         (const uint8_t*)c, n_ch, (double2*)cp_y, (double2*)cp_x);
    else
      hipLaunchKernelGGL((k_pack<double, double>), image_grid(p), dim3(256), 0, st, p->gd,
                         (const double*)c, n_ch, (double2*)cp_y, (double2*)cp_x);
  } else {
    hipLaunchKernelGGL((k_pack<float, float>), image_grid(p), dim3(256), 0, st, p->gd,
                       (const float*)c, n_ch, (float2*)cp_y, (float2*)cp_x);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_zero_tail(p, cp_x, dbl, st);
}

// Zero the packed_tail_elems elements after the x-major copy (which follows
// the natural copy with no gap): the forward projectors read them for rays
// outside the slices and for idle lanes, so they must hold zeros (0 x NaN
// would not vanish).
hipError_t launch_zero_tail(const deam_plan* p, void* cp_x, bool dbl, hipStream_t st) {
  const size_t e2 = dbl ? sizeof(double2) : sizeof(float2);
  const size_t n = packed_tail_elems(p->gd.nx, p->gd.ny);
  return launch_fill_u32((uint32_t*)((char*)cp_x + (size_t)p->gd.V * e2), 0u,
                         (int64_t)(n * e2 / 4), st);
}

template <typename T, int MODE>
static void fp_dispatch(const deam_plan* p, const void* cp_y, const void* cp_x, const float* d,
                        const uint8_t* mask, void* out, double* partial,
                        double tthr, uint8_t* mask_out, double* Tout, hipStream_t st, int nout = 2,
                        uint32_t* wmap = nullptr) {
  using T2 = typename Vec2<T>::type;
  const WMapDev M = wmap_dev(p->gd, wmap);
  const dim3 grid((unsigned)p->ray_blocks), blk(kFpBlock);
  const EBin<T>* eb = (const EBin<T>*)p->d_energy;
  // the x-major copy follows the natural one in the same allocation
  const uint32_t xoff = (uint32_t)(((const T2*)cp_x) - ((const T2*)cp_y));
  if (p->gd.is3d) {
    constexpr int RG = fp3_rows<T>();
    const dim3 grid3((unsigned)fp3_blocks(p->gd.nvl, p->gd.n_rows, p->gd.n_cols, RG));
    hipLaunchKernelGGL((k_fp3<T, MODE, RG>), grid3, dim3(64 * kFp3Views), 0, st, p->gd,
                       (const T2*)cp_y, xoff,
                       eb, p->nE, d, mask, (T*)out, partial, tthr, mask_out, Tout, nout, M);
  } else
    hipLaunchKernelGGL((k_fp<T, false, MODE>), grid, blk, 0, st, p->gd, (const T2*)cp_y, xoff,
                       eb, p->nE, d, mask, (T*)out, partial, tthr, mask_out, Tout, nout, M);
}

hipError_t launch_forward(const deam_plan* p, const void* cp_y, const void* cp_x, void* l,
                          int n_out, hipStream_t st) {
  if (p->precision == DEAM_PREC_FP64)
    fp_dispatch<double, PM_L>(p, cp_y, cp_x, nullptr, nullptr, l, nullptr, 0.0, nullptr,
                              nullptr, st, n_out);
  else
    fp_dispatch<float, PM_L>(p, cp_y, cp_x, nullptr, nullptr, l, nullptr, 0.0, nullptr,
                             nullptr, st, n_out);
  return hipGetLastError();
}

hipError_t launch_metal_trace(const deam_plan* p, const void* cp_y, const void* cp_x, double t,
                              uint8_t* mask, double* T, hipStream_t st) {
  fp_dispatch<double, PM_TRACE>(p, cp_y, cp_x, nullptr, nullptr, nullptr, nullptr, t,
                                mask, T, st);
  return hipGetLastError();
}

hipError_t launch_fp_poly(const deam_plan* p, const void* cp_y, const void* cp_x, const float* d,
                          const uint8_t* mask, int mode, void* w, double* partial,
                          hipStream_t st, uint32_t* wmap) {
  const bool dbl = p->precision == DEAM_PREC_FP64;
  if (mode == PM_AM) {
    if (dbl) fp_dispatch<double, PM_AM>(p, cp_y, cp_x, d, mask, w, partial, 0, nullptr, nullptr, st, 2, wmap);
    else fp_dispatch<float, PM_AM>(p, cp_y, cp_x, d, mask, w, partial, 0, nullptr, nullptr, st, 2, wmap);
  } else if (mode == PM_GRAD) {
    if (dbl) fp_dispatch<double, PM_GRAD>(p, cp_y, cp_x, d, mask, w, partial, 0, nullptr, nullptr, st, 2, wmap);
    else fp_dispatch<float, PM_GRAD>(p, cp_y, cp_x, d, mask, w, partial, 0, nullptr, nullptr, st, 2, wmap);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
static void poly_dispatch(const deam_plan* p, const void* l, const float* d, const uint8_t* mask,
                          int mode, const void* v, void* w, void* g, double* partial,
                          hipStream_t st, uint32_t* wmap) {
  const int64_t R = p->gd.R;
  const WMapDev M = wmap_dev(p->gd, wmap);
  const dim3 grid((unsigned)((R + kFpBlock - 1) / kFpBlock)), blk(kFpBlock);
  const EBin<T>* eb = (const EBin<T>*)p->d_energy;
  if (mode == PM_AM)
    hipLaunchKernelGGL((k_poly<T, PM_AM>), grid, blk, 0, st, R, eb, p->nE, (const T*)l, d, mask,
                       (const T*)v, (T*)w, (T*)g, partial, p->gd.n_cols,
                       (const T*)p->gd.bowtie, M);
  else if (mode == PM_GRAD)
    hipLaunchKernelGGL((k_poly<T, PM_GRAD>), grid, blk, 0, st, R, eb, p->nE, (const T*)l, d,
                       mask, (const T*)v, (T*)w, (T*)g, partial, p->gd.n_cols,
                       (const T*)p->gd.bowtie, M);
  else if (mode == PM_VJP)
    hipLaunchKernelGGL((k_poly<T, PM_VJP>), grid, blk, 0, st, R, eb, p->nE, (const T*)l, d, mask,
                       (const T*)v, (T*)w, (T*)g, partial, p->gd.n_cols,
                       (const T*)p->gd.bowtie, M);
  else
    hipLaunchKernelGGL((k_poly<T, PM_STEP>), grid, blk, 0, st, R, eb, p->nE, (const T*)l, d, mask,
                       (const T*)v, (T*)w, (T*)g, partial, p->gd.n_cols,
                       (const T*)p->gd.bowtie, M);
}

hipError_t launch_poly(const deam_plan* p, const void* l, const float* d, const uint8_t* mask,
                       int mode, const void* v, void* w, void* g, double* partial,
                       hipStream_t st, uint32_t* wmap) {
  if (p->precision == DEAM_PREC_FP64)
    poly_dispatch<double>(p, l, d, mask, mode, v, w, g, partial, st, wmap);
  else
    poly_dispatch<float>(p, l, d, mask, mode, v, w, g, partial, st, wmap);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partial, int64_t n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, st, partial, n, out);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* ptr, uint32_t v, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ptr, v, n);
  return hipGetLastError();
}

hipError_t launch_absmax(const deam_plan* p, const void* w, int n_ch, uint32_t* wmap,
                         hipStream_t st) {
  const int64_t R = p->gd.R;
  hipError_t e = launch_fill_u32(wmap, 0u, wmap_words(p->gd), st);
  if (e != hipSuccess) return e;
  const WMapDev M = wmap_dev(p->gd, wmap);
  const unsigned nb = (unsigned)((R + kFpBlock - 1) / kFpBlock);
  if (p->precision == DEAM_PREC_FP64)
    hipLaunchKernelGGL(k_absmax<double>, dim3(nb), dim3(kFpBlock), 0, st, R, n_ch,
                       (const double*)w, M);
  else
    hipLaunchKernelGGL(k_absmax<float>, dim3(nb), dim3(kFpBlock), 0, st, R, n_ch,
                       (const float*)w, M);
  return hipGetLastError();
}

// Bound of the number of terms one voxel receives in one view batch: per view
// at most nk channels and nr rows pass through it (the factors of the plan's
// geometric bound), each ray one term, doubled for safety.
static double batch_terms(const deam_plan* p) {
  return 2.0 * (double)kViewBatch * p->bp_rays_per_voxel;
}

// The packed backprojector's per-tile bound applies to the plan's own view
// set (all views, in order): the batches it was measured on.
static const float* plan_hbt(const deam_plan* p) {
  const GeomDev& G = p->gd;
  return (G.voff == 0 && G.vsub == 1 && G.nvl == G.n_views) ? (const float*)p->d_hbt : nullptr;
}

template <typename T, bool Z3, int NCH, bool NONNEG, bool SM>
static hipError_t bp_tiles(const deam_plan* p, const void* w, const uint32_t* wmap, float* tmax,
                           void* b, hipStream_t st, float* hbt_out = nullptr) {
  using BT = BpTile<Z3, NCH, NONNEG && sizeof(T) == 4 && NCH == 4, SM>;
  Tiling TL{BT::tx, BT::ty, BT::tz, 0, 0, 0};
  TL.ntx = (p->gd.nx + BT::tx - 1) / BT::tx;
  TL.nty = (p->gd.ny + BT::ty - 1) / BT::ty;
  TL.ntz = ((Z3 ? p->gd.nz : 1) + BT::tz - 1) / BT::tz;
  const size_t lds = BT::lds_bytes;
  const unsigned nt = (unsigned)(TL.ntx * TL.nty * TL.ntz);
  if ((int64_t)nt > max_tiles(p->gd)) return hipErrorInvalidValue;   // tmax holds max_tiles
  hipError_t e;
  if (!hbt_out) {   // the bound pass takes every weight as 1 and needs no maxima
    hipLaunchKernelGGL(k_tile_max, dim3(nt), dim3(256), 0, st, p->gd, TL,
                       wmap_dev(p->gd, const_cast<uint32_t*>(wmap)), NCH, tmax);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  auto kern = k_bp<T, Z3, NCH, NONNEG, SM>;
  e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(nt), dim3(BT::block), lds, st, p->gd, TL, (const T*)w,
                     (const float*)tmax, p->h1_bound, p->hmax, (T*)b, plan_hbt(p), hbt_out,
                     batch_terms(p));
  return hipGetLastError();
}

// 2D: whole-CU 32 x 32 tiles when there are enough of them to give every
// compute unit one, else 16 x 16 tiles (four per CU)
template <typename T, bool Z3, int NCH, bool NONNEG>
static hipError_t bp_go(const deam_plan* p, const void* w, const uint32_t* wmap, float* tmax,
                        void* b, hipStream_t st, float* hbt_out = nullptr) {
  if constexpr (Z3) {
    return bp_tiles<T, Z3, NCH, NONNEG, false>(p, w, wmap, tmax, b, st, hbt_out);
  } else {
    const int64_t n32 = (int64_t)((p->gd.nx + 31) / 32) * ((p->gd.ny + 31) / 32);
    return n32 >= p->n_cu ? bp_tiles<T, Z3, NCH, NONNEG, false>(p, w, wmap, tmax, b, st, hbt_out)
                          : bp_tiles<T, Z3, NCH, NONNEG, true>(p, w, wmap, tmax, b, st, hbt_out);
  }
}

hipError_t launch_bp_bound(const deam_plan* p, float* hbt_out, hipStream_t st) {
  if (p->precision != DEAM_PREC_MIXED) return hipErrorInvalidValue;
  return p->gd.is3d ? bp_go<float, true, 4, true>(p, nullptr, nullptr, nullptr, nullptr, st, hbt_out)
                    : bp_go<float, false, 4, true>(p, nullptr, nullptr, nullptr, nullptr, st, hbt_out);
}

template <typename T, bool Z3>
static hipError_t bp_by_channels(const deam_plan* p, const void* w, int n_ch, bool nonneg,
                                 const uint32_t* wmap, float* tmax, void* b, hipStream_t st) {
  switch (n_ch) {
    case 1: return bp_go<T, Z3, 1, false>(p, w, wmap, tmax, b, st);
    case 2: return bp_go<T, Z3, 2, false>(p, w, wmap, tmax, b, st);
    case 4:
      return nonneg ? bp_go<T, Z3, 4, true>(p, w, wmap, tmax, b, st)
                    : bp_go<T, Z3, 4, false>(p, w, wmap, tmax, b, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_backproject(const deam_plan* p, const void* w, int n_ch, bool nonneg,
                              const uint32_t* wmap, float* tmax, void* b, hipStream_t st) {
  if (p->precision == DEAM_PREC_FP64)
    return p->gd.is3d ? bp_by_channels<double, true>(p, w, n_ch, nonneg, wmap, tmax, b, st)
                      : bp_by_channels<double, false>(p, w, n_ch, nonneg, wmap, tmax, b, st);
  return p->gd.is3d ? bp_by_channels<float, true>(p, w, n_ch, nonneg, wmap, tmax, b, st)
                    : bp_by_channels<float, false>(p, w, n_ch, nonneg, wmap, tmax, b, st);
}

hipError_t launch_step_u(const deam_plan* p, const double* G, const void* b, double z1, double z2,
                         void* u, hipStream_t st) {
  const int64_t V = p->gd.V;
  const dim3 grid((unsigned)((V + 255) / 256));
  if (p->precision == DEAM_PREC_FP64)
    hipLaunchKernelGGL(k_step_u<double>, grid, dim3(256), 0, st, V, G, (const double*)b, 1.0 / z1,
                       1.0 / z2, (double*)u);
  else
    hipLaunchKernelGGL(k_step_u<float>, grid, dim3(256), 0, st, V, G, (const float*)b, 1.0 / z1,
                       1.0 / z2, (float*)u);
  return hipGetLastError();
}

hipError_t launch_add_g(const deam_plan* p, const double* G, const void* bl, double* out,
                        hipStream_t st) {
  const int64_t n = 2 * p->gd.V;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (p->precision == DEAM_PREC_FP64)
    hipLaunchKernelGGL(k_add_g<double>, grid, dim3(256), 0, st, n, G, (const double*)bl, out);
  else
    hipLaunchKernelGGL(k_add_g<float>, grid, dim3(256), 0, st, n, G, (const float*)bl, out);
  return hipGetLastError();
}

hipError_t launch_update(const deam_plan* p, double* c64, const void* b, double z1, double z2,
                         void* c_proj, void* cp_y, void* cp_x, hipStream_t st, const void* b2) {
  if (p->precision == DEAM_PREC_FP64)
    hipLaunchKernelGGL(k_update<double>, image_grid(p), dim3(256), 0, st, p->gd, c64,
                       (const double*)b, (const double*)b2, 1.0 / z1, 1.0 / z2, (double*)c_proj,
                       (double2*)cp_y, (double2*)cp_x);
  else
    hipLaunchKernelGGL(k_update<float>, image_grid(p), dim3(256), 0, st, p->gd, c64,
                       (const float*)b, (const float*)b2, 1.0 / z1, 1.0 / z2, (float*)c_proj,
                       (float2*)cp_y, (float2*)cp_x);
  return hipGetLastError();
}

static PenArgs pen_args(const deam_plan* p, const double* c_prev, double z1, double z2,
                        double lambda, double delta) {
  PenArgs a{};
  a.c_prev = c_prev;
  a.z1 = z1;
  a.z2 = z2;
  a.lam2 = 2.0 * lambda;
  a.lam4 = 4.0 * lambda;
  a.idelta = 1.0 / delta;
  a.delta2 = delta * delta;
  for (int k = 0; k < 7; ++k) {
    const int m = k + 1;
    const double ddx = (m & 1) ? p->gd.dx : 0.0, ddy = (m & 2) ? p->gd.dy : 0.0,
                 ddz = (m & 4) ? p->gd.dz : 0.0;
    a.w[k] = 1.0 / std::sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
  }
  return a;
}

hipError_t launch_update_pen(const deam_plan* p, const double* c_prev, double* c64, const void* b,
                             double z1, double z2, double lambda, double delta, void* c_proj,
                             void* cp_y, void* cp_x, hipStream_t st) {
  const PenArgs a = pen_args(p, c_prev, z1, z2, lambda, delta);
  const bool z3 = p->gd.is3d && p->gd.nz > 1;
  const dim3 grid((p->gd.nx + 31) / 32, (p->gd.ny + 7) / 8, p->gd.is3d ? p->gd.nz : 1);
  if (p->precision == DEAM_PREC_FP64) {
    if (z3)
      hipLaunchKernelGGL((k_update_pen<double, true>), grid, dim3(256), 0, st, p->gd, a,
                         c64, (const double*)b, (double*)c_proj, (double2*)cp_y, (double2*)cp_x);
    else
      hipLaunchKernelGGL((k_update_pen<double, false>), grid, dim3(256), 0, st, p->gd, a,
                         c64, (const double*)b, (double*)c_proj, (double2*)cp_y, (double2*)cp_x);
  } else {
    if (z3)
      hipLaunchKernelGGL((k_update_pen<float, true>), grid, dim3(256), 0, st, p->gd, a,
                         c64, (const float*)b, (float*)c_proj, (float2*)cp_y, (float2*)cp_x);
    else
      hipLaunchKernelGGL((k_update_pen<float, false>), grid, dim3(256), 0, st, p->gd, a,
                         c64, (const float*)b, (float*)c_proj, (float2*)cp_y, (float2*)cp_x);
  }
  return hipGetLastError();
}

int64_t pen_blocks(const deam_plan* p) {
  const dim3 g = image_grid(p);
  return (int64_t)g.x * g.y * g.z;
}

hipError_t launch_penalty(const deam_plan* p, const double* c, double lambda, double delta,
                          double* partial, hipStream_t st) {
  const PenArgs a = pen_args(p, nullptr, 1.0, 1.0, lambda, delta);
  if (p->gd.is3d && p->gd.nz > 1)
    hipLaunchKernelGGL(k_penalty<true>, image_grid(p), dim3(256), 0, st, p->gd, a, lambda, c,
                       partial);
  else
    hipLaunchKernelGGL(k_penalty<false>, image_grid(p), dim3(256), 0, st, p->gd, a, lambda, c,
                       partial);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// MAR initialisation launchers
// ---------------------------------------------------------------------------
hipError_t launch_line_integrals(const deam_plan* p, const float* d, void* out, hipStream_t st) {
  const int64_t R = p->gd.R;
  const dim3 grid((unsigned)((R + 255) / 256));
  const double lt1 = std::log(p->i0sum[0]), lt2 = std::log(p->i0sum[1]);
  if (p->precision == DEAM_PREC_FP64)
    hipLaunchKernelGGL(k_line_integrals<double>, grid, dim3(256), 0, st, R, d, lt1, lt2,
                       (double*)out);
  else
    hipLaunchKernelGGL(k_line_integrals<float>, grid, dim3(256), 0, st, R, d, lt1, lt2,
                       (float*)out);
  return hipGetLastError();
}

hipError_t launch_fbp(const deam_plan* p, const void* sino, int n_ch, void* q, void* img,
                      hipStream_t st) {
  const int n = p->gd.n_cols;
  const dim3 fgrid((unsigned)p->gd.n_views, (unsigned)n_ch);
  const size_t lds = (size_t)2 * n * sizeof(double);
  const int64_t V = (int64_t)p->gd.nx * p->gd.ny;
  const dim3 bgrid((unsigned)((V + 255) / 256));
  const double scale = 2.0 * M_PI / p->gd.n_views;
  // the weighted row and the kernel sit in LDS (up to 64 KiB at 4096 channels)
  hipError_t e = hipFuncSetAttribute(
      p->precision == DEAM_PREC_FP64 ? (const void*)k_fbp_filter<double> : (const void*)k_fbp_filter<float>,
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (p->precision == DEAM_PREC_FP64) {
    hipLaunchKernelGGL(k_fbp_filter<double>, fgrid, dim3(256), lds, st, n, p->gd.R,
                       (const double*)sino, p->d_fbp, p->gd.dgamma, (double*)q);
    hipLaunchKernelGGL(k_fbp_bp<double>, bgrid, dim3(256), 0, st, p->gd, n_ch, (const double*)q,
                       scale, (double*)img);
  } else {
    hipLaunchKernelGGL(k_fbp_filter<float>, fgrid, dim3(256), lds, st, n, p->gd.R,
                       (const float*)sino, p->d_fbp, p->gd.dgamma, (float*)q);
    hipLaunchKernelGGL(k_fbp_bp<float>, bgrid, dim3(256), 0, st, p->gd, n_ch, (const float*)q,
                       scale, (float*)img);
  }
  return hipGetLastError();
}

hipError_t launch_nmar(const deam_plan* p, const void* sino, const uint8_t* mask, const void* pp,
                       double eps, void* out, hipStream_t st) {
  const dim3 grid((unsigned)p->gd.n_views);
  if (p->precision == DEAM_PREC_FP64)
    hipLaunchKernelGGL(k_nmar<double>, grid, dim3(256), 0, st, p->gd.n_cols, p->gd.R,
                       (const double*)sino, mask, (const double*)pp, eps, (double*)out);
  else
    hipLaunchKernelGGL(k_nmar<float>, grid, dim3(256), 0, st, p->gd.n_cols, p->gd.R,
                       (const float*)sino, mask, (const float*)pp, eps, (float*)out);
  return hipGetLastError();
}

hipError_t launch_mar_classes(const deam_plan* p, const void* mu0, const double water[2],
                              double fa, double fb, double fm, uint8_t* M, void* prior,
                              hipStream_t st) {
  const int64_t V = p->gd.V;
  const dim3 grid((unsigned)((V + 255) / 256));
  if (p->precision == DEAM_PREC_FP64)
    hipLaunchKernelGGL(k_mar_classes<double>, grid, dim3(256), 0, st, V, (const double*)mu0,
                       water[0], water[1], fa, fb, fm, M, (double*)prior);
  else
    hipLaunchKernelGGL(k_mar_classes<float>, grid, dim3(256), 0, st, V, (const float*)mu0,
                       water[0], water[1], fa, fb, fm, M, (float*)prior);
  return hipGetLastError();
}

hipError_t launch_decompose(const deam_plan* p, const void* mu, double* c64, hipStream_t st) {
  const int64_t V = p->gd.V;
  const dim3 grid((unsigned)((V + 255) / 256));
  const double* a = &p->mu_eff_inv[0][0];
  if (p->precision == DEAM_PREC_FP64)
    hipLaunchKernelGGL(k_decompose<double>, grid, dim3(256), 0, st, V, (const double*)mu, a[0],
                       a[1], a[2], a[3], c64);
  else
    hipLaunchKernelGGL(k_decompose<float>, grid, dim3(256), 0, st, V, (const float*)mu, a[0], a[1],
                       a[2], a[3], c64);
  return hipGetLastError();
}

hipError_t launch_dilate(const deam_plan* p, const uint8_t* mask, int radius, uint8_t* out,
                         hipStream_t st) {
  const int64_t R = p->gd.R;
  hipLaunchKernelGGL(k_dilate, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, st, R,
                     p->gd.n_cols, radius, mask, out);
  return hipGetLastError();
}

hipError_t launch_validate(const deam_plan* p, const double* c64, const float* d,
                           unsigned long long* cnt, hipStream_t st) {
  const int64_t nc = c64 ? 2 * p->gd.V : 0, nd = d ? 2 * p->gd.R : 0;
  const int64_t n = max(nc, nd);
  const int64_t nb = (n + 255) / 256;
  const unsigned blocks = (unsigned)(nb < 4096 ? nb : 4096);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate, dim3(blocks), dim3(256), 0, st, c64, nc, d, nd, cnt);
  return hipGetLastError();
}

hipError_t noalloc_scratch(void** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

hipError_t launch_pack_mask(const deam_plan* p, const uint8_t* mask, uint32_t* bits,
                            hipStream_t st) {
  const int64_t nw = (p->gd.R + 31) / 32;
  hipLaunchKernelGGL(k_pack_mask, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, st, p->gd.R,
                     mask, bits);
  return hipGetLastError();
}

}  // namespace deam





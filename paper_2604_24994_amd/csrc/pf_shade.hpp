// Per-(ray, cell) device math shared by the rasteriser, the ray walk and the
// backward pass, so that the two renderers evaluate every contribution's
// geometry with the same instructions (the radiance's lobe softmaxes are
// taken without the max shift in the rasteriser and with it in the walk,
// which holds the texture per lane in fewer registers; the two agree up to
// rounding).
//
// Numerics: the ray is generated in float64 and, per cell, re-expressed in
// the cell's local frame in float64: q = closest-approach offset from p_i,
// s = t - t_closest, so that x(t) - p_i = q + s d.  All lengths below are
// then small numbers near the cell, computed in float32 (IEEE division and
// square root are replaced by the hardware reciprocal and square root,
// <= 1 ulp).  The sphere discriminant is
// formed in float64 (it cancels near tangency).
#pragma once

#include <hip/hip_runtime.h>

#include "pf_internal.hpp"

namespace pf {

struct RayD {
  double ox, oy, oz;   // camera centre
  double dx, dy, dz;   // unit direction
  float fx, fy, fz;    // direction rounded to float
  bool valid;
};

// Equidistant fisheye: camera-frame direction at polar angle th of the
// pixel offset (ex, ey), rho = |(ex, ey)|.  Out of line, so that the float64
// sine and cosine constants stay in this function instead of occupying
// registers across the loops of the kernels that generate rays.
__device__ __attribute__((noinline)) double3 fisheye_dir(double ex, double ey, double rho, double th) {
  const double st = sin(th);
  double3 d;
  d.x = rho > 0.0 ? st * ex / rho : 0.0;
  d.y = rho > 0.0 ? st * ey / rho : 0.0;
  d.z = cos(th);
  return d;
}

// Ray through pixel-centre coordinates (u, v).
__device__ inline RayD make_ray(const pf_camera& c, double u, double v) {
  RayD r;
  double dcx, dcy, dcz;
  r.valid = true;
  if (c.model == 0) {
    dcx = (u - (double)c.cx) / (double)c.fx;
    dcy = (v - (double)c.cy) / (double)c.fy;
    dcz = 1.0;
  } else {
    const double ex = u - (double)c.cx, ey = v - (double)c.cy;
    const double rho = sqrt(ex * ex + ey * ey);
    const double th = rho / (double)c.f_fish;
    r.valid = th <= (double)c.theta_max;
    const double3 d = fisheye_dir(ex, ey, rho, th);
    dcx = d.x;
    dcy = d.y;
    dcz = d.z;
  }
  const float* m = c.c2w;
  double wx = (double)m[0] * dcx + (double)m[1] * dcy + (double)m[2] * dcz;
  double wy = (double)m[4] * dcx + (double)m[5] * dcy + (double)m[6] * dcz;
  double wz = (double)m[8] * dcx + (double)m[9] * dcy + (double)m[10] * dcz;
  // 1/|w|: hardware reciprocal square root refined by two Newton steps
  const double w2 = wx * wx + wy * wy + wz * wz;
  double inv = __builtin_amdgcn_rsq(w2);
  inv = inv * fma(-0.5 * w2 * inv, inv, 1.5);
  inv = inv * fma(-0.5 * w2 * inv, inv, 1.5);
  r.dx = wx * inv;
  r.dy = wy * inv;
  r.dz = wz * inv;
  r.ox = m[3];
  r.oy = m[7];
  r.oz = m[11];
  r.fx = (float)r.dx;
  r.fy = (float)r.dy;
  r.fz = (float)r.dz;
  return r;
}

__device__ inline float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
// Hardware square root (<= 1 ulp; the correctly rounded expansion costs a
// dozen instructions).
__device__ inline float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

constexpr float LOG2E_F = 1.4426950408889634f;

// exp(x - shift) as one fused multiply-add and the hardware exp2, with
// shift_l2 = shift * log2(e) formed once per softmax.
__device__ inline float exp_shifted(float x, float shift_l2) {
  return __builtin_amdgcn_exp2f(fmaf(x, LOG2E_F, -shift_l2));
}

// Local frame of the ray at a cell: q (float), beta = s at t = 0, and the
// squared closest-approach distance in float64.
struct Local {
  float qx, qy, qz;
  float beta;
  double qq;
  double b;          // float64 beta
  double dqx, dqy, dqz;  // float64 q
};

__device__ inline Local make_local(const RayD& R, float px, float py, float pz) {
  Local L;
  const double ocx = R.ox - (double)px, ocy = R.oy - (double)py, ocz = R.oz - (double)pz;
  const double b = ocx * R.dx + ocy * R.dy + ocz * R.dz;
  const double qx = ocx - b * R.dx, qy = ocy - b * R.dy, qz = ocz - b * R.dz;
  L.qx = (float)qx;
  L.qy = (float)qy;
  L.qz = (float)qz;
  L.dqx = qx;
  L.dqy = qy;
  L.dqz = qz;
  L.qq = qx * qx + qy * qy + qz * qz;
  L.b = b;
  L.beta = (float)b;
  return L;
}

// h - q.m of face plane (m, h) = pl as one fused chain from h, given -q: the
// ray x = p_i + q + s d meets the plane at s = (h - q.m) / (d.m).
__device__ inline float face_offset(const float4 pl, float nqx, float nqy, float nqz) {
  return fmaf(nqz, pl.z, fmaf(nqy, pl.y, fmaf(nqx, pl.x, pl.w)));
}

// Duff et al., "Building an Orthonormal Basis, Revisited" (JCGT 2017).
__device__ inline void onb(float nx, float ny, float nz, float& t1x, float& t1y, float& t1z, float& t2x,
                           float& t2y, float& t2z) {
  const float sign = copysignf(1.0f, nz);
  const float a = -frcp(sign + nz);   // |sign + nz| >= 1
  const float b = nx * ny * a;
  t1x = 1.0f + sign * nx * nx * a;
  t1y = sign * b;
  t1z = -sign * nx;
  t2x = b;
  t2y = sign + ny * ny * a;
  t2z = -ny;
}

// Softmax of up to 8 base-2 logits z into p (normalised in place by the
// caller): p_k = 2^z_k, returned sum.  The logits are exponentiated
// unshifted (2^z is exact in float range), and only when the sum leaves
// [2^-100, 2^100] (a logit near the range's ends) are they shifted by their
// largest, as a softmax usually is; *shift receives the shift (0 or that
// largest logit).  Saves the max and the subtraction on every call.
template <int N>
__device__ inline float softmax2_sum(const float (&z)[N], float (&p)[N], float* shift) {
  float sum = 0.0f;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    p[k] = __builtin_amdgcn_exp2f(z[k]);
    sum += p[k];
  }
  float sh = 0.0f;
  if (!(sum >= 0x1p-100f && sum <= 0x1p100f)) {
    sh = z[0];
#pragma unroll
    for (int k = 1; k < N; ++k) sh = fmaxf(sh, z[k]);
    sum = 0.0f;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      p[k] = __builtin_amdgcn_exp2f(z[k] - sh);
      sum += p[k];
    }
  }
  *shift = sh;
  return sum;
}

// Soft-Voronoi weights over the K detail sites at face point u (Sec. 3.4,
// Eq. svdisp / Eq. svrad).  The logits are shifted by tau*|u| and written as
//   |u - s_k| - |u| = (|s_k|^2 - 2 u.s_k) / (|u - s_k| + |u|),
// which keeps them accurate when u is far from the sites (grazing rays).
__device__ inline void sv_weights(const float* __restrict__ tx, float ux, float uy, float tau, float* w) {
  const float un = fsqrt(ux * ux + uy * uy);
  float mx = -INFINITY;
#pragma unroll
  for (int k = 0; k < KD; ++k) {
    const float sx = tx[k * TEXW + 0], sy = tx[k * TEXW + 1];
    const float ex = ux - sx, ey = uy - sy;
    const float dist = fsqrt(ex * ex + ey * ey);
    const float num = sx * sx + sy * sy - 2.0f * (ux * sx + uy * sy);
    const float den = dist + un;
    const float e = den > 0.0f ? num * frcp(den) : 0.0f;
    w[k] = -tau * e;
    mx = fmaxf(mx, w[k]);
  }
  float sum = 0.0f;
  const float mxl = mx * LOG2E_F;
#pragma unroll
  for (int k = 0; k < KD; ++k) {
    w[k] = exp_shifted(w[k], mxl);
    sum += w[k];
  }
  const float inv = frcp(sum);
#pragma unroll
  for (int k = 0; k < KD; ++k) w[k] *= inv;
}

// Sums of detail site t's M Spherical-Voronoi lobes for direction g = d log2(e):
// *sum = sum_m 2^(a_m.g - shift), (sr, sg, sb) = sum_m 2^(a_m.g - shift) c_m;
// returns the base-2 shift (softmax2_sum).
__device__ inline float sv_lobes(const float* __restrict__ t, float gx, float gy, float gz, float& sum, float& sr,
                                 float& sg, float& sb) {
  float lg[MA], e[MA], sh;
#pragma unroll
  for (int m = 0; m < MA; ++m) lg[m] = t[3 + 3 * m] * gx + t[4 + 3 * m] * gy + t[5 + 3 * m] * gz;
  sum = softmax2_sum(lg, e, &sh);
  sr = sg = sb = 0.0f;
#pragma unroll
  for (int m = 0; m < MA; ++m) {
    sr += e[m] * t[3 + 3 * MA + 3 * m];
    sg += e[m] * t[4 + 3 * MA + 3 * m];
    sb += e[m] * t[5 + 3 * MA + 3 * m];
  }
  return sh;
}

// Geometry of one (ray, cell) piece: bounded interval, dipole split and
// opacity.  faces/nfaces: the cell's raster faces.  Returns alpha (0 when
// the piece is empty) and the texture point u, plus what the backward needs.
struct Piece {
  float alpha;
  float ux, uy;       // texture point in the face frame
  float s0, s1;       // bounded interval (local s)
  float j0, j1;       // dense part
  int bind0, bind1;   // binding constraint of s0 / s1: -1 sphere, -2 camera, f >= 0 face index
  float den, sx, sbar, delta;
  float t1x, t1y, t1z, t2x, t2y, t2z;
};

// WAVE_CELL: every lane of the wave evaluates the same cell (the
// rasteriser).  Its faces and texture are then read through the scalar
// cache, the wave leaves the face loop as soon as no lane's interval is left,
// and, before the displacement weights, it tests whether the dense part is
// empty for every displacement the sites allow (for the walk's per-lane loads
// that test costs more than it saves).  Either way alpha is the same.
template <bool WAVE_CELL>
__device__ inline Piece piece_geometry(const RayD& R, const Local& L, float r, const float4* __restrict__ faces,
                                       int nfaces, float4 nrm, const float* __restrict__ tx, float tau) {
  Piece P;
  P.alpha = 0.0f;
  P.ux = P.uy = 0.0f;
  P.bind0 = P.bind1 = -1;
  const double D = (double)r * (double)r - L.qq;
  P.s0 = 1.0f;
  P.s1 = 0.0f;
  if (D <= 0.0) return P;
  const float sq = fsqrt((float)D);
  float s0 = -sq, s1 = sq;
  int b0 = -1, b1 = -1;
  const float fx = R.fx, fy = R.fy, fz = R.fz;
  // exit (a >= 0) and entry (a < 0) bounds by selects rather than branches.
  // a = d.m + 0 is never -0, so a face parallel to the ray (a = +0) gives
  // s = bb * (1/+0): -inf when the ray lies on its outer side (bb < 0),
  // which empties the interval, +inf (or NaN for bb = 0) otherwise, which
  // leaves it.  Once empty, an interval stays empty.
  const float nqx = -L.qx, nqy = -L.qy, nqz = -L.qz;
  auto clip = [&](const float4 pl, int f) {
    const float a = (fx * pl.x + fy * pl.y + fz * pl.z) + 0.0f;
    const float s = face_offset(pl, nqx, nqy, nqz) * frcp(a);
    const bool exits = a >= 0.0f;
    const bool out = exits && s < s1;
    const bool in = !exits && s > s0;
    s1 = out ? s : s1;
    b1 = out ? f : b1;
    s0 = in ? s : s0;
    b0 = in ? f : b0;
  };
  if constexpr (WAVE_CELL) {
    // two faces per step from one wave-uniform (scalar) address
    int f = 0;
    bool more = nfaces >= 2;
    float4 c0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), c1 = c0;
    if (more) {
      c0 = faces[0];
      c1 = faces[1];
    }
    while (more) {
      const float4 p0 = c0, p1 = c1;
      const int fn = f + 2;
      if (fn + 2 <= nfaces) {   // the next pair is loaded while this one is tested
        const float4* fp = faces + __builtin_amdgcn_readfirstlane(fn);
        c0 = fp[0];
        c1 = fp[1];
      }
      clip(p0, f);
      clip(p1, f + 1);
      f = fn;
      more = f + 2 <= nfaces && __any(s0 < s1);
    }
    if (f + 1 == nfaces) clip(faces[__builtin_amdgcn_readfirstlane(f)], f);
  } else {
    // (the next face is loaded while this one is tested)
    float4 nxt = nfaces > 0 ? faces[0] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (int f = 0; f < nfaces; ++f) {
      const float4 pl = nxt;
      if (f + 1 < nfaces) nxt = faces[f + 1];
      clip(pl, f);
    }
  }
  if (L.beta > s0) { s0 = L.beta; b0 = -2; }
  P.s0 = s0;
  P.s1 = s1;
  P.bind0 = b0;
  P.bind1 = b1;
  if (!(s0 < s1)) return P;

  // dipole face with displacement (Sec. 3.3, Sec. 3.4)
  const float nx = nrm.x, ny = nrm.y, nz = nrm.z;
  onb(nx, ny, nz, P.t1x, P.t1y, P.t1z, P.t2x, P.t2y, P.t2z);
  const float den = fx * nx + fy * ny + fz * nz;
  const float qn = L.qx * nx + L.qy * ny + L.qz * nz;
  const float qt1 = L.qx * P.t1x + L.qy * P.t1y + L.qz * P.t1z;
  const float qt2 = L.qx * P.t2x + L.qy * P.t2y + L.qz * P.t2z;
  const float dt1 = fx * P.t1x + fy * P.t1y + fz * P.t1z;
  const float dt2 = fx * P.t2x + fy * P.t2y + fz * P.t2z;
  P.den = den;
  float j0 = s0, j1 = s1;
  if (den != 0.0f) {
    const float idn = frcp(den);
    // The displacement is a convex combination of the sites' d_k, so the
    // displaced face lies between the faces moved by min d_k and max d_k.
    // When even the face moved by max d_k leaves [s0, s1] on the empty side
    // (beyond s1 going in, before s0 going out), the dense part is empty
    // whatever the weights: alpha = 0 without evaluating them.  The test
    // keeps a relative margin far above the rounding of the exact path, so
    // it only fires where that path gives an empty dense part too.
    if constexpr (WAVE_CELL) {
      float dmax = tx[2], dabs = fabsf(tx[2]);
#pragma unroll
      for (int k = 1; k < KD; ++k) {
        dmax = fmaxf(dmax, tx[k * TEXW + 2]);
        dabs = fmaxf(dabs, fabsf(tx[k * TEXW + 2]));
      }
      const float bound = (dmax + 1e-5f * dabs - qn) * idn;
      const float tol = 1e-4f * (fabsf(s0) + fabsf(s1) + fabsf(bound)) + 1e-30f;
      if (den > 0.0f ? bound + tol <= s0 : bound - tol >= s1) return P;
    }
    const float sbar = -qn * idn;
    float w[KD];
    sv_weights(tx, qt1 + sbar * dt1, qt2 + sbar * dt2, tau, w);
    float delta = 0.0f;
#pragma unroll
    for (int k = 0; k < KD; ++k) delta += w[k] * tx[k * TEXW + 2];
    const float sxx = (delta - qn) * idn;
    if (den > 0.0f) j1 = fminf(s1, sxx);
    else j0 = fmaxf(s0, sxx);
    P.ux = qt1 + sxx * dt1;
    P.uy = qt2 + sxx * dt2;
    P.sx = sxx;
    P.sbar = sbar;
    P.delta = delta;
  } else {
    const float sm = 0.5f * (s0 + s1);
    P.ux = qt1 + sm * dt1;
    P.uy = qt2 + sm * dt2;
    P.sx = 0.0f;
    P.sbar = 0.0f;
    P.delta = 0.0f;
    if (!(qn < 0.0f)) j1 = j0;
  }
  P.j0 = j0;
  P.j1 = j1;
  const float ell = fmaxf(j1 - j0, 0.0f);
  P.alpha = 1.0f - __expf(-nrm.w * ell);
  return P;
}

// Radiance at texture point u for direction d: base colour plus the
// soft-Voronoi blend of the detail sites' Spherical-Voronoi colours.
// WAVE_CELL = true (the rasteriser, one cell per wave, texture in scalar
// registers): the lobes are exponentiated in base 2 without the max shift;
// if any site's sum leaves [2^-100, 2^100], the colour is evaluated again
// with each site's logits shifted by their largest (as in softmax2_sum).
// That rare pass runs over the sites in a loop that is not unrolled, so that
// its texture reads are its own and the common pass holds no texture values
// for it.
template <bool WAVE_CELL>
__device__ inline void radiance(const float* __restrict__ tx, const float* __restrict__ rgb, float ux, float uy,
                                float fx, float fy, float fz, float tau, float& cr, float& cg, float& cb) {
  float w[KD];
  sv_weights(tx, ux, uy, tau, w);
  const float gx = fx * LOG2E_F, gy = fy * LOG2E_F, gz = fz * LOG2E_F;
  cr = rgb[0];
  cg = rgb[1];
  cb = rgb[2];
  bool in_range = true;
#pragma unroll
  for (int k = 0; k < KD; ++k) {
    const float* t = tx + k * TEXW;
    float sum = 0.0f, sr = 0.0f, sg = 0.0f, sb = 0.0f;
#pragma unroll
    for (int m = 0; m < MA; ++m) {
      const float e = __builtin_amdgcn_exp2f(t[3 + 3 * m] * gx + t[4 + 3 * m] * gy + t[5 + 3 * m] * gz);
      sum += e;
      sr += e * t[3 + 3 * MA + 3 * m];
      sg += e * t[4 + 3 * MA + 3 * m];
      sb += e * t[5 + 3 * MA + 3 * m];
    }
    in_range = in_range && sum >= 0x1p-100f && sum <= 0x1p100f;
    const float sc = w[k] * frcp(sum);
    cr += sc * sr;
    cg += sc * sg;
    cb += sc * sb;
  }
  if (!in_range) {
    cr = rgb[0];
    cg = rgb[1];
    cb = rgb[2];
#pragma unroll 1
    for (int k = 0; k < KD; ++k) {
      float wk = w[0];
#pragma unroll
      for (int j = 1; j < KD; ++j) wk = (k == j) ? w[j] : wk;
      const float* t = tx + k * TEXW;
      float mx = -INFINITY;
      for (int m = 0; m < MA; ++m) mx = fmaxf(mx, t[3 + 3 * m] * gx + t[4 + 3 * m] * gy + t[5 + 3 * m] * gz);
      float sum = 0.0f, sr = 0.0f, sg = 0.0f, sb = 0.0f;
      for (int m = 0; m < MA; ++m) {
        const float e =
            __builtin_amdgcn_exp2f(t[3 + 3 * m] * gx + t[4 + 3 * m] * gy + t[5 + 3 * m] * gz - mx);
        sum += e;
        sr += e * t[3 + 3 * MA + 3 * m];
        sg += e * t[4 + 3 * MA + 3 * m];
        sb += e * t[5 + 3 * MA + 3 * m];
      }
      const float sc = wk * frcp(sum);
      cr += sc * sr;
      cg += sc * sg;
      cb += sc * sb;
    }
  }
}


// WAVE_CELL = false (the walk: a cell per lane, the texture read per lane):
// every softmax shifted by its largest logit, which keeps fewer values live
// than the unshifted form with its rare shifted pass (the walk is held to 80
// VGPRs).
template <>
__device__ inline void radiance<false>(const float* __restrict__ tx, const float* __restrict__ rgb, float ux, float uy,
                                       float fx, float fy, float fz, float tau, float& cr, float& cg, float& cb) {
  float w[KD];
  sv_weights(tx, ux, uy, tau, w);
  cr = rgb[0];
  cg = rgb[1];
  cb = rgb[2];
#pragma unroll
  for (int k = 0; k < KD; ++k) {
    const float* t = tx + k * TEXW;
    float lg[MA];
    float mx = -INFINITY;
#pragma unroll
    for (int m = 0; m < MA; ++m) {
      lg[m] = t[3 + 3 * m] * fx + t[4 + 3 * m] * fy + t[5 + 3 * m] * fz;
      mx = fmaxf(mx, lg[m]);
    }
    float sum = 0.0f, sr = 0.0f, sg = 0.0f, sb = 0.0f;
    const float mxl = mx * LOG2E_F;
#pragma unroll
    for (int m = 0; m < MA; ++m) {
      const float e = exp_shifted(lg[m], mxl);
      sum += e;
      sr += e * t[3 + 3 * MA + 3 * m];
      sg += e * t[4 + 3 * MA + 3 * m];
      sb += e * t[5 + 3 * MA + 3 * m];
    }
    const float sc = w[k] * frcp(sum);
    cr += sc * sr;
    cg += sc * sg;
    cb += sc * sb;
  }
}

}  // namespace pf

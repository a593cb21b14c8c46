#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

// The FP32 Kalman filter shared by the tracklet constructor (tpc_track.hip)
// and the track refit (tpc_refit.hip): one track per lane.  Internal header of
// the library.
//
// State at plane x: (y, z, sin(phi), tan(lambda), q/pT); curvature C = k q/pT.
// Exact helix transport: sin2 = sin1 + C dx, dy = dx (sin1+sin2)/(cos1+cos2),
// dz = tan(lambda) s_T with s_T = sign(dx) L asin(u)/u, L = |(dx,dy)|, u = |C|L/2;
// analytic Jacobian for the covariance; no process noise.

namespace tpc_kf {

// Two forms of the state, which differ only in where the covariance (lower
// triangle, row-major, 15 entries) lives: KState keeps it in LDS, entry k at
// c[k * 64] (the lane's column of a [15][64] block, so the lanes of a wave
// hit distinct banks); KStateR keeps it in registers.  The functions below
// take either and reach entry k through cv(s, k).
struct KState {
  float p[5];
  float *c;
  float x, chi2;
};
struct KStateR {
  float p[5];
  float c[15];
  float x, chi2;
};
__device__ __forceinline__ float &cv(KState &s, int k) { return s.c[k * 64]; }
__device__ __forceinline__ float &cv(KStateR &s, int k) { return s.c[k]; }

__device__ __forceinline__ float asin_over(float u) {  // asin(u)/u
  const float u2 = u * u;
  if (u < 0.03f) return 1.f + u2 * (1.f / 6.f + u2 * (3.f / 40.f));
  return asinf(u) / u;
}
__device__ __forceinline__ float asin_over_dd(float u) {  // (d/du asin(u)/u) / u
  const float u2 = u * u;
  if (u < 0.2f) return 1.f / 3.f + u2 * (0.3f + u2 * (15.f / 56.f + u2 * (35.f / 144.f)));
  return (u / sqrtf(1.f - u2) - asinf(u)) / (u2 * u);
}

// Transport of the state to a plane x2, parameter part; kept so that the
// covariance part can follow once a hit is found in that row.
struct Step {
  float dx, C, s1, s2, c1, c2, D, N, iD, dy, L, u, fu, sT, sg;
};

template <class S>
__device__ __forceinline__ bool step_prepare(const S &s, float x2, float k, float sinmax, Step &t) {
  t.dx = x2 - s.x;
  t.C = k * s.p[4];
  t.s1 = s.p[2];
  t.s2 = t.s1 + t.C * t.dx;
  if (!(fabsf(t.s1) < sinmax) || !(fabsf(t.s2) < sinmax)) return false;
  t.c1 = sqrtf(1.f - t.s1 * t.s1);
  t.c2 = sqrtf(1.f - t.s2 * t.s2);
  t.D = t.c1 + t.c2;
  t.N = t.s1 + t.s2;
  t.iD = 1.f / t.D;
  t.dy = t.dx * t.N * t.iD;
  t.L = sqrtf(t.dx * t.dx + t.dy * t.dy);
  t.u = fabsf(t.C) * t.L * 0.5f;
  if (!(t.u < 1.f)) return false;
  t.sg = t.dx < 0.f ? -1.f : 1.f;
  t.fu = asin_over(t.u);
  t.sT = t.sg * t.L * t.fu;
  return true;
}

// Apply a prepared step: parameters, and the covariance through the analytic
// Jacobian.
template <class S>
__device__ __forceinline__ void step_apply(S &s, const Step &t, float x2, float k) {
  const float dx = t.dx, s1 = t.s1, s2 = t.s2, c1 = t.c1, c2 = t.c2, D = t.D, N = t.N, iD = t.iD;
  const float dy = t.dy, L = t.L, u = t.u, fu = t.fu, sT = t.sT, sg = t.sg, C = t.C;
  const float tgl = s.p[3];
  const float iD2 = iD * iD;
  const float a = dx * (2.f * D + N * (s1 / c1 + s2 / c2)) * iD2;
  const float b = dx * k * dx * (D + N * s2 / c2) * iD2;
  const float g = asin_over_dd(u);
  const float dsdy = L > 0.f ? sg * (dy / L) * (fu + u * u * g) : 0.f;
  const float dsdC = sg * C * L * L * L * g * 0.25f;
  const float cc = tgl * dsdy * a;
  const float d = sT;
  const float e = tgl * (dsdy * b + dsdC * k);
  const float f = k * dx;
  s.p[0] += dy;
  s.p[1] += tgl * sT;
  s.p[2] = s2;
  s.x = x2;
  // cov <- F cov F^T, F = I + {(0,2)=a, (0,4)=b, (1,2)=cc, (1,3)=d, (1,4)=e, (2,4)=f}
  const float P00 = cv(s, 0), P10 = cv(s, 1), P11 = cv(s, 2), P20 = cv(s, 3), P21 = cv(s, 4),
              P22 = cv(s, 5), P30 = cv(s, 6), P31 = cv(s, 7), P32 = cv(s, 8), P33 = cv(s, 9),
              P40 = cv(s, 10), P41 = cv(s, 11), P42 = cv(s, 12), P43 = cv(s, 13), P44 = cv(s, 14);
  // T = F P, rows 0..2
  const float T00 = P00 + a * P20 + b * P40, T02 = P20 + a * P22 + b * P42,
              T04 = P40 + a * P42 + b * P44;
  const float T10 = P10 + cc * P20 + d * P30 + e * P40, T11 = P11 + cc * P21 + d * P31 + e * P41,
              T12 = P21 + cc * P22 + d * P32 + e * P42, T13 = P31 + cc * P32 + d * P33 + e * P43,
              T14 = P41 + cc * P42 + d * P43 + e * P44;
  const float T20 = P20 + f * P40, T21 = P21 + f * P41, T22 = P22 + f * P42, T23 = P32 + f * P43,
              T24 = P42 + f * P44;
  cv(s, 0) = T00 + a * T02 + b * T04;
  cv(s, 1) = T10 + a * T12 + b * T14;
  cv(s, 2) = T11 + cc * T12 + d * T13 + e * T14;
  cv(s, 3) = T20 + a * T22 + b * T24;
  cv(s, 4) = T21 + cc * T22 + d * T23 + e * T24;
  cv(s, 5) = T22 + f * T24;
  cv(s, 6) = P30 + a * P32 + b * P43;
  cv(s, 7) = P31 + cc * P32 + d * P33 + e * P43;
  cv(s, 8) = P32 + f * P43;
  cv(s, 10) = P40 + a * P42 + b * P44;
  cv(s, 11) = P41 + cc * P42 + d * P43 + e * P44;
  cv(s, 12) = P42 + f * P44;
}

template <class S>
__device__ __forceinline__ void kf_update(S &s, float my, float mz, float sy2, float sz2) {
  const float r0 = my - s.p[0], r1 = mz - s.p[1];
  const float S00 = cv(s, 0) + sy2, S01 = cv(s, 1), S11 = cv(s, 2) + sz2;
  const float idet = 1.f / (S00 * S11 - S01 * S01);
  const float I00 = S11 * idet, I01 = -S01 * idet, I11 = S00 * idet;
  // columns 0 and 1 of P (P_i0, P_i1)
  const float q0[5] = {cv(s, 0), cv(s, 1), cv(s, 3), cv(s, 6), cv(s, 10)};
  const float q1[5] = {cv(s, 1), cv(s, 2), cv(s, 4), cv(s, 7), cv(s, 11)};
  float K0[5], K1[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    K0[i] = q0[i] * I00 + q1[i] * I01;
    K1[i] = q0[i] * I01 + q1[i] * I11;
    s.p[i] += K0[i] * r0 + K1[i] * r1;
  }
  int k = 0;
#pragma unroll
  for (int i = 0; i < 5; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j, ++k) cv(s, k) -= K0[i] * q0[j] + K1[i] * q1[j];
  s.chi2 += r0 * (I00 * r0 + I01 * r1) + r1 * (I01 * r0 + I11 * r1);
}

template <class S>
__device__ __forceinline__ void cov_reset(S &s, const float *cov0) {
#pragma unroll
  for (int i = 0; i < 15; ++i) cv(s, i) = 0.f;
  cv(s, 0) = cov0[0];
  cv(s, 2) = cov0[1];
  cv(s, 5) = cov0[2];
  cv(s, 9) = cov0[3];
  cv(s, 14) = cov0[4];
}

// measurement of hit h relative to the reference (exact: integer difference)
template <class S>
__device__ __forceinline__ void upd_hit(S &s, int2 yz, int Yr, int Zr, float sy2, float sz2) {
  kf_update(s, float(yz.x - Yr) * (1.f / 256.f), float(yz.y - Zr) * (1.f / 256.f), sy2, sz2);
}

// Three-point seed: the circle through (x0, 0), (x1, y1), (x2, y2) gives the
// curvature C and sin(phi) at the first point; tan(lambda) = z2 / s_T, with s_T
// the transverse arc length from the first point to the third.  y and z are
// relative to the first point.  The state starts at x0 with the diagonal
// covariance cov0.  False when the points are not distinct, the circle cannot
// join them or |sin(phi)| reaches smx.
template <class S>
__device__ __forceinline__ bool seed3(S &s, float x0, float x1, float x2, float y1, float y2, float z2,
                                      float k, float smx, const float *cov0) {
  const float ax = x1 - x0, ay = y1, bx = x2 - x0, by = y2, cx = x2 - x1, cy = y2 - y1;
  const float d12 = sqrtf(ax * ax + ay * ay), d13 = sqrtf(bx * bx + by * by), d23 = sqrtf(cx * cx + cy * cy);
  bool ok = d12 > 0.f && d13 > 0.f && d23 > 0.f;
  const float C = ok ? 2.f * (ax * by - ay * bx) / (d12 * d13 * d23) : 0.f;
  const float sa = ok ? C * d13 * 0.5f : 0.f;
  ok = ok && fabsf(sa) < 1.f;
  const float ca = sqrtf(fmaxf(0.f, 1.f - sa * sa));
  const float sphi = ok ? (by / d13) * ca - (bx / d13) * sa : 0.f;
  ok = ok && fabsf(sphi) < smx;
  const float sT = ok ? d13 * asin_over(fabsf(sa)) : 1.f;
  s.p[0] = 0.f;
  s.p[1] = 0.f;
  s.p[2] = sphi;
  s.p[3] = z2 / sT;
  s.p[4] = k != 0.f ? C / k : 0.f;
  s.x = x0;
  s.chi2 = 0.f;
  cov_reset(s, cov0);
  return ok;
}

}  // namespace tpc_kf

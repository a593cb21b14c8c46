/*
 * Closed-form crossings of charged-particle helices with the pad-row planes of
 * a TPC made of 2 x 18 trapezoidal sectors.  Part of the seeded synthetic-input
 * generator; it holds no step of the tracking method.
 *
 * Geometry (global frame, cm): sector s (0..35) has azimuth
 *   alpha_s = (s mod 18) * 20 deg + 10 deg,
 * sectors 0..17 see z > 0 (A side), 18..35 see z < 0 (C side).  Pad row i of a
 * sector is the straight line {P : P . e_s = x_i}, e_s = (cos a, sin a), limited
 * to |y_local| <= x_i * tan(half_open), y_local = P . (-sin a, cos a).
 *
 * Helix: vertex v, transverse direction phi0, signed curvature C = dphi/ds
 * (C = -kappa * Bz * q / pT), z = vz + tgl * s with s the transverse arc length.
 * Position at arc length s:  P(s) = c + (1/C) (sin phi, -cos phi),
 * phi = phi0 + C s, centre c = v + (1/C) (-sin phi0, cos phi0).
 * A crossing with row line (s, i) satisfies sin(phi - alpha) = C (x_i - c.e);
 * its local y is c.e_perp - cos(phi - alpha)/C.  The helix is followed for at
 * most max_turns full turns and while |z| <= z_max; with r_exit > 0 also only
 * up to the arc length where it first leaves the cylinder r = r_exit around
 * the beam axis (a particle that leaves the TPC through its outer wall does not
 * come back; loopers that stay inside keep their turns).
 *
 * Output: one record per crossing, ordered by (track, sector, row, arc length),
 * so the result does not depend on the number of threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define TWO_PI 6.283185307179586476925287

typedef struct {
  int32_t sector, row;
  double y, z, s;
  double sinphi_local; /* direction of the helix at the crossing, local frame */
  double cosphi_local;
} xing_t;

/* Arc length at which the helix first reaches distance r_exit from the beam
 * axis (the vertex lies inside), or infinity when it never does or r_exit <= 0. */
static double exit_arc(double vx, double vy, double curv, double phi0, double r_exit) {
  if (r_exit <= 0.0) return INFINITY;
  if (curv == 0.0) { /* |v + s u| = r_exit, u = (cos phi0, sin phi0), the positive root */
    const double vu = vx * cos(phi0) + vy * sin(phi0);
    return -vu + sqrt(vu * vu - (vx * vx + vy * vy) + r_exit * r_exit);
  }
  const double R = 1.0 / curv; /* signed */
  const double cx = vx - R * sin(phi0), cy = vy + R * cos(phi0);
  const double dc = sqrt(cx * cx + cy * cy);
  if (dc + fabs(R) <= r_exit) return INFINITY;
  /* |P|^2 = dc^2 + R^2 + 2 R dc sin(phi - psi), psi the direction of the centre */
  const double kap = (r_exit * r_exit - dc * dc - R * R) / (2.0 * R * dc);
  if (fabs(kap) > 1.0) return INFINITY;
  const double psi = atan2(cy, cx), a0 = asin(kap);
  double best = INFINITY;
  for (int k = 0; k < 2; ++k) {
    const double phi_star = psi + (k == 0 ? a0 : M_PI - a0);
    double dphi = fmod((phi_star - phi0) * (curv > 0 ? 1.0 : -1.0), TWO_PI);
    if (dphi < 0) dphi += TWO_PI;
    if (dphi / fabs(curv) < best) best = dphi / fabs(curv);
  }
  return best;
}

/* Enumerate crossings of one helix; store up to cap of them in out, return the count. */
static int64_t one_track(double vx, double vy, double vz, double curv, double phi0,
                         double tgl, int n_rows, const double *row_x, double tan_half,
                         double z_max, double max_turns, double r_exit, xing_t *out, int64_t cap) {
  int64_t n = 0;
  const double s_exit = exit_arc(vx, vy, curv, phi0, r_exit);
  for (int sec = 0; sec < 36; ++sec) {
    const double a = ((sec % 18) * 20.0 + 10.0) * (M_PI / 180.0);
    const double ca = cos(a), sa = sin(a);
    const int side = sec < 18 ? 1 : -1;
    for (int i = 0; i < n_rows; ++i) {
      const double xi = row_x[i];
      const double yhw = xi * tan_half;
      double cand_s[64];
      double cand_y[64];
      double cand_sp[64];
      double cand_cp[64];
      int nc = 0;
      if (curv == 0.0) {
        /* straight line: P = v + s (cos phi0, sin phi0) */
        const double den = cos(phi0 - a);
        if (den == 0.0) continue;
        const double s = (xi - (vx * ca + vy * sa)) / den;
        if (s <= 0.0) continue;
        const double px = vx + s * cos(phi0), py = vy + s * sin(phi0);
        cand_s[nc] = s;
        cand_y[nc] = -px * sa + py * ca;
        cand_sp[nc] = sin(phi0 - a);
        cand_cp[nc] = cos(phi0 - a);
        ++nc;
      } else {
        const double R = 1.0 / curv; /* signed */
        const double cx = vx - R * sin(phi0), cy = vy + R * cos(phi0);
        const double ce = cx * ca + cy * sa, cp = -cx * sa + cy * ca;
        const double w = curv * (xi - ce);
        if (fabs(w) > 1.0) continue;
        const double root = sqrt(1.0 - w * w);
        for (int br = 0; br < 2; ++br) {
          const double cosv = br == 0 ? root : -root; /* cos(phi - alpha) */
          const double yl = cp - cosv * R;
          if (fabs(yl) > yhw) continue;
          const double phi_star = a + atan2(w, cosv);
          double dphi = (phi_star - phi0) * (curv > 0 ? 1.0 : -1.0);
          dphi = fmod(dphi, TWO_PI);
          if (dphi < 0) dphi += TWO_PI;
          const double turn_len = TWO_PI / fabs(curv);
          for (int k = 0; k < 8; ++k) {
            const double s = dphi / fabs(curv) + k * turn_len;
            if (s > max_turns * turn_len) break;
            if (nc < 64) {
              cand_s[nc] = s;
              cand_y[nc] = yl;
              /* local direction: phi - alpha, with cos(phi - alpha) = cosv */
              cand_sp[nc] = w;
              cand_cp[nc] = cosv;
              ++nc;
            }
          }
        }
      }
      /* order by arc length, keep the ones inside the drift volume on this side */
      for (int p = 1; p < nc; ++p)
        for (int q = p; q > 0 && cand_s[q] < cand_s[q - 1]; --q) {
          double t;
          t = cand_s[q]; cand_s[q] = cand_s[q - 1]; cand_s[q - 1] = t;
          t = cand_y[q]; cand_y[q] = cand_y[q - 1]; cand_y[q - 1] = t;
          t = cand_sp[q]; cand_sp[q] = cand_sp[q - 1]; cand_sp[q - 1] = t;
          t = cand_cp[q]; cand_cp[q] = cand_cp[q - 1]; cand_cp[q - 1] = t;
        }
      for (int p = 0; p < nc; ++p) {
        const double z = vz + tgl * cand_s[p];
        if (fabs(z) > z_max || cand_s[p] > s_exit) continue;
        if ((side > 0 && !(z > 0.0)) || (side < 0 && !(z < 0.0))) continue;
        if (n < cap) {
          out[n].sector = sec;
          out[n].row = i;
          out[n].y = cand_y[p];
          out[n].z = z;
          out[n].s = cand_s[p];
          out[n].sinphi_local = cand_sp[p];
          out[n].cosphi_local = cand_cp[p];
        }
        ++n;
      }
    }
  }
  return n;
}

/*
 * Count (out_* == NULL) or fill the crossings of n_trk helices.
 * counts[t] receives the number of crossings of track t (count pass) and must
 * hold them on the fill pass; records of track t start at sum(counts[0..t)).
 * Returns the total number of crossings.
 */
int64_t synth_crossings(int64_t n_trk, const double *vx, const double *vy, const double *vz,
                        const double *curv, const double *phi0, const double *tgl,
                        int n_rows, const double *row_x, double tan_half, double z_max,
                        double max_turns, double r_exit, int64_t *counts, int32_t *out_sector,
                        int32_t *out_row, int32_t *out_track, double *out_y, double *out_z,
                        double *out_s, double *out_sinphi, double *out_cosphi) {
  const int fill = out_sector != NULL;
  int64_t *starts = NULL;
  if (fill) {
    starts = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_trk + 1));
    starts[0] = 0;
    for (int64_t t = 0; t < n_trk; ++t) starts[t + 1] = starts[t] + counts[t];
  }
  int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
  for (int64_t t = 0; t < n_trk; ++t) {
    xing_t buf[4096];
    xing_t *b = buf;
    int64_t cap = 4096;
    if (fill && counts[t] > cap) {
      b = (xing_t *)malloc(sizeof(xing_t) * (size_t)counts[t]);
      cap = counts[t];
    }
    int64_t n = one_track(vx[t], vy[t], vz[t], curv[t], phi0[t], tgl[t], n_rows, row_x,
                          tan_half, z_max, max_turns, r_exit, b, cap);
    if (!fill) {
      counts[t] = n;
    } else {
      const int64_t o = starts[t];
      for (int64_t j = 0; j < n && j < cap; ++j) {
        out_sector[o + j] = b[j].sector;
        out_row[o + j] = b[j].row;
        out_track[o + j] = (int32_t)t;
        out_y[o + j] = b[j].y;
        out_z[o + j] = b[j].z;
        out_s[o + j] = b[j].s;
        out_sinphi[o + j] = b[j].sinphi_local;
        out_cosphi[o + j] = b[j].cosphi_local;
      }
    }
    if (b != buf) free(b);
    total += n;
  }
  free(starts);
  return total;
}

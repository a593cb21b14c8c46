/*
 * TPC sector track finding: plain CPU reference ("oracle").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code, header or table with the HIP library:
 * both read the same input arrays and parameter values and nothing else.
 *
 * Precision: every discrete decision in int64 on quantized coordinates; the
 * Kalman fit in FP64.  Plain loops, no blocking, no fusion: each function
 * follows one step of the method in order, so it can be read against the
 * description it cites.
 *
 * What the paper fixes: TPC track finding over all hits of a time frame is the
 * dominant synchronous workload (paper §2.1); it runs on continuous-readout data
 * with overlapping collisions and no a-priori absolute z (paper §2.3); its cost
 * grows with the number of fitted tracks and attached clusters (paper §3.2).
 * The paper does not spell out the algorithm's steps; the steps below are the
 * readings this build adopts (hit grid, row-pair neighbours, reciprocal
 * cleaning, cellular-automaton chains, two-pass Kalman tracklet construction,
 * ownership-based selection), each stated at the function that implements it.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>

#define M_PI_ORC 3.14159265358979323846
#endif

#define KAPPA 0.00299792458 /* GeV / (T cm): pT = KAPPA * B * R */

typedef struct {
  int32_t q_shift;      /* quantum = 2^-q_shift cm; only 8 is accepted */
  int32_t tan_half_q16; /* tan(half sector opening) * 2^16 */
  int32_t bin_y_q;      /* grid bin width in y, quanta */
  int32_t bin_occ;      /* target hits per grid bin */
  int32_t bin_zmin_q;   /* smallest grid bin length in z, quanta */
  int32_t win_y_q;      /* neighbour window, y, quanta */
  int32_t win_z_q;      /* neighbour window, z, quanta */
  int32_t w_y, w_z;     /* residual weights */
  int32_t pad0;
  int64_t smax_k;       /* score cut S_max(i) = smax_k (X_{i+1} - X_{i-1})^2 */
  int32_t l_min;        /* minimum chain length for a seed */
  int32_t ext_win_y_q;  /* pickup window, y */
  int32_t ext_win_z_q;  /* pickup window, z */
  int32_t ext_edge_q;   /* stop when |Y_pred| > H + ext_edge_q */
  int32_t max_miss;     /* consecutive misses before a walk stops */
  int32_t n_min;        /* selector: minimum owned hits */
  int32_t f_min_q8;     /* selector: minimum owned fraction * 256 */
  int32_t brute;        /* 1: search whole rows instead of the grid (pin mode) */
  double sinphi_max;
  double sigma_y, sigma_z;
  double cov0[5];
  double fragile_eps;   /* rounding-boundary margin (quanta) for the fragile flag */
} orc_params_t;

typedef struct {
  int64_t n, n_units, n_rows, n_seg, n_cells, n_tracklets, n_tracks, n_track_hits;
  int32_t status;
  int32_t pad;
  /* per sorted position (global index space) */
  int32_t *perm, *up, *dn, *upc, *dnc;
  uint32_t *owner;
  /* per input cluster */
  int32_t *cluster_track;
  /* per (unit,row) segment */
  int32_t *seg_start, *seg_count, *seg_zmin, *seg_zmax, *seg_ny, *seg_nz, *seg_by, *seg_bz,
      *seg_cell_base;
  int32_t *cell_start; /* [n_cells + 1], sorted position of each cell's first hit */
  /* per tracklet (ordered by unit, then by grid position of the start hit) */
  int32_t *trk_start, *trk_unit, *trk_len, *trk_nfit, *trk_p1n, *trk_owned, *trk_keep,
      *trk_fragile;
  uint32_t *trk_key;
  double *trk_params, *trk_cov, *trk_xref, *trk_chi2;
  int32_t *trk_hits; /* [n_tracklets][n_rows], pass-2 order (outermost first), -1 padded */
  /* per kept track */
  int32_t *track_tracklet, *track_first_hit, *track_n_hits, *track_hits; /* hits: cluster ids */
  double time_s[8];
} orc_result_t;

enum { ORC_OK = 0, ORC_INVALID = -1 };

/* ------------------------------------------------------------------------- */
/* integer helpers                                                            */

static int64_t floor_div(int64_t a, int64_t b) { /* b > 0 */
  int64_t q = a / b;
  if ((a % b != 0) && (a < 0)) --q;
  return q;
}
static int64_t clamp64(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return ts.tv_sec + 1e-9 * ts.tv_nsec;
}

/* ------------------------------------------------------------------------- */
/* O1 quantization.  Reading: every decision uses coordinates rounded to      */
/* 1/256 cm, round-half-to-even; scaling by a power of two is exact, so the   */
/* integers do not depend on the precision the rounding is done in.           */

static int64_t quantize(double v) { return (int64_t)nearbyint(v * 256.0); }

/* ------------------------------------------------------------------------- */
/* O2 hit grid.  Per (unit,row): y range [-H, H] with H = (X tan_half) >> 16; */
/* z range = data-driven [Zmin, Zmax] over the row's hits (continuous readout */
/* gives no a-priori z, paper §2.3); z bins adapt to the row's occupancy.     */

typedef struct {
  int64_t H, by, ny, zmin, zmax, bz, nz;
} seg_geom_t;

static seg_geom_t seg_geometry(int64_t X, int64_t count, int64_t zmin, int64_t zmax,
                               const orc_params_t *P) {
  seg_geom_t g;
  g.H = (X * P->tan_half_q16) >> 16;
  g.by = P->bin_y_q;
  if (g.by < 2 * g.H / 63 + 1) g.by = 2 * g.H / 63 + 1; /* at most 63 y bins */
  g.ny = 2 * g.H / g.by + 1;
  if (count == 0) { zmin = 0; zmax = 0; }
  g.zmin = zmin;
  g.zmax = zmax;
  const int64_t span = zmax - zmin;
  const int64_t per = (int64_t)P->bin_occ * g.ny;
  int64_t nz_occ = (count + per - 1) / per;
  if (nz_occ < 1) nz_occ = 1;
  const int64_t nz_span = span / P->bin_zmin_q + 1;
  g.nz = nz_occ < nz_span ? nz_occ : nz_span;
  if (g.nz < 1) g.nz = 1;
  g.bz = span / g.nz + 1;
  return g;
}

static int64_t bin_of(const seg_geom_t *g, int64_t Y, int64_t Z) {
  const int64_t iy = clamp64(Y + g->H, 0, 2 * g->H) / g->by;
  const int64_t iz = (Z - g->zmin) / g->bz;
  return iz * g->ny + iy;
}

typedef struct {
  int64_t row, bin, id;
} sort_key_t;

static int cmp_key(const void *a, const void *b) {
  const sort_key_t *x = (const sort_key_t *)a, *y = (const sort_key_t *)b;
  if (x->row != y->row) return x->row < y->row ? -1 : 1;
  if (x->bin != y->bin) return x->bin < y->bin ? -1 : 1;
  if (x->id != y->id) return x->id < y->id ? -1 : 1;
  return 0;
}

/* ------------------------------------------------------------------------- */
/* per-unit working state                                                     */

typedef struct {
  const orc_params_t *P;
  int64_t a, b;          /* unit range in the global index space */
  int64_t n_rows;
  const int64_t *X;      /* quantized row positions */
  const double *xr;      /* row positions, cm */
  int64_t *Ys, *Zs;      /* quantized coordinates by sorted position (global index space) */
  seg_geom_t *sg;        /* [n_rows] of this unit */
  int64_t *rstart;       /* [n_rows + 1] sorted start of each row */
  int64_t *cbase;        /* [n_rows] first global cell of each row */
  const int32_t *cell_start;
  const int32_t *perm;
  double k;              /* -KAPPA * Bz: curvature per unit q/pT */
} unit_ctx_t;

/* Candidate positions of row j for a window; grid mode visits the bins that
 * cover [ylo, yhi] x [zlo, zhi], brute mode the whole row.  The caller applies
 * the exact predicate, so both modes give the same decisions. */
typedef struct {
  int64_t p, pend;        /* current position / end of the current run */
  int64_t iy0, iy1, iz, iz1;
  int64_t row;
  int brute;
  const unit_ctx_t *u;
} cand_iter_t;

static void cand_begin(cand_iter_t *it, const unit_ctx_t *u, int64_t row, int64_t ylo,
                       int64_t yhi, int64_t zlo, int64_t zhi) {
  it->u = u;
  it->row = row;
  it->brute = u->P->brute;
  if (it->brute) {
    it->p = u->rstart[row];
    it->pend = u->rstart[row + 1];
    it->iz = it->iz1 = 0;
    return;
  }
  const seg_geom_t *g = &u->sg[row];
  it->p = it->pend = 0;
  if (u->rstart[row + 1] == u->rstart[row] || zhi < g->zmin || zlo > g->zmax || yhi < ylo ||
      zhi < zlo) {
    it->iz = 1;
    it->iz1 = 0; /* empty */
    return;
  }
  const int64_t span = g->zmax - g->zmin;
  it->iy0 = clamp64(ylo + g->H, 0, 2 * g->H) / g->by;
  it->iy1 = clamp64(yhi + g->H, 0, 2 * g->H) / g->by;
  it->iz = clamp64(zlo - g->zmin, 0, span) / g->bz;
  it->iz1 = clamp64(zhi - g->zmin, 0, span) / g->bz;
  it->iz -= 1; /* advanced on first call */
}

/* Returns the next candidate sorted position, or -1. */
static int64_t cand_next(cand_iter_t *it) {
  for (;;) {
    if (it->p < it->pend) return it->p++;
    if (it->brute) return -1;
    it->iz += 1;
    if (it->iz > it->iz1) return -1;
    const unit_ctx_t *u = it->u;
    const seg_geom_t *g = &u->sg[it->row];
    const int64_t c0 = u->cbase[it->row] + it->iz * g->ny + it->iy0;
    const int64_t c1 = u->cbase[it->row] + it->iz * g->ny + it->iy1;
    it->p = u->cell_start[c0];
    it->pend = u->cell_start[c1 + 1];
  }
}

/* ------------------------------------------------------------------------- */
/* O3 neighbour finder.  Reading: for hit m in row i (1 <= i <= n_rows-2),     */
/* candidates n in rows j = i -/+ 1 must lie in an origin-pointing window in   */
/* y (|Y_n X_i - Y_m X_j| <= W_y X_i; the collision vertex is at the          */
/* transverse origin) and a plain window in z (|Z_n - Z_m| <= W_z; no vertex   */
/* pointing in z because continuous readout has no absolute z, paper §2.3).   */
/* Over all pairs (d below, u above) the straight-line residual at m,          */
/*   R = (V_d - V_m)(X_u - X_i) + (V_u - V_m)(X_i - X_d)  for V = Y, Z,         */
/* gives score = w_y R_y^2 + w_z R_z^2; the pair with the least                 */
/* (score, id_d, id_u) is kept if score <= smax_k (X_{i+1} - X_{i-1})^2.       */

static int in_window(const unit_ctx_t *u, int64_t n, int64_t m, int64_t Xi, int64_t Xj) {
  const orc_params_t *P = u->P;
  const int64_t lhs = u->Ys[n] * Xi - u->Ys[m] * Xj;
  if (llabs(lhs) > (int64_t)P->win_y_q * Xi) return 0;
  if (llabs(u->Zs[n] - u->Zs[m]) > P->win_z_q) return 0;
  return 1;
}

static void window_bounds(const unit_ctx_t *u, int64_t m, int64_t Xi, int64_t Xj, int64_t *ylo,
                          int64_t *yhi, int64_t *zlo, int64_t *zhi) {
  const orc_params_t *P = u->P;
  *ylo = floor_div(u->Ys[m] * Xj - (int64_t)P->win_y_q * Xi, Xi);
  *yhi = floor_div(u->Ys[m] * Xj + (int64_t)P->win_y_q * Xi, Xi) + 1;
  *zlo = u->Zs[m] - P->win_z_q;
  *zhi = u->Zs[m] + P->win_z_q;
}

static void find_neighbours(const unit_ctx_t *u, int32_t *up, int32_t *dn) {
  const orc_params_t *P = u->P;
  for (int64_t p = u->a; p < u->b; ++p) up[p] = dn[p] = -1;
  for (int64_t i = 1; i + 1 < u->n_rows; ++i) {
    const int64_t Xi = u->X[i], Xd = u->X[i - 1], Xu = u->X[i + 1];
    const int64_t dxd = Xi - Xd, dxu = Xu - Xi;
    const int64_t smax = P->smax_k * (Xu - Xd) * (Xu - Xd);
    for (int64_t m = u->rstart[i]; m < u->rstart[i + 1]; ++m) {
      int64_t best_s = INT64_MAX, best_d = -1, best_u = -1, best_id_d = 0, best_id_u = 0;
      int64_t ylo, yhi, zlo, zhi;
      cand_iter_t itd;
      window_bounds(u, m, Xi, Xd, &ylo, &yhi, &zlo, &zhi);
      cand_begin(&itd, u, i - 1, ylo, yhi, zlo, zhi);
      for (int64_t d; (d = cand_next(&itd)) >= 0;) {
        if (!in_window(u, d, m, Xi, Xd)) continue;
        int64_t ylo2, yhi2, zlo2, zhi2;
        cand_iter_t itu;
        window_bounds(u, m, Xi, Xu, &ylo2, &yhi2, &zlo2, &zhi2);
        cand_begin(&itu, u, i + 1, ylo2, yhi2, zlo2, zhi2);
        for (int64_t w; (w = cand_next(&itu)) >= 0;) {
          if (!in_window(u, w, m, Xi, Xu)) continue;
          const int64_t Ry = (u->Ys[d] - u->Ys[m]) * dxu + (u->Ys[w] - u->Ys[m]) * dxd;
          const int64_t Rz = (u->Zs[d] - u->Zs[m]) * dxu + (u->Zs[w] - u->Zs[m]) * dxd;
          const __int128 s128 = (__int128)P->w_y * Ry * Ry + (__int128)P->w_z * Rz * Rz;
          if (s128 > smax) continue;
          const int64_t s = (int64_t)s128;
          const int64_t idd = u->perm[d], idu = u->perm[w];
          if (s < best_s || (s == best_s && (idd < best_id_d || (idd == best_id_d && idu < best_id_u)))) {
            best_s = s;
            best_d = d;
            best_u = w;
            best_id_d = idd;
            best_id_u = idu;
          }
        }
      }
      if (best_d >= 0) {
        dn[m] = (int32_t)best_d;
        up[m] = (int32_t)best_u;
      }
    }
  }
}

/* ------------------------------------------------------------------------- */
/* O4 cleaner.  Reading: a link survives only if it is mutual.                 */

static void clean_links(int64_t a, int64_t b, const int32_t *up, const int32_t *dn, int32_t *upc,
                        int32_t *dnc) {
  for (int64_t m = a; m < b; ++m) {
    upc[m] = (up[m] >= 0 && dn[up[m]] == m) ? up[m] : -1;
    dnc[m] = (dn[m] >= 0 && up[dn[m]] == m) ? dn[m] : -1;
  }
}

/* ------------------------------------------------------------------------- */
/* Helix model for the Kalman filter.  State at plane x:                      */
/*   p = (y, z, sin(phi), tan(lambda), q/pT),  curvature C = k q/pT,           */
/*   k = -KAPPA Bz, C = dphi/ds (s = transverse arc length).                   */
/* Exact helix transport along x:                                              */
/*   sin(phi2) = sin(phi1) + C dx,                                             */
/*   dy = dx (sin1 + sin2) / (cos1 + cos2),                                    */
/*   dz = tan(lambda) s_T,  s_T = sign(dx) L asin(u)/u,  L = |(dx,dy)|, u = |C| L/2. */

static double asin_over(double u) { /* asin(u)/u */
  if (u < 1e-3) return 1.0 + u * u / 6.0;
  return asin(u) / u;
}
static double asin_over_d(double u) { /* (d/du asin(u)/u) / u */
  if (u < 1e-3) return 1.0 / 3.0 + 0.3 * u * u;
  return (u / sqrt(1.0 - u * u) - asin(u)) / (u * u * u);
}

/* Propagate p from x1 to x2.  F (if not NULL) receives the 5x5 Jacobian,
 * row-major.  Returns 0, or -1 when the helix cannot reach x2 within
 * |sin(phi)| < sinphi_max. */
int orc_propagate(const double p[5], double x1, double x2, double k, double sinphi_max,
                  double out[5], double F[25]) {
  const double dx = x2 - x1;
  const double C = k * p[4];
  const double s1 = p[2], s2 = s1 + C * dx;
  if (fabs(s1) >= sinphi_max || fabs(s2) >= sinphi_max) return -1;
  const double c1 = sqrt(1.0 - s1 * s1), c2 = sqrt(1.0 - s2 * s2);
  const double D = c1 + c2, N = s1 + s2;
  const double dy = dx * N / D;
  const double L = sqrt(dx * dx + dy * dy);
  const double u = fabs(C) * L * 0.5;
  if (u >= 1.0) return -1;
  const double sgn = dx < 0 ? -1.0 : 1.0;
  const double fu = asin_over(u);
  const double sT = sgn * L * fu;
  out[0] = p[0] + dy;
  out[1] = p[1] + p[3] * sT;
  out[2] = s2;
  out[3] = p[3];
  out[4] = p[4];
  if (F) {
    memset(F, 0, 25 * sizeof(double));
    for (int i = 0; i < 5; ++i) F[i * 5 + i] = 1.0;
    /* d dy / d sin1 and d dy / d(q/pT) */
    const double dT_ds1 = (2.0 * D + N * (s1 / c1 + s2 / c2)) / (D * D);
    const double dT_dq = k * dx * (D + N * s2 / c2) / (D * D);
    const double a = dx * dT_ds1, b = dx * dT_dq;
    /* s_T as a function of dy and C */
    const double g = asin_over_d(u);
    const double dsT_ddy = (L > 0) ? sgn * (dy / L) * (fu + u * u * g) : 0.0;
    const double dsT_dC = sgn * C * L * L * L * g * 0.25;
    F[0 * 5 + 2] = a;
    F[0 * 5 + 4] = b;
    F[1 * 5 + 2] = p[3] * dsT_ddy * a;
    F[1 * 5 + 3] = sT;
    F[1 * 5 + 4] = p[3] * (dsT_ddy * b + dsT_dC * k);
    F[2 * 5 + 4] = k * dx;
  }
  return 0;
}

/* cov <- F cov F^T (full 5x5 products). */
static void transport_cov(const double F[25], double cov[25]) {
  double T[25], R[25];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) {
      double s = 0;
      for (int l = 0; l < 5; ++l) s += F[i * 5 + l] * cov[l * 5 + j];
      T[i * 5 + j] = s;
    }
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) {
      double s = 0;
      for (int l = 0; l < 5; ++l) s += T[i * 5 + l] * F[j * 5 + l];
      R[i * 5 + j] = s;
    }
  memcpy(cov, R, sizeof(R));
}

/* Kalman measurement update with (my, mz), R = diag(sy^2, sz^2).  Adds the
 * residual's chi2 to *chi2. */
static void kf_update(double p[5], double cov[25], double my, double mz, double sy, double sz,
                      double *chi2) {
  const double r0 = my - p[0], r1 = mz - p[1];
  const double S00 = cov[0] + sy * sy, S01 = cov[1], S11 = cov[6] + sz * sz;
  const double det = S00 * S11 - S01 * S01;
  const double I00 = S11 / det, I01 = -S01 / det, I11 = S00 / det;
  double K[5][2];
  for (int i = 0; i < 5; ++i) {
    K[i][0] = cov[i * 5 + 0] * I00 + cov[i * 5 + 1] * I01;
    K[i][1] = cov[i * 5 + 0] * I01 + cov[i * 5 + 1] * I11;
  }
  for (int i = 0; i < 5; ++i) p[i] += K[i][0] * r0 + K[i][1] * r1;
  double nc[25];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j)
      nc[i * 5 + j] = cov[i * 5 + j] - (K[i][0] * cov[0 * 5 + j] + K[i][1] * cov[1 * 5 + j]);
  memcpy(cov, nc, sizeof(nc));
  *chi2 += r0 * (I00 * r0 + I01 * r1) + r1 * (I01 * r0 + I11 * r1);
}

/* Seed from three points (Reading): the circle through (x,y) of the first,
 * middle and last chain hits gives the curvature C and sin(phi) at the first
 * hit; tan(lambda) = (z3 - z1) / s_T(1 -> 3).  Returns 0 or -1. */
int orc_seed(const double x[3], const double y[3], const double z[3], double k,
             double sinphi_max, double p[5]) {
  const double ax = x[1] - x[0], ay = y[1] - y[0];
  const double bx = x[2] - x[0], by = y[2] - y[0];
  const double cx = x[2] - x[1], cy = y[2] - y[1];
  const double d12 = sqrt(ax * ax + ay * ay), d13 = sqrt(bx * bx + by * by),
               d23 = sqrt(cx * cx + cy * cy);
  if (d12 <= 0 || d13 <= 0 || d23 <= 0) return -1;
  const double cross = ax * by - ay * bx;
  const double C = 2.0 * cross / (d12 * d13 * d23);
  const double sa = C * d13 * 0.5; /* sin of half the turning angle 1 -> 3 */
  if (fabs(sa) >= 1.0) return -1;
  const double ca = sqrt(1.0 - sa * sa);
  const double spsi = by / d13, cpsi = bx / d13;
  const double sphi = spsi * ca - cpsi * sa;
  if (fabs(sphi) >= sinphi_max) return -1;
  const double sT = d13 * asin_over(fabs(sa));
  p[0] = y[0];
  p[1] = z[0];
  p[2] = sphi;
  p[3] = (z[2] - z[0]) / sT;
  p[4] = (k != 0.0) ? C / k : 0.0;
  return 0;
}

/* ------------------------------------------------------------------------- */
/* O6 tracklet constructor.                                                    */
/* Reading: pass 1 fits the chain from its inner end upward and then extends   */
/* it row by row to the last row, picking in each row the hit nearest to the    */
/* rounded prediction inside a fixed window (least (w_y dY^2 + w_z dZ^2, id)),  */
/* stopping after more than max_miss consecutive empty rows, when |sin(phi)|    */
/* reaches sinphi_max or when the prediction leaves the sector.  Pass 2 starts  */
/* at the outermost pass-1 hit with the covariance reset, walks down to row 0,  */
/* reuses the pass-1 hits, picks hits in the other rows by the same rule, and   */
/* its last update gives the tracklet's parameters at its innermost hit.       */

typedef struct {
  int found;      /* picked sorted position or -1 */
  int stop;       /* 1 = the prediction left the sector */
} pick_t;

static pick_t pick_with(const unit_ctx_t *u, int64_t row, int64_t Yp, int64_t Zp) {
  const orc_params_t *P = u->P;
  pick_t r = {-1, 0};
  const seg_geom_t *g = &u->sg[row];
  if (llabs(Yp) > g->H + P->ext_edge_q) {
    r.stop = 1;
    return r;
  }
  int64_t best_s = INT64_MAX, best_id = INT64_MAX, best = -1;
  cand_iter_t it;
  cand_begin(&it, u, row, Yp - P->ext_win_y_q, Yp + P->ext_win_y_q, Zp - P->ext_win_z_q,
             Zp + P->ext_win_z_q);
  for (int64_t c; (c = cand_next(&it)) >= 0;) {
    const int64_t dY = u->Ys[c] - Yp, dZ = u->Zs[c] - Zp;
    if (llabs(dY) > P->ext_win_y_q || llabs(dZ) > P->ext_win_z_q) continue;
    const int64_t s = (int64_t)P->w_y * dY * dY + (int64_t)P->w_z * dZ * dZ;
    const int64_t id = u->perm[c];
    if (s < best_s || (s == best_s && id < best_id)) {
      best_s = s;
      best_id = id;
      best = c;
    }
  }
  r.found = (int)best;
  return r;
}

/* Rounded prediction and pick; flags the decision fragile when another
 * rounding of a value within fragile_eps of a rounding boundary would change
 * it (a different pick or a different stop). */
static pick_t pick(const unit_ctx_t *u, int64_t row, double yp, double zp, int *fragile) {
  const double vy = yp * 256.0, vz = zp * 256.0;
  if (!(fabs(vy) < 4e15) || !(fabs(vz) < 4e15)) {
    pick_t r = {-1, 1};
    return r;
  }
  const int64_t Yp = (int64_t)nearbyint(vy), Zp = (int64_t)nearbyint(vz);
  pick_t r = pick_with(u, row, Yp, Zp);
  const double eps = u->P->fragile_eps;
  if (eps > 0) {
    const double fy = vy - floor(vy), fz = vz - floor(vz);
    const int ny = fabs(fy - 0.5) < eps, nz = fabs(fz - 0.5) < eps;
    if (ny || nz) {
      const int64_t ay[2] = {(int64_t)floor(vy), (int64_t)floor(vy) + 1};
      const int64_t az[2] = {(int64_t)floor(vz), (int64_t)floor(vz) + 1};
      for (int i = 0; i < (ny ? 2 : 1); ++i)
        for (int j = 0; j < (nz ? 2 : 1); ++j) {
          const int64_t Y2 = ny ? ay[i] : Yp, Z2 = nz ? az[j] : Zp;
          pick_t r2 = pick_with(u, row, Y2, Z2);
          if (r2.found != r.found || r2.stop != r.stop) *fragile = 1;
        }
    }
  }
  return r;
}

typedef struct {
  double p[5], cov[25], x, chi2;
} kstate_t;

static void cov_init(double cov[25], const orc_params_t *P) {
  memset(cov, 0, 25 * sizeof(double));
  for (int i = 0; i < 5; ++i) cov[i * 5 + i] = P->cov0[i];
}

/* one propagation step with covariance; flags closeness to the sin(phi) limit */
static int step_to(kstate_t *s, double x2, double k, const orc_params_t *P, int *fragile) {
  double np[5], F[25];
  if (orc_propagate(s->p, s->x, x2, k, P->sinphi_max, np, F) != 0) {
    const double s2 = s->p[2] + k * s->p[4] * (x2 - s->x);
    if (fabs(fabs(s2) - P->sinphi_max) < 1e-5) *fragile = 1;
    return -1;
  }
  if (fabs(fabs(np[2]) - P->sinphi_max) < 1e-5) *fragile = 1;
  memcpy(s->p, np, sizeof(np));
  transport_cov(F, s->cov);
  s->x = x2;
  return 0;
}

static void upd(kstate_t *s, const unit_ctx_t *u, int64_t h) {
  kf_update(s->p, s->cov, (double)u->Ys[h] / 256.0, (double)u->Zs[h] / 256.0, u->P->sigma_y,
            u->P->sigma_z, &s->chi2);
}

static int64_t row_of(const unit_ctx_t *u, int64_t h) {
  int64_t lo = 0, hi = u->n_rows - 1; /* last row r with rstart[r] <= h */
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (u->rstart[mid] <= h) lo = mid; else hi = mid - 1;
  }
  return lo;
}

typedef struct {
  int32_t len, nfit, p1n, fragile;
  double p[5], cov[15], xref, chi2;
  int32_t *hits; /* [n_rows] pass-2 hits, outermost first */
} tracklet_out_t;

static void pack_cov(const double c[25], double out[15]) {
  int k = 0;
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j <= i; ++j) out[k++] = c[i * 5 + j];
}

static void construct(const unit_ctx_t *u, int64_t start, const int32_t *upc, tracklet_out_t *t) {
  const orc_params_t *P = u->P;
  const int64_t R = u->n_rows;
  int64_t *chain = (int64_t *)malloc(sizeof(int64_t) * (size_t)R);
  int64_t *p1hit = (int64_t *)malloc(sizeof(int64_t) * (size_t)R);
  int64_t L = 0;
  for (int64_t h = start; h >= 0 && L < R; h = upc[h]) chain[L++] = h;
  t->len = (int32_t)L;
  t->nfit = 0;
  t->p1n = 0;
  t->fragile = 0;
  t->chi2 = 0;
  t->xref = 0;
  memset(t->p, 0, sizeof(t->p));
  memset(t->cov, 0, sizeof(t->cov));
  for (int64_t r = 0; r < R; ++r) t->hits[r] = -1;
  if (L < P->l_min) goto done;
  {
    const int64_t r1 = row_of(u, chain[0]);
    double sx[3], sy[3], sz[3];
    const int64_t idx[3] = {0, L / 2, L - 1};
    for (int i = 0; i < 3; ++i) {
      const int64_t h = chain[idx[i]];
      sx[i] = u->xr[r1 + idx[i]];
      sy[i] = (double)u->Ys[h] / 256.0;
      sz[i] = (double)u->Zs[h] / 256.0;
    }
    kstate_t s;
    if (orc_seed(sx, sy, sz, u->k, P->sinphi_max, s.p) != 0) goto done;
    cov_init(s.cov, P);
    s.x = u->xr[r1];
    s.chi2 = 0;
    for (int64_t r = 0; r < R; ++r) p1hit[r] = -1;
    /* pass 1: chain */
    kstate_t last = s;
    int64_t r_out = r1;
    int chain_ok = 1;
    int p1n = 0;
    for (int64_t j = 0; j < L; ++j) {
      if (j > 0 && step_to(&s, u->xr[r1 + j], u->k, P, &t->fragile) != 0) {
        chain_ok = 0;
        break;
      }
      upd(&s, u, chain[j]);
      p1hit[r1 + j] = chain[j];
      ++p1n;
      last = s;
      r_out = r1 + j;
    }
    /* pass 1: extension upward */
    if (chain_ok) {
      int misses = 0;
      for (int64_t r = r1 + L; r < R; ++r) {
        if (step_to(&s, u->xr[r], u->k, P, &t->fragile) != 0) break;
        pick_t pk = pick(u, r, s.p[0], s.p[1], &t->fragile);
        if (pk.stop) break;
        if (pk.found >= 0) {
          upd(&s, u, pk.found);
          p1hit[r] = pk.found;
          ++p1n;
          last = s;
          r_out = r;
          misses = 0;
        } else if (++misses > P->max_miss) {
          break;
        }
      }
    }
    t->p1n = p1n;
    /* pass 2: from the outermost pass-1 hit down to row 0 */
    s = last;
    cov_init(s.cov, P);
    s.chi2 = 0;
    int nfit = 0;
    upd(&s, u, p1hit[r_out]);
    t->hits[nfit++] = (int32_t)p1hit[r_out];
    last = s;
    int misses = 0;
    for (int64_t r = r_out - 1; r >= 0; --r) {
      if (step_to(&s, u->xr[r], u->k, P, &t->fragile) != 0) break;
      if (r >= r1 && p1hit[r] >= 0) {
        upd(&s, u, p1hit[r]);
        t->hits[nfit++] = (int32_t)p1hit[r];
        last = s;
        continue;
      }
      pick_t pk = pick(u, r, s.p[0], s.p[1], &t->fragile);
      if (pk.stop) break;
      if (pk.found >= 0) {
        upd(&s, u, pk.found);
        t->hits[nfit++] = pk.found;
        last = s;
        misses = 0;
      } else if (r < r1 && ++misses > P->max_miss) {
        break;
      }
    }
    t->nfit = nfit;
    memcpy(t->p, last.p, sizeof(t->p));
    pack_cov(last.cov, t->cov);
    t->xref = last.x;
    t->chi2 = last.chi2;
  }
done:
  free(chain);
  free(p1hit);
}

/* ------------------------------------------------------------------------- */
/* helpers exported for the pins                                               */

/* The fit's arithmetic type (a build of this file that evaluates the fit in
 * single precision turns it into float; the batch refit below the driver
 * keeps its double interface either way). */
typedef double fit_real;

/* Two-pass fit of a fixed list of hits (no pickups): pass 1 from hit 0 to hit
 * n-1 starting from the three-point seed, pass 2 back from hit n-1 to hit 0
 * with the covariance reset.  Output at hit 0; p1_out / cov1_out (each
 * optional) receive pass 1's state at hit n-1; *fragile_out (optional) is set
 * when a transport came within 1e-5 of the sin(phi) limit.  Returns 0 or -1. */
static int fit_two_pass(int n, const fit_real *x, const fit_real *y, const fit_real *z, fit_real k,
                        const orc_params_t *P, fit_real p_out[5], fit_real cov_out[15], fit_real *chi2,
                        fit_real p1_out[5], fit_real cov1_out[15], int *fragile_out) {
  if (n < 3) return -1;
  double sx[3] = {x[0], x[n / 2], x[n - 1]}, sy[3] = {y[0], y[n / 2], y[n - 1]},
         sz[3] = {z[0], z[n / 2], z[n - 1]};
  kstate_t s;
  int fr = 0;
  if (orc_seed(sx, sy, sz, k, P->sinphi_max, s.p) != 0) return -1;
  cov_init(s.cov, P);
  s.x = x[0];
  s.chi2 = 0;
  for (int j = 0; j < n; ++j) {
    if (j > 0 && step_to(&s, x[j], k, P, &fr) != 0) {
      if (fragile_out) *fragile_out = fr;
      return -1;
    }
    kf_update(s.p, s.cov, y[j], z[j], P->sigma_y, P->sigma_z, &s.chi2);
  }
  if (p1_out) memcpy(p1_out, s.p, sizeof(s.p));
  if (cov1_out) pack_cov(s.cov, cov1_out);
  cov_init(s.cov, P);
  s.chi2 = 0;
  kf_update(s.p, s.cov, y[n - 1], z[n - 1], P->sigma_y, P->sigma_z, &s.chi2);
  for (int j = n - 2; j >= 0; --j) {
    if (step_to(&s, x[j], k, P, &fr) != 0) {
      if (fragile_out) *fragile_out = fr;
      return -1;
    }
    kf_update(s.p, s.cov, y[j], z[j], P->sigma_y, P->sigma_z, &s.chi2);
  }
  memcpy(p_out, s.p, sizeof(s.p));
  if (cov_out) pack_cov(s.cov, cov_out);
  if (chi2) *chi2 = s.chi2;
  if (fragile_out) *fragile_out = fr;
  return 0;
}

int orc_fit_two_pass(int n, const double *x, const double *y, const double *z, double k,
                     const orc_params_t *P, double p_out[5], double cov_out[15], double *chi2,
                     double p1_out[5]) {
  return fit_two_pass(n, x, y, z, k, P, p_out, cov_out, chi2, p1_out, NULL, NULL);
}

/* The turn between sector frames (used by the merger below the driver and by
 * the chain fit here; see the merger's section for the derivation). */
/* Turn state p at plane x by d.  Returns 0, or -1 when the direction reaches
 * |sin(phi')| >= sinphi_max or cos(phi') <= 0 (the state cannot describe a
 * track moving inward in the new frame). */
int orc_rotate(const double p[5], double x, double d, double k, double sinphi_max, double out[5], double *x_out,
               double J[25]) {
  const double cd = cos(d), sd = sin(d);
  const double s = p[2];
  if (!(fabs(s) < 1.0)) return -1;
  const double c = sqrt(1.0 - s * s);
  const double s2 = s * cd - c * sd, c2 = c * cd + s * sd;
  if (!(c2 > 0.0) || !(fabs(s2) < sinphi_max)) return -1;
  *x_out = x * cd + p[0] * sd;
  out[0] = -x * sd + p[0] * cd;
  out[1] = p[1];
  out[2] = s2;
  out[3] = p[3];
  out[4] = p[4];
  if (J) {
    memset(J, 0, 25 * sizeof(double));
    for (int i = 0; i < 5; ++i) J[i * 5 + i] = 1.0;
    J[0 * 5 + 0] = c / c2;
    J[1 * 5 + 0] = -sd * p[3] / c2;
    J[2 * 5 + 0] = -k * p[4] * sd;
    J[2 * 5 + 2] = c2 / c;
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Fit of a merged chain of segments (Reading R-25): the hits of linked       */
/* segments in chain order (segment by segment, rows increasing inside each), */
/* hit j measured in its unit's frame (angle unit_alpha[u[j]]) at x[j] with   */
/* y[j], z[j].  Seed: the three-point circle through the first, middle (n/2)  */
/* and last hit, their positions turned into the first hit's frame.  Pass 1   */
/* from hit 0: before a hit of another frame the state, and its covariance by */
/* the turn's Jacobian, is turned into that frame, then carried to the hit    */
/* and updated.  Pass 2 from hit n-1 back, the covariance reset, turning back */
/* at each change of frame.  Output: the state at hit 0, in its frame.        */

static int turn_state(kstate_t *s, double d_raw, double k, const orc_params_t *P) {
  const double d = remainder(d_raw, 2.0 * M_PI_ORC);
  double q[5], xq, J[25];
  if (orc_rotate(s->p, s->x, d, k, P->sinphi_max, q, &xq, J) != 0) return -1;
  memcpy(s->p, q, sizeof(q));
  s->x = xq;
  transport_cov(J, s->cov);
  return 0;
}

/* Returns 0, or -1 when n < 3 or the seed, a turn or a transport fails. */
int orc_fit_chain(int n, const fit_real *x, const fit_real *y, const fit_real *z, const int32_t *u,
                  const fit_real *unit_alpha, fit_real k, const orc_params_t *P, fit_real p_out[5],
                  fit_real cov_out[15], fit_real *chi2) {
  if (n < 3) return -1;
  const int js[3] = {0, n / 2, n - 1};
  double sx[3], sy[3], sz[3];
  for (int i = 0; i < 3; ++i) { /* the point of hit js[i] in hit 0's frame */
    const int j = js[i];
    const double d = remainder(unit_alpha[u[0]] - unit_alpha[u[j]], 2.0 * M_PI_ORC);
    const double cd = cos(d), sd = sin(d);
    sx[i] = x[j] * cd + y[j] * sd;
    sy[i] = -x[j] * sd + y[j] * cd;
    sz[i] = z[j];
  }
  kstate_t s;
  int fr = 0, cu = u[0];
  if (orc_seed(sx, sy, sz, k, P->sinphi_max, s.p) != 0) return -1;
  cov_init(s.cov, P);
  s.x = x[0];
  s.chi2 = 0;
  for (int j = 0; j < n; ++j) {
    if (j > 0) {
      if (u[j] != cu) {
        if (turn_state(&s, unit_alpha[u[j]] - unit_alpha[cu], k, P) != 0) return -1;
        cu = u[j];
      }
      if (step_to(&s, x[j], k, P, &fr) != 0) return -1;
    }
    kf_update(s.p, s.cov, y[j], z[j], P->sigma_y, P->sigma_z, &s.chi2);
  }
  cov_init(s.cov, P);
  s.chi2 = 0;
  kf_update(s.p, s.cov, y[n - 1], z[n - 1], P->sigma_y, P->sigma_z, &s.chi2);
  for (int j = n - 2; j >= 0; --j) {
    if (u[j] != cu) {
      if (turn_state(&s, unit_alpha[u[j]] - unit_alpha[cu], k, P) != 0) return -1;
      cu = u[j];
    }
    if (step_to(&s, x[j], k, P, &fr) != 0) return -1;
    kf_update(s.p, s.cov, y[j], z[j], P->sigma_y, P->sigma_z, &s.chi2);
  }
  memcpy(p_out, s.p, sizeof(s.p));
  pack_cov(s.cov, cov_out);
  *chi2 = s.chi2;
  return 0;
}

int orc_kf_update(double p[5], double cov15[15], double my, double mz, double sy, double sz,
                  double *chi2) {
  double c[25];
  int k = 0;
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j <= i; ++j) {
      c[i * 5 + j] = c[j * 5 + i] = cov15[k++];
    }
  kf_update(p, c, my, mz, sy, sz, chi2);
  pack_cov(c, cov15);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* driver                                                                      */

int64_t orc_max_cells(int64_t n, int64_t n_units, int64_t n_rows, const orc_params_t *P) {
  return n / (P->bin_occ > 0 ? P->bin_occ : 1) + n_units * n_rows * 65 + 1;
}

static void *xcalloc(size_t n, size_t sz) {
  void *p = calloc(n ? n : 1, sz);
  if (!p) {
    fprintf(stderr, "oracle: out of memory\n");
    abort();
  }
  return p;
}

void orc_free(orc_result_t *r) {
  void **ptrs[] = {(void **)&r->perm, (void **)&r->up, (void **)&r->dn, (void **)&r->upc,
                   (void **)&r->dnc, (void **)&r->owner, (void **)&r->cluster_track,
                   (void **)&r->seg_start, (void **)&r->seg_count, (void **)&r->seg_zmin,
                   (void **)&r->seg_zmax, (void **)&r->seg_ny, (void **)&r->seg_nz,
                   (void **)&r->seg_by, (void **)&r->seg_bz, (void **)&r->seg_cell_base,
                   (void **)&r->cell_start, (void **)&r->trk_start, (void **)&r->trk_unit,
                   (void **)&r->trk_len, (void **)&r->trk_nfit, (void **)&r->trk_p1n,
                   (void **)&r->trk_owned, (void **)&r->trk_keep, (void **)&r->trk_fragile,
                   (void **)&r->trk_key, (void **)&r->trk_params, (void **)&r->trk_cov,
                   (void **)&r->trk_xref, (void **)&r->trk_chi2, (void **)&r->trk_hits,
                   (void **)&r->track_tracklet, (void **)&r->track_first_hit,
                   (void **)&r->track_n_hits, (void **)&r->track_hits};
  for (size_t i = 0; i < sizeof(ptrs) / sizeof(ptrs[0]); ++i) {
    free(*ptrs[i]);
    *ptrs[i] = NULL;
  }
}

static int valid_params(const orc_params_t *P) {
  return P->q_shift == 8 && P->tan_half_q16 > 0 && P->bin_y_q > 0 && P->bin_occ > 0 &&
         P->bin_zmin_q > 0 && P->win_y_q >= 0 && P->win_z_q >= 0 && P->w_y >= 0 && P->w_y <= 15 &&
         P->w_z >= 0 && P->w_z <= 15 && P->smax_k >= 0 && P->smax_k < ((int64_t)1 << 30) &&
         P->l_min >= 3 && P->ext_win_y_q >= 0 && P->ext_win_y_q < 8192 && P->ext_win_z_q >= 0 &&
         P->ext_win_z_q < 8192 &&
         P->max_miss >= 0 && P->n_min >= 0 && P->f_min_q8 >= 0 && P->sinphi_max > 0 &&
         P->sinphi_max < 1 && P->sigma_y > 0 && P->sigma_z > 0;
}

/*
 * Run the whole method on host arrays.  y, z, row: [n]; unit_offsets:
 * [n_units + 1]; row_x: [n_rows].  Fills *res (arrays owned by res; release
 * with orc_free).  Returns ORC_OK or ORC_INVALID (then res->status says so and
 * nothing else is filled).
 */
int orc_run(int64_t n, int64_t n_units, const int64_t *unit_offsets, const float *y,
            const float *z, const uint16_t *row, int64_t n_rows, const float *row_x, float bz,
            const orc_params_t *P, orc_result_t *res) {
  memset(res, 0, sizeof(*res));
  res->n = n;
  res->n_units = n_units;
  res->n_rows = n_rows;
  res->status = ORC_INVALID;
  /* ingest: validate (step a1) */
  if (!valid_params(P) || n < 0 || n_units < 1 || n_rows < 3 || n_rows > 255 || n > INT32_MAX / 2)
    return ORC_INVALID;
  if (unit_offsets[0] != 0 || unit_offsets[n_units] != n) return ORC_INVALID;
  for (int64_t u = 0; u < n_units; ++u)
    if (unit_offsets[u + 1] < unit_offsets[u] || unit_offsets[u + 1] - unit_offsets[u] >= (1 << 24))
      return ORC_INVALID;
  /* pad rows between 1 cm and 8192 cm from the axis, increasing */
  for (int64_t r = 0; r < n_rows; ++r)
    if (!(row_x[r] >= 1.0f) || !(row_x[r] < 8192.0f) || (r > 0 && !(row_x[r] > row_x[r - 1])))
      return ORC_INVALID;
  /* rows two apart at most 32 cm apart: keeps the neighbour cut below 2^56 */
  for (int64_t r = 1; r + 1 < n_rows; ++r)
    if (quantize((double)row_x[r + 1]) - quantize((double)row_x[r - 1]) >= 8192) return ORC_INVALID;
  for (int64_t i = 0; i < n; ++i)
    if (row[i] >= n_rows || !(fabsf(y[i]) <= 8192.0f) || !(fabsf(z[i]) <= 8192.0f)) return ORC_INVALID;
  res->status = ORC_OK;

  const int64_t S = n_units * n_rows;
  res->n_seg = S;
  int64_t *X = (int64_t *)xcalloc((size_t)n_rows, sizeof(int64_t));
  double *xr = (double *)xcalloc((size_t)n_rows, sizeof(double));
  for (int64_t r = 0; r < n_rows; ++r) {
    X[r] = quantize((double)row_x[r]);
    xr[r] = (double)row_x[r];
  }
  int64_t *Y = (int64_t *)xcalloc((size_t)n, sizeof(int64_t));
  int64_t *Z = (int64_t *)xcalloc((size_t)n, sizeof(int64_t));
  int64_t *Ys = (int64_t *)xcalloc((size_t)n, sizeof(int64_t));
  int64_t *Zs = (int64_t *)xcalloc((size_t)n, sizeof(int64_t));
  res->perm = (int32_t *)xcalloc((size_t)n, 4);
  res->up = (int32_t *)xcalloc((size_t)n, 4);
  res->dn = (int32_t *)xcalloc((size_t)n, 4);
  res->upc = (int32_t *)xcalloc((size_t)n, 4);
  res->dnc = (int32_t *)xcalloc((size_t)n, 4);
  res->owner = (uint32_t *)xcalloc((size_t)n, 4);
  res->cluster_track = (int32_t *)xcalloc((size_t)n, 4);
  res->seg_start = (int32_t *)xcalloc((size_t)S, 4);
  res->seg_count = (int32_t *)xcalloc((size_t)S, 4);
  res->seg_zmin = (int32_t *)xcalloc((size_t)S, 4);
  res->seg_zmax = (int32_t *)xcalloc((size_t)S, 4);
  res->seg_ny = (int32_t *)xcalloc((size_t)S, 4);
  res->seg_nz = (int32_t *)xcalloc((size_t)S, 4);
  res->seg_by = (int32_t *)xcalloc((size_t)S, 4);
  res->seg_bz = (int32_t *)xcalloc((size_t)S, 4);
  res->seg_cell_base = (int32_t *)xcalloc((size_t)S, 4);
  seg_geom_t *SG = (seg_geom_t *)xcalloc((size_t)S, sizeof(seg_geom_t));
  int64_t *rstart = (int64_t *)xcalloc((size_t)(n_units * (n_rows + 1)), sizeof(int64_t));
  int64_t *cbase = (int64_t *)xcalloc((size_t)S, sizeof(int64_t));

  double t0 = now_s();
  /* O1 quantization */
  for (int64_t i = 0; i < n; ++i) {
    Y[i] = quantize((double)y[i]);
    Z[i] = quantize((double)z[i]);
  }
  /* O2 hit grid: per-row counts and z extent, bin geometry, then one sort by
   * (row, bin, id) per unit */
  for (int64_t u = 0; u < n_units; ++u) {
    int64_t *cnt = (int64_t *)xcalloc((size_t)n_rows, sizeof(int64_t));
    int64_t *zmn = (int64_t *)xcalloc((size_t)n_rows, sizeof(int64_t));
    int64_t *zmx = (int64_t *)xcalloc((size_t)n_rows, sizeof(int64_t));
    for (int64_t r = 0; r < n_rows; ++r) { zmn[r] = INT64_MAX; zmx[r] = INT64_MIN; }
    for (int64_t i = unit_offsets[u]; i < unit_offsets[u + 1]; ++i) {
      const int64_t r = row[i];
      ++cnt[r];
      if (Z[i] < zmn[r]) zmn[r] = Z[i];
      if (Z[i] > zmx[r]) zmx[r] = Z[i];
    }
    int64_t pos = unit_offsets[u];
    for (int64_t r = 0; r < n_rows; ++r) {
      const int64_t s = u * n_rows + r;
      SG[s] = seg_geometry(X[r], cnt[r], zmn[r], zmx[r], P);
      rstart[u * (n_rows + 1) + r] = pos;
      res->seg_start[s] = (int32_t)pos;
      res->seg_count[s] = (int32_t)cnt[r];
      res->seg_zmin[s] = (int32_t)SG[s].zmin;
      res->seg_zmax[s] = (int32_t)SG[s].zmax;
      res->seg_ny[s] = (int32_t)SG[s].ny;
      res->seg_nz[s] = (int32_t)SG[s].nz;
      res->seg_by[s] = (int32_t)SG[s].by;
      res->seg_bz[s] = (int32_t)SG[s].bz;
      pos += cnt[r];
    }
    rstart[u * (n_rows + 1) + n_rows] = pos;
    free(cnt);
    free(zmn);
    free(zmx);
  }
  int64_t n_cells = 0;
  for (int64_t s = 0; s < S; ++s) {
    cbase[s] = n_cells;
    res->seg_cell_base[s] = (int32_t)n_cells;
    n_cells += SG[s].ny * SG[s].nz;
  }
  res->n_cells = n_cells;
  res->cell_start = (int32_t *)xcalloc((size_t)(n_cells + 1), 4);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t u = 0; u < n_units; ++u) {
    const int64_t a = unit_offsets[u], b = unit_offsets[u + 1];
    sort_key_t *keys = (sort_key_t *)xcalloc((size_t)(b - a), sizeof(sort_key_t));
    for (int64_t i = a; i < b; ++i) {
      const int64_t r = row[i];
      keys[i - a].row = r;
      keys[i - a].bin = bin_of(&SG[u * n_rows + r], Y[i], Z[i]);
      keys[i - a].id = i;
    }
    qsort(keys, (size_t)(b - a), sizeof(sort_key_t), cmp_key);
    for (int64_t k = 0; k < b - a; ++k) {
      res->perm[a + k] = (int32_t)keys[k].id;
      Ys[a + k] = Y[keys[k].id];
      Zs[a + k] = Z[keys[k].id];
    }
    /* cell starts: first sorted position whose (row, bin) >= the cell */
    int64_t k = 0;
    for (int64_t r = 0; r < n_rows; ++r) {
      const int64_t s = u * n_rows + r;
      const int64_t nb = SG[s].ny * SG[s].nz;
      for (int64_t c = 0; c < nb; ++c) {
        while (k < b - a && (keys[k].row < r || (keys[k].row == r && keys[k].bin < c))) ++k;
        res->cell_start[cbase[s] + c] = (int32_t)(a + k);
      }
    }
    free(keys);
  }
  res->cell_start[n_cells] = (int32_t)n;
  double t1 = now_s();
  res->time_s[0] = t1 - t0;

  /* O3 - O4 per unit */
  const double kcurv = -KAPPA * (double)bz;
  unit_ctx_t *U = (unit_ctx_t *)xcalloc((size_t)n_units, sizeof(unit_ctx_t));
  for (int64_t u = 0; u < n_units; ++u) {
    U[u].P = P;
    U[u].a = unit_offsets[u];
    U[u].b = unit_offsets[u + 1];
    U[u].n_rows = n_rows;
    U[u].X = X;
    U[u].xr = xr;
    U[u].Ys = Ys;
    U[u].Zs = Zs;
    U[u].sg = &SG[u * n_rows];
    U[u].rstart = &rstart[u * (n_rows + 1)];
    U[u].cbase = &cbase[u * n_rows];
    U[u].cell_start = res->cell_start;
    U[u].perm = res->perm;
    U[u].k = kcurv;
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t u = 0; u < n_units; ++u) find_neighbours(&U[u], res->up, res->dn);
  double t2 = now_s();
  res->time_s[1] = t2 - t1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t u = 0; u < n_units; ++u)
    clean_links(U[u].a, U[u].b, res->up, res->dn, res->upc, res->dnc);
  /* start hits: have a cleaned upward link and no cleaned downward link;
   * tracklets are numbered in (unit, grid position) order */
  int64_t K = 0;
  for (int64_t p = 0; p < n; ++p)
    if (res->upc[p] >= 0 && res->dnc[p] < 0) ++K;
  res->n_tracklets = K;
  res->trk_start = (int32_t *)xcalloc((size_t)K, 4);
  res->trk_unit = (int32_t *)xcalloc((size_t)K, 4);
  res->trk_len = (int32_t *)xcalloc((size_t)K, 4);
  res->trk_nfit = (int32_t *)xcalloc((size_t)K, 4);
  res->trk_p1n = (int32_t *)xcalloc((size_t)K, 4);
  res->trk_owned = (int32_t *)xcalloc((size_t)K, 4);
  res->trk_keep = (int32_t *)xcalloc((size_t)K, 4);
  res->trk_fragile = (int32_t *)xcalloc((size_t)K, 4);
  res->trk_key = (uint32_t *)xcalloc((size_t)K, 4);
  res->trk_params = (double *)xcalloc((size_t)K * 5, 8);
  res->trk_cov = (double *)xcalloc((size_t)K * 15, 8);
  res->trk_xref = (double *)xcalloc((size_t)K, 8);
  res->trk_chi2 = (double *)xcalloc((size_t)K, 8);
  res->trk_hits = (int32_t *)xcalloc((size_t)(K * n_rows), 4);
  int64_t *unit_trk0 = (int64_t *)xcalloc((size_t)(n_units + 1), sizeof(int64_t));
  {
    int64_t k = 0;
    for (int64_t u = 0; u < n_units; ++u) {
      unit_trk0[u] = k;
      for (int64_t p = unit_offsets[u]; p < unit_offsets[u + 1]; ++p)
        if (res->upc[p] >= 0 && res->dnc[p] < 0) {
          res->trk_start[k] = (int32_t)p;
          res->trk_unit[k] = (int32_t)u;
          ++k;
        }
    }
    unit_trk0[n_units] = k;
  }
  double t3 = now_s();
  res->time_s[2] = t3 - t2;

  /* O5 + O6: chains and tracklet construction */
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t u = 0; u < n_units; ++u) {
    for (int64_t t = unit_trk0[u]; t < unit_trk0[u + 1]; ++t) {
      tracklet_out_t o;
      o.hits = &res->trk_hits[t * n_rows];
      construct(&U[u], res->trk_start[t], res->upc, &o);
      res->trk_len[t] = o.len;
      res->trk_nfit[t] = o.nfit;
      res->trk_p1n[t] = o.p1n;
      res->trk_fragile[t] = o.fragile;
      memcpy(&res->trk_params[t * 5], o.p, sizeof(o.p));
      memcpy(&res->trk_cov[t * 15], o.cov, sizeof(o.cov));
      res->trk_xref[t] = o.xref;
      res->trk_chi2[t] = o.chi2;
      if (o.nfit > 0) {
        const uint32_t local = (uint32_t)(res->perm[res->trk_start[t]] - unit_offsets[u]);
        res->trk_key[t] = ((uint32_t)o.nfit << 24) | (0xFFFFFFu - local);
      }
    }
  }
  double t4 = now_s();
  res->time_s[3] = t4 - t3;

  /* Owner of a hit: the largest key (n hits, then the earliest start id) over
   * the tracklets that use it (Reading). */
  for (int64_t p = 0; p < n; ++p) res->owner[p] = 0;
  for (int64_t t = 0; t < K; ++t)
    for (int64_t j = 0; j < res->trk_nfit[t]; ++j) {
      const int64_t h = res->trk_hits[t * n_rows + j];
      if (res->trk_key[t] > res->owner[h]) res->owner[h] = res->trk_key[t];
    }
  /* O7 selector (Reading): keep a tracklet when it owns at least n_min hits
   * and at least f_min of its hits; no refit. */
  int64_t n_tracks = 0, n_track_hits = 0;
  for (int64_t t = 0; t < K; ++t) {
    int owned = 0;
    for (int64_t j = 0; j < res->trk_nfit[t]; ++j)
      if (res->owner[res->trk_hits[t * n_rows + j]] == res->trk_key[t]) ++owned;
    res->trk_owned[t] = owned;
    res->trk_keep[t] = res->trk_nfit[t] > 0 && owned >= P->n_min &&
                       (int64_t)owned * 256 >= (int64_t)P->f_min_q8 * res->trk_nfit[t];
    if (res->trk_keep[t]) {
      ++n_tracks;
      n_track_hits += owned;
    }
  }
  res->n_tracks = n_tracks;
  res->n_track_hits = n_track_hits;
  res->track_tracklet = (int32_t *)xcalloc((size_t)n_tracks, 4);
  res->track_first_hit = (int32_t *)xcalloc((size_t)n_tracks, 4);
  res->track_n_hits = (int32_t *)xcalloc((size_t)n_tracks, 4);
  res->track_hits = (int32_t *)xcalloc((size_t)n_track_hits, 4);
  for (int64_t i = 0; i < n; ++i) res->cluster_track[i] = -1;
  {
    int64_t tr = 0, hp = 0;
    for (int64_t t = 0; t < K; ++t) {
      if (!res->trk_keep[t]) continue;
      res->track_tracklet[tr] = (int32_t)t;
      res->track_first_hit[tr] = (int32_t)hp;
      res->track_n_hits[tr] = res->trk_owned[t];
      /* owned hits in increasing row order = reverse of the pass-2 order */
      for (int64_t j = res->trk_nfit[t] - 1; j >= 0; --j) {
        const int64_t h = res->trk_hits[t * n_rows + j];
        if (res->owner[h] == res->trk_key[t]) {
          res->track_hits[hp++] = res->perm[h];
          res->cluster_track[res->perm[h]] = (int32_t)tr;
        }
      }
      ++tr;
    }
  }
  double t5 = now_s();
  res->time_s[4] = t5 - t4;
  res->time_s[5] = t5 - t0;

  free(X);
  free(xr);
  free(Y);
  free(Z);
  free(Ys);
  free(Zs);
  free(SG);
  free(rstart);
  free(cbase);
  free(U);
  free(unit_trk0);
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Collision assignment in continuous readout (a step after track finding).    */
/* The paper states that in continuous readout the collisions overlap in the   */
/* drift volume and that tracks are assigned to collisions only after tracking */
/* (§2, §2.3); it does not say how.  Reading used here: the measured z' of a   */
/* cluster is z - side v_d t0, so every track of one collision on one side of  */
/* the TPC carries the same z' at the vertex, z_vertex - side v_d t0.  A       */
/* track's z' at its transverse point of closest approach to the beam axis     */
/* estimates it.  That estimate is unambiguous only for a track whose circle   */
/* does not fit inside the TPC (|C| < c_max = 2 / outer radius): a looper may  */
/* be seen on a later leg or turn, where z' is off by the z advance per turn.  */
/* Per side, the z' of those "forming" tracks are histogrammed in bins of      */
/* width w over [-zmax, zmax); a candidate collision is a bin holding at least */
/* n_min of them that is the largest within `reach` bins on either side (ties  */
/* go to the lower bin).  Every track in the range (loopers too) joins the     */
/* candidate whose bin is nearest to its own within `reach` bins (ties to the  */
/* lower bin), else none.  A candidate's z' is the mean over the forming       */
/* tracks it holds, its t0 = -side z' / v_d with the vertex taken at z = 0     */
/* (the spread of vertex z is the resolution of t0 here).                      */

/* z' at the transverse point of closest approach to the beam axis (x = y = 0
 * of the sector frame) of the helix with state p at plane x, curvature k p[4].
 * The closest point of a circle to the origin lies on the line from the
 * circle's centre to the origin; the arc length to it follows from the signed
 * angle it turns about the centre.  *sT: transverse arc length from the
 * reference point (negative toward the beam); *turn: that angle (radians). */
double orc_zdca(const double p[5], double x, double k, double *sT_out, double *turn_out) {
  const double y = p[0], z = p[1], sphi = p[2], tgl = p[3];
  const double C = k * p[4];
  const double cphi = sqrt(1.0 - sphi * sphi);
  double sT = 0.0, turn = 0.0;
  if (C == 0.0) {  /* straight line: foot of the perpendicular from the origin */
    sT = -(x * cphi + y * sphi);
  } else {
    const double xc = x - sphi / C, yc = y + cphi / C; /* centre of the circle */
    const double dc = sqrt(xc * xc + yc * yc);
    if (dc > 0.0) {
      const double R = 1.0 / fabs(C);
      const double px = xc * (1.0 - R / dc), py = yc * (1.0 - R / dc);
      const double ax = x - xc, ay = y - yc, bx = px - xc, by = py - yc;
      turn = atan2(ax * by - ay * bx, ax * bx + ay * by);
      sT = turn / C;
    }
  }
  if (sT_out) *sT_out = sT;
  if (turn_out) *turn_out = turn;
  return z + tgl * sT;
}

/* Histogram bin of a z' value (range [-zmax, zmax) in nb bins of width w), or
 * -1; a value just below zmax whose quotient rounds up to nb is in the last bin. */
static int64_t col_bin(double z, double w, double zmax, int64_t nb) {
  if (!(z >= -zmax && z < zmax)) return -1;
  const int64_t b = (int64_t)floor((z + zmax) / w);
  return b < nb ? b : nb - 1;
}

/* Collision candidates of n_tracks tracks (state at x_ref in the frame of
 * their unit, unit_side[unit] = +1 or -1).  Outputs per track: zdca, t0 (us,
 * the track's own estimate), collision (-1 none; candidates are numbered side
 * A first, then by increasing bin) and fragile (1 when another rounding of its
 * z' could move it to the next bin: within eps of a bin edge or of the range
 * ends, or a closest point half a turn away); per candidate (capacity: all
 * bins of both sides): side, bin, tracks assigned, forming tracks assigned,
 * mean z' and t0.  Returns the number of candidates. */
int64_t orc_collisions(int64_t n_tracks, const double *params, const double *x_ref, const int32_t *unit,
                       const int32_t *unit_side, double k, double v_drift, double w, double zmax,
                       double c_max, int32_t n_min, int32_t reach, double eps, double *zdca, double *t0,
                       int32_t *collision, int32_t *fragile, int32_t *c_side, int32_t *c_bin,
                       int32_t *c_count, int32_t *c_form, double *c_zdca, double *c_t0) {
  const int64_t nb = (int64_t)ceil(2.0 * zmax / w);
  int32_t *hist = (int32_t *)xcalloc((size_t)(2 * nb), sizeof(int32_t)); /* [side A, side C][bin] */
  int64_t *cand = (int64_t *)xcalloc((size_t)(2 * nb), sizeof(int64_t)); /* candidate of a bin, -1 */
  for (int64_t t = 0; t < n_tracks; ++t) {
    const int32_t side = unit_side[unit[t]];
    double turn = 0.0;
    zdca[t] = orc_zdca(&params[t * 5], x_ref[t], k, NULL, &turn);
    t0[t] = -(double)side * zdca[t] / v_drift;
    const double f = (zdca[t] + zmax) / w;
    fragile[t] = fabs(f - nearbyint(f)) * w < eps || fabs(fabs(turn) - 3.14159265358979323846) < eps;
    const int64_t b = col_bin(zdca[t], w, zmax, nb);
    if (b >= 0 && fabs(k * params[t * 5 + 4]) < c_max) hist[(side > 0 ? 0 : nb) + b] += 1;
  }
  int64_t nc = 0;
  for (int s = 0; s < 2; ++s) {
    const int32_t *h = hist + s * nb;
    for (int64_t b = 0; b < nb; ++b) {
      cand[s * nb + b] = -1;
      if (h[b] < n_min) continue;
      int peak = 1;
      for (int64_t d = 1; d <= reach && peak; ++d) {
        if (b - d >= 0 && h[b - d] >= h[b]) peak = 0; /* a lower bin as large wins */
        if (b + d < nb && h[b + d] > h[b]) peak = 0;
      }
      if (!peak) continue;
      cand[s * nb + b] = nc;
      c_side[nc] = s == 0 ? 1 : -1;
      c_bin[nc] = (int32_t)b;
      c_count[nc] = 0;
      c_form[nc] = 0;
      c_zdca[nc] = 0.0;
      ++nc;
    }
  }
  for (int64_t t = 0; t < n_tracks; ++t) {
    collision[t] = -1;
    const int32_t side = unit_side[unit[t]];
    const int64_t b = col_bin(zdca[t], w, zmax, nb);
    if (b < 0) continue;
    const int64_t *cs = cand + (side > 0 ? 0 : nb);
    for (int64_t d = 0; d <= reach; ++d) { /* nearest candidate bin, the lower one first */
      if (b - d >= 0 && cs[b - d] >= 0) { collision[t] = (int32_t)cs[b - d]; break; }
      if (b + d < nb && cs[b + d] >= 0) { collision[t] = (int32_t)cs[b + d]; break; }
    }
    const int32_t c = collision[t];
    if (c < 0) continue;
    c_count[c] += 1;
    if (fabs(k * params[t * 5 + 4]) < c_max) {
      c_form[c] += 1;
      c_zdca[c] += zdca[t];
    }
  }
  for (int64_t c = 0; c < nc; ++c) { /* a candidate holds the >= n_min forming tracks of its own bin */
    c_zdca[c] /= c_form[c];
    c_t0[c] = -(double)c_side[c] * c_zdca[c] / v_drift;
  }
  free(hist);
  free(cand);
  return nc;
}

/* ------------------------------------------------------------------------- */
/* Clusterizer: raw ADC digits to clusters (the producer of the tracker's      */
/* input).  The paper states that a clusterizing algorithm turns the raw ADC   */
/* values into hits (§2.1) and that it runs much faster on GPUs than on CPUs   */
/* (§3.2); it does not describe it.  Reading used here: digits are grouped by  */
/* (unit, row, pad), times increasing inside a pad.  A digit of charge v at    */
/* (pad p, time t) is a peak when v >= q_min and every digit among its eight   */
/* neighbours (pads p-1..p+1 of the same row, times t-1..t+1) is smaller, or   */
/* equal and later in (pad, time) order -- so a plateau of equal charges has   */
/* one peak, its first digit.  The cluster of a peak sums the digits of the    */
/* 3x3 window around it: Q = sum v, Sp = sum v (p' - p), St = sum v (t' - t);  */
/* its centre is (p + Sp/Q, t + St/Q) in FP64; y = (pad + 0.5 - half) pw and   */
/* z' = (time + 0.5) tb - zoff, rounded once to FP32.  Clusters come in the    */
/* order of their peaks.                                                       */

/* digits of pad j with time in [t0, t1]: the index range [*a, *b) */
static void pad_range(const int64_t *pad_offsets, const uint16_t *time, int64_t j, int32_t t0, int32_t t1,
                      int64_t *a, int64_t *b) {
  int64_t lo = pad_offsets[j], hi = pad_offsets[j + 1];
  while (lo < hi && time[lo] < t0) ++lo;
  int64_t e = lo;
  while (e < hi && time[e] <= t1) ++e;
  *a = lo;
  *b = e;
}

/* Clusters of all digits.  half[n_rows]: half the pad count of each row
 * (rows have 2 half[r] pads; pads_total = sum of them); pad_offsets has
 * n_units * pads_total + 1 entries.  Outputs (capacity: the number of
 * digits): unit, row, peak pad and time, qmax, Q, Sp, St, and the float
 * centre (pad, time) and position (y, z').  Returns the cluster count. */
int64_t orc_clusterize(int32_t n_units, int32_t n_rows, const int32_t *half, const int64_t *pad_offsets,
                       const uint16_t *time, const uint16_t *q, int32_t q_min, double pw, double tb, double zoff,
                       int32_t *c_unit, int32_t *c_row, int32_t *c_pad, int32_t *c_time, int32_t *c_qmax,
                       int32_t *c_q, int32_t *c_sp, int32_t *c_st, float *c_padf, float *c_timef, float *c_y,
                       float *c_z) {
  int64_t pads_total = 0;
  for (int r = 0; r < n_rows; ++r) pads_total += 2 * (int64_t)half[r];
  int64_t nc = 0;
  for (int32_t u = 0; u < n_units; ++u) {
    int64_t base = (int64_t)u * pads_total;
    for (int32_t r = 0; r < n_rows; ++r) {
      const int32_t np = 2 * half[r];
      for (int32_t p = 0; p < np; ++p) {
        const int64_t j = base + p;
        for (int64_t d = pad_offsets[j]; d < pad_offsets[j + 1]; ++d) {
          const int32_t t = time[d], v = q[d];
          if (v < q_min) continue;
          int peak = 1;
          int32_t Q = 0, Sp = 0, St = 0;
          for (int dp = -1; dp <= 1 && peak; ++dp) {
            if (p + dp < 0 || p + dp >= np) continue; /* neighbours stay in the row */
            int64_t a, b;
            pad_range(pad_offsets, time, j + dp, t - 1, t + 1, &a, &b);
            for (int64_t e = a; e < b; ++e) {
              const int32_t dt = (int32_t)time[e] - t, w = q[e];
              const int later = dp > 0 || (dp == 0 && dt > 0);
              if (!(dp == 0 && dt == 0) && !(w < v || (w == v && later))) {
                peak = 0;
                break;
              }
              Q += w;
              Sp += w * dp;
              St += w * dt;
            }
          }
          if (!peak) continue;
          const double padf = (double)p + (double)Sp / (double)Q;
          const double timef = (double)t + (double)St / (double)Q;
          c_unit[nc] = u;
          c_row[nc] = r;
          c_pad[nc] = p;
          c_time[nc] = t;
          c_qmax[nc] = v;
          c_q[nc] = Q;
          c_sp[nc] = Sp;
          c_st[nc] = St;
          c_padf[nc] = (float)padf;
          c_timef[nc] = (float)timef;
          c_y[nc] = (float)((padf + 0.5 - (double)half[r]) * pw);
          c_z[nc] = (float)((timef + 0.5) * tb - zoff);
          ++nc;
        }
      }
      base += np;
    }
  }
  return nc;
}

/* ------------------------------------------------------------------------- */
/* Hit removal and track-model compression (the consumer of the tracks).  The  */
/* paper states that hits of tracks not used for physics are removed and the  */
/* remaining hits go through entropy-reduction steps such as the track model  */
/* compression (§2.1); it does not give them.  Reading used here: a cluster   */
/* attached to a track with pT below pt_remove (|q/pT| pt_remove > 1: loopers */
/* that curl inside the chamber) is removed; a cluster attached to another    */
/* track is stored as its residual to the track model -- the track's state at */
/* x_ref carried along the helix to the cluster's row -- in steps of `step`   */
/* cm, rounded half to even; a cluster attached to no track, or whose track   */
/* cannot reach its row within |sin(phi)| < sinphi_max, is stored by its      */
/* position in the same steps.  The entropy coder that would follow is out of */
/* scope; the codes' histograms give its size.                                */

/* Codes of n clusters.  cls: 0 no track (position codes), 1 residual codes,
 * 2 removed, 3 attached without a model (position codes).  fragile: a
 * residual code whose unrounded value lies within eps of a rounding boundary,
 * so another rounding of the prediction could change it. */
void orc_compress(int64_t n, const float *y, const float *z, const uint16_t *row, const int32_t *cluster_track,
                  const float *params, const float *x_ref, const float *row_x, double k, double step,
                  double pt_remove, double sinphi_max, double eps, uint8_t *cls, int32_t *code_y, int32_t *code_z,
                  uint8_t *fragile) {
  for (int64_t c = 0; c < n; ++c) {
    const int32_t t = cluster_track[c];
    double vy = (double)y[c] / step, vz = (double)z[c] / step;
    cls[c] = 0;
    if (t >= 0) {
      double p[5], out[5];
      for (int i = 0; i < 5; ++i) p[i] = (double)params[(int64_t)t * 5 + i];
      if (fabs(p[4]) * pt_remove > 1.0) {
        cls[c] = 2;
        code_y[c] = code_z[c] = 0;
        fragile[c] = 0;
        continue;
      }
      if (orc_propagate(p, (double)x_ref[t], (double)row_x[row[c]], k, sinphi_max, out, NULL) == 0) {
        cls[c] = 1;
        vy = ((double)y[c] - out[0]) / step;
        vz = ((double)z[c] - out[1]) / step;
      } else {
        cls[c] = 3;
      }
    }
    code_y[c] = (int32_t)nearbyint(vy);
    code_z[c] = (int32_t)nearbyint(vz);
    /* a position code is one correctly rounded quotient of the inputs, the
     * same everywhere, and so is a residual at the state's own plane (the
     * helix carries nothing there); other residual codes depend on the
     * helix's rounding */
    const double fy = vy - floor(vy), fz = vz - floor(vz);
    fragile[c] = cls[c] == 1 && row_x[row[c]] != x_ref[t] && (fabs(fy - 0.5) < eps || fabs(fz - 0.5) < eps);
  }
}

/* ------------------------------------------------------------------------- */
/* Refit of the selected tracks (the step after the selector, which may have
 * taken hits away from a tracklet): track t's hits are the cluster ids
 * hits[first[t] .. first[t] + nh[t]), in increasing row order.  Each hit is
 * measured at x = row_x[row] with y and z in quanta of 1/256 cm, rounded half
 * to even, as the tracker measures them; the fit is the two-pass fit of the
 * helpers above (fit_two_pass).  Per track: ok = 1 when the fit succeeded
 * (else every output is zero), the pass-2 state at the first hit (p_in,
 * cov_in, x_in, chi2), the pass-1 state at the last hit (p_out, cov_out,
 * x_out), and fragile = 1 when a transport came within 1e-5 of the sin(phi)
 * limit. */
void orc_refit_tracks(int64_t n_tracks, const int32_t *first, const int32_t *nh, const int32_t *hits,
                      const float *y, const float *z, const uint16_t *row, const double *row_x, double k,
                      const orc_params_t *P, double *p_in, double *cov_in, double *x_in, double *chi2,
                      double *p_out, double *cov_out, double *x_out, int8_t *ok, int8_t *fragile) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t t = 0; t < n_tracks; ++t) {
    const int n = nh[t];
    fit_real *X = (fit_real *)malloc(sizeof(fit_real) * 3 * (size_t)(n > 0 ? n : 1));
    fit_real *Y = X + n, *Z = X + 2 * n;
    for (int j = 0; j < n; ++j) {
      const int32_t h = hits[first[t] + j];
      X[j] = row_x[row[h]];
      Y[j] = nearbyint(256.0 * (double)y[h]) / 256.0;
      Z[j] = nearbyint(256.0 * (double)z[h]) / 256.0;
    }
    fit_real pi[5], ci[15], ch = 0, po[5], co[15];
    int fr = 0;
    const int st = fit_two_pass(n, X, Y, Z, (fit_real)k, P, pi, ci, &ch, po, co, &fr);
    ok[t] = st == 0;
    fragile[t] = (int8_t)fr;
    for (int q = 0; q < 5; ++q) {
      p_in[t * 5 + q] = st == 0 ? (double)pi[q] : 0.0;
      p_out[t * 5 + q] = st == 0 ? (double)po[q] : 0.0;
    }
    for (int q = 0; q < 15; ++q) {
      cov_in[t * 15 + q] = st == 0 ? (double)ci[q] : 0.0;
      cov_out[t * 15 + q] = st == 0 ? (double)co[q] : 0.0;
    }
    chi2[t] = st == 0 ? (double)ch : 0.0;
    x_in[t] = st == 0 ? (double)X[0] : 0.0;
    x_out[t] = st == 0 ? (double)X[n - 1] : 0.0;
    free(X);
  }
}

/* ------------------------------------------------------------------------- */
/* Merging of track segments across sector boundaries (Reading R-24: the      */
/* paper asks for full tracking and does not describe the merger).            */
/*                                                                             */
/* A sector's local frame is the global one turned by the sector's angle a     */
/* (x along the sector's centre line).  Turning a state from the frame at a1   */
/* to the frame at a2 (d = a2 - a1): the point (x, y) becomes                  */
/* (x cos d + y sin d, -x sin d + y cos d), the direction phi becomes phi - d; */
/* z, tan(lambda) and q/pT do not change.  The new state lives at the plane    */
/* x' of the turned point.  Its Jacobian against the old state: a shift dy of  */
/* the track along the old y axis moves the point by (sin d, cos d) dy in the  */
/* new frame, and taking it back to the plane x' along the track (a step of    */
/* -sin d dy in x) gives dy' = (cos d - sin d tan phi') dy = cos phi / cos      */
/* phi' dy, dz' = -sin d tan(lambda) / cos phi' dy and dsin(phi') = -C sin d   */
/* dy; a turn of the direction gives dsin(phi') = cos phi' / cos phi           */
/* dsin(phi); everything else is unchanged to first order.                     */

/* S^-1 r . r for a symmetric positive definite 5x5 S (Cholesky); -1 when S
 * is not positive definite. */
static double chi2_of(const double S[25], const double r[5]) {
  double L[25] = {0};
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j <= i; ++j) {
      double v = S[i * 5 + j];
      for (int m = 0; m < j; ++m) v -= L[i * 5 + m] * L[j * 5 + m];
      if (i == j) {
        if (!(v > 0.0)) return -1.0;
        L[i * 5 + i] = sqrt(v);
      } else {
        L[i * 5 + j] = v / L[j * 5 + j];
      }
    }
  double w[5], q = 0.0;
  for (int i = 0; i < 5; ++i) {  /* w = L^-1 r */
    double v = r[i];
    for (int m = 0; m < i; ++m) v -= L[i * 5 + m] * w[m];
    w[i] = v / L[i * 5 + i];
    q += w[i] * w[i];
  }
  return q;
}

static void unpack_cov15(const double c15[15], double c[25]) {
  int m = 0;
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j <= i; ++j) c[i * 5 + j] = c[j * 5 + i] = c15[m++];
}

/* The match of segment a's outer end (state p_out at x_out in a's frame) to
 * segment b's inner end (state p_in at x_in in b's frame): a's state turned
 * into b's frame (when the units differ), carried along the helix to b's
 * x_in with its covariance, and chi2 = r^T (C_a + C_b)^-1 r over the five
 * parameters, r = p_b - p_a.  Returns chi2, or -1 when a's state cannot be
 * turned or carried, or the summed covariance is not positive definite. */
static double match_chi2(const double pa[5], const double ca15[15], double xa, double d, const double pb[5],
                         const double cb15[15], double xb, double k, double sinphi_max) {
  double p[5], C[25], x = xa, J[25], q[5], F[25];
  unpack_cov15(ca15, C);
  memcpy(p, pa, sizeof(p));
  if (d != 0.0) {
    if (orc_rotate(pa, xa, d, k, sinphi_max, p, &x, J) != 0) return -1.0;
    transport_cov(J, C);
  }
  if (orc_propagate(p, x, xb, k, sinphi_max, q, F) != 0) return -1.0;
  transport_cov(F, C);
  double Cb[25], S[25], r[5];
  unpack_cov15(cb15, Cb);
  for (int i = 0; i < 25; ++i) S[i] = C[i] + Cb[i];
  for (int i = 0; i < 5; ++i) r[i] = pb[i] - q[i];
  return chi2_of(S, r);
}

/* Links between the refitted segments of a tracking call (Reading R-24).
 * Segment b is a candidate continuation of segment a when both are refitted,
 * their units lie on the same side with |a2 - a1| <= max_dalpha (the same
 * unit included), b's first hit row follows a's last one by 1 .. max_gap rows,
 * the z' of b's inner state lies within dz_max of the z' of a's outer state,
 * the y of b's inner state within dy_max of the y of a's outer state turned
 * into b's frame and carried along the helix to b's x_in, and
 * match_chi2 <= chi2_max.  Each segment takes its best candidate in
 * each direction (the least chi2, then the smaller index); a and b are linked
 * when each is the other's best.  Output per segment: next (outer partner) and
 * prev (inner partner), -1 for none, and the link's chi2 in link_chi2 (at the
 * inner segment).  fragile = 1 on a segment whose link decision comes within
 * eps (relative) of the cut or of a tie.  Returns the number of candidate
 * pairs. */
int64_t orc_merge(int64_t T, const int32_t *unit, const int32_t *first_row, const int32_t *last_row,
                  const int8_t *ok, const double *p_in, const double *cov_in, const double *x_in,
                  const double *p_out, const double *cov_out, const double *x_out, int32_t n_units,
                  const double *unit_alpha, const int32_t *unit_side, int32_t n_rows, double k,
                  double sinphi_max, double max_dalpha, int32_t max_gap, double dz_max, double dy_max,
                  double chi2_max, double eps, int32_t *next, int32_t *prev, double *link_chi2,
                  int8_t *fragile) {
  /* segments by (unit, first row) */
  const int64_t nb = (int64_t)n_units * n_rows;
  int64_t *start = (int64_t *)calloc((size_t)nb + 1, sizeof(int64_t));
  int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)(T > 0 ? T : 1));
  for (int64_t t = 0; t < T; ++t)
    if (ok[t]) ++start[(int64_t)unit[t] * n_rows + first_row[t] + 1];
  for (int64_t b = 0; b < nb; ++b) start[b + 1] += start[b];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nb + 1));
  memcpy(fill, start, sizeof(int64_t) * (size_t)(nb + 1));
  for (int64_t t = 0; t < T; ++t)
    if (ok[t]) idx[fill[(int64_t)unit[t] * n_rows + first_row[t]]++] = t;
  free(fill);
  /* best candidate of each segment outward (ob) and inward (ib), with the
   * runner-up chi2 for the fragile flag */
  double *ob_c = (double *)malloc(sizeof(double) * (size_t)(T > 0 ? T : 1));
  double *ib_c = (double *)malloc(sizeof(double) * (size_t)(T > 0 ? T : 1));
  double *ob_2 = (double *)malloc(sizeof(double) * (size_t)(T > 0 ? T : 1));
  double *ib_2 = (double *)malloc(sizeof(double) * (size_t)(T > 0 ? T : 1));
  int64_t *ob = (int64_t *)malloc(sizeof(int64_t) * (size_t)(T > 0 ? T : 1));
  int64_t *ib = (int64_t *)malloc(sizeof(int64_t) * (size_t)(T > 0 ? T : 1));
  int8_t *near_cut = (int8_t *)calloc((size_t)(T > 0 ? T : 1), 1);
  for (int64_t t = 0; t < T; ++t) {
    ob[t] = ib[t] = -1;
    ob_c[t] = ib_c[t] = ob_2[t] = ib_2[t] = INFINITY;
  }
  int64_t n_cand = 0;
  for (int64_t a = 0; a < T; ++a) {
    if (!ok[a]) continue;
    for (int32_t w = 0; w < n_units; ++w) {
      if (unit_side[w] != unit_side[unit[a]]) continue;
      const double d = remainder(unit_alpha[w] - unit_alpha[unit[a]], 2.0 * M_PI_ORC);
      if (!(fabs(d) <= max_dalpha)) continue;
      /* a's outer state in w's frame (parameters only) */
      double pw[5], xw = x_out[a];
      memcpy(pw, p_out + a * 5, sizeof(pw));
      if (w != unit[a] && orc_rotate(p_out + a * 5, x_out[a], d, k, sinphi_max, pw, &xw, NULL) != 0) continue;
      for (int32_t r = last_row[a] + 1; r <= last_row[a] + max_gap && r < n_rows; ++r) {
        const int64_t bin = (int64_t)w * n_rows + r;
        for (int64_t q = start[bin]; q < start[bin + 1]; ++q) {
          const int64_t b = idx[q];
          if (!(fabs(p_in[b * 5 + 1] - p_out[a * 5 + 1]) <= dz_max)) continue;
          double yc[5];
          if (orc_propagate(pw, xw, x_in[b], k, sinphi_max, yc, NULL) != 0) continue;
          if (!(fabs(p_in[b * 5] - yc[0]) <= dy_max)) continue;
          const double c2 = match_chi2(p_out + a * 5, cov_out + a * 15, x_out[a], w == unit[a] ? 0.0 : d,
                                       p_in + b * 5, cov_in + b * 15, x_in[b], k, sinphi_max);
          if (c2 < 0.0) continue;
          if (fabs(c2 - chi2_max) <= eps * chi2_max) near_cut[a] = near_cut[b] = 1;
          if (c2 > chi2_max) continue;
          ++n_cand;
          if (c2 < ob_c[a] || (c2 == ob_c[a] && b < ob[a])) {
            ob_2[a] = ob_c[a];
            ob_c[a] = c2;
            ob[a] = b;
          } else if (c2 < ob_2[a]) {
            ob_2[a] = c2;
          }
          if (c2 < ib_c[b] || (c2 == ib_c[b] && a < ib[b])) {
            ib_2[b] = ib_c[b];
            ib_c[b] = c2;
            ib[b] = a;
          } else if (c2 < ib_2[b]) {
            ib_2[b] = c2;
          }
        }
      }
    }
  }
  for (int64_t t = 0; t < T; ++t) {
    next[t] = prev[t] = -1;
    link_chi2[t] = 0.0;
  }
  for (int64_t a = 0; a < T; ++a) {
    const int64_t b = ob[a];
    if (b >= 0 && ib[b] == a) {
      next[a] = (int32_t)b;
      prev[b] = (int32_t)a;
      link_chi2[a] = ob_c[a];
    }
  }
  for (int64_t t = 0; t < T; ++t) {
    int fr = near_cut[t];
    if (ob[t] >= 0 && ob_2[t] - ob_c[t] <= eps * ob_c[t]) fr = 1;
    if (ib[t] >= 0 && ib_2[t] - ib_c[t] <= eps * ib_c[t]) fr = 1;
    fragile[t] = (int8_t)fr;
  }
  free(start);
  free(idx);
  free(ob_c);
  free(ib_c);
  free(ob_2);
  free(ib_2);
  free(ob);
  free(ib);
  free(near_cut);
  return n_cand;
}

/* The chains of a batch: chain c's hits are the cluster ids
 * hits[first[c] .. first[c] + nh[c]) with units hit_unit[...], measured as the
 * tracker measures them (quanta of 1/256 cm at the rows' x).  ok[c] = 1 when
 * the fit succeeded, else every output of the chain is zero. */
void orc_refit_chains(int64_t n_chains, const int32_t *first, const int32_t *nh, const int32_t *hits,
                      const int32_t *hit_unit, const float *y, const float *z, const uint16_t *row,
                      const double *row_x, const double *unit_alpha, int32_t n_units, double k,
                      const orc_params_t *P, double *p, double *cov, double *x_ref, double *chi2, int8_t *ok) {
  fit_real *ua = (fit_real *)malloc(sizeof(fit_real) * (size_t)(n_units > 0 ? n_units : 1));
  for (int32_t u = 0; u < n_units; ++u) ua[u] = unit_alpha[u];
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t c = 0; c < n_chains; ++c) {
    const int n = nh[c];
    fit_real *X = (fit_real *)malloc(sizeof(fit_real) * 3 * (size_t)(n > 0 ? n : 1));
    fit_real *Y = X + n, *Z = X + 2 * n;
    for (int j = 0; j < n; ++j) {
      const int32_t h = hits[first[c] + j];
      X[j] = row_x[row[h]];
      Y[j] = nearbyint(256.0 * (double)y[h]) / 256.0;
      Z[j] = nearbyint(256.0 * (double)z[h]) / 256.0;
    }
    fit_real pp[5], cc[15], ch = 0;
    const int st = orc_fit_chain(n, X, Y, Z, hit_unit + first[c], ua, (fit_real)k, P, pp, cc, &ch);
    ok[c] = st == 0;
    for (int q = 0; q < 5; ++q) p[c * 5 + q] = st == 0 ? (double)pp[q] : 0.0;
    for (int q = 0; q < 15; ++q) cov[c * 15 + q] = st == 0 ? (double)cc[q] : 0.0;
    chi2[c] = st == 0 ? (double)ch : 0.0;
    x_ref[c] = st == 0 ? (double)X[0] : 0.0;
    free(X);
  }
  free(ua);
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the following calls (timing only; results do not depend on it). */
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

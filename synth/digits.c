/*
 * Raw ADC digits of the clusters of an event, for the clusterizer: per
 * cluster a charge spread over pads and time bins by Gaussian response
 * functions (the fraction of each bin under the Gaussian), summed where
 * clusters overlap, noise added, rounded, zero-suppressed and clipped to 10
 * bits.  Part of the seeded synthetic-input generator; it holds no step of
 * the clusterizer.
 *
 * Pads: row r has 2 * half[r] pads of width pw; pad p is centred at
 * y = (p + 0.5 - half[r]) * pw.  Time bins: bin t is centred at
 * z' = (t + 0.5) * tb - zoff.
 *
 * Output: digits grouped by (unit, row, pad), times increasing inside a pad;
 * pad_counts[(unit * n_rows + row) * max_pads + pad] receives the number of
 * digits of each pad.  Noise comes from a counter-based generator (splitmix64
 * of the seed and the digit's coordinates) so the result does not depend on
 * the number of threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define FOOT 2 /* footprint: +-2 pads, +-2 time bins around the centre bin */

static uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

/* standard normal from two uniforms of the counter-based stream (Box-Muller) */
static double normal_at(uint64_t seed, uint64_t key) {
  const uint64_t a = splitmix64(seed ^ splitmix64(key));
  const uint64_t b = splitmix64(a ^ 0x5851F42D4C957F2Dull);
  const double u1 = ((double)(a >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double u2 = (double)(b >> 11) * (1.0 / 9007199254740992.0);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* fraction of a unit Gaussian (centre c, width s) inside [a, b] */
static double frac(double a, double b, double c, double s) {
  const double k = 1.0 / (s * 1.4142135623730951);
  return 0.5 * (erf((b - c) * k) - erf((a - c) * k));
}

/*
 * n_rows rows; half[r] half the pad count of row r (max_pads >= 2 * half[r]).
 * Clusters: positions y, z (cm), row, charge q (ADC sum), grouped by
 * (unit, row) through ur_offsets[n_units * n_rows + 1] over the order `order`.
 * Count pass (out_time == NULL) fills pad_counts and returns the total; the
 * fill pass writes out_time / out_q at the offsets the caller derived from
 * pad_counts (pad_starts, same layout).
 */
int64_t synth_digits(int32_t n_units, int32_t n_rows, const int32_t *half, int32_t max_pads, double pw,
                     double tb, double zoff, double sig_pad, double sig_time, double noise, int32_t thr,
                     uint64_t seed, const int64_t *ur_offsets, const int64_t *order, const float *y,
                     const float *z, const double *q, int64_t *pad_counts, const int64_t *pad_starts,
                     uint16_t *out_time, uint16_t *out_q) {
  const int fill = out_time != NULL;
  int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : total)
  for (int64_t ur = 0; ur < (int64_t)n_units * n_rows; ++ur) {
    const int r = (int)(ur % n_rows);
    const int np = 2 * half[r];
    const int64_t a = ur_offsets[ur], b = ur_offsets[ur + 1];
    int64_t *cnt = pad_counts + ur * max_pads;
    if (!fill) memset(cnt, 0, sizeof(int64_t) * (size_t)max_pads);
    if (a == b) continue;
    /* time extent of this row's clusters */
    double tmin = 1e300, tmax = -1e300;
    for (int64_t k = a; k < b; ++k) {
      const double tc = ((double)z[order[k]] + zoff) / tb - 0.5;
      if (tc < tmin) tmin = tc;
      if (tc > tmax) tmax = tc;
    }
    int64_t t0 = (int64_t)floor(tmin) - FOOT - 1, t1 = (int64_t)floor(tmax) + FOOT + 2;
    if (t0 < 0) t0 = 0;
    if (t1 > 65535) t1 = 65535;
    if (t1 < t0) continue;
    const int64_t nt = t1 - t0 + 1;
    float *map = (float *)calloc((size_t)(np * nt), sizeof(float));
    uint8_t *hit = (uint8_t *)calloc((size_t)(np * nt), 1);
    for (int64_t k = a; k < b; ++k) {
      const int64_t c = order[k];
      const double pc = (double)y[c] / pw + half[r] - 0.5; /* continuous pad coordinate */
      const double tc = ((double)z[c] + zoff) / tb - 0.5;   /* continuous time coordinate */
      const int64_t p0 = (int64_t)floor(pc + 0.5), tt0 = (int64_t)floor(tc + 0.5);
      for (int dp = -FOOT; dp <= FOOT; ++dp) {
        const int64_t p = p0 + dp;
        if (p < 0 || p >= np) continue;
        const double fp = frac(p - 0.5, p + 0.5, pc, sig_pad);
        for (int dt = -FOOT; dt <= FOOT; ++dt) {
          const int64_t t = tt0 + dt;
          if (t < t0 || t > t1) continue;
          const double ft = frac(t - 0.5, t + 0.5, tc, sig_time);
          map[p * nt + (t - t0)] += (float)(q[c] * fp * ft);
          hit[p * nt + (t - t0)] = 1;
        }
      }
    }
    for (int p = 0; p < np; ++p) {
      int64_t o = fill ? pad_starts[ur * max_pads + p] : 0;
      int64_t m = 0;
      for (int64_t j = 0; j < nt; ++j) {
        if (!hit[p * nt + j]) continue;
        const uint64_t key = (((uint64_t)ur * 4096u + (uint64_t)p) << 20) ^ (uint64_t)(t0 + j);
        double v = map[p * nt + j] + noise * normal_at(seed, key);
        long a2 = lrint(v);
        if (a2 < thr) continue;
        if (a2 > 1023) a2 = 1023;
        if (fill) {
          out_time[o] = (uint16_t)(t0 + j);
          out_q[o] = (uint16_t)a2;
          ++o;
        }
        ++m;
      }
      if (!fill) cnt[p] = m;
      total += m;
    }
    free(map);
    free(hit);
  }
  return total;
}

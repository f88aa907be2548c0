/*
 * CPU oracle for atlas-based fiber bundle segmentation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * source with the GPU library.
 *
 * What it computes (Vazquez et al., "Parallel optimization of fiber bundle
 * segmentation for massive tractography datasets"):
 *
 *   d_E(a_i, b_i) = || a_i - b_i ||_2                         (Eq. 1)
 *   d_ME(a, b)    = min( max_i d_E(a_i, b_i),
 *                        max_i d_E(a_i, b_{20-i}) )           (Eq. 2; the
 *                   inverse order pairs point i with point 20-i, 0-based)
 *   a fiber matches a centroid when d_ME is not above the threshold of the
 *   centroid's bundle (section 2.3); among matching centroids the fiber takes
 *   the bundle of the closest one (section 2.4, "Classification of fibers";
 *   Algorithm 1 keeps the first centroid found at equal distance, i.e. the
 *   lowest index in bundle-major order).
 *
 * Readings of points the paper leaves open (each is listed with its reason in
 * the design notes of the repository):
 *   - comparison is done on squared distances: D = d_ME^2 against
 *     T2 = fl32(T*T); a bundle with T < 0 never matches;
 *   - "under the threshold" is inclusive: accept iff D <= T2;
 *   - the float32 point distance is evaluated with one fixed expression and
 *     no other contraction:
 *         dx = fl(a.x - b.x), dy = ..., dz = ...
 *         d2 = fmaf(dz, dz, fmaf(dy, dy, fl(dx * dx)))
 *     (this file must be compiled with -ffp-contract=off);
 *   - a fiber with no matching centroid gets label -1 and distance +inf;
 *   - the reported distance is d_ME (no length term), sqrt of D rounded once.
 *
 * Two evaluation modes reach the same result:
 *   ORACLE_BRUTE  every pair, every point, both orders (the definition);
 *   ORACLE_CUT    the paper's progressive discard (section 2.3, "Progressive
 *                 fiber discarding", and section 2.4): center point, then the
 *                 two end points, then four intermediate points, then all
 *                 points, with an exit as soon as a point distance exceeds
 *                 the threshold in an order; an order dies on its first
 *                 exceeding point and a pair dies when both orders died.
 *                 The four intermediate points are 4, 8, 12 and 16 (the paper
 *                 does not name them; any choice gives the same result).
 * Metric variants (oracle_segment_ext_f32), flags:
 *   VAR_TN   length normalisation (section 2.3, Eq. 3): for an accepted pair the
 *            complete metric is  d_ME + TN,  TN = (|l_S - l_C| / max(l_S, l_C) + 1)^2 - 1
 *            with l the arc length of the 21-point polyline; the pair is kept
 *            when D <= T2 and d_ME + TN <= T, and the fiber takes the bundle of
 *            the smallest complete metric (readings: the metric is compared
 *            with the threshold, TN = 0 when both lengths are 0, the reported
 *            distance is the complete metric);
 *   VAR_DIR  direction inference (section 2.4, "Inference of fiber
 *            direction"): the order with the smaller largest end-point
 *            distance (direct on ties) is the fiber's direction and D is the
 *            largest point distance of that order only.
 *   float32 expressions: segment length sqrtf(fmaf(dz, dz, fmaf(dy, dy,
 *   dx * dx))) of p[i+1] - p[i], summed in point order; r = |lS - lC| / max
 *   (rounded once), u = r + 1, TN = u * u - 1 (each rounded); the complete
 *   metric sqrtf(D) + TN (rounded once).
 * Several labels per fiber (oracle_segment_multi_f32), the classification of
 *   the previous version of the algorithm (section 2.4, "Classification of
 *   fibers": a fiber may be assigned to every bundle whose threshold test it
 *   passes): the fiber is a member of bundle B when some centroid of B passes
 *   the test above (with the metric variant's rules); its distance to B is
 *   the smallest value over those centroids (sqrtf(D), or the complete
 *   metric with VAR_TN).  Output: per fiber, its bundles in increasing id
 *   with their distances, as rows of a CSR table, and the number of members
 *   of each bundle.
 * Resampling (oracle_resample_f32), the step before the comparison: every
 *   subject fiber is brought to 21 points equidistant in arc length (section
 *   2.3, classification algorithm; section 2.2: the atlas centroids carry 21
 *   equidistant points).  A raw streamline is a polyline of P >= 1 points.
 *   The arc length is accumulated exactly, in fixed point, so that it does
 *   not depend on the order of summation:
 *     segment length  g_j = sqrtf of the float32 squared length of
 *                     d = fl(p_{j+1} - p_j), the same expression as the
 *                     point distance (and the arc length above);
 *     fixed point     q_j = g_j in units of 2^-24 mm, rounded to nearest
 *                     (ties to even); 2^38 (16.384 m) for g_j >= 2^14 mm or
 *                     a non-finite g_j;
 *     cumulative      S_0 = 0, S_{j+1} = S_j + q_j (exact 64-bit integers),
 *                     L = S_{P-1};
 *     targets         t_k = floor(k L / 20), k = 1..19 (exact);
 *     point k         on the first segment j with t_k <= S_{j+1}, at
 *                     w = fl(fl(t_k - S_j) / fl(q_j)) (integer differences
 *                     converted to float32, rounded to nearest), clamped to
 *                     [0, 1], 0 when q_j = 0: out = fmaf(w, fl(p_{j+1} -
 *                     p_j), p_j) per coordinate;
 *     end points      out_0 = p_0 and out_20 = p_{P-1}, copied;
 *     one point       all 21 outputs are that point.
 *   A streamline without points or of more than 2^24 points (so that its
 *   sum stays below 2^62), or offsets outside [0, npts] or decreasing, is an
 *   error.
 * Precisions:
 *   *_f32  the float32 decision above (labels must match it bit for bit);
 *   *_f64  the same definition in double precision with exact differences,
 *          accept iff D64 <= (double)T * (double)T.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define NP 21
#define CENTER 10

enum { ORACLE_BRUTE = 0, ORACLE_CUT = 1 };
enum { VAR_TN = 1, VAR_DIR = 2 };

/* ---------------------------------------------------------------- float32 */

static float d2_f32(const float* a, const float* b) {
  float dx = a[0] - b[0];
  float dy = a[1] - b[1];
  float dz = a[2] - b[2];
  return fmaf(dz, dz, fmaf(dy, dy, dx * dx));
}

/* Squared threshold of a bundle; -1 encodes "never matches". */
static float thr2_f32(float t) { return t >= 0.0f ? t * t : -1.0f; }

/* Definition: both orders over all 21 points. */
void oracle_pair_f32(const float* a, const float* b, float* d_dir, float* d_inv) {
  float md = 0.0f, mi = 0.0f;
  for (int i = 0; i < NP; ++i) {
    float x = d2_f32(a + 3 * i, b + 3 * i);
    float y = d2_f32(a + 3 * i, b + 3 * (NP - 1 - i));
    md = x > md ? x : md;
    mi = y > mi ? y : mi;
  }
  *d_dir = md;
  *d_inv = mi;
}

/* Brute evaluation of one pair: returns 1 and D when accepted. */
static int eval_brute_f32(const float* a, const float* b, float t2, float* D) {
  float md, mi;
  oracle_pair_f32(a, b, &md, &mi);
  float d = md < mi ? md : mi;
  if (d <= t2) {
    *D = d;
    return 1;
  }
  return 0;
}

/* Progressive discard of one pair (paper's tests 1-4). */
static int eval_cut_f32(const float* a, const float* b, float t2, float* D) {
  static const int four[4] = {4, 8, 12, 16};
  /* test1: the center point pairs with itself in both orders */
  float c = d2_f32(a + 3 * CENTER, b + 3 * CENTER);
  if (c > t2) return 0;
  float md = c, mi = c;
  int alive_d = 1, alive_i = 1;
  /* test2: end points */
  {
    float x0 = d2_f32(a, b), x1 = d2_f32(a + 3 * (NP - 1), b + 3 * (NP - 1));
    if (x0 > t2 || x1 > t2) alive_d = 0;
    else { md = x0 > md ? x0 : md; md = x1 > md ? x1 : md; }
    float y0 = d2_f32(a, b + 3 * (NP - 1)), y1 = d2_f32(a + 3 * (NP - 1), b);
    if (y0 > t2 || y1 > t2) alive_i = 0;
    else { mi = y0 > mi ? y0 : mi; mi = y1 > mi ? y1 : mi; }
  }
  if (!alive_d && !alive_i) return 0;
  /* test3: four intermediate points, exit at the first exceeding distance */
  for (int k = 0; k < 4 && alive_d; ++k) {
    int i = four[k];
    float x = d2_f32(a + 3 * i, b + 3 * i);
    if (x > t2) alive_d = 0; else md = x > md ? x : md;
  }
  for (int k = 0; k < 4 && alive_i; ++k) {
    int i = four[k];
    float y = d2_f32(a + 3 * i, b + 3 * (NP - 1 - i));
    if (y > t2) alive_i = 0; else mi = y > mi ? y : mi;
  }
  if (!alive_d && !alive_i) return 0;
  /* test4: the remaining points */
  for (int i = 1; i < NP - 1 && alive_d; ++i) {
    if (i == CENTER || i == 4 || i == 8 || i == 12 || i == 16) continue;
    float x = d2_f32(a + 3 * i, b + 3 * i);
    if (x > t2) alive_d = 0; else md = x > md ? x : md;
  }
  for (int i = 1; i < NP - 1 && alive_i; ++i) {
    if (i == CENTER || i == 4 || i == 8 || i == 12 || i == 16) continue;
    float y = d2_f32(a + 3 * i, b + 3 * (NP - 1 - i));
    if (y > t2) alive_i = 0; else mi = y > mi ? y : mi;
  }
  if (alive_d && alive_i) *D = md < mi ? md : mi;
  else if (alive_d) *D = md;
  else if (alive_i) *D = mi;
  else return 0;
  return 1;
}

static int check_args(int64_t n, int64_t m, const int32_t* bid, int32_t nb) {
  if (n < 0 || m < 0) return -1;
  if (m > 0 && nb <= 0) return -1;
  for (int64_t c = 0; c < m; ++c)
    if (bid[c] < 0 || bid[c] >= nb) return -2;
  return 0;
}

/*
 * labels[N] int32, dists[N] float32, best[N] int32 (winning centroid index or
 * -1; may be NULL).  Returns 0, -1 on bad sizes, -2 on a bundle id out of
 * range.  nthreads <= 0 uses the OpenMP default.
 */
int oracle_segment_f32(const float* fibers, int64_t n, const float* cen, int64_t m,
                       const int32_t* bid, const float* thr, int32_t nb, int mode,
                       int nthreads, int32_t* labels, float* dists, int32_t* best) {
  int rc = check_args(n, m, bid, nb);
  if (rc) return rc;
  float* t2 = (float*)malloc(sizeof(float) * (size_t)(nb > 0 ? nb : 1));
  for (int32_t b = 0; b < nb; ++b) t2[b] = thr2_f32(thr[b]);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t f = 0; f < n; ++f) {
    const float* a = fibers + (size_t)f * 3 * NP;
    float bestd = 0.0f;
    int64_t bestc = -1;
    for (int64_t c = 0; c < m; ++c) {
      float D;
      const float* b = cen + (size_t)c * 3 * NP;
      float tt = t2[bid[c]];
      int ok = mode == ORACLE_CUT ? eval_cut_f32(a, b, tt, &D) : eval_brute_f32(a, b, tt, &D);
      if (ok && (bestc < 0 || D < bestd)) {
        bestd = D;
        bestc = c;
      }
    }
    if (bestc < 0) {
      labels[f] = -1;
      dists[f] = INFINITY;
    } else {
      labels[f] = bid[bestc];
      dists[f] = sqrtf(bestd);
    }
    if (best) best[f] = (int32_t)bestc;
  }
  free(t2);
  return 0;
}

/*
 * Every accepted (fiber, centroid) pair, in fiber-major then centroid order.
 * Writes at most cap pairs into pairs[2*k], pairs[2*k+1]; returns the total
 * count (which may exceed cap), or a negative code.  Single-threaded.
 */
int64_t oracle_accepted_pairs_f32(const float* fibers, int64_t n, const float* cen, int64_t m,
                                  const int32_t* bid, const float* thr, int32_t nb,
                                  int64_t* pairs, int64_t cap) {
  int rc = check_args(n, m, bid, nb);
  if (rc) return rc;
  int64_t cnt = 0;
  for (int64_t f = 0; f < n; ++f) {
    const float* a = fibers + (size_t)f * 3 * NP;
    for (int64_t c = 0; c < m; ++c) {
      float D;
      if (eval_brute_f32(a, cen + (size_t)c * 3 * NP, thr2_f32(thr[bid[c]]), &D)) {
        if (cnt < cap) {
          pairs[2 * cnt] = f;
          pairs[2 * cnt + 1] = c;
        }
        ++cnt;
      }
    }
  }
  return cnt;
}

/* ---------------------------------------------------------------- variants */

/* Arc length of a 21-point polyline (float32, segments summed in order). */
float oracle_arc_length_f32(const float* p) {
  float l = 0.0f;
  for (int i = 0; i + 1 < NP; ++i) {
    float dx = p[3 * (i + 1)] - p[3 * i];
    float dy = p[3 * (i + 1) + 1] - p[3 * i + 1];
    float dz = p[3 * (i + 1) + 2] - p[3 * i + 2];
    l = l + sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
  }
  return l;
}

/* Length term of Eq. 3. */
float oracle_tn_f32(float ls, float lc) {
  float mx = ls > lc ? ls : lc;
  if (!(mx > 0.0f)) return 0.0f;
  float r = fabsf(ls - lc) / mx;
  float u = r + 1.0f;
  float uu = u * u;
  return uu - 1.0f;
}

/* Direction inference, brute form: the order with the smaller largest
   end-point distance, then every point of that order. */
static int eval_dir_brute_f32(const float* a, const float* b, float t2, float* D) {
  float ed = d2_f32(a, b), ed2 = d2_f32(a + 3 * (NP - 1), b + 3 * (NP - 1));
  float ei = d2_f32(a, b + 3 * (NP - 1)), ei2 = d2_f32(a + 3 * (NP - 1), b);
  ed = ed2 > ed ? ed2 : ed;
  ei = ei2 > ei ? ei2 : ei;
  int direct = ed <= ei;
  float mx = 0.0f;
  for (int i = 0; i < NP; ++i) {
    float x = d2_f32(a + 3 * i, b + 3 * (direct ? i : NP - 1 - i));
    mx = x > mx ? x : mx;
  }
  if (mx <= t2) {
    *D = mx;
    return 1;
  }
  return 0;
}

/* Direction inference as the paper runs it: center, end points (which fix
   the direction), then the four intermediate points and the rest in that
   direction only, leaving at the first point above the threshold. */
static int eval_dir_cut_f32(const float* a, const float* b, float t2, float* D) {
  static const int four[4] = {4, 8, 12, 16};
  float c = d2_f32(a + 3 * CENTER, b + 3 * CENTER);
  if (c > t2) return 0;
  float x0 = d2_f32(a, b), x1 = d2_f32(a + 3 * (NP - 1), b + 3 * (NP - 1));
  float y0 = d2_f32(a, b + 3 * (NP - 1)), y1 = d2_f32(a + 3 * (NP - 1), b);
  float ed = x1 > x0 ? x1 : x0, ei = y1 > y0 ? y1 : y0;
  int direct = ed <= ei;
  float mx = direct ? ed : ei;
  if (mx > t2) return 0;
  mx = c > mx ? c : mx;
  for (int k = 0; k < 4; ++k) {
    int i = four[k];
    float x = d2_f32(a + 3 * i, b + 3 * (direct ? i : NP - 1 - i));
    if (x > t2) return 0;
    mx = x > mx ? x : mx;
  }
  for (int i = 1; i < NP - 1; ++i) {
    if (i == CENTER || i == 4 || i == 8 || i == 12 || i == 16) continue;
    float x = d2_f32(a + 3 * i, b + 3 * (direct ? i : NP - 1 - i));
    if (x > t2) return 0;
    mx = x > mx ? x : mx;
  }
  *D = mx;
  return 1;
}

/*
 * The float32 decision with metric variants (flags: VAR_TN | VAR_DIR).
 * Outputs as oracle_segment_f32; dists holds the complete metric with
 * VAR_TN, sqrtf(D) otherwise.  flags = 0 gives oracle_segment_f32's result.
 */
int oracle_segment_ext_f32(const float* fibers, int64_t n, const float* cen, int64_t m,
                           const int32_t* bid, const float* thr, int32_t nb, int mode, int flags,
                           int nthreads, int32_t* labels, float* dists, int32_t* best) {
  int rc = check_args(n, m, bid, nb);
  if (rc) return rc;
  float* t2 = (float*)malloc(sizeof(float) * (size_t)(nb > 0 ? nb : 1));
  float* lc = (float*)malloc(sizeof(float) * (size_t)(m > 0 ? m : 1));
  for (int32_t b = 0; b < nb; ++b) t2[b] = thr2_f32(thr[b]);
  for (int64_t c = 0; c < m; ++c) lc[c] = oracle_arc_length_f32(cen + (size_t)c * 3 * NP);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t f = 0; f < n; ++f) {
    const float* a = fibers + (size_t)f * 3 * NP;
    const float ls = oracle_arc_length_f32(a);
    float bestv = 0.0f;
    int64_t bestc = -1;
    for (int64_t c = 0; c < m; ++c) {
      float D;
      const float* b = cen + (size_t)c * 3 * NP;
      float tt = t2[bid[c]];
      int ok;
      if (flags & VAR_DIR)
        ok = mode == ORACLE_CUT ? eval_dir_cut_f32(a, b, tt, &D) : eval_dir_brute_f32(a, b, tt, &D);
      else
        ok = mode == ORACLE_CUT ? eval_cut_f32(a, b, tt, &D) : eval_brute_f32(a, b, tt, &D);
      if (!ok) continue;
      float v = D;
      if (flags & VAR_TN) {
        v = sqrtf(D) + oracle_tn_f32(ls, lc[c]);
        if (!(v <= thr[bid[c]])) continue;
      }
      if (bestc < 0 || v < bestv) {
        bestv = v;
        bestc = c;
      }
    }
    if (bestc < 0) {
      labels[f] = -1;
      dists[f] = INFINITY;
    } else {
      labels[f] = bid[bestc];
      dists[f] = (flags & VAR_TN) ? bestv : sqrtf(bestv);
    }
    if (best) best[f] = (int32_t)bestc;
  }
  free(lc);
  free(t2);
  return 0;
}

/* ---------------------------------------------------------------- several labels */

/* Bundles of fiber a: best[b] = smallest accepted value over the centroids
   of bundle b, seen[b] = whether any centroid of b was accepted. */
static void multi_one_f32(const float* a, const float* cen, int64_t m, const int32_t* bid,
                          const float* thr, const float* t2, const float* lc, int mode, int flags,
                          float* best, char* seen) {
  const float ls = oracle_arc_length_f32(a);
  for (int64_t c = 0; c < m; ++c) {
    float D;
    const float* b = cen + (size_t)c * 3 * NP;
    float tt = t2[bid[c]];
    int ok;
    if (flags & VAR_DIR)
      ok = mode == ORACLE_CUT ? eval_dir_cut_f32(a, b, tt, &D) : eval_dir_brute_f32(a, b, tt, &D);
    else
      ok = mode == ORACLE_CUT ? eval_cut_f32(a, b, tt, &D) : eval_brute_f32(a, b, tt, &D);
    if (!ok) continue;
    float v = D;
    if (flags & VAR_TN) {
      v = sqrtf(D) + oracle_tn_f32(ls, lc[c]);
      if (!(v <= thr[bid[c]])) continue;
    }
    int32_t k = bid[c];
    if (!seen[k] || v < best[k]) best[k] = v;
    seen[k] = 1;
  }
}

/*
 * Several labels per fiber.  offsets [n + 1]: fiber f's entries are
 * bundles/dists[offsets[f] .. offsets[f+1]), bundles increasing; entries
 * beyond `cap` are not written.  bundle_counts [nb] (may be NULL).  Returns
 * the number of entries, or a negative error.
 */
int64_t oracle_segment_multi_f32(const float* fibers, int64_t n, const float* cen, int64_t m,
                                 const int32_t* bid, const float* thr, int32_t nb, int mode,
                                 int flags, int nthreads, int64_t* offsets, int32_t* bundles,
                                 float* dists, int64_t cap, int64_t* bundle_counts) {
  int rc = check_args(n, m, bid, nb);
  if (rc) return rc;
  const size_t nbs = (size_t)(nb > 0 ? nb : 1);
  float* t2 = (float*)malloc(sizeof(float) * nbs);
  float* lc = (float*)malloc(sizeof(float) * (size_t)(m > 0 ? m : 1));
  for (int32_t b = 0; b < nb; ++b) t2[b] = thr2_f32(thr[b]);
  for (int64_t c = 0; c < m; ++c) lc[c] = oracle_arc_length_f32(cen + (size_t)c * 3 * NP);
  /* pass 1: number of bundles of each fiber; pass 2: the entries */
  for (int pass = 0; pass < 2; ++pass) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
      float* best = (float*)malloc(sizeof(float) * nbs);
      char* seen = (char*)malloc(nbs);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
      for (int64_t f = 0; f < n; ++f) {
        memset(seen, 0, nbs);
        multi_one_f32(fibers + (size_t)f * 3 * NP, cen, m, bid, thr, t2, lc, mode, flags, best,
                      seen);
        int64_t k = 0;
        for (int32_t b = 0; b < nb; ++b) {
          if (!seen[b]) continue;
          if (pass == 1) {
            int64_t at = offsets[f] + k;
            if (at < cap) {
              bundles[at] = b;
              dists[at] = (flags & VAR_TN) ? best[b] : sqrtf(best[b]);
            }
          }
          ++k;
        }
        if (pass == 0) offsets[f + 1] = k;
      }
      free(seen);
      free(best);
    }
    if (pass == 0) {
      offsets[0] = 0;
      for (int64_t f = 0; f < n; ++f) offsets[f + 1] += offsets[f];
    }
  }
  if (bundle_counts) {
    for (int32_t b = 0; b < nb; ++b) bundle_counts[b] = 0;
    for (int64_t i = 0; i < offsets[n] && i < cap; ++i) bundle_counts[bundles[i]] += 1;
  }
  free(lc);
  free(t2);
  return offsets[n];
}

/* ---------------------------------------------------------------- resampling */

/* Fixed-point length of one segment (units of 2^-24 mm). */
static int64_t seg_fixed(float g) {
  if (!(g < 16384.0f)) return (int64_t)1 << 38;
  return (int64_t)rintf(g * 16777216.0f);
}

/* One streamline of P >= 1 points to 21 points; S is scratch of P sums. */
static void resample_one_f32(const float* p, int64_t P, int64_t* S, float* out) {
  S[0] = 0;
  for (int64_t j = 0; j + 1 < P; ++j) {
    float dx = p[3 * (j + 1)] - p[3 * j];
    float dy = p[3 * (j + 1) + 1] - p[3 * j + 1];
    float dz = p[3 * (j + 1) + 2] - p[3 * j + 2];
    S[j + 1] = S[j] + seg_fixed(sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx * dx))));
  }
  int64_t L = S[P - 1];
  for (int c = 0; c < 3; ++c) {
    out[c] = p[c];
    out[3 * (NP - 1) + c] = p[3 * (P - 1) + c];
  }
  for (int k = 1; k < NP - 1; ++k) {
    int64_t t = (L / 20) * k + ((L % 20) * k) / 20;
    int64_t j = 0;
    while (j + 1 < P && !(t <= S[j + 1])) ++j;
    if (j + 1 >= P) {  /* a single point */
      for (int c = 0; c < 3; ++c) out[3 * k + c] = p[3 * (P - 1) + c];
      continue;
    }
    int64_t q = S[j + 1] - S[j];
    float w = q > 0 ? (float)(t - S[j]) / (float)q : 0.0f;
    w = w < 0.0f ? 0.0f : (w > 1.0f ? 1.0f : w);
    for (int c = 0; c < 3; ++c) {
      float a = p[3 * j + c], b = p[3 * (j + 1) + c];
      out[3 * k + c] = fmaf(w, b - a, a);
    }
  }
}

int oracle_resample_f32(const float* pts, const int64_t* off, int64_t n, int64_t npts,
                        int nthreads, float* out) {
  if (n < 0 || npts < 0) return -1;
  int64_t pmax = 1;
  for (int64_t i = 0; i < n; ++i) {
    if (off[i] < 0 || off[i + 1] > npts || off[i + 1] <= off[i]) return -2;
    if (off[i + 1] - off[i] > ((int64_t)1 << 24)) return -2;
    if (off[i + 1] - off[i] > pmax) pmax = off[i + 1] - off[i];
  }
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
  {
    int64_t* s = (int64_t*)malloc((size_t)pmax * sizeof(int64_t));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 256)
#endif
    for (int64_t i = 0; i < n; ++i)
      resample_one_f32(pts + 3 * off[i], off[i + 1] - off[i], s, out + (size_t)i * 3 * NP);
    free(s);
  }
  return 0;
}

/* ---------------------------------------------------------------- float64 */

static double d2_f64(const float* a, const float* b) {
  double dx = (double)a[0] - (double)b[0];
  double dy = (double)a[1] - (double)b[1];
  double dz = (double)a[2] - (double)b[2];
  return dx * dx + dy * dy + dz * dz;
}

void oracle_pair_f64(const float* a, const float* b, double* d_dir, double* d_inv) {
  double md = 0.0, mi = 0.0;
  for (int i = 0; i < NP; ++i) {
    double x = d2_f64(a + 3 * i, b + 3 * i);
    double y = d2_f64(a + 3 * i, b + 3 * (NP - 1 - i));
    md = x > md ? x : md;
    mi = y > mi ? y : mi;
  }
  *d_dir = md;
  *d_inv = mi;
}

int oracle_segment_f64(const float* fibers, int64_t n, const float* cen, int64_t m,
                       const int32_t* bid, const float* thr, int32_t nb, int nthreads,
                       int32_t* labels, double* dists, int32_t* best) {
  int rc = check_args(n, m, bid, nb);
  if (rc) return rc;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t f = 0; f < n; ++f) {
    const float* a = fibers + (size_t)f * 3 * NP;
    double bestd = 0.0;
    int64_t bestc = -1;
    for (int64_t c = 0; c < m; ++c) {
      double t = (double)thr[bid[c]];
      if (!(t >= 0.0)) continue;
      double md, mi;
      oracle_pair_f64(a, cen + (size_t)c * 3 * NP, &md, &mi);
      double d = md < mi ? md : mi;
      if (d <= t * t && (bestc < 0 || d < bestd)) {
        bestd = d;
        bestc = c;
      }
    }
    labels[f] = bestc < 0 ? -1 : bid[bestc];
    dists[f] = bestc < 0 ? INFINITY : sqrt(bestd);
    if (best) best[f] = (int32_t)bestc;
  }
  return 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

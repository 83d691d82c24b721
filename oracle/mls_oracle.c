/*
 * mls_oracle.c -- plain, slow, FP64 CPU oracle for moving-least-squares (MLS)
 * field evaluation and marching-squares contour extraction.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent definition that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the GPU library never
 * does, and the two share no source, header, table or helper.
 *
 * What it computes (Muelder et al., "A Moving Least Squares Based Approach
 * for Contour Visualization of Multi-Dimensional Data", Sec. 3.3):
 *
 *   For every evaluation position p and data point i (position x_i, values
 *   f_i in R^D) take a radial weight w_i(p) and the polynomial basis
 *   b(u) = [1, u_x, u_y, u_x^2, u_x u_y, u_y^2] (truncated to m = 1, 3, 6
 *   terms for degree 0, 1, 2) with u = (x_i - p) / h, i.e. centred on p.
 *   The moving least-squares fit minimises sum_i w_i |b(u_i)^T c - f_i|^2;
 *   its normal equations are
 *       M c = R,   M = sum_i w_i b_i b_i^T,   R = sum_i w_i b_i f_i^T,
 *   and because the basis is centred on p the fitted value at p is the
 *   constant coefficient c_0.  Degree 1 is the affine MLS of Eq. 6-8 (the
 *   weighted-centroid form is the same minimiser), degree 0 is the weighted
 *   mean of Eq. 5.  Weights: the paper's inverse-distance power (Eq. 4),
 *   a Gaussian exp(-r^2/h^2), and the compactly supported Wendland C2
 *   function (1 - r/h)^4 (4 r/h + 1) for r < h.
 *
 * Readings where the paper is silent (each one is also listed in the design
 * notes):
 *   - Sums run sequentially in point-index order in FP64, no FMA contraction.
 *   - If sum_i w_i < weight_floor the value is undetermined: NaN, code 255.
 *   - Otherwise a degree ladder: for k' = k, k-1, ..., 0 take the leading
 *     m(k') x m(k') block M' (lower degrees are prefixes of the basis),
 *     equilibrate A = S M' S with S = diag(M'_jj^-1/2), run Cholesky on A
 *     and accept k' if every pivot (Schur-complement diagonal) is >= tau.
 *     Degree 0 always succeeds (A = [1]).  The smallest accepted pivot is
 *     reported as d_min.
 *   - Inverse-distance weight with a point exactly at p: the value is the
 *     mean of the coincident points' values (point identity, Sec. 3.3
 *     criterion 2), code 254.
 *   - Gradient output: the slope of the local fit, (c_1, c_2) / h.
 *
 * Rigid MLS (Eq. 9-10) maps a position to 2-vector values q_i by the
 * rotation-and-translation fit; see rigid_one for the formula and readings.
 *
 * Marching squares (Sec. 3.4 draws contour lines of the MLS output; the
 * extraction rule is this library's reading, the usual 16-case table):
 *   cell (i, j) has corners v0 = f[i][j], v1 = f[i][j+1], v2 = f[i+1][j+1],
 *   v3 = f[i+1][j]; bit k of the case is (v_k >= iso); any NaN corner gives
 *   case 255 and no segment.  Edge crossings interpolate from the edge
 *   endpoint with the smaller (row, col), so a shared edge gives the same
 *   point in both cells.  Segments are oriented with the >= iso region on
 *   their left.  Saddles (cases 5, 10) use the centre value
 *   ((v0 + v1) + (v2 + v3)) * 0.25: centre >= iso joins the above corners.
 *   The f32 variant rounds every arithmetic step of the case and crossing
 *   computation to binary32, for comparing against contours of FP32 fields.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_W_GAUSSIAN = 0, OR_W_WENDLAND_C2 = 1, OR_W_INVPOW = 2 };
enum { OR_DEG_NAN = 255, OR_DEG_HIT = 254 };
enum { OR_MAXM = 6 };

static int terms_for_degree(int degree) {
  return degree == 0 ? 1 : (degree == 1 ? 3 : 6);
}

/* Monomial basis centred on the evaluation point, in units of h. */
static void eval_basis(double ux, double uy, int m, double* b) {
  b[0] = 1.0;
  if (m >= 3) {
    b[1] = ux;
    b[2] = uy;
  }
  if (m >= 6) {
    b[3] = ux * ux;
    b[4] = ux * uy;
    b[5] = uy * uy;
  }
}

/* Radial weight of a point at squared distance rho2. */
static double eval_weight(int kind, double rho2, double h, double alpha) {
  if (kind == OR_W_GAUSSIAN) {
    return exp(-(rho2 / (h * h)));
  } else if (kind == OR_W_WENDLAND_C2) {
    double s = sqrt(rho2) / h;
    if (s >= 1.0) return 0.0;
    double t = 1.0 - s;
    return t * t * t * t * (4.0 * s + 1.0);
  } else {
    /* Eq. 4: 1 / |p_i - v|^(2 alpha), expressed in units of h. */
    return pow(rho2 / (h * h), -alpha);
  }
}

/*
 * Solve the normal equations of one position through the degree ladder.
 * M is m x m (row-major, full), R is m x D (row-major).  Writes D values
 * to out[d * out_stride], the accepted degree and the smallest accepted
 * equilibrated pivot.  If grad is not NULL it also receives the gradient of
 * the local fit at the position, (c_1, c_2) / h for each attribute (the
 * basis is centred on the position and scaled by h, so these are the
 * fitted slopes; zero when the ladder accepts the constant basis, NaN where
 * the value is NaN), at grad[(2 d + axis) * out_stride].
 */
static void ladder_solve(const double* M, const double* R, int m, int D,
                         double tau, double floor_w, double h, double* out,
                         int64_t out_stride, double* grad, uint8_t* deg_out,
                         double* dmin_out) {
  if (!(M[0] >= floor_w)) {
    if (grad)
      for (int d = 0; d < 2 * D; ++d) grad[(int64_t)d * out_stride] = NAN;
    for (int d = 0; d < D; ++d) out[(int64_t)d * out_stride] = NAN;
    *deg_out = OR_DEG_NAN;
    *dmin_out = 0.0;
    return;
  }
  int degree = (m == 6) ? 2 : (m == 3 ? 1 : 0);
  for (int k = degree; k >= 0; --k) {
    int mk = terms_for_degree(k);
    double s[OR_MAXM], A[OR_MAXM][OR_MAXM], L[OR_MAXM][OR_MAXM];
    int ok = 1;
    for (int j = 0; j < mk; ++j) {
      double mjj = M[j * m + j];
      if (!(mjj > 0.0)) { ok = 0; break; }
      s[j] = 1.0 / sqrt(mjj);
    }
    if (!ok) continue;
    for (int r = 0; r < mk; ++r)
      for (int c = 0; c < mk; ++c) A[r][c] = s[r] * M[r * m + c] * s[c];
    double pmin = INFINITY;
    for (int j = 0; j < mk && ok; ++j) {
      double piv = A[j][j];
      for (int q = 0; q < j; ++q) piv -= L[j][q] * L[j][q];
      if (!(piv >= tau)) { ok = 0; break; }
      if (piv < pmin) pmin = piv;
      L[j][j] = sqrt(piv);
      for (int r = j + 1; r < mk; ++r) {
        double v = A[r][j];
        for (int q = 0; q < j; ++q) v -= L[r][q] * L[j][q];
        L[r][j] = v / L[j][j];
      }
    }
    if (!ok) continue;
    /* A y = S R_d, then c = S y; the value at p is c_0. */
    for (int d = 0; d < D; ++d) {
      double z[OR_MAXM], y[OR_MAXM];
      for (int r = 0; r < mk; ++r) {
        double v = s[r] * R[r * D + d];
        for (int q = 0; q < r; ++q) v -= L[r][q] * z[q];
        z[r] = v / L[r][r];
      }
      for (int r = mk - 1; r >= 0; --r) {
        double v = z[r];
        for (int q = r + 1; q < mk; ++q) v -= L[q][r] * y[q];
        y[r] = v / L[r][r];
      }
      out[(int64_t)d * out_stride] = s[0] * y[0];
      if (grad) {
        grad[(int64_t)(2 * d) * out_stride] = mk >= 3 ? s[1] * y[1] / h : 0.0;
        grad[(int64_t)(2 * d + 1) * out_stride] = mk >= 3 ? s[2] * y[2] / h : 0.0;
      }
    }
    *deg_out = (uint8_t)k;
    *dmin_out = pmin;
    return;
  }
  /* Unreachable: degree 0 always passes once M_00 >= floor > 0. */
  if (grad)
    for (int d = 0; d < 2 * D; ++d) grad[(int64_t)d * out_stride] = NAN;
  for (int d = 0; d < D; ++d) out[(int64_t)d * out_stride] = NAN;
  *deg_out = OR_DEG_NAN;
  *dmin_out = 0.0;
}

/* The MLS value at one position (px, py). */
static void fit_one(const float* pts, const float* vals, int64_t n, int D,
                    int degree, int wkind, double h, double alpha, double px,
                    double py, double tau, double floor_w, double* out,
                    int64_t out_stride, double* grad, uint8_t* deg_out,
                    double* dmin_out, double* work /* m*D */) {
  int m = terms_for_degree(degree);
  double M[OR_MAXM * OR_MAXM];
  double* R = work;
  memset(M, 0, sizeof(M));
  memset(R, 0, sizeof(double) * (size_t)m * (size_t)D);
  if (wkind == OR_W_INVPOW) {
    /* Exact hit: the weight is infinite, the value is the point's own. */
    int64_t hits = 0;
    for (int64_t i = 0; i < n; ++i) {
      double dx = (double)pts[2 * i] - px, dy = (double)pts[2 * i + 1] - py;
      if (dx * dx + dy * dy == 0.0) {
        for (int d = 0; d < D; ++d) R[d] += (double)vals[i * D + d];
        ++hits;
      }
    }
    if (hits > 0) {
      /* the field jumps to the points' own value: no slope there */
      if (grad)
        for (int d = 0; d < 2 * D; ++d) grad[(int64_t)d * out_stride] = NAN;
      for (int d = 0; d < D; ++d) out[(int64_t)d * out_stride] = R[d] / (double)hits;
      *deg_out = OR_DEG_HIT;
      *dmin_out = 1.0;
      return;
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    double dx = (double)pts[2 * i] - px, dy = (double)pts[2 * i + 1] - py;
    double rho2 = dx * dx + dy * dy;
    double w = eval_weight(wkind, rho2, h, alpha);
    if (w == 0.0) continue;
    double b[OR_MAXM];
    eval_basis(dx / h, dy / h, m, b);
    for (int r = 0; r < m; ++r) {
      double wb = w * b[r];
      for (int c = r; c < m; ++c) M[r * m + c] += wb * b[c];
      for (int d = 0; d < D; ++d) R[r * D + d] += wb * (double)vals[i * D + d];
    }
  }
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < r; ++c) M[r * m + c] = M[c * m + r];
  ladder_solve(M, R, m, D, tau, floor_w, h, out, out_stride, grad, deg_out, dmin_out);
}

static int check_common(const float* pts, const float* vals, int64_t n, int D,
                        int degree, int wkind, double h) {
  if (!pts || !vals || n < 1 || D < 1) return -1;
  if (degree < 0 || degree > 2) return -1;
  if (wkind < 0 || wkind > 2) return -1;
  if (!(h > 0.0) || !isfinite(h)) return -1;
  return 0;
}

/*
 * MLS values at arbitrary positions pos[P][2].  Outputs: fields[D][P],
 * degree codes deg[P], smallest accepted pivot dmin[P], and, if grads is
 * not NULL, the gradients grads[D][2][P] (see ladder_solve).
 * Returns 0, or -1 on invalid arguments.
 */
int oracle_fit_at(const float* pts, const float* vals, int64_t n, int32_t D,
                  int32_t degree, int32_t wkind, double h, double alpha,
                  const double* pos, int64_t npos, double tau, double floor_w,
                  int32_t nthreads, double* fields, uint8_t* deg, double* dmin,
                  double* grads) {
  if (check_common(pts, vals, n, D, degree, wkind, h) || !pos || npos < 0 ||
      !fields || !deg || !dmin)
    return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  int m = terms_for_degree(degree);
#pragma omp parallel
  {
    double* work = (double*)malloc(sizeof(double) * (size_t)m * (size_t)D);
#pragma omp for schedule(static)
    for (int64_t k = 0; k < npos; ++k)
      fit_one(pts, vals, n, D, degree, wkind, h, alpha, pos[2 * k], pos[2 * k + 1],
              tau, floor_w, fields + k, npos, grads ? grads + k : NULL, deg + k,
              dmin + k, work);
    free(work);
  }
  return 0;
}

/*
 * MLS values at grid nodes.  Node (r, c) sits at (x0 + c*dx, y0 + r*dy);
 * pixels[] lists linear node indices r*W + c (NULL means all H*W nodes in
 * row-major order, npix = H*W).  Outputs fields[D][npix], deg[npix],
 * dmin[npix], and, if grads is not NULL, grads[D][2][npix].  Returns 0, or
 * -1 on invalid arguments.
 */
int oracle_fit_grid(const float* pts, const float* vals, int64_t n, int32_t D,
                    int32_t degree, int32_t wkind, double h, double alpha,
                    double x0, double y0, double dx, double dy, int32_t W,
                    int32_t H, const int64_t* pixels, int64_t npix, double tau,
                    double floor_w, int32_t nthreads, double* fields,
                    uint8_t* deg, double* dmin, double* grads) {
  if (check_common(pts, vals, n, D, degree, wkind, h) || W < 1 || H < 1 ||
      !fields || !deg || !dmin)
    return -1;
  if (!pixels && npix != (int64_t)W * H) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  int m = terms_for_degree(degree);
  int bad = 0;
#pragma omp parallel
  {
    double* work = (double*)malloc(sizeof(double) * (size_t)m * (size_t)D);
#pragma omp for schedule(static)
    for (int64_t k = 0; k < npix; ++k) {
      int64_t lin = pixels ? pixels[k] : k;
      if (lin < 0 || lin >= (int64_t)W * H) {
        bad = 1;
        continue;
      }
      int64_t r = lin / W, c = lin % W;
      double px = x0 + (double)c * dx, py = y0 + (double)r * dy;
      fit_one(pts, vals, n, D, degree, wkind, h, alpha, px, py, tau, floor_w,
              fields + k, npix, grads ? grads + k : NULL, deg + k, dmin + k, work);
    }
    free(work);
  }
  return bad ? -1 : 0;
}

/* ---------------------------------------------------------------------- */
/* Rigid MLS (Sec. 3.3, Eq. 9-10)                                          */
/* ---------------------------------------------------------------------- */

/* v^perp for a row vector v = (x, y). */
static void perp(const double v[2], double out[2]) {
  out[0] = -v[1];
  out[1] = v[0];
}

/*
 * Rigid MLS of 2-vector values q_i (vals[i][0..1]) at position v = (px, py),
 * in the paper's notation: p* and q* the weighted centroids (Eq. 7, 8),
 * dp_i = p_i - p*, dq_i = q_i - q*, dv = v - p*,
 *   f'(v) = sum_i w_i dq_i [dp_i ; -dp_i^perp] [dv ; -dv^perp]^T
 *   f(v)  = |dv| f'(v) / |f'(v)| + q*.
 * Readings: the index on dv in the printed Eq. 10 is a typo (dv does not
 * depend on i); v^perp = (-y, x); where |f'| = 0 (no rotation defined) or
 * dv = 0 the value is q*; sum w < floor gives NaN (code 255); an exact hit
 * of the inverse-distance weight gives the mean of the coincident q_i (code
 * 254); otherwise code 1.
 */
static void rigid_one(const float* pts, const float* vals, int64_t n, int wkind,
                      double h, double alpha, double px, double py, double floor_w,
                      double* out, int64_t out_stride, uint8_t* deg_out) {
  if (wkind == OR_W_INVPOW) {
    double s0 = 0.0, s1 = 0.0;
    int64_t hits = 0;
    for (int64_t i = 0; i < n; ++i) {
      double dx = (double)pts[2 * i] - px, dy = (double)pts[2 * i + 1] - py;
      if (dx * dx + dy * dy == 0.0) {
        s0 += (double)vals[2 * i];
        s1 += (double)vals[2 * i + 1];
        ++hits;
      }
    }
    if (hits > 0) {
      out[0] = s0 / (double)hits;
      out[out_stride] = s1 / (double)hits;
      *deg_out = OR_DEG_HIT;
      return;
    }
  }
  double sw = 0.0, sp[2] = {0.0, 0.0}, sq[2] = {0.0, 0.0};
  for (int64_t i = 0; i < n; ++i) {
    double dx = (double)pts[2 * i] - px, dy = (double)pts[2 * i + 1] - py;
    double w = eval_weight(wkind, dx * dx + dy * dy, h, alpha);
    sw += w;
    sp[0] += w * (double)pts[2 * i];
    sp[1] += w * (double)pts[2 * i + 1];
    sq[0] += w * (double)vals[2 * i];
    sq[1] += w * (double)vals[2 * i + 1];
  }
  if (!(sw >= floor_w)) {
    out[0] = NAN;
    out[out_stride] = NAN;
    *deg_out = OR_DEG_NAN;
    return;
  }
  const double ps[2] = {sp[0] / sw, sp[1] / sw}, qs[2] = {sq[0] / sw, sq[1] / sw};
  const double dv[2] = {px - ps[0], py - ps[1]};
  double dvp[2];
  perp(dv, dvp);
  /* B = [dv ; -dv^perp]^T (2 x 2, columns dv and -dv^perp) */
  const double B[2][2] = {{dv[0], -dvp[0]}, {dv[1], -dvp[1]}};
  double fr[2] = {0.0, 0.0};
  for (int64_t i = 0; i < n; ++i) {
    double dx = (double)pts[2 * i] - px, dy = (double)pts[2 * i + 1] - py;
    double w = eval_weight(wkind, dx * dx + dy * dy, h, alpha);
    if (w == 0.0) continue;
    const double dp[2] = {(double)pts[2 * i] - ps[0], (double)pts[2 * i + 1] - ps[1]};
    const double dq[2] = {(double)vals[2 * i] - qs[0], (double)vals[2 * i + 1] - qs[1]};
    double dpp[2];
    perp(dp, dpp);
    /* P = [dp ; -dp^perp] (rows dp and -dp^perp) */
    const double P[2][2] = {{dp[0], dp[1]}, {-dpp[0], -dpp[1]}};
    double A[2][2];
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) A[r][c] = P[r][0] * B[0][c] + P[r][1] * B[1][c];
    fr[0] += w * (dq[0] * A[0][0] + dq[1] * A[1][0]);
    fr[1] += w * (dq[0] * A[0][1] + dq[1] * A[1][1]);
  }
  const double nf = sqrt(fr[0] * fr[0] + fr[1] * fr[1]);
  const double nv = sqrt(dv[0] * dv[0] + dv[1] * dv[1]);
  if (nf > 0.0 && nv > 0.0) {
    out[0] = nv * fr[0] / nf + qs[0];
    out[out_stride] = nv * fr[1] / nf + qs[1];
  } else {
    out[0] = qs[0];
    out[out_stride] = qs[1];
  }
  *deg_out = 1;
}

/*
 * Rigid MLS at grid nodes (as oracle_fit_grid, D = 2 fixed): outputs
 * fields[2][npix] and deg[npix].  Returns 0, or -1 on invalid arguments.
 */
int oracle_rigid_grid(const float* pts, const float* vals, int64_t n, int32_t wkind,
                      double h, double alpha, double x0, double y0, double dx, double dy,
                      int32_t W, int32_t H, const int64_t* pixels, int64_t npix,
                      double floor_w, int32_t nthreads, double* fields, uint8_t* deg) {
  if (check_common(pts, vals, n, 2, 1, wkind, h) || W < 1 || H < 1 || !fields || !deg)
    return -1;
  if (!pixels && npix != (int64_t)W * H) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  int bad = 0;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < npix; ++k) {
    int64_t lin = pixels ? pixels[k] : k;
    if (lin < 0 || lin >= (int64_t)W * H) {
      bad = 1;
      continue;
    }
    int64_t r = lin / W, c = lin % W;
    const double px = x0 + dx * (double)c, py = y0 + dy * (double)r;
    rigid_one(pts, vals, n, wkind, h, alpha, px, py, floor_w, fields + k, npix, deg + k);
  }
  return bad ? -1 : 0;
}

/* ---------------------------------------------------------------------- */
/* Planarity-preserving force-directed layout (Sec. 3.2, Eq. 1-3)          */
/* ---------------------------------------------------------------------- */

/*
 * One node's move in one iteration, from the positions at the start of the
 * iteration (every node reads the same snapshot).  Forces, as printed:
 *   repulsion from every other node u:   C V / (|V|^3 + eta),  V = v - u
 *   spring along each mesh edge (v, u):  |V| log((|V| + eta) / D) (-V)
 *   node-edge repulsion for each triangle (v, a, b) around v:
 *                                        -C R / (|R|^2 + eta),
 *     R the vector from v to the line through a and b (to the foot of the
 *     perpendicular).
 * Readings: the summed force is the move, shortened to the temperature t if
 * it is longer; then the planarity constraint: each triangle (v, a, b) has
 * three limiting lines, each through the midpoints of two of its edges (so
 * parallel to the third edge and halfway between it and the opposite
 * vertex), and v may cross none of them.  For the line parallel to ab the
 * perpendicular from v is R / 2; for the line parallel to vb (resp. va),
 * v lies on that edge, and the perpendicular from v is half of a's (resp.
 * b's) offset from the line vb (resp. va).  The move's component along each
 * such R_i may not exceed |R_i| - eta; the whole move is scaled down to the
 * tightest bound (scaling keeps every half-plane constraint that already
 * holds, so all hold at once).  A triangle with a zero-length edge defines
 * no line and is skipped.
 */
static void layout_move(const double* x, int64_t n, int64_t v, const int32_t* adj_start,
                        const int32_t* adj, const int32_t* fan_start, const int32_t* fan,
                        double C, double D, double eta, double t, double* mv) {
  const double vx = x[2 * v], vy = x[2 * v + 1];
  double fx = 0.0, fy = 0.0;
  for (int64_t u = 0; u < n; ++u) {
    if (u == v) continue;
    const double ax = vx - x[2 * u], ay = vy - x[2 * u + 1];
    const double L = sqrt(ax * ax + ay * ay);
    const double s = C / (L * L * L + eta);
    fx += s * ax;
    fy += s * ay;
  }
  for (int32_t k = adj_start[v]; k < adj_start[v + 1]; ++k) {
    const int32_t u = adj[k];
    const double ax = vx - x[2 * u], ay = vy - x[2 * u + 1];
    const double L = sqrt(ax * ax + ay * ay);
    const double s = L * log((L + eta) / D);
    fx -= s * ax;
    fy -= s * ay;
  }
  for (int32_t k = fan_start[v]; k < fan_start[v + 1]; ++k) {
    const int32_t a = fan[2 * k], b = fan[2 * k + 1];
    const double ex = x[2 * b] - x[2 * a], ey = x[2 * b + 1] - x[2 * a + 1];
    const double e2 = ex * ex + ey * ey;
    if (!(e2 > 0.0)) continue;
    const double tt = ((vx - x[2 * a]) * ex + (vy - x[2 * a + 1]) * ey) / e2;
    const double rx = x[2 * a] + tt * ex - vx, ry = x[2 * a + 1] + tt * ey - vy;
    const double s = -C / (rx * rx + ry * ry + eta);
    fx += s * rx;
    fy += s * ry;
  }
  const double fl = sqrt(fx * fx + fy * fy);
  if (fl > t) {
    fx *= t / fl;
    fy *= t / fl;
  }
  double scale = 1.0;
  for (int32_t k = fan_start[v]; k < fan_start[v + 1]; ++k) {
    /* the triangle's vertices, v first; line i is parallel to the edge
       opposite corner i, halfway to corner i */
    const double P[3][2] = {{vx, vy},
                            {x[2 * fan[2 * k]], x[2 * fan[2 * k] + 1]},
                            {x[2 * fan[2 * k + 1]], x[2 * fan[2 * k + 1] + 1]}};
    for (int i = 0; i < 3; ++i) {
      const double* c = P[i];
      const double* e0 = P[(i + 1) % 3];
      const double* e1 = P[(i + 2) % 3];
      const double ex = e1[0] - e0[0], ey = e1[1] - e0[1];
      const double e2 = ex * ex + ey * ey;
      if (!(e2 > 0.0)) continue;
      /* offset of corner i from the opposite edge's line; the limiting
         line sits at half of it */
      const double tt = ((c[0] - e0[0]) * ex + (c[1] - e0[1]) * ey) / e2;
      const double ox = c[0] - (e0[0] + tt * ex), oy = c[1] - (e0[1] + tt * ey);
      /* perpendicular from v to the limiting line: from v's own line
         (i = 0: v is the corner, the line is half-way towards the edge;
         i > 0: v lies on the edge's line, the line is half-way towards the
         corner) */
      const double rx = i == 0 ? -0.5 * ox : 0.5 * ox, ry = i == 0 ? -0.5 * oy : 0.5 * oy;
      const double rl = sqrt(rx * rx + ry * ry);
      if (!(rl > 0.0)) {
        scale = 0.0;
        continue;
      }
      const double proj = (fx * rx + fy * ry) / rl;
      if (proj > 0.0) {
        const double room = rl - eta > 0.0 ? rl - eta : 0.0;
        if (proj * scale > room) scale = room / proj;
      }
    }
  }
  mv[0] = fx * scale;
  mv[1] = fy * scale;
}

/*
 * `iterations` layout iterations from pos_in[n][2] (float64), temperature
 * t_k = t0 lambda^k in iteration k.  Mesh: CSR neighbour lists
 * adj[adj_start[v] .. adj_start[v+1]) and triangle fans, the other two
 * vertices (a, b) of each triangle around v at fan[2 k], fan[2 k + 1] for
 * k in [fan_start[v], fan_start[v+1]).  Writes pos_out[n][2].
 * Returns 0, or -1 on invalid arguments.
 */
int oracle_layout(const double* pos_in, int64_t n, const int32_t* adj_start,
                  const int32_t* adj, const int32_t* fan_start, const int32_t* fan,
                  double C, double D, double eta, double t0, double lambda,
                  int32_t iterations, int32_t nthreads, double* pos_out) {
  if (!pos_in || !pos_out || n < 1 || !adj_start || !fan_start || iterations < 0 ||
      !(D > 0.0) || !(eta > 0.0) || !(t0 >= 0.0) || !(lambda > 0.0))
    return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  double* a = (double*)malloc(sizeof(double) * 2 * (size_t)n);
  double* b = (double*)malloc(sizeof(double) * 2 * (size_t)n);
  if (!a || !b) {
    free(a);
    free(b);
    return -1;
  }
  memcpy(a, pos_in, sizeof(double) * 2 * (size_t)n);
  double t = t0;
  for (int32_t it = 0; it < iterations; ++it) {
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < n; ++v) {
      double mv[2];
      layout_move(a, n, v, adj_start, adj, fan_start, fan, C, D, eta, t, mv);
      b[2 * v] = a[2 * v] + mv[0];
      b[2 * v + 1] = a[2 * v + 1] + mv[1];
    }
    double* tmp = a;
    a = b;
    b = tmp;
    t *= lambda;
  }
  memcpy(pos_out, a, sizeof(double) * 2 * (size_t)n);
  free(a);
  free(b);
  return 0;
}

/*
 * One layout iteration at temperature t for the listed nodes only:
 * pos_out[2 i], pos_out[2 i + 1] is node nodes[i] after the iteration, from
 * the positions pos_in[n][2] (the same move as oracle_layout's first
 * iteration, so large meshes can be checked on a sample of nodes).
 * Returns 0, or -1 on invalid arguments.
 */
int oracle_layout_step_nodes(const double* pos_in, int64_t n, const int32_t* adj_start,
                             const int32_t* adj, const int32_t* fan_start, const int32_t* fan,
                             double C, double D, double eta, double t, const int64_t* nodes,
                             int64_t m, int32_t nthreads, double* pos_out) {
  if (!pos_in || !pos_out || n < 1 || !adj_start || !fan_start || !nodes || m < 0 ||
      !(D > 0.0) || !(eta > 0.0) || !(t >= 0.0))
    return -1;
  for (int64_t i = 0; i < m; ++i)
    if (nodes[i] < 0 || nodes[i] >= n) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    const int64_t v = nodes[i];
    double mv[2];
    layout_move(pos_in, n, v, adj_start, adj, fan_start, fan, C, D, eta, t, mv);
    pos_out[2 * i] = pos_in[2 * v] + mv[0];
    pos_out[2 * i + 1] = pos_in[2 * v + 1] + mv[1];
  }
  return 0;
}

/* ---------------------------------------------------------------------- */
/* Marching squares                                                        */
/* ---------------------------------------------------------------------- */

/* Round to binary32 when emulating FP32 arithmetic, identity otherwise. */
static double rnd(double v, int f32) { return f32 ? (double)(float)v : v; }

/*
 * Edges: 0 bottom (v0-v1), 1 right (v1-v2), 2 top (v3-v2), 3 left (v0-v3).
 * The crossing on an edge, from its smaller-(row, col) endpoint a toward b.
 */
static void edge_point(int e, double v0, double v1, double v2, double v3,
                       double iso, int64_t i, int64_t j, double x0, double y0,
                       double dx, double dy, int f32, double* x, double* y) {
  double va, vb;
  switch (e) {
    case 0: va = v0; vb = v1; break;
    case 1: va = v1; vb = v2; break;
    case 2: va = v3; vb = v2; break;
    default: va = v0; vb = v3; break;
  }
  double t = rnd(rnd(iso - va, f32) / rnd(vb - va, f32), f32);
  switch (e) {
    case 0: *x = x0 + ((double)j + t) * dx; *y = y0 + (double)i * dy; break;
    case 1: *x = x0 + (double)(j + 1) * dx; *y = y0 + ((double)i + t) * dy; break;
    case 2: *x = x0 + ((double)j + t) * dx; *y = y0 + (double)(i + 1) * dy; break;
    default: *x = x0 + (double)j * dx; *y = y0 + ((double)i + t) * dy; break;
  }
}

/*
 * Segment list of a case as (from-edge, to-edge) pairs.  Walking the cell
 * boundary counter-clockwise (v0, e0, v1, e1, v2, e2, v3, e3), each run of
 * above corners is entered through one edge and left through another; the
 * segment runs from the leaving edge back to the entering edge, which puts
 * the above side on its left.
 */
static int case_segments(int cs, int joined, int seg[2][2]) {
  static const signed char single[16][2] = {
      {-1, -1}, {0, 3}, {1, 0}, {1, 3}, {2, 1}, {-1, -1}, {2, 0}, {2, 3},
      {3, 2},   {0, 2}, {-1, -1}, {1, 2}, {3, 1}, {0, 1}, {3, 0}, {-1, -1}};
  if (cs == 5) {
    if (joined) { seg[0][0] = 0; seg[0][1] = 1; seg[1][0] = 2; seg[1][1] = 3; }
    else        { seg[0][0] = 0; seg[0][1] = 3; seg[1][0] = 2; seg[1][1] = 1; }
    return 2;
  }
  if (cs == 10) {
    if (joined) { seg[0][0] = 3; seg[0][1] = 0; seg[1][0] = 1; seg[1][1] = 2; }
    else        { seg[0][0] = 1; seg[0][1] = 0; seg[1][0] = 3; seg[1][1] = 2; }
    return 2;
  }
  if (single[cs][0] < 0) return 0;
  seg[0][0] = single[cs][0];
  seg[0][1] = single[cs][1];
  return 1;
}

static int64_t contour_impl(const double* field, int32_t H, int32_t W, double x0,
                            double y0, double dx, double dy, const double* iso,
                            int32_t n_iso, int32_t field_index, uint8_t* cases,
                            double* segs, int32_t* ids, int64_t cap, int f32) {
  int64_t count = 0;
  int64_t cw = W - 1, ch = H - 1;
  for (int32_t k = 0; k < n_iso; ++k) {
    double lv = iso[k];
    for (int64_t i = 0; i < ch; ++i) {
      for (int64_t j = 0; j < cw; ++j) {
        double v0 = field[i * W + j], v1 = field[i * W + j + 1];
        double v2 = field[(i + 1) * W + j + 1], v3 = field[(i + 1) * W + j];
        int64_t cell = i * cw + j;
        int cs;
        if (isnan(v0) || isnan(v1) || isnan(v2) || isnan(v3)) {
          cs = 255;
        } else {
          cs = (v0 >= lv ? 1 : 0) | (v1 >= lv ? 2 : 0) | (v2 >= lv ? 4 : 0) |
               (v3 >= lv ? 8 : 0);
        }
        if (cases) cases[(int64_t)k * ch * cw + cell] = (uint8_t)cs;
        if (cs == 255) continue;
        int joined = 0;
        if (cs == 5 || cs == 10) {
          double c = rnd(rnd(rnd(v0 + v1, f32) + rnd(v2 + v3, f32), f32) * 0.25, f32);
          joined = (c >= lv);
        }
        int seg[2][2];
        int ns = case_segments(cs, joined, seg);
        for (int q = 0; q < ns; ++q) {
          if (count < cap && segs) {
            double* o = segs + 4 * count;
            edge_point(seg[q][0], v0, v1, v2, v3, lv, i, j, x0, y0, dx, dy, f32, &o[0], &o[1]);
            edge_point(seg[q][1], v0, v1, v2, v3, lv, i, j, x0, y0, dx, dy, f32, &o[2], &o[3]);
            if (ids) {
              ids[3 * count] = field_index;
              ids[3 * count + 1] = k;
              ids[3 * count + 2] = (int32_t)cell;
            }
          }
          ++count;
        }
      }
    }
  }
  return count;
}

/*
 * Contours of one H x W field at n_iso isovalues.  cases[n_iso][H-1][W-1]
 * (may be NULL); segments written in (iso, cell, k) order as
 * segs[q] = (x_from, y_from, x_to, y_to) and ids[q] = (field_index, iso, cell)
 * while q < cap.  Returns the total segment count (may exceed cap), or -1.
 */
int64_t oracle_contour_f64(const double* field, int32_t H, int32_t W, double x0,
                           double y0, double dx, double dy, const double* iso,
                           int32_t n_iso, int32_t field_index, uint8_t* cases,
                           double* segs, int32_t* ids, int64_t cap) {
  if (!field || H < 2 || W < 2 || n_iso < 0 || (n_iso > 0 && !iso)) return -1;
  return contour_impl(field, H, W, x0, y0, dx, dy, iso, n_iso, field_index, cases,
                      segs, ids, cap, 0);
}

/* Same as oracle_contour_f64 on binary32 values with binary32 arithmetic. */
int64_t oracle_contour_f32(const float* field, int32_t H, int32_t W, double x0,
                           double y0, double dx, double dy, const float* iso,
                           int32_t n_iso, int32_t field_index, uint8_t* cases,
                           double* segs, int32_t* ids, int64_t cap) {
  if (!field || H < 2 || W < 2 || n_iso < 0 || (n_iso > 0 && !iso)) return -1;
  int64_t nn = (int64_t)H * W;
  double* f = (double*)malloc(sizeof(double) * (size_t)nn);
  double* lv = (double*)malloc(sizeof(double) * (size_t)(n_iso > 0 ? n_iso : 1));
  if (!f || !lv) { free(f); free(lv); return -1; }
  for (int64_t q = 0; q < nn; ++q) f[q] = (double)field[q];
  for (int32_t k = 0; k < n_iso; ++k) lv[k] = (double)iso[k];
  int64_t r = contour_impl(f, H, W, x0, y0, dx, dy, lv, n_iso, field_index, cases,
                           segs, ids, cap, 1);
  free(f);
  free(lv);
  return r;
}

/* ---------------------------------------------------------------------- */
/* Space mappings of the fields (Sec. 3.4, Fig. 5b-d)                      */
/* ---------------------------------------------------------------------- */

/*
 * Discrete colours (Fig. 5b): each region between isovalues takes one
 * colour, so a node's colour is decided by its band, the number of
 * isovalues at or below its value (the same "at or above counts as above"
 * tie rule as the contour cases).  NaN values get band 255.  The isovalues
 * need not be sorted.  fields[D][P], iso[D][n_iso], bands[D][P].
 */
int oracle_map_bands(const float* fields, int32_t D, int64_t P, const float* iso,
                     int32_t n_iso, uint8_t* bands) {
  if (!fields || !bands || D < 1 || P < 0 || n_iso < 1 || n_iso > 254 || !iso) return -1;
  for (int32_t d = 0; d < D; ++d) {
    for (int64_t q = 0; q < P; ++q) {
      float v = fields[(int64_t)d * P + q];
      if (isnan(v)) {
        bands[(int64_t)d * P + q] = 255;
        continue;
      }
      int b = 0;
      for (int32_t k = 0; k < n_iso; ++k)
        if (v >= iso[(int64_t)d * n_iso + k]) ++b;
      bands[(int64_t)d * P + q] = (uint8_t)b;
    }
  }
  return 0;
}

/*
 * Adaptive contour lines (Fig. 5d): the gradient of the field sets the
 * local spacing of the lines on screen, finer lines fade in where that
 * spacing is wide (space expanded) and out where it is narrow (space
 * compressed).  Reading (the paper gives no formula):
 *   - level j = 0 .. n_levels-1 has lines at origin + k spacing / 2^j;
 *   - at a node with value f and gradient g = (g_x, g_y) the field changes
 *     by r = |(g_x dx, g_y dy)| per pixel along its steepest pixel
 *     direction (the gradient in pixel coordinates), and level j's lines
 *     are s_j = (spacing / 2^j) / r pixels apart;
 *   - level 0 is always drawn; level j >= 1 with opacity
 *     a_j = clamp((s_j - fade_lo) / (fade_hi - fade_lo), 0, 1);
 *   - the distance in pixels to the nearest level-j line is
 *     e_j = |t - round(t)| s_j with t = (f - origin) / (spacing / 2^j);
 *   - the line intensity is max_j a_j max(0, 1 - e_j / halfwidth), in
 *     [0, 1]; NaN where f is NaN, 0 where r is 0 or not finite.
 * fields[D][P], grads[D][2][P] (d/dx, d/dy), levels[D][2] (origin,
 * spacing), out[D][P].
 */
int oracle_map_adaptive(const float* fields, const float* grads, int32_t D, int64_t P,
                        const float* levels, double dx, double dy, int32_t n_levels,
                        double halfwidth, double fade_lo, double fade_hi, double* out) {
  if (!fields || !grads || !levels || !out || D < 1 || P < 0 || n_levels < 1 ||
      n_levels > 30 || !(halfwidth > 0.0) || !(fade_hi > fade_lo))
    return -1;
  for (int32_t d = 0; d < D; ++d) {
    double origin = (double)levels[2 * d], spacing = (double)levels[2 * d + 1];
    for (int64_t q = 0; q < P; ++q) {
      double f = (double)fields[(int64_t)d * P + q];
      double gx = (double)grads[((int64_t)2 * d) * P + q];
      double gy = (double)grads[((int64_t)2 * d + 1) * P + q];
      double* o = out + (int64_t)d * P + q;
      if (isnan(f)) {
        *o = NAN;
        continue;
      }
      double px = gx * dx, py = gy * dy;
      double per_px = sqrt(px * px + py * py);
      if (!(per_px > 0.0) || !isfinite(per_px) || !(spacing > 0.0)) {
        *o = 0.0;
        continue;
      }
      double best = 0.0;
      for (int32_t j = 0; j < n_levels; ++j) {
        double step = spacing / ldexp(1.0, j);
        double s = step / per_px;
        double a = 1.0;
        if (j > 0) {
          a = (s - fade_lo) / (fade_hi - fade_lo);
          if (a < 0.0) a = 0.0;
          if (a > 1.0) a = 1.0;
        }
        double t = (f - origin) / step;
        double e = fabs(t - round(t)) * s;
        double line = 1.0 - e / halfwidth;
        if (line < 0.0) line = 0.0;
        if (a * line > best) best = a * line;
      }
      *o = best;
    }
  }
  return 0;
}

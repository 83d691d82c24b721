// Per-node float64 solve of the MLS normal equations (Muelder et al.,
// Sec. 3.3, Eq. 6-8 generalised to polynomial bases).
//
// The contraction kernels accumulate, per node, the weighted moments of the
// basis in a tile frame: u = (x_i - c_T) / h with c_T the tile anchor, i.e.
//   g[mono(a, b)]           = sum_i w_i u_x^a u_y^b      (a + b <= 2 deg)
//   g[nmom + j * D + d]     = sum_i w_i b_j(u_i) f_{i,d}  (j < m)
// The node's own frame is u_p = u - delta with delta = (p - c_T) / h.  A
// shift of a complete polynomial space is an invertible linear map T with
// b(u_p) = T b(u), so the node-frame normal matrix is M_p = T M_t T^T and
// its right-hand sides R_p = T R_t.  The degree ladder (equilibrated
// Cholesky, every pivot >= tau, else drop a degree) runs on M_p exactly as
// the definition states, and the value at the node is
//   field_d = e_0^T M_p'^{-1} R_p' = y^T R_t,  y = T'^T z,  z = M_p'^{-1} e_0
// so one factorisation and D dot products of length m give all D fields.
// The slope of the local fit at the node is (c_1, c_2) / h with
// c_j = e_j^T M_p'^{-1} R_p' = y_j^T R_t, y_j = T'^T M_p'^{-1} e_j: two more
// triangular solves with the same factor (only when gradients are asked for).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mls {

// Index of the monomial u_x^a u_y^b in the moment vector (ordered by total
// degree t = a + b, then by the power of u_y).
__device__ __forceinline__ constexpr int mono_index(int a, int b) {
  return (a + b) * (a + b + 1) / 2 + b;
}

// Exponents (a, b) of the basis terms [1, ux, uy, ux^2, ux uy, uy^2].
__device__ __forceinline__ constexpr int basis_ax(int j) {
  return j == 1 ? 1 : (j == 3 ? 2 : (j == 4 ? 1 : 0));
}
__device__ __forceinline__ constexpr int basis_ay(int j) {
  return j == 2 ? 1 : (j == 5 ? 2 : (j == 4 ? 1 : 0));
}

// Row r of the shift map T (b(u - delta) = T b(u)), entry c.
__device__ __forceinline__ double shift_entry(int r, int c, double ex, double ey) {
  switch (r) {
    case 0: return c == 0 ? 1.0 : 0.0;
    case 1: return c == 0 ? -ex : (c == 1 ? 1.0 : 0.0);
    case 2: return c == 0 ? -ey : (c == 2 ? 1.0 : 0.0);
    case 3: return c == 0 ? ex * ex : (c == 1 ? -2.0 * ex : (c == 3 ? 1.0 : 0.0));
    case 4: return c == 0 ? ex * ey : (c == 1 ? -ey : (c == 2 ? -ex : (c == 4 ? 1.0 : 0.0)));
    default: return c == 0 ? ey * ey : (c == 2 ? -2.0 * ey : (c == 5 ? 1.0 : 0.0));
  }
}

// The degree ladder at one node: the tile-frame moments g[0 .. nmom) are
// shifted to the node (M_p = T M_t T^T), then for k' = DEG, DEG-1, .. 0 the
// equilibrated matrix S M_p' S is factored (L, every pivot >= tau) until a
// degree is accepted.  Fills the factor and y = T'^T M_p'^{-1} e_0, the
// tile-frame coefficients of the node's shape function: the fitted value
// is y^T R_t.  The reciprocal of each diagonal entry of L is kept (r), so
// the triangular solves multiply instead of dividing.  Returns the accepted degree, or 255 when the weight sum
// (divided by wscale) is below the floor or no degree is accepted.
template <int DEG>
struct Ladder {
  static constexpr int m = DEG == 0 ? 1 : (DEG == 1 ? 3 : 6);
  double T[m][m], L[m][m], r[m], s[m], q[m], w[m], y[m];
  int mk;
};

template <int DEG, typename Acc>
__device__ __forceinline__ int ladder_solve(const Acc* g, double ex, double ey, double tau,
                                            double floor_w, double wscale, Ladder<DEG>& lad) {
  constexpr int m = Ladder<DEG>::m;
  const double sumw = (double)g[0] / wscale;
  if (!(sumw >= floor_w)) return 255;
  double Mt[m][m];
#pragma unroll
  for (int j = 0; j < m; ++j)
#pragma unroll
    for (int k = 0; k < m; ++k)
      Mt[j][k] = (double)g[mono_index(basis_ax(j) + basis_ax(k), basis_ay(j) + basis_ay(k))];
#pragma unroll
  for (int r = 0; r < m; ++r)
#pragma unroll
    for (int c = 0; c < m; ++c) lad.T[r][c] = shift_entry(r, c, ex, ey);
  // Mp = T Mt T^T (lower triangle is all the ladder reads)
  double TM[m][m];
#pragma unroll
  for (int r = 0; r < m; ++r)
#pragma unroll
    for (int c = 0; c < m; ++c) {
      double v = 0.0;
#pragma unroll
      for (int q = 0; q <= r; ++q) v += lad.T[r][q] * Mt[q][c];
      TM[r][c] = v;
    }
  double Mp[m][m];
#pragma unroll
  for (int r = 0; r < m; ++r)
#pragma unroll
    for (int c = 0; c <= r; ++c) {
      double v = 0.0;
#pragma unroll
      for (int q = 0; q <= c; ++q) v += TM[r][q] * lad.T[c][q];
      Mp[r][c] = v;
    }
#pragma unroll
  for (int kd = DEG; kd >= 0; --kd) {
    const int mk = kd == 0 ? 1 : (kd == 1 ? 3 : 6);
    bool ok = true;
#pragma unroll
    for (int j = 0; j < m; ++j) {
      if (j < mk) {
        ok = ok && (Mp[j][j] > 0.0);
        lad.s[j] = ok ? 1.0 / sqrt(Mp[j][j]) : 0.0;
      }
    }
    if (!ok) continue;
#pragma unroll
    for (int j = 0; j < m; ++j) {
      if (j >= mk || !ok) continue;
      double piv = lad.s[j] * Mp[j][j] * lad.s[j];
#pragma unroll
      for (int q = 0; q < j; ++q) piv -= lad.L[j][q] * lad.L[j][q];
      if (!(piv >= tau)) {
        ok = false;
        continue;
      }
      lad.L[j][j] = sqrt(piv);
      const double inv = 1.0 / lad.L[j][j];
      lad.r[j] = inv;
#pragma unroll
      for (int r = j + 1; r < m; ++r) {
        if (r >= mk) continue;
        double v = lad.s[r] * Mp[r][j] * lad.s[j];
#pragma unroll
        for (int q = 0; q < j; ++q) v -= lad.L[r][q] * lad.L[j][q];
        lad.L[r][j] = v * inv;
      }
    }
    if (!ok) continue;
    // z = S A^{-1} S e0:  L q = s0 e0,  L^T w = q,  z = S w
#pragma unroll
    for (int r = 0; r < m; ++r) {
      if (r >= mk) continue;
      double v = r == 0 ? lad.s[0] : 0.0;
#pragma unroll
      for (int c = 0; c < r; ++c) v -= lad.L[r][c] * lad.q[c];
      lad.q[r] = v * lad.r[r];
    }
#pragma unroll
    for (int r = m - 1; r >= 0; --r) {
      if (r >= mk) continue;
      double v = lad.q[r];
#pragma unroll
      for (int c = r + 1; c < m; ++c)
        if (c < mk) v -= lad.L[c][r] * lad.w[c];
      lad.w[r] = v * lad.r[r];
    }
    // y = T'^T z over the accepted rows
#pragma unroll
    for (int c = 0; c < m; ++c) {
      double v = 0.0;
#pragma unroll
      for (int r = 0; r < m; ++r)
        if (r < mk) v += lad.T[r][c] * (lad.s[r] * lad.w[r]);
      lad.y[c] = v;
    }
    lad.mk = mk;
    return kd;
  }
  return 255;   // only when sum w == 0 passes a zero floor
}

// Solve one node.  `g` points at the node's F accumulated features
// (consecutive values, float64 or float32), `ex, ey` is delta.  Writes
// field_d to fields[d * plane] (float32) and returns the accepted degree
// code.  If `shift` is given, the attributes were fitted as
// (f_d - shift[d]) / scale[d] and the value is mapped back.  `wscale`
// divides the weight sum before the floor test (weights that were scaled
// by a common factor).  If `grads` is given, the slopes d f_d / dx and
// d f_d / dy go to grads[(2 d) * plane] and grads[(2 d + 1) * plane]
// (zero when the constant basis is accepted, NaN where the field is).
template <int DEG, typename Acc>
__device__ __forceinline__ uint8_t solve_node(const Acc* g, int D, double ex, double ey,
                              double tau, double floor_w, float* fields,
                              int64_t plane, const float* shift = nullptr,
                              const float* scale = nullptr, double wscale = 1.0,
                              float* grads = nullptr, double inv_h = 1.0) {
  constexpr int m = Ladder<DEG>::m;
  constexpr int nmom = DEG == 0 ? 1 : (DEG == 1 ? 6 : 15);
  Ladder<DEG> lad;
  const int accepted = ladder_solve<DEG>(g, ex, ey, tau, floor_w, wscale, lad);
  if (accepted == 255) {
    for (int d = 0; d < D; ++d) fields[(int64_t)d * plane] = __builtin_nan("");
    if (grads)
      for (int d = 0; d < 2 * D; ++d) grads[(int64_t)d * plane] = __builtin_nan("");
    return 255;
  }
  const int mk = lad.mk;
  if (grads) {
    // slopes: the same two triangular solves with S e_1 and S e_2
    const Acc* Rg = g + nmom;
#pragma unroll 1
    for (int a = 1; a <= 2; ++a) {
      double ya[m];
#pragma unroll
      for (int c = 0; c < m; ++c) ya[c] = 0.0;
      if (mk >= 3) {
#pragma unroll
        for (int r = 0; r < m; ++r) {
          if (r >= mk) continue;
          double v = r == a ? lad.s[r] : 0.0;
#pragma unroll
          for (int c = 0; c < r; ++c) v -= lad.L[r][c] * lad.q[c];
          lad.q[r] = v * lad.r[r];
        }
#pragma unroll
        for (int r = m - 1; r >= 0; --r) {
          if (r >= mk) continue;
          double v = lad.q[r];
#pragma unroll
          for (int c = r + 1; c < m; ++c)
            if (c < mk) v -= lad.L[c][r] * lad.w[c];
          lad.w[r] = v * lad.r[r];
        }
#pragma unroll
        for (int c = 0; c < m; ++c) {
          double v = 0.0;
#pragma unroll
          for (int r = 0; r < m; ++r)
            if (r < mk) v += lad.T[r][c] * (lad.s[r] * lad.w[r]);
          ya[c] = v;
        }
      }
      for (int d = 0; d < D; ++d) {
        double v = 0.0;
#pragma unroll
        for (int c = 0; c < m; ++c) v += ya[c] * (double)Rg[c * D + d];
        if (scale) v *= (double)scale[d];
        grads[(int64_t)(2 * d + a - 1) * plane] = (float)(v * inv_h);
      }
    }
  }
  const Acc* R = g + nmom;
  for (int d = 0; d < D; ++d) {
    double v = 0.0;
#pragma unroll
    for (int c = 0; c < m; ++c) v += lad.y[c] * (double)R[c * D + d];
    if (shift) v = (double)shift[d] + (double)scale[d] * v;
    fields[(int64_t)d * plane] = (float)v;
  }
  return (uint8_t)accepted;
}

// Rigid MLS (Eq. 9-10) of 2-vector values at one node, from the linear-basis
// moments of the tile frame (g[0..5], then R[c * 2 + d] for c = 1, u_x, u_y).
// With dp_i, dq_i the offsets from the weighted centroids p*, q* and
// dv = v - p*, each term dq_i [dp_i; -dp_i^perp][dv; -dv^perp]^T of the
// printed sum is (dq_i . dp_i) dv rotated by a quarter turn's share of
// (dq_i x dp_i), so
//   f'(v) = (dv_x mu + dv_y nu, -dv_x nu + dv_y mu),
//   mu = sum w dq . dp,   nu = sum w (dq_x dp_y - dq_y dp_x),
// and f = |dv| f' / |f'| + q* = (dv_x mu + dv_y nu, -dv_x nu + dv_y mu) / rho
// + q*, rho = sqrt(mu^2 + nu^2).  These sums are the first moments and the
// basis x value moments shifted to the node (u_p = u - delta), scaled by h.
// Where rho = 0 or dv = 0 the value is q*.  Returns the degree code (1, or
// 255 below the weight floor).
template <typename Acc>
__device__ __forceinline__ uint8_t rigid_node(const Acc* g, double ex, double ey, double h,
                                              double floor_w, float* fields, int64_t plane) {
  const double w0 = (double)g[0];
  if (!(w0 >= floor_w)) {
    fields[0] = __builtin_nanf("");
    fields[plane] = __builtin_nanf("");
    return 255;
  }
  const Acc* R = g + 6;
  const double sx = (double)g[1] - ex * w0, sy = (double)g[2] - ey * w0;
  const double q0 = (double)R[0], q1 = (double)R[1];
  const double sxq0 = (double)R[2] - ex * q0, sxq1 = (double)R[3] - ex * q1;
  const double syq0 = (double)R[4] - ey * q0, syq1 = (double)R[5] - ey * q1;
  const double P0 = h * sx / w0, P1 = h * sy / w0;   // p* - v
  const double Q0 = q0 / w0, Q1 = q1 / w0;           // q*
  // c_ad = sum w dp_a dq_d
  const double c00 = h * sxq0 - w0 * P0 * Q0, c01 = h * sxq1 - w0 * P0 * Q1;
  const double c10 = h * syq0 - w0 * P1 * Q0, c11 = h * syq1 - w0 * P1 * Q1;
  const double mu = c00 + c11, nu = c10 - c01;
  const double d0 = -P0, d1 = -P1;                   // v - p*
  const double rho = sqrt(mu * mu + nu * nu);
  double f0 = Q0, f1 = Q1;
  if (rho > 0.0 && (d0 != 0.0 || d1 != 0.0)) {
    f0 += (d0 * mu + d1 * nu) / rho;
    f1 += (-d0 * nu + d1 * mu) / rho;
  }
  fields[0] = (float)f0;
  fields[plane] = (float)f1;
  return 1;
}

}  // namespace mls

// Planarity-preserving force-directed layout of a triangulated point set
// (Muelder et al., Sec. 3.2, Eq. 1-3): every iteration moves each node by
// the sum of
//   - inverse-square repulsion from every other node, C V / (|V|^3 + eta);
//   - a logarithmic spring along each mesh edge, |V| log((|V| + eta) / D) (-V);
//   - node-edge repulsion from the opposite edge of each incident triangle,
//     -C R / (|R|^2 + eta), R the perpendicular from the node to that edge;
// shortened to the iteration's temperature t_k = t0 lambda^k, then scaled
// down so that the node crosses none of the three limiting lines of any of
// its triangles (each through the midpoints of two edges, i.e. halfway
// between an edge and the opposite corner), keeping eta clear of them.  The
// section proves that no triangle can then flip even though all nodes move
// at once, which is what lets every node move in parallel.
//
// Parallel form: nodes read the positions at the start of the iteration
// (ping-pong buffers, float64).  A workgroup of 256 lanes owns NB nodes and
// gives each SP = 256 / NB adjacent lanes of one wave; the lanes of a node
// split its all-pairs repulsion by source and its spring and node-edge terms
// by list entry, then add their partial forces with an xor butterfly (every
// lane ends with the same bits, and the order does not depend on
// scheduling).  NB falls as n falls so that the paper's sizes (a few
// thousand nodes) still fill the chip.  Sources are staged into LDS in
// tiles, the next tile's loads in flight while the current one is used; the
// list ranges, each lane's first spring and triangle and the first tile are
// all requested before any of them is waited on.  The same lanes then share the node's triangles
// for the limiting-line test and take the minimum of their step scales.
// The exact all-pairs sum replaces the paper's kd-tree far field: at the
// sizes the paper lays out it costs microseconds.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mls_internal.h"

namespace mls {
namespace {

constexpr int kLanes = 256;     // lanes per workgroup

struct LayoutParams {
  const double* x;              // [n][2] positions at the start of the iteration
  double* y;                    // [n][2] positions after it
  int64_t n;
  const int32_t* adj_start;
  const int32_t* adj;
  int64_t n_adj;                // entries of adj
  const int32_t* fan_start;
  const int32_t* fan;
  int64_t n_fan;                // triangles in fan (pairs)
  double C, D, eta, t;
};

// Entries [start[v], start[v+1]) of a CSR list, clipped to [0, total): the
// lists come from the caller, and a malformed one must not read past them.
__device__ __forceinline__ void csr_range(const int32_t* start, int64_t v, int64_t total,
                                          int64_t* k0, int64_t* k1) {
  int64_t a = start[v], b = start[v + 1];
  a = a < 0 ? 0 : (a > total ? total : a);
  b = b < a ? a : (b > total ? total : b);
  *k0 = a;
  *k1 = b;
}

__device__ __forceinline__ double2 load_pos(const double* x, int64_t u) {
  return *reinterpret_cast<const double2*>(x + 2 * u);
}

// Spring of Eq. 2 on v from the neighbour at (ux, uy), added to (fx, fy).
__device__ __forceinline__ void add_spring(double vx, double vy, double ux, double uy,
                                           double D, double eta, double& fx, double& fy) {
#pragma clang fp contract(off)
  const double ax = vx - ux, ay = vy - uy;
  const double L = sqrt(ax * ax + ay * ay);
  const double q = L * log((L + eta) / D);
  fx -= q * ax;
  fy -= q * ay;
}

// Node-edge repulsion of Eq. 3 on v from the edge (a, b), added to (fx, fy).
__device__ __forceinline__ void add_edge(double vx, double vy, double ax0, double ay0,
                                         double bx, double by, double C, double eta, double& fx,
                                         double& fy) {
#pragma clang fp contract(off)
  const double ex = bx - ax0, ey = by - ay0;
  const double e2 = ex * ex + ey * ey;
  if (!(e2 > 0.0)) return;
  const double tt = ((vx - ax0) * ex + (vy - ay0) * ey) / e2;
  const double rx = ax0 + tt * ex - vx, ry = ay0 + tt * ey - vy;
  const double q = -C / (rx * rx + ry * ry + eta);
  fx += q * rx;
  fy += q * ry;
}

// Largest fraction of the move (fx, fy) that keeps node v (corner 0 of the
// triangle v, a, b) eta clear of the triangle's three limiting lines.
// Corner i's line lies halfway between corner i and the opposite edge; the
// offset from v to it is half of -(v's offset from its opposite edge) for
// i = 0 and half of corner i's offset from the edge through v for i = 1, 2.
__device__ __forceinline__ double triangle_scale(double vx, double vy, double ax, double ay,
                                                 double bx, double by, double fx, double fy,
                                                 double eta) {
#pragma clang fp contract(off)
  const double P[3][2] = {{vx, vy}, {ax, ay}, {bx, by}};
  double scale = 1.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double* c = P[i];
    const double* e0 = P[(i + 1) % 3];
    const double* e1 = P[(i + 2) % 3];
    const double ex = e1[0] - e0[0], ey = e1[1] - e0[1];
    const double e2 = ex * ex + ey * ey;
    if (!(e2 > 0.0)) continue;
    const double tt = ((c[0] - e0[0]) * ex + (c[1] - e0[1]) * ey) / e2;
    const double ox = c[0] - (e0[0] + tt * ex), oy = c[1] - (e0[1] + tt * ey);
    const double rx = i == 0 ? -0.5 * ox : 0.5 * ox, ry = i == 0 ? -0.5 * oy : 0.5 * oy;
    const double rl = sqrt(rx * rx + ry * ry);
    if (!(rl > 0.0)) {
      scale = 0.0;
      continue;
    }
    const double proj = (fx * rx + fy * ry) / rl;
    if (proj > 0.0) {
      const double room = rl - eta > 0.0 ? rl - eta : 0.0;
      const double lim = room / proj;
      scale = lim < scale ? lim : scale;
    }
  }
  return scale;
}

// C / (|V|^3 + eta) for |V|^2 = r2, the factor of V in the repulsion of
// Eq. 1.  |V| comes from the hardware reciprocal square root and the
// quotient from the hardware reciprocal (each an estimate good to about 23
// bits), refined by one Newton step each (about 46 bits) and a final
// residual step on the quotient: within about 1e-14 of the correctly
// rounded value, in about half the instructions of the IEEE square root and
// division, and without a branch.  V = 0 (the node itself, or a coincident
// node) takes |V| = 1 so that the factor stays finite and its product with
// V is exactly zero.
__device__ __forceinline__ double repulsion_factor(double r2, double C, double eta) {
  const double a = r2 > 0.0 ? r2 : 1.0;
  double y = __builtin_amdgcn_rsq(a);
  y = fma(y, fma(-(a * y), 0.5 * y, 0.5), y);      // y <- y (3 - a y^2) / 2
  const double L = a * y;
  const double den = a * L + eta;
  double r = __builtin_amdgcn_rcp(den);
  r = fma(r, fma(-den, r, 1.0), r);                // r <- r (2 - den r)
  const double q = C * r;
  return fma(fma(-den, q, C), r, q);
}

template <int SP>
__device__ __forceinline__ double group_sum(double a) {
#pragma unroll
  for (int w = 1; w < SP; w *= 2) a = a + __shfl_xor(a, w, SP);
  return a;
}

template <int SP>
__device__ __forceinline__ double group_min(double a) {
#pragma unroll
  for (int w = 1; w < SP; w *= 2) {
    const double o = __shfl_xor(a, w, SP);
    a = o < a ? o : a;
  }
  return a;
}

// NB nodes per workgroup; TILE sources staged into LDS per round.
template <int NB, int TILE>
__global__ __launch_bounds__(kLanes) void layout_step_kernel(LayoutParams p) {
#pragma clang fp contract(off)
  constexpr int SP = kLanes / NB;         // lanes per node, within one wave
  constexpr int PER = TILE / kLanes;      // sources each lane stages per round
  static_assert(SP <= 64 && TILE % kLanes == 0, "node groups must sit inside a wave");
  __shared__ double2 src[TILE];
  const int t = threadIdx.x;
  const int j = t / SP, s = t % SP;       // node slot, lane within the node
  const int64_t v = (int64_t)blockIdx.x * NB + j;
  const bool live = v < p.n;
  // requests that depend on nothing: the node, its list ranges, tile 0
  const double2 pv = live ? load_pos(p.x, v) : make_double2(0.0, 0.0);
  const double vx = pv.x, vy = pv.y;
  int64_t k0 = 0, k1 = 0, f0 = 0, f1 = 0;
  if (live) {
    csr_range(p.adj_start, v, p.n_adj, &k0, &k1);
    csr_range(p.fan_start, v, p.n_fan, &f0, &f1);
  }
  double2 st[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int64_t u = t + (int64_t)i * kLanes;
    st[i] = u < p.n ? load_pos(p.x, u) : make_double2(0.0, 0.0);
  }
  // each lane's first spring and triangle (their latency overlaps the
  // repulsion below)
  bool has_u = false, has_ab = false;
  double2 pu = make_double2(0.0, 0.0), pa = pu, pb = pu;
  if (k0 + s < k1) {
    const int32_t u = p.adj[k0 + s];
    if (u >= 0 && u < p.n) {
      has_u = true;
      pu = load_pos(p.x, u);
    }
  }
  if (f0 + s < f1) {
    const int32_t a = p.fan[2 * (f0 + s)], b = p.fan[2 * (f0 + s) + 1];
    if (a >= 0 && a < p.n && b >= 0 && b < p.n) {
      has_ab = true;
      pa = load_pos(p.x, a);
      pb = load_pos(p.x, b);
    }
  }
  // repulsion (Eq. 1) from the sources base + e, e = s, s + SP, ...; the
  // node itself adds exactly zero, so it needs no test
  double fx = 0.0, fy = 0.0;
  for (int64_t base = 0; base < p.n; base += TILE) {
    __syncthreads();                       // the previous round is done with src
#pragma unroll
    for (int i = 0; i < PER; ++i) src[t + i * kLanes] = st[i];
    __syncthreads();
    const int64_t next = base + TILE;
    if (next < p.n) {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int64_t u = next + t + (int64_t)i * kLanes;
        st[i] = u < p.n ? load_pos(p.x, u) : make_double2(0.0, 0.0);
      }
    }
    const int cnt = (int)((p.n - base) < TILE ? (p.n - base) : TILE);
#pragma unroll 4
    for (int e = s; e < cnt; e += SP) {
      const double2 q2 = src[e];
      const double ax = vx - q2.x, ay = vy - q2.y;
      const double q = repulsion_factor(ax * ax + ay * ay, p.C, p.eta);
      fx += q * ax;
      fy += q * ay;
    }
  }
  // springs (Eq. 2) and node-edge repulsion (Eq. 3)
  if (has_u) add_spring(vx, vy, pu.x, pu.y, p.D, p.eta, fx, fy);
  for (int64_t k = k0 + s + SP; k < k1; k += SP) {
    const int32_t u = p.adj[k];
    if (u < 0 || u >= p.n) continue;
    const double2 q2 = load_pos(p.x, u);
    add_spring(vx, vy, q2.x, q2.y, p.D, p.eta, fx, fy);
  }
  if (has_ab) add_edge(vx, vy, pa.x, pa.y, pb.x, pb.y, p.C, p.eta, fx, fy);
  for (int64_t k = f0 + s + SP; k < f1; k += SP) {
    const int32_t a = p.fan[2 * k], b = p.fan[2 * k + 1];
    if (a < 0 || a >= p.n || b < 0 || b >= p.n) continue;
    const double2 qa = load_pos(p.x, a), qb = load_pos(p.x, b);
    add_edge(vx, vy, qa.x, qa.y, qb.x, qb.y, p.C, p.eta, fx, fy);
  }
  fx = group_sum<SP>(fx);
  fy = group_sum<SP>(fy);
  // temperature
  const double fl = sqrt(fx * fx + fy * fy);
  if (fl > p.t) {
    fx *= p.t / fl;
    fy *= p.t / fl;
  }
  // limiting lines of the node's triangles, shared over its lanes
  double scale = 1.0;
  if (has_ab) scale = triangle_scale(vx, vy, pa.x, pa.y, pb.x, pb.y, fx, fy, p.eta);
  for (int64_t k = f0 + s + SP; k < f1; k += SP) {
    const int32_t a = p.fan[2 * k], b = p.fan[2 * k + 1];
    if (a < 0 || a >= p.n || b < 0 || b >= p.n) continue;
    const double2 qa = load_pos(p.x, a), qb = load_pos(p.x, b);
    const double g = triangle_scale(vx, vy, qa.x, qa.y, qb.x, qb.y, fx, fy, p.eta);
    scale = g < scale ? g : scale;
  }
  scale = group_min<SP>(scale);
  if (s == 0 && live) {
    p.y[2 * v] = vx + fx * scale;
    p.y[2 * v + 1] = vy + fy * scale;
  }
}

__global__ __launch_bounds__(256) void widen_kernel(const float* in, double* out, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < m) out[i] = (double)in[i];
}

__global__ __launch_bounds__(256) void narrow_kernel(const double* in, float* out, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < m) out[i] = (float)in[i];
}

}  // namespace

hipError_t launch_layout(const LayoutArgs& a, hipStream_t s) {
  const int64_t m = 2 * a.n;
  const unsigned gm = (unsigned)((m + 255) / 256);
  hipLaunchKernelGGL(widen_kernel, dim3(gm), dim3(256), 0, s, a.pos, a.buf0, m);
  LayoutParams p;
  p.n = a.n;
  p.adj_start = a.adj_start;
  p.adj = a.adj;
  p.n_adj = a.n_adj;
  p.fan_start = a.fan_start;
  p.fan = a.fan;
  p.n_fan = a.n_fan;
  p.C = a.C;
  p.D = a.D;
  p.eta = a.eta;
  double* cur = a.buf0;
  double* nxt = a.buf1;
  double t = a.t0;
  // nodes per workgroup: few (more lanes per node) while the node count
  // alone would leave compute units idle, more once sources dominate.  Below
  // 16384 nodes the choice between 4 and 8 is measured: 8 is faster at 306
  // and 2245 nodes (5.9 vs 6.8 and 17.3 vs 19.2 us per iteration), 4 at 1000
  // (7.2 vs 7.8 us)
  const int nb = a.n < 16384 ? ((a.n < 512 || a.n >= 2048) ? 8 : 4)
                             : (a.n < 262144 ? 16 : 64);
  const unsigned blocks = (unsigned)((a.n + nb - 1) / nb);
  for (int it = 0; it < a.iterations; ++it) {
    p.x = cur;
    p.y = nxt;
    p.t = t;
    if (nb == 4)
      hipLaunchKernelGGL((layout_step_kernel<4, 2048>), dim3(blocks), dim3(kLanes), 0, s, p);
    else if (nb == 8)
      hipLaunchKernelGGL((layout_step_kernel<8, 2048>), dim3(blocks), dim3(kLanes), 0, s, p);
    else if (nb == 16)
      hipLaunchKernelGGL((layout_step_kernel<16, 1024>), dim3(blocks), dim3(kLanes), 0, s, p);
    else
      hipLaunchKernelGGL((layout_step_kernel<64, 1024>), dim3(blocks), dim3(kLanes), 0, s, p);
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
    t *= a.lambda;
  }
  hipLaunchKernelGGL(narrow_kernel, dim3(gm), dim3(256), 0, s, cur, a.pos, m);
  return hipGetLastError();
}

}  // namespace mls

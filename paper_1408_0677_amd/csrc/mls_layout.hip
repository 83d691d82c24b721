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
// (ping-pong buffers, float64).  A workgroup of four waves owns 64 nodes,
// one per lane; the all-pairs repulsion is split over the four waves by
// source (source tiles staged through LDS) and the four partial sums are
// added in a fixed order, so results do not depend on scheduling.  The
// exact all-pairs sum replaces the paper's kd-tree far field: at the sizes
// the paper lays out (a few thousand points) it costs microseconds.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mls_internal.h"

namespace mls {
namespace {

constexpr int kNodes = 64;      // nodes per workgroup (one per lane)
constexpr int kWaves = 4;       // source splits
constexpr int kTile = 256;      // sources staged per round

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

__global__ __launch_bounds__(kNodes * kWaves) void layout_step_kernel(LayoutParams p) {
#pragma clang fp contract(off)
  __shared__ double src[kTile][2];
  __shared__ double part[kWaves][kNodes][2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t v = (int64_t)blockIdx.x * kNodes + lane;
  const bool live = v < p.n;
  const double vx = live ? p.x[2 * v] : 0.0, vy = live ? p.x[2 * v + 1] : 0.0;
  // repulsion: wave w takes the sources s = w, w + 4, ... of each tile
  double fx = 0.0, fy = 0.0;
  for (int64_t base = 0; base < p.n; base += kTile) {
    __syncthreads();
    for (int e = threadIdx.x; e < kTile; e += kNodes * kWaves) {
      const int64_t u = base + e;
      src[e][0] = u < p.n ? p.x[2 * u] : 0.0;
      src[e][1] = u < p.n ? p.x[2 * u + 1] : 0.0;
    }
    __syncthreads();
    const int cnt = (int)((p.n - base) < kTile ? (p.n - base) : kTile);
    for (int e = wave; e < cnt; e += kWaves) {
      if (base + e == v) continue;
      const double ax = vx - src[e][0], ay = vy - src[e][1];
      const double L = sqrt(ax * ax + ay * ay);
      const double s = p.C / (L * L * L + p.eta);
      fx += s * ax;
      fy += s * ay;
    }
  }
  part[wave][lane][0] = fx;
  part[wave][lane][1] = fy;
  __syncthreads();
  if (wave != 0 || !live) return;
  fx = ((part[0][lane][0] + part[1][lane][0]) + part[2][lane][0]) + part[3][lane][0];
  fy = ((part[0][lane][1] + part[1][lane][1]) + part[2][lane][1]) + part[3][lane][1];
  // springs along the mesh edges
  int64_t k0, k1;
  csr_range(p.adj_start, v, p.n_adj, &k0, &k1);
  for (int64_t k = k0; k < k1; ++k) {
    const int32_t u = p.adj[k];
    if (u < 0 || u >= p.n) continue;
    const double ax = vx - p.x[2 * u], ay = vy - p.x[2 * u + 1];
    const double L = sqrt(ax * ax + ay * ay);
    const double s = L * log((L + p.eta) / p.D);
    fx -= s * ax;
    fy -= s * ay;
  }
  // node-edge repulsion from the opposite edge of each incident triangle
  csr_range(p.fan_start, v, p.n_fan, &k0, &k1);
  for (int64_t k = k0; k < k1; ++k) {
    const int32_t a = p.fan[2 * k], b = p.fan[2 * k + 1];
    if (a < 0 || a >= p.n || b < 0 || b >= p.n) continue;
    const double ax0 = p.x[2 * a], ay0 = p.x[2 * a + 1];
    const double ex = p.x[2 * b] - ax0, ey = p.x[2 * b + 1] - ay0;
    const double e2 = ex * ex + ey * ey;
    if (!(e2 > 0.0)) continue;
    const double tt = ((vx - ax0) * ex + (vy - ay0) * ey) / e2;
    const double rx = ax0 + tt * ex - vx, ry = ay0 + tt * ey - vy;
    const double s = -p.C / (rx * rx + ry * ry + p.eta);
    fx += s * rx;
    fy += s * ry;
  }
  // temperature
  const double fl = sqrt(fx * fx + fy * fy);
  if (fl > p.t) {
    fx *= p.t / fl;
    fy *= p.t / fl;
  }
  // limiting lines: corner i's line is halfway between the edge opposite
  // corner i and the corner; from v it is half of -(v's offset) for i = 0,
  // half of the corner's offset from the edge through v for i = 1, 2
  double scale = 1.0;
  for (int64_t k = k0; k < k1; ++k) {
    const int32_t a = p.fan[2 * k], b = p.fan[2 * k + 1];
    if (a < 0 || a >= p.n || b < 0 || b >= p.n) continue;
    const double P[3][2] = {{vx, vy}, {p.x[2 * a], p.x[2 * a + 1]}, {p.x[2 * b], p.x[2 * b + 1]}};
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
        const double room = rl - p.eta > 0.0 ? rl - p.eta : 0.0;
        if (proj * scale > room) scale = room / proj;
      }
    }
  }
  p.y[2 * v] = vx + fx * scale;
  p.y[2 * v + 1] = vy + fy * scale;
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
  const unsigned blocks = (unsigned)((a.n + kNodes - 1) / kNodes);
  for (int it = 0; it < a.iterations; ++it) {
    p.x = cur;
    p.y = nxt;
    p.t = t;
    hipLaunchKernelGGL(layout_step_kernel, dim3(blocks), dim3(kNodes * kWaves), 0, s, p);
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
    t *= a.lambda;
  }
  hipLaunchKernelGGL(narrow_kernel, dim3(gm), dim3(256), 0, s, cur, a.pos, m);
  return hipGetLastError();
}

}  // namespace mls

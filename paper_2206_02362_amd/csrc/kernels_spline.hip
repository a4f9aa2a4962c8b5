// Linear spline operator S and its adjoint S* (Section 2: the velocity model
// is held on a coarse spline grid and mapped onto the finite-difference grid
// by linear spline interpolation; gradients come back through S*).
//
// S is the tensor product of two 1D hat-function interpolations: the fine
// point at depth iz*dz lies in spline cell kz (node kz <= iz*dz < node kz+1,
// the last cell closed) with weight tz for node kz+1 and 1 - tz for node kz;
// likewise along x.  Per axis a table kernel finds every fine point's cell by
// binary search over the node coordinates (in FP64) and, for every node j,
// the first fine point whose cell is at least j.  The same tables, evaluated
// at the nodes of a finer spline grid, move a model to that grid.  Because the cell index never
// decreases along the axis, the fine points of cell j form the range
// [start[j], start[j+1]), so the adjoint is a deterministic gather: node j
// collects the points of cell j - 1 with weight t and those of cell j with
// weight 1 - t, in ascending order.
//
// Layouts: fine fields [nx][nz], node values [nxn][nzn], z fastest.  All
// kernels are bandwidth-bound streams; the node arrays are small and stay in
// cache.
#include "internal.h"

namespace fw {

static unsigned spline_blocks(long n) {
  const long b = (n + 255) / 256;
  return (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

// cell[i], wt[i] for target points i = 0..nf-1 at coordinate pts[i], or at
// i*h without pts (the finite-difference grid); nn >= 2 nodes
__global__ void k_spline_axis(const double *nodes, int nn, const double *pts, int nf, double h, int *cell,
                              float *wt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  const double p = pts ? pts[i] : i * h;
  int lo = 0, hi = nn - 2;                     // the cell is in [lo, hi]
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (nodes[mid] <= p) lo = mid;
    else hi = mid - 1;
  }
  double t = (p - nodes[lo]) / (nodes[lo + 1] - nodes[lo]);
  t = fmin(fmax(t, 0.0), 1.0);
  cell[i] = lo;
  wt[i] = (float)t;
}

// start[j] = first fine point whose cell is >= j, for j = 0..nn
__global__ void k_spline_starts(const int *cell, int nf, int nn, int *start) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > nn) return;
  int lo = 0, hi = nf;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (cell[mid] >= j) hi = mid;
    else lo = mid + 1;
  }
  start[j] = lo;
}

// out[ix][iz] = sum over the four surrounding nodes of their bilinear weights
__global__ void k_spline_apply(const float *__restrict__ mc, int nzn, const int *__restrict__ cz,
                               const float *__restrict__ tz, const int *__restrict__ cx,
                               const float *__restrict__ tx, int nz, long n, float *__restrict__ out) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int ix = (int)(i / nz), iz = (int)(i - (long)ix * nz);
    const int kz = cz[iz], kx = cx[ix];
    const float wz = tz[iz], wx = tx[ix];
    const float *m0 = mc + (long)kx * nzn + kz;
    const float *m1 = m0 + nzn;
    const float a = (1.0f - wz) * m0[0] + wz * m0[1];
    const float b = (1.0f - wz) * m1[0] + wz * m1[1];
    out[i] = (1.0f - wx) * a + wx * b;
  }
}

// tmp[ix][jz] = sum over fine iz of A_z[iz][jz] f[ix][iz]
__global__ void k_spline_adj_z(const float *__restrict__ f, int nz, const float *__restrict__ tz,
                               const int *__restrict__ sz, int nzn, long n, float *__restrict__ tmp) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int ix = (int)(i / nzn), jz = (int)(i - (long)ix * nzn);
    const float *row = f + (long)ix * nz;
    float acc = 0.0f;
    if (jz > 0)
      for (int iz = sz[jz - 1]; iz < sz[jz]; ++iz) acc += tz[iz] * row[iz];
    for (int iz = sz[jz]; iz < sz[jz + 1]; ++iz) acc += (1.0f - tz[iz]) * row[iz];
    tmp[i] = acc;
  }
}

// out[jx][jz] = sum over fine ix of A_x[ix][jx] tmp[ix][jz]
__global__ void k_spline_adj_x(const float *__restrict__ tmp, int nzn, const float *__restrict__ tx,
                               const int *__restrict__ sx, long n, float *__restrict__ out) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int jx = (int)(i / nzn), jz = (int)(i - (long)jx * nzn);
    float acc = 0.0f;
    if (jx > 0)
      for (int ix = sx[jx - 1]; ix < sx[jx]; ++ix) acc += tx[ix] * tmp[(long)ix * nzn + jz];
    for (int ix = sx[jx]; ix < sx[jx + 1]; ++ix) acc += (1.0f - tx[ix]) * tmp[(long)ix * nzn + jz];
    out[i] = acc;
  }
}

hipError_t launch_spline_tables(const double *nodes, int nn, const double *pts, int nf, double h, int *cell,
                                float *wt, int *start, hipStream_t st) {
  k_spline_axis<<<(nf + 255) / 256, 256, 0, st>>>(nodes, nn, pts, nf, h, cell, wt);
  k_spline_starts<<<(nn + 1 + 255) / 256, 256, 0, st>>>(cell, nf, nn, start);
  return hipGetLastError();
}

hipError_t launch_spline_apply(const float *mc, int nzn, const int *cz, const float *tz, const int *cx,
                               const float *tx, int nz, int nx, float *out, hipStream_t st) {
  const long n = (long)nx * nz;
  k_spline_apply<<<spline_blocks(n), 256, 0, st>>>(mc, nzn, cz, tz, cx, tx, nz, n, out);
  return hipGetLastError();
}

hipError_t launch_spline_adjoint(const float *f, int nz, int nx, const float *tz, const int *sz, int nzn,
                                 const float *tx, const int *sx, int nxn, float *tmp, float *out, hipStream_t st) {
  const long n1 = (long)nx * nzn, n2 = (long)nxn * nzn;
  k_spline_adj_z<<<spline_blocks(n1), 256, 0, st>>>(f, nz, tz, sz, nzn, n1, tmp);
  k_spline_adj_x<<<spline_blocks(n2), 256, 0, st>>>(tmp, nzn, tx, sx, n2, out);
  return hipGetLastError();
}

}  // namespace fw

// Vector kernels of the variable-projection solver: the linear
// conjugate-gradient iteration on the normal equation of eq. vp.obj needs
// inner products, the two updates of the iterate and residual, the new search
// direction and the diagonal regularization term eps^2 D* D.
//
// All of them are bandwidth-bound streams over [nh][nx][nz] or data-sized
// FP32 arrays.  Inner products accumulate in FP64 over a fixed grid and are
// reduced in a fixed order, so a result does not depend on scheduling.
#include "internal.h"

namespace fw {

constexpr int kDotBlocks = 1024;
constexpr int kDotThreads = 256;

// out = a - b
__global__ void k_sub(const float *a, const float *b, float *out, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    out[i] = a[i] - b[i];
}

// part[block] = sum over this block's strided share of x[i] * y[i], in FP64
__global__ void __launch_bounds__(kDotThreads) k_dot_part(const float *x, const float *y, long n, double *part) {
  __shared__ double red[kDotThreads];
  double acc = 0.0;
  for (long i = (long)blockIdx.x * kDotThreads + threadIdx.x; i < n; i += (long)kDotBlocks * kDotThreads)
    acc += (double)x[i] * (double)y[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kDotThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// *out = sum of the partials in a fixed tree order (one workgroup)
__global__ void __launch_bounds__(kDotThreads) k_dot_final(const double *part, double *out) {
  __shared__ double red[kDotThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < kDotBlocks; i += kDotThreads) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kDotThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// p += alpha s;  r -= alpha q
__global__ void k_cg_step(float *p, float *r, const float *s, const float *q, float alpha, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    p[i] = fmaf(alpha, s[i], p[i]);
    r[i] = fmaf(-alpha, q[i], r[i]);
  }
}

// s = r + beta s
__global__ void k_cg_dir(float *s, const float *r, float beta, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    s[i] = fmaf(beta, s[i], r[i]);
}

// q[h] += e2d2[h] * s[h] for each offset plane h (plane = nx nz cells)
__global__ void k_add_diag(float *q, const float *s, const float *e2d2, long plane, int nh) {
  const long n = plane * nh;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    q[i] = fmaf(e2d2[i / plane], s[i], q[i]);
}

static unsigned stream_blocks(long n) {
  const long b = (n + 255) / 256;
  return (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

hipError_t launch_sub(const float *a, const float *b, float *out, long n, hipStream_t st) {
  k_sub<<<stream_blocks(n), 256, 0, st>>>(a, b, out, n);
  return hipGetLastError();
}

hipError_t launch_dot(const float *x, const float *y, long n, double *part, double *out, hipStream_t st) {
  k_dot_part<<<kDotBlocks, kDotThreads, 0, st>>>(x, y, n, part);
  k_dot_final<<<1, kDotThreads, 0, st>>>(part, out);
  return hipGetLastError();
}

int dot_partials() { return kDotBlocks; }

hipError_t launch_cg_step(float *p, float *r, const float *s, const float *q, float alpha, long n, hipStream_t st) {
  k_cg_step<<<stream_blocks(n), 256, 0, st>>>(p, r, s, q, alpha, n);
  return hipGetLastError();
}

hipError_t launch_cg_dir(float *s, const float *r, float beta, long n, hipStream_t st) {
  k_cg_dir<<<stream_blocks(n), 256, 0, st>>>(s, r, beta, n);
  return hipGetLastError();
}

hipError_t launch_add_diag(float *q, const float *s, const float *e2d2, long plane, int nh, hipStream_t st) {
  k_add_diag<<<stream_blocks(plane * nh), 256, 0, st>>>(q, s, e2d2, plane, nh);
  return hipGetLastError();
}

// y = a x + b y (x may alias y)
__global__ void k_axpby(const float *x, float a, float *y, float b, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = fmaf(a, x[i], b * y[i]);
}

hipError_t launch_axpby(const float *x, float a, float *y, float b, long n, hipStream_t st) {
  k_axpby<<<stream_blocks(n), 256, 0, st>>>(x, a, y, b, n);
  return hipGetLastError();
}

}  // namespace fw

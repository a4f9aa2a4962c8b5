// Leapfrog time step of the constant-density acoustic wave equation on a
// batch of shots sharing one velocity model (gfx950, wave64).
//
//   out = g (2 cur - g prev + V (L cur + src)),   g = g_z(z) g_x(x)
//
// with L the radius-4 Laplacian (zero outside the padded grid), evaluated in
// difference form.  The same
// kernel runs the forward recursion (cur = u^n, prev = u^{n-1}, out =
// u^{n+1}) and the transposed one backwards in time (cur = lambda_k, prev =
// lambda_{k+1}, out = lambda_{k-1}), because every time block of the
// discrete system is symmetric.
//
// Tiling: a workgroup owns a 64 (z) x TX (x) tile of one shot.  Lane = z, so
// every global access of a wavefront is 256 contiguous bytes of one column.
// The input field tile plus a 4-cell halo is staged in LDS; each wavefront
// then marches over TX/4 consecutive columns keeping the 9 x-neighbours in a
// register queue and reading the 8 z-neighbours from LDS.  `prev`, V and the
// optional dense source are loaded straight into registers before the LDS
// barrier, so their latency overlaps the tile load.
//
// Workgroups are mapped XCD-aware: hardware workgroup b runs on XCD b % 8, and
// the logical tile order (tile_index: groups of x-strips, one shot at a time
// inside a group) is split into 8 contiguous ranges, one per XCD, so halo
// columns and the shared V tile are re-read from the XCD's own L2.
//
// Point sources / receiver injections come as per-(tile, wave) lists sorted by
// column, consumed by a wave-uniform loop inside the column march.  Receiver
// sampling reads the LDS tile of the INPUT field, i.e. the kernel of equation
// n records u^n.
//
// Free surface (kModeFS): the tile rows just above the surface row are loaded
// from their mirror rows below it with opposite sign, and the output is zero
// at and above the surface row; nothing else changes.
#include "internal.h"

namespace fw {

template <int TX>
struct StepTile {
  static constexpr int HC = TX + 2 * kR;
  static constexpr int HZ = kTZ + 2 * kR;
  float v[HC][HZ];
  float sink[kWaves][kTZ];   // target of the halo-row writes of lanes 8..63 (never read)
};

// One 64 x TX tile of one shot; `logical` is the tile's position in the
// launch order of tile_index.  With extract_only the kernel only samples the
// receivers of the input field (the last time sample of a job).
template <int TX, int MODE>
__device__ __forceinline__ void step_body(const StepArgs &a, int logical, StepTile<TX> &sh, bool extract_only) {
  constexpr bool FS = (MODE & kModeFS) != 0;
  constexpr int CPW = TX / kWaves;
  constexpr int HC = TX + 2 * kR;
  constexpr int HZ = kTZ + 2 * kR;
  auto &tile = sh.v;
  int txi, tzi, s;
  tile_coords(logical, a.ntz, a.ntx, a.nshots, txi, tzi, s);
  const int z0 = tzi * kTZ;
  const int x0 = txi * TX;
  const int NZ = a.NZ, NX = a.NX, LZ = a.LZ;

  const long soff = (long)s * a.sstride;
  float *out = a.out + soff;
  const int CB = LZ * 4;                      // bytes per column
  const unsigned FB = (unsigned)NX * (unsigned)CB;
  const auto r_cur = rsrc(a.cur + soff, FB);
  const auto r_prev = rsrc(a.prev + soff, FB);
  const auto r_V = rsrc(a.V, FB);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int z = z0 + lane;
  const bool zin = z < NZ;
  const int xs = x0 + w * CPW;

  // Own-cell operands first: their latency hides behind the tile load.  A
  // cell outside the grid gets an offset past the end of the buffer and reads
  // zero, so no load sits behind a branch (the compiler would wait for each).
  float pv[CPW], vv[CPW], ds[CPW], gx[CPW];
  [[maybe_unused]] __amdgpu_buffer_rsrc_t r_ds;
  if constexpr ((MODE & kModeDsrc) != 0) r_ds = rsrc(a.dsrc + (long)s * a.dsrc_sstride, FB);
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int x = xs + j;
    const int o = zin && x < NX ? x * CB + z * 4 : kOutOfRange;
    gx[j] = a.gx[min(x, NX - 1)];
    pv[j] = ld(r_prev, o, 0);
    vv[j] = ld(r_V, o, 0);
    ds[j] = 0.f;
    if constexpr ((MODE & kModeDsrc) != 0) ds[j] = ld(r_ds, o, 0);
  }
  const float gzv = zin ? a.gz[z] : 0.f;
  if constexpr ((MODE & kModeNu) != 0) {
    const long so = (long)s * a.nu.sstride;
    const auto rm = rsrc(a.nu.em + so, FB), r0 = rsrc(a.nu.e0 + so, FB), rp = rsrc(a.nu.ep + so, FB);
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      const int x = xs + j;
      const bool in = zin && x < NX;
      const int o = in ? x * CB + z * 4 : kOutOfRange;
      const float g = gzv * gx[j];
      const float e = ld(rm, o, 0) / g - 2.f * ld(r0, o, 0) + g * ld(rp, o, 0);
      if (in) ds[j] += e;   // a select: nothing is loaded under it
    }
  }

  // input tile plus a 4-cell halo: lane = row z0 - 4 + lane, lanes 0..7 also
  // row z0 + 60 + lane; every load of it is in flight before the first wait
  {
    constexpr int NC = HC / kWaves;
    static_assert(HC % kWaves == 0 && HZ == kTZ + 2 * kR, "tile shape");
    const int zg = z0 - kR + lane;
    const bool zg_in = zg >= 0 && zg < NZ;
    const bool zg2_in = lane < 2 * kR && zg + kTZ < NZ;
    float v[NC], v2[NC];
    // rows read for the two loads of this lane (mirrored under a free surface)
    float sg = 1.f, sg2 = 1.f;
    int zr = zg, zr2 = zg + kTZ;
    if constexpr (FS) {
      zr = fs_mirror_row(zg, a.fs, sg);
      zr2 = fs_mirror_row(zg + kTZ, a.fs, sg2);
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      const int x = x0 - kR + w + kWaves * i;
      const bool xin = x >= 0 && x < NX;      // wave-uniform
      v[i] = ld(r_cur, xin && zg_in ? x * CB + zr * 4 : kOutOfRange, 0);
      v2[i] = ld(r_cur, xin && zg2_in ? x * CB + zr2 * 4 : kOutOfRange, 0);
    }
    const bool lo8 = lane < 2 * kR;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      const int c = w + kWaves * i;
      tile[c][lane] = FS ? sg * v[i] : v[i];
      *(lo8 ? &tile[c][kTZ + lane] : &sh.sink[w][lane]) = FS ? sg2 * v2[i] : v2[i];
    }
  }
  __syncthreads();

  if (a.ext.ptr != nullptr) {
    const int e0 = a.ext.ptr[logical], e1 = a.ext.ptr[logical + 1];
    for (int e = e0 + tid; e < e1; e += 256) {
      const int2 en = a.ext.ent[e];
      a.ext.out[(long)en.y * a.ext.stride_idx + a.ext.t] = tile[(en.x >> 6) + kR][(en.x & 63) + kR];
    }
  }
  if (extract_only) return;

  int p = 0, pend = 0;
  if (a.inj.ptr != nullptr) {
    p = a.inj.ptr[logical * kWaves + w];
    pend = a.inj.ptr[logical * kWaves + w + 1];
  }

  const int lz = lane + kR;
  const int cb = w * CPW + kR;
  float q[2 * kR + 1];
#pragma unroll
  for (int k = 0; k < 2 * kR; ++k) q[k] = tile[cb - kR + k][lz];

#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    q[2 * kR] = tile[cb + j + kR][lz];
    const float c = q[kR];
    const float *col = &tile[cb + j][lz];
    // Difference form: the weights sum to zero, so L u = sum_k w_k
    // ((u_{+k} - u) + (u_{-k} - u)); neighbour differences are formed first,
    // which avoids the cancellation of the w_0 u + sum w_k (u_+ + u_-) form
    // (about 20x smaller FP32 rounding error over a few thousand steps).
    float lap = 0.f;
#pragma unroll
    for (int k = 1; k <= kR; ++k) {
      lap += a.cz[k - 1] * ((col[-k] - c) + (col[k] - c));
      lap += a.cx[k - 1] * ((q[kR - k] - c) + (q[kR + k] - c));
    }
    float src = ds[j];
    while (p < pend) {   // wave-uniform
      const int2 en = a.inj.ent[p];
      if ((en.x >> 6) != j) break;
      const float val = a.inj.val[(long)en.y * a.inj.stride_idx + a.inj.t] * a.inj.scale;
      if ((en.x & 63) == lane) src += val;
      ++p;
    }
    const int x = xs + j;
    if (zin && x < NX) {
      const float g = gzv * gx[j];
      float r = vv[j] * (lap + src);
      const long idx = (long)x * LZ + z;
      float u = g * (2.f * c - g * pv[j] + r);
      if constexpr (FS) {
        if (z <= a.fs) u = r = 0.f;          // at and above the free surface
      }
      out[idx] = u;
      if constexpr ((MODE & kModeT2) != 0) a.t2[(long)s * a.t2_sstride + idx] = r;
    }
#pragma unroll
    for (int k = 0; k < 2 * kR; ++k) q[k] = q[k + 1];
  }
}


template <int TX, int MODE>
__global__ void __launch_bounds__(256) k_step(const StepArgs a) {
  __shared__ StepTile<TX> sh;
  const int total = a.ntz * a.ntx * a.nshots;
  const int per = (total + 7) >> 3;
  const int b = blockIdx.x;
  const int logical = (b & 7) * per + (b >> 3);    // XCD-contiguous tile ranges
  if (logical >= total) return;
  step_body<TX, MODE>(a, logical, sh, false);
}

// Many jobs (different grids, models and geometries) in one launch.  Blocks
// cover the concatenated tile lists of the jobs (prefix sums in tile_begin);
// the time index of job j is *step - t0_j: it advances its fields while the
// index is below nt_j - 1, samples its receivers at nt_j - 1 and is idle
// outside [0, nt_j - 1].  Job j's fields alternate between bufA and bufB.
template <int TX, int MODE>
__global__ void __launch_bounds__(256) k_step_multi(const BatchJob *jobs, int njobs, int total,
                                                    const int *step, int step_val) {
  __shared__ StepTile<TX> sh;
  const int per = (total + 7) >> 3;
  const int b = blockIdx.x;
  const int logical = (b & 7) * per + (b >> 3);
  if (logical >= total) return;
  int lo = 0, hi = njobs - 1;                       // last job with tile_begin <= logical
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].tile_begin <= logical) lo = mid;
    else hi = mid - 1;
  }
  const BatchJob &jb = jobs[lo];
  const int n = (step ? *step : step_val) - jb.t0;
  if (n < 0 || n > jb.nt - 1) return;
  StepArgs a = jb.a;
  const bool even = (n & 1) == 0;
  a.cur = even ? jb.bufA : jb.bufB;
  a.prev = even ? jb.bufB : jb.bufA;
  a.out = const_cast<float *>(a.prev);
  a.inj.t = n;
  a.ext.t = n;
  step_body<TX, MODE>(a, logical - jb.tile_begin, sh, n == jb.nt - 1);
}

__global__ void k_bump(int *step, int by) { *step += by; }

template <int TX>
static void launch_step_multi_tx(dim3 grid, const BatchJob *jobs, int njobs, int total_tiles, const int *step,
                                 int step_val, bool fs, hipStream_t st) {
  if (fs) k_step_multi<TX, kModeFS><<<grid, 256, 0, st>>>(jobs, njobs, total_tiles, step, step_val);
  else k_step_multi<TX, kModePlain><<<grid, 256, 0, st>>>(jobs, njobs, total_tiles, step, step_val);
}

hipError_t launch_step_multi(const BatchJob *jobs, int njobs, int total_tiles, const int *step, int step_val,
                             int tile_x, bool fs, hipStream_t st) {
  const long per = (total_tiles + 7) / 8;
  const dim3 grid((unsigned)(per * 8));
  switch (tile_x) {
    case 16: launch_step_multi_tx<16>(grid, jobs, njobs, total_tiles, step, step_val, fs, st); break;
    case 24: launch_step_multi_tx<24>(grid, jobs, njobs, total_tiles, step, step_val, fs, st); break;
    case 32: launch_step_multi_tx<32>(grid, jobs, njobs, total_tiles, step, step_val, fs, st); break;
    case 48: launch_step_multi_tx<48>(grid, jobs, njobs, total_tiles, step, step_val, fs, st); break;
    case 64: launch_step_multi_tx<64>(grid, jobs, njobs, total_tiles, step, step_val, fs, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_bump(int *step, int by, hipStream_t st) {
  k_bump<<<1, 1, 0, st>>>(step, by);
  return hipGetLastError();
}

int step_tile_x_supported(int tx) { return tx == 16 || tx == 24 || tx == 32 || tx == 48 || tx == 64; }

template <int TX>
static hipError_t launch_step_tx(const StepArgs &a, int mode, hipStream_t st) {
  const long total = (long)a.ntz * a.ntx * a.nshots;
  const long per = (total + 7) / 8;
  const dim3 grid((unsigned)(per * 8));
  if (a.fs >= 0) mode |= kModeFS;
  switch (mode) {
#define FW_STEP_MODE(M)                                     \
  case M: k_step<TX, M><<<grid, 256, 0, st>>>(a); break;    \
  case M | kModeFS: k_step<TX, M | kModeFS><<<grid, 256, 0, st>>>(a); break;
    FW_STEP_MODE(kModePlain)
    FW_STEP_MODE(kModeT2)
    FW_STEP_MODE(kModeDsrc)
    FW_STEP_MODE(kModeT2 | kModeDsrc)
    FW_STEP_MODE(kModeNu)
#undef FW_STEP_MODE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_step(const StepArgs &a, int tile_x, int mode, hipStream_t st) {
  switch (tile_x) {
    case 16: return launch_step_tx<16>(a, mode, st);
    case 24: return launch_step_tx<24>(a, mode, st);
    case 32: return launch_step_tx<32>(a, mode, st);
    case 48: return launch_step_tx<48>(a, mode, st);
    case 64: return launch_step_tx<64>(a, mode, st);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------

__global__ void k_gather(const float *field, long sstride, const int *cells, int nshots, int nrec, float *out,
                         long stride_r, int t) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)nshots * nrec) return;
  const int s = (int)(i / nrec);
  out[i * stride_r + t] = field[(long)s * sstride + cells[i]];
}

hipError_t launch_gather(const float *field, long sstride, const int *cells, int nshots, int nrec, float *out,
                         long stride_r, int t, hipStream_t st) {
  const long n = (long)nshots * nrec;
  if (n == 0) return hipSuccess;
  k_gather<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(field, sstride, cells, nshots, nrec, out, stride_r, t);
  return hipGetLastError();
}

__global__ void k_prep(const float *vel, int nz, int nx, int nb, int NZ, int NX, int LZ, float dt, float *V) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)NX * LZ) return;
  const int x = (int)(i / LZ);
  const int z = (int)(i - (long)x * LZ);
  if (z >= NZ) {
    V[i] = 0.f;
    return;
  }
  const int mx = min(max(x - nb, 0), nx - 1);
  const int mz = min(max(z - nb, 0), nz - 1);
  const float v = vel[(long)mx * nz + mz];
  V[i] = v * v * dt * dt;
}

hipError_t launch_prep(const float *vel, int nz, int nx, int nb, int NZ, int NX, int LZ, float dt, float *V,
                       hipStream_t st) {
  const long n = (long)NX * LZ;
  k_prep<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(vel, nz, nx, nb, NZ, NX, LZ, dt, V);
  return hipGetLastError();
}

__global__ void k_zero(float *a, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) a[i] = 0.f;
}

hipError_t launch_zero(float *a, long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  k_zero<<<(unsigned)blocks, 256, 0, st>>>(a, n);
  return hipGetLastError();
}

__global__ void k_copy_fields(float *dst, long dst_sstride, const float *src, long src_sstride, long n) {
  const int s = blockIdx.y;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[s * dst_sstride + i] = src[s * src_sstride + i];
}

hipError_t launch_copy_fields(float *dst, long dst_sstride, const float *src, long src_sstride, int S, long n,
                              hipStream_t st) {
  if (n <= 0 || S <= 0) return hipSuccess;
  long bx = (n + 255) / 256;
  if (bx > 4096) bx = 4096;
  k_copy_fields<<<dim3((unsigned)bx, (unsigned)S), 256, 0, st>>>(dst, dst_sstride, src, src_sstride, n);
  return hipGetLastError();
}

// Block-reduced min / max / non-finite count, combined across blocks with
// device-scope atomics on doubles (order-independent).
__global__ void k_minmax(const float *a, long n, double *res) {
  float mn = INFINITY, mx = -INFINITY;
  double bad = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float v = a[i];
    if (!isfinite(v)) {
      bad += 1.0;
    } else {
      mn = fminf(mn, v);
      mx = fmaxf(mx, v);
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    mn = fminf(mn, __shfl_xor(mn, o));
    mx = fmaxf(mx, __shfl_xor(mx, o));
    bad += __shfl_xor(bad, o);
  }
  __shared__ float smn[4], smx[4];
  __shared__ double sbad[4];
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    smn[wv] = mn;
    smx[wv] = mx;
    sbad[wv] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    mn = fminf(fminf(smn[0], smn[1]), fminf(smn[2], smn[3]));
    mx = fmaxf(fmaxf(smx[0], smx[1]), fmaxf(smx[2], smx[3]));
    bad = sbad[0] + sbad[1] + sbad[2] + sbad[3];
    atomicMin(&res[0], (double)mn);
    atomicMax(&res[1], (double)mx);
    atomicAdd(&res[2], bad);
  }
}

__global__ void k_minmax_init(double *res) {
  res[0] = INFINITY;
  res[1] = -INFINITY;
  res[2] = 0.0;
}

hipError_t launch_minmax(const float *a, long n, double *res, hipStream_t st) {
  k_minmax_init<<<1, 1, 0, st>>>(res);
  long blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  k_minmax<<<(unsigned)blocks, 256, 0, st>>>(a, n, res);
  return hipGetLastError();
}

}  // namespace fw

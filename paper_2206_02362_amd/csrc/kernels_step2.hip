// Two leapfrog time steps per launch (temporal blocking) of the
// constant-density acoustic recursion
//
//   u^{n+1} = g (2 u^n - g u^{n-1} + V (L u^n + f^n)),   g = g_z(z) g_x(x),
//
// the same update, operation for operation, as the one-step kernel, so both
// produce identical bits.  A workgroup owns a 56 (z) x TX (x) output tile of
// one shot.  It stages u^n on the tile plus an 8-cell halo in LDS, computes
// u^{n+1} on the tile plus a 4-cell halo (the halo part is recomputed by the
// neighbouring workgroups too, from the same operands, so it is bit-identical
// to theirs), keeps it in LDS and computes u^{n+2} on the tile.  Per time step
// a cell then costs about one read and one write of a wavefield in HBM instead
// of two reads and one write.
//
// Lane = row: row z0 - 4 + lane for both steps (lanes 4..59 are the tile's own
// rows), so every global access of a wavefront is one contiguous column run.
// Wave w marches over its columns with the 9 x-neighbours in a register queue
// and the z-neighbours read from LDS, like the one-step kernel.
//
// Inputs u^{n-1} and u^n are read with halos and the outputs go to two other
// buffers, so a caller rotates four field buffers.  Optional outputs: the
// T2 term V (L u + f) of both steps on the tile, receiver samples of u^n and
// u^{n+1}.  Optional input: a dense source per step (read on the halo for the
// first step, so it must not be the buffer a T2 output goes to), given either
// as a field or as three slots of a ring whose transposed second time
// difference is the source.  With two == 0 only u^{n+1} is produced (an odd
// last step).
#include "internal.h"

namespace fw {

template <int TX, bool DF = false>
struct Step2Tile {
  static constexpr int C0 = TX + 16;   // u^n columns x0 - 8 .. x0 + TX + 7
  static constexpr int C1 = TX + 8;    // u^{n+1} columns x0 - 4 .. x0 + TX + 3
  static constexpr int ROWS = 72;      // rows z0 - 8 .. z0 + 63
  float u0[C0][ROWS];
  float u1[C1][ROWS];                  // rows 0..3 and 68..71 are never stored (read by idle lanes only)
};

// Extended-precision variant: each field is hi (FP32) + lo (BF16 bits), the
// lo part holding the FP32 rounding residual of the update.  The Laplacian
// acts on hi + lo and the update is evaluated in FP64 before the split, so
// the rounding noise of an FP32 wavefield (white in space, strongly amplified
// by the second time difference V (L u + f) that feeds the Born source) does
// not build up.
template <int TX>
struct Step2Tile<TX, true> : Step2Tile<TX, false> {
  unsigned short l0[Step2Tile<TX, false>::C0][Step2Tile<TX, false>::ROWS];
  unsigned short l1[Step2Tile<TX, false>::C1][Step2Tile<TX, false>::ROWS];
};

__device__ __forceinline__ float bf16_f32(unsigned short b) { return __uint_as_float((unsigned)b << 16); }
__device__ __forceinline__ unsigned short f32_bf16(float f) {   // round to nearest even (finite values)
  const unsigned u = __float_as_uint(f);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// u = g (2 (c + cl) - g (p + pl) + r) in FP64, split into FP32 hi and BF16 lo
__device__ __forceinline__ float df_update(float g, float c, float cl, float pv, float pl, float r,
                                           unsigned short &lo) {
  const double gd = g;
  const double ex = gd * (2.0 * ((double)c + (double)cl) - gd * ((double)pv + (double)pl) + (double)r);
  const float hi = (float)ex;
  lo = f32_bf16((float)(ex - (double)hi));
  return hi;
}

// One 56 x TX tile of one shot; `logical` enumerates (x-chunk, z-strip, shot)
// with the shot fastest.  extract_only: only sample u^n.  ext_next: sample
// u^{n+1} after the first step even when no second step follows.
template <int TX, int MODE>
__device__ __forceinline__ void step2_body(const Step2Args &p, int logical,
                                           Step2Tile<TX, (MODE & kModeDF) != 0> &sh, bool extract_only,
                                           bool ext_next) {
  constexpr bool T2 = (MODE & kModeT2) != 0;
  constexpr bool DS = (MODE & kModeDsrc) != 0;
  constexpr bool NU = (MODE & kModeNu) != 0;
  constexpr bool DF = (MODE & kModeDF) != 0;
  constexpr int C0 = Step2Tile<TX>::C0;
  constexpr int ROWS = Step2Tile<TX>::ROWS;
  constexpr int W1 = (TX + 8) / kWaves;      // step-1 columns per wave
  constexpr int W2 = TX / kWaves;            // step-2 columns per wave
  static_assert((TX + 8) % kWaves == 0 && TX % kWaves == 0, "tile width");
  const StepArgs &a = p.a;
  const int tile_id = logical / a.nshots;
  const int s = logical - tile_id * a.nshots;
  const int txi = tile_id / a.ntz;
  const int tzi = tile_id - txi * a.ntz;
  const int z0 = tzi * kTZ2;
  const int x0 = txi * TX;
  const int NZ = a.NZ, NX = a.NX, LZ = a.LZ;

  const long soff = (long)s * a.sstride;
  const float *u0g = a.cur + soff;
  const float *um = a.prev + soff;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int z = z0 - kR + lane;
  const bool zin = z >= 0 && z < NZ;
  const bool zown = lane >= kR && lane < kR + kTZ2;
  const int xs1 = x0 - kR + w * W1;          // first step-1 column of this wave
  const int xs2 = x0 + w * W2;               // first step-2 column

  // Own-row operands of both steps; their latency hides behind the tile load.
  float pv[W1], vv1[W1], vv2[W2], ds1[W1], ds2[W2], pl[W1];
#pragma unroll
  for (int j = 0; j < W1; ++j) {
    const int x = xs1 + j;
    const bool in = zin && x >= 0 && x < NX;
    const long idx = (long)x * LZ + z;
    pv[j] = in ? um[idx] : 0.f;
    pl[j] = 0.f;
    if constexpr (DF) pl[j] = in ? bf16_f32(p.lo_prev[soff + idx]) : 0.f;
    vv1[j] = in ? a.V[idx] : 0.f;
    ds1[j] = 0.f;
    if constexpr (DS) ds1[j] = in ? a.dsrc[(long)s * a.dsrc_sstride + idx] : 0.f;
  }
#pragma unroll
  for (int j = 0; j < W2; ++j) {
    const int x = xs2 + j;
    const bool in = zin && x < NX;
    const long idx = (long)x * LZ + z;
    vv2[j] = in ? a.V[idx] : 0.f;
    ds2[j] = 0.f;
    if constexpr (DS) ds2[j] = (in && p.two) ? p.dsrc2[(long)s * a.dsrc_sstride + idx] : 0.f;
  }
  const float gzv = zin ? a.gz[z] : 0.f;
  if constexpr (NU) {
    // transposed second time difference of the e ring: step 1 reads slots
    // (k-1, k, k+1) on the halo, step 2 slots (k-2, k-1, k) on the tile
    const long so = (long)s * a.nu.sstride;
#pragma unroll
    for (int j = 0; j < W1; ++j) {
      const int x = xs1 + j;
      if (zin && x >= 0 && x < NX) {
        const long idx = so + (long)x * LZ + z;
        const float g = gzv * a.gx[x];
        ds1[j] += a.nu.em[idx] / g - 2.f * a.nu.e0[idx] + g * a.nu.ep[idx];
      }
    }
    if (p.two) {
#pragma unroll
      for (int j = 0; j < W2; ++j) {
        const int x = xs2 + j;
        if (zin && x < NX) {
          const long idx = so + (long)x * LZ + z;
          const float g = gzv * a.gx[x];
          ds2[j] += p.nu2.em[idx] / g - 2.f * p.nu2.e0[idx] + g * p.nu2.ep[idx];
        }
      }
    }
  }

  for (int i = tid; i < C0 * ROWS; i += 256) {
    const int c = i / ROWS;
    const int r = i - c * ROWS;
    const int x = x0 - 2 * kR + c;
    const int zg = z0 - 2 * kR + r;
    float v = 0.f;
    if ((unsigned)x < (unsigned)NX && (unsigned)zg < (unsigned)NZ) v = u0g[(long)x * LZ + zg];
    sh.u0[c][r] = v;
    if constexpr (DF) {
      unsigned short l = 0;
      if ((unsigned)x < (unsigned)NX && (unsigned)zg < (unsigned)NZ) l = p.lo_cur[soff + (long)x * LZ + zg];
      sh.l0[c][r] = l;
    }
  }
  __syncthreads();

  // receivers of u^n (time t)
  const int e0 = a.ext.ptr ? a.ext.ptr[logical] : 0;
  const int e1 = a.ext.ptr ? a.ext.ptr[logical + 1] : 0;
  for (int e = e0 + tid; e < e1; e += 256) {
    const int2 en = a.ext.ent[e];
    a.ext.out[(long)en.y * a.ext.stride_idx + a.ext.t] = sh.u0[(en.x >> 6) + 2 * kR][(en.x & 63) + 2 * kR];
  }
  if (extract_only) return;

  const int lz = lane + kR;                  // LDS row of this lane's row
  // ---- step 1: u^{n+1} on the tile plus a 4-cell halo --------------------
  {
    int q0 = 0, qend = 0;
    if (a.inj.ptr != nullptr) {
      q0 = a.inj.ptr[logical * kWaves + w];
      qend = a.inj.ptr[logical * kWaves + w + 1];
    }
    float *out = a.out + soff;
    const int cb = w * W1 + kR;              // u0 column of the wave's first column
    float q[2 * kR + 1], ql[2 * kR + 1];
#pragma unroll
    for (int k = 0; k < 2 * kR; ++k) {
      q[k] = sh.u0[cb - kR + k][lz];
      if constexpr (DF) ql[k] = bf16_f32(sh.l0[cb - kR + k][lz]);
    }
#pragma unroll
    for (int j = 0; j < W1; ++j) {
      q[2 * kR] = sh.u0[cb + j + kR][lz];
      const float c = q[kR];
      const float *col = &sh.u0[cb + j][lz];
      float lap = 0.f;
#pragma unroll
      for (int k = 1; k <= kR; ++k) {
        lap += a.cz[k - 1] * ((col[-k] - c) + (col[k] - c));
        lap += a.cx[k - 1] * ((q[kR - k] - c) + (q[kR + k] - c));
      }
      float cl = 0.f;
      if constexpr (DF) {
        ql[2 * kR] = bf16_f32(sh.l0[cb + j + kR][lz]);
        cl = ql[kR];
        const unsigned short *cll = &sh.l0[cb + j][lz];
        float lapl = 0.f;
#pragma unroll
        for (int k = 1; k <= kR; ++k) {
          lapl += a.cz[k - 1] * ((bf16_f32(cll[-k]) - cl) + (bf16_f32(cll[k]) - cl));
          lapl += a.cx[k - 1] * ((ql[kR - k] - cl) + (ql[kR + k] - cl));
        }
        lap += lapl;
      }
      float src = ds1[j];
      while (q0 < qend) {   // wave-uniform
        const int2 en = a.inj.ent[q0];
        if ((en.x >> 6) != j) break;
        const float val = a.inj.val[(long)en.y * a.inj.stride_idx + a.inj.t] * a.inj.scale;
        if ((en.x & 63) == lane) src += val;
        ++q0;
      }
      const int x = xs1 + j;
      float u1 = 0.f;
      unsigned short u1l = 0;
      if (zin && x >= 0 && x < NX) {
        const float g = gzv * a.gx[x];
        const float r = vv1[j] * (lap + src);
        if constexpr (DF) u1 = df_update(g, c, cl, pv[j], pl[j], r, u1l);
        else u1 = g * (2.f * c - g * pv[j] + r);
        if (zown && x >= x0 && x < x0 + TX) {
          const long idx = (long)x * LZ + z;
          out[idx] = u1;
          if constexpr (DF) p.lo_out[soff + idx] = u1l;
          if constexpr (T2) a.t2[(long)s * a.t2_sstride + idx] = r;
        }
      }
      sh.u1[w * W1 + j][lz] = u1;
      if constexpr (DF) sh.l1[w * W1 + j][lz] = u1l;
#pragma unroll
      for (int k = 0; k < 2 * kR; ++k) {
        q[k] = q[k + 1];
        if constexpr (DF) ql[k] = ql[k + 1];
      }
    }
  }
  if (!p.two && !ext_next) return;
  __syncthreads();

  // receivers of u^{n+1} (time t + 1)
  for (int e = e0 + tid; e < e1; e += 256) {
    const int2 en = a.ext.ent[e];
    a.ext.out[(long)en.y * a.ext.stride_idx + a.ext.t + 1] = sh.u1[(en.x >> 6) + kR][(en.x & 63) + 2 * kR];
  }
  if (!p.two) return;

  // ---- step 2: u^{n+2} on the tile ----------------------------------------
  {
    int q0 = 0, qend = 0;
    if (p.inj2.ptr != nullptr) {
      q0 = p.inj2.ptr[logical * kWaves + w];
      qend = p.inj2.ptr[logical * kWaves + w + 1];
    }
    float *out = p.out2 + soff;
    const int cb = w * W2 + kR;              // u1 column of the wave's first column
    float q[2 * kR + 1], ql[2 * kR + 1];
#pragma unroll
    for (int k = 0; k < 2 * kR; ++k) {
      q[k] = sh.u1[cb - kR + k][lz];
      if constexpr (DF) ql[k] = bf16_f32(sh.l1[cb - kR + k][lz]);
    }
#pragma unroll
    for (int j = 0; j < W2; ++j) {
      q[2 * kR] = sh.u1[cb + j + kR][lz];
      const float c = q[kR];
      const float *col = &sh.u1[cb + j][lz];
      float lap = 0.f;
#pragma unroll
      for (int k = 1; k <= kR; ++k) {
        lap += a.cz[k - 1] * ((col[-k] - c) + (col[k] - c));
        lap += a.cx[k - 1] * ((q[kR - k] - c) + (q[kR + k] - c));
      }
      float cl = 0.f;
      if constexpr (DF) {
        ql[2 * kR] = bf16_f32(sh.l1[cb + j + kR][lz]);
        cl = ql[kR];
        const unsigned short *cll = &sh.l1[cb + j][lz];
        float lapl = 0.f;
#pragma unroll
        for (int k = 1; k <= kR; ++k) {
          lapl += a.cz[k - 1] * ((bf16_f32(cll[-k]) - cl) + (bf16_f32(cll[k]) - cl));
          lapl += a.cx[k - 1] * ((ql[kR - k] - cl) + (ql[kR + k] - cl));
        }
        lap += lapl;
      }
      float src = ds2[j];
      while (q0 < qend) {   // wave-uniform
        const int2 en = p.inj2.ent[q0];
        if ((en.x >> 6) != j) break;
        const float val = p.inj2.val[(long)en.y * p.inj2.stride_idx + p.inj2.t] * p.inj2.scale;
        if ((en.x & 63) == lane) src += val;
        ++q0;
      }
      const int x = xs2 + j;
      if (zown && zin && x < NX) {
        const float g = gzv * a.gx[x];
        const float un = sh.u0[cb + j + kR][lz];
        const float r = vv2[j] * (lap + src);
        const long idx = (long)x * LZ + z;
        if constexpr (DF) {
          unsigned short l;
          out[idx] = df_update(g, c, cl, un, bf16_f32(sh.l0[cb + j + kR][lz]), r, l);
          p.lo_out2[soff + idx] = l;
        } else {
          out[idx] = g * (2.f * c - g * un + r);
        }
        if constexpr (T2) p.t2b[(long)s * a.t2_sstride + idx] = r;
      }
#pragma unroll
      for (int k = 0; k < 2 * kR; ++k) {
        q[k] = q[k + 1];
        if constexpr (DF) ql[k] = ql[k + 1];
      }
    }
  }
}

template <int TX, int MODE>
__global__ void __launch_bounds__(256) k_step2(const Step2Args p) {
  __shared__ Step2Tile<TX, (MODE & kModeDF) != 0> sh;
  const int total = p.a.ntz * p.a.ntx * p.a.nshots;
  const int per = (total + 7) >> 3;
  const int b = blockIdx.x;
  const int logical = (b & 7) * per + (b >> 3);      // XCD-contiguous tile ranges
  if (logical >= total) return;
  step2_body<TX, MODE>(p, logical, sh, false, p.two != 0);
}

// Many jobs (grids, models, geometries) in one launch, two steps per launch.
// The time index of job j is n = *step - t0_j (the counter advances by 2).
// Job j's fields rotate through buf[0..3] (prev = buf[n % 4]).  At
// n = nt_j - 2 it takes one step and samples u^n and u^{n+1}; at n = nt_j - 1
// it only samples u^n; outside [0, nt_j - 1] it is idle.
template <int TX>
__global__ void __launch_bounds__(256) k_step2_multi(const BatchJob2 *jobs, int njobs, int total, const int *step) {
  __shared__ Step2Tile<TX> sh;
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
  const BatchJob2 &jb = jobs[lo];
  const int n = *step - jb.t0;
  if (n < 0 || n > jb.nt - 1) return;
  Step2Args p = jb.p;
  p.a.prev = jb.buf[n & 3];
  p.a.cur = jb.buf[(n + 1) & 3];
  p.a.out = jb.buf[(n + 2) & 3];
  p.out2 = jb.buf[(n + 3) & 3];
  p.two = n + 2 <= jb.nt - 1;
  p.a.inj.t = n;
  p.inj2.t = n + 1;
  p.a.ext.t = n;
  step2_body<TX, kModePlain>(p, logical - jb.tile_begin, sh, n == jb.nt - 1, true);
}

hipError_t launch_step2_multi(const BatchJob2 *jobs, int njobs, int total_tiles, const int *step, int tile_x,
                              hipStream_t st) {
  const long per = (total_tiles + 7) / 8;
  const dim3 grid((unsigned)(per * 8));
  switch (tile_x) {
    case 16: k_step2_multi<16><<<grid, 256, 0, st>>>(jobs, njobs, total_tiles, step); break;
    case 32: k_step2_multi<32><<<grid, 256, 0, st>>>(jobs, njobs, total_tiles, step); break;
    case 64: k_step2_multi<64><<<grid, 256, 0, st>>>(jobs, njobs, total_tiles, step); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int TX>
static hipError_t launch_step2_tx(const Step2Args &p, int mode, hipStream_t st) {
  const long total = (long)p.a.ntz * p.a.ntx * p.a.nshots;
  const dim3 grid((unsigned)((total + 7) / 8 * 8));
  switch (mode) {
    case kModePlain: k_step2<TX, kModePlain><<<grid, 256, 0, st>>>(p); break;
    case kModeT2: k_step2<TX, kModeT2><<<grid, 256, 0, st>>>(p); break;
    case kModeDsrc: k_step2<TX, kModeDsrc><<<grid, 256, 0, st>>>(p); break;
    case kModeNu: k_step2<TX, kModeNu><<<grid, 256, 0, st>>>(p); break;
    case kModeDF: k_step2<TX, kModeDF><<<grid, 256, 0, st>>>(p); break;
    case kModeT2 | kModeDF: k_step2<TX, kModeT2 | kModeDF><<<grid, 256, 0, st>>>(p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_step2(const Step2Args &p, int tile_x, int mode, hipStream_t st) {
  switch (tile_x) {
    case 16: return launch_step2_tx<16>(p, mode, st);
    case 32: return launch_step2_tx<32>(p, mode, st);
    case 64: return launch_step2_tx<64>(p, mode, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fw

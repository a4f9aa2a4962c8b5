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
//
// Free surface (kModeFS): rows fs-4 .. fs-1 of the u^n tile are loaded from
// their mirror rows fs+4 .. fs+1 with opposite sign; u^{n+1} and u^{n+2} are
// zero at and above row fs, and the u^{n+1} tile's rows fs-4 .. fs-1 take the
// negated values of the mirror rows, which the same wavefront holds whenever
// a row below the surface reads them (a lane shuffle).
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
__device__ __forceinline__ float df_update(float g, float c, float cl, float pv, float pl, double r,
                                           unsigned short &lo) {
  const double gd = g;
  const double ex = gd * (2.0 * ((double)c + (double)cl) - gd * ((double)pv + (double)pl) + r);
  const float hi = (float)ex;
  lo = f32_bf16((float)(ex - (double)hi));
  return hi;
}

// Adds a wavefront's point sources to its per-column source registers, in list
// order (the order in which the one-step kernel adds them).  Done before the
// column march so that the march itself has no loop inside.  Lane l fetches
// entry l of each batch of 64 and its sample, so a batch costs two dependent
// loads however many entries it has; the entries are then broadcast one by
// one from registers.
template <int W>
__device__ __forceinline__ void fold_sources(const Inject &inj, int logical, int w, int lane, float (&src)[W]) {
  if (inj.ptr == nullptr) return;
  const int e1 = inj.ptr[logical * kWaves + w + 1];
  for (int b = inj.ptr[logical * kWaves + w]; b < e1; b += 64) {   // wave-uniform
    const int cnt = min(64, e1 - b);
    int key = 0;
    float val = 0.f;
    if (lane < cnt) {
      const int2 en = inj.ent[b + lane];
      key = en.x;
      val = inj.val[(long)en.y * inj.stride_idx + inj.t] * inj.scale;
    }
    for (int k = 0; k < cnt; ++k) {
      const int kx = __builtin_amdgcn_readlane(key, k);
      const float kv = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, val), k));
      const int j = kx >> 6;
      if ((kx & 63) == lane) {
#pragma unroll
        for (int jj = 0; jj < W; ++jj)
          if (jj == j) src[jj] += kv;
      }
    }
  }
}

// One 56 x TX tile of one shot; `logical` is the tile's position in the
// launch order of tile_index.  extract_only: only sample u^n.  ext_next: sample
// u^{n+1} after the first step even when no second step follows.
template <int TX, int MODE, bool EARLY2 = true>
__device__ __forceinline__ void step2_body(const Step2Args &p, int logical,
                                           Step2Tile<TX, (MODE & kModeDF) != 0> &sh, bool extract_only,
                                           bool ext_next) {
  constexpr bool T2 = (MODE & kModeT2) != 0;
  constexpr bool DS = (MODE & kModeDsrc) != 0;
  constexpr bool NU = (MODE & kModeNu) != 0;
  constexpr bool DF = (MODE & kModeDF) != 0;
  constexpr bool FS = (MODE & kModeFS) != 0;
  constexpr int C0 = Step2Tile<TX>::C0;
  constexpr int ROWS = Step2Tile<TX>::ROWS;
  constexpr int W1 = (TX + 8) / kWaves;      // step-1 columns per wave
  constexpr int W2 = TX / kWaves;            // step-2 columns per wave
  static_assert((TX + 8) % kWaves == 0 && TX % kWaves == 0 && C0 % kWaves == 0, "tile width");
  static_assert(EARLY2 || (MODE & ~kModeFS) == kModePlain, "late step-2 operand loads: plain mode only");
  const StepArgs &a = p.a;
  int txi, tzi, s;
  tile_coords(logical, a.ntz, a.ntx, a.nshots, txi, tzi, s);
  const int z0 = tzi * kTZ2;
  const int x0 = txi * TX;
  const int NZ = a.NZ, NX = a.NX, LZ = a.LZ;
  const int CB = LZ * 4;                      // bytes per column
  const unsigned FB = (unsigned)NX * (unsigned)CB;

  const long soff = (long)s * a.sstride;
  const auto r_cur = rsrc(a.cur + soff, FB);
  const auto r_prev = rsrc(a.prev + soff, FB);
  const auto r_V = rsrc(a.V, FB);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int z = z0 - kR + lane;
  const bool zin = z >= 0 && z < NZ;
  const bool zown = lane >= kR && lane < kR + kTZ2;
  const int vz = z * 4;                       // byte offset of this lane's row
  // Branch-free stores (the multi-job kernel): a row the lane does not own
  // (or outside the grid) goes past the end of the buffer, and a column the
  // wave must not write goes to a resource of size zero; the hardware drops
  // both, so no store needs an exec-mask branch.
  [[maybe_unused]] const int vz_st = zin && zown ? vz : kOutOfRange;
  [[maybe_unused]] const int vz16_st = zin && zown ? z * 2 : kOutOfRange;
  const int xs1 = x0 - kR + w * W1;          // first step-1 column of this wave
  const int xs2 = x0 + w * W2;               // first step-2 column

  // Own-row operands of both steps; their latency hides behind the tile load.
  // (the second step's operands are loaded after the first step, to keep the
  // register footprint of the first step small).  They only feed cells whose
  // results are stored, or zeroed when outside the grid, so they are read
  // unconditionally at the nearest cell inside the grid: no guard, no branch.
  const int vzc = min(max(z, 0), NZ - 1) * 4;                     // clamped row
  float pv[W1], vv1[W1], ds1[W1], pl[W1], gx1[W1];
  [[maybe_unused]] __amdgpu_buffer_rsrc_t r_ds1, r_lprev, r_lcur;
  if constexpr (DS) r_ds1 = rsrc(a.dsrc + (long)s * a.dsrc_sstride, FB);
  if constexpr (DF) {
    r_lprev = rsrc(p.lo_prev + soff, FB / 2);
    r_lcur = rsrc(p.lo_cur + soff, FB / 2);
  }
#pragma unroll
  for (int j = 0; j < W1; ++j) {
    const int xc = min(max(xs1 + j, 0), NX - 1);                 // clamped column
    gx1[j] = a.gx[xc];
    pv[j] = ld(r_prev, vzc, xc * CB);
    vv1[j] = ld(r_V, vzc, xc * CB);
    ds1[j] = pl[j] = 0.f;
    if constexpr (DS) ds1[j] = ld(r_ds1, vzc, xc * CB);
    if constexpr (DF) pl[j] = bf16_f32(ld16(r_lprev, vzc / 2, xc * (CB / 2)));
  }
  const float gzv = zin ? a.gz[z] : 0.f;
  // transposed second time difference of the e ring: step 1 reads slots
  // (k-1, k, k+1) on the halo, step 2 slots (k-2, k-1, k) on the tile; the
  // values are combined once every load of the prologue is in flight
  [[maybe_unused]] float em1[W1], e01[W1], ep1[W1];
  if constexpr (NU) {
    const long so = (long)s * a.nu.sstride;
    const auto rm = rsrc(a.nu.em + so, FB), r0 = rsrc(a.nu.e0 + so, FB), rp = rsrc(a.nu.ep + so, FB);
#pragma unroll
    for (int j = 0; j < W1; ++j) {
      const int xc = min(max(xs1 + j, 0), NX - 1);
      em1[j] = ld(rm, vzc, xc * CB);
      e01[j] = ld(r0, vzc, xc * CB);
      ep1[j] = ld(rp, vzc, xc * CB);
    }
  }

  float vv2[W2], ds2[W2], gx2[W2];
  auto load_step2_operands = [&]() {
#pragma unroll
    for (int j = 0; j < W2; ++j) {
      const int xc = min(xs2 + j, NX - 1);
      gx2[j] = a.gx[xc];
      vv2[j] = ld(r_V, vzc, xc * CB);
      ds2[j] = 0.f;
    }
  };

  // u^n tile, one column per wavefront access: lane = row z0 - 8 + lane, and
  // lanes 0..7 also row z0 + 56 + lane.  No branch: a cell outside the grid
  // gets a per-lane offset past the end of the buffer (the whole offset is in
  // the per-lane register, which the range check covers), so it reads as
  // zero, and every load of the tile is in flight before the first LDS write
  // waits for one.
  {
    constexpr int NC = C0 / kWaves;
    constexpr int kOut = kOutOfRange;
    const int zt = z0 - 2 * kR + lane;
    const bool zt_in = zt >= 0 && zt < NZ;
    const bool zt2_in = lane < 2 * kR && zt + 64 < NZ;
    float v[NC], v2[NC];
    [[maybe_unused]] unsigned short l[NC], l2[NC];
    // rows read for the two loads of this lane (mirrored under a free surface)
    [[maybe_unused]] float sg = 1.f, sg2 = 1.f;
    int zr = zt, zr2 = zt + 64;
    if constexpr (FS) {
      zr = fs_mirror_row(zt, a.fs, sg);
      zr2 = fs_mirror_row(zt + 64, a.fs, sg2);
    }
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      const int x = x0 - 2 * kR + w + kWaves * i;
      const bool xin = x >= 0 && x < NX;      // wave-uniform
      const int o1 = xin && zt_in ? x * CB + zr * 4 : kOut;
      const int o2 = xin && zt2_in ? x * CB + zr2 * 4 : kOut;
      v[i] = ld(r_cur, o1, 0);
      v2[i] = ld(r_cur, o2, 0);
      if constexpr (DF) {
        l[i] = ld16(r_lcur, o1 == kOut ? kOut : o1 / 2, 0);
        l2[i] = ld16(r_lcur, o2 == kOut ? kOut : o2 / 2, 0);
      }
    }
    if constexpr (FS) {
#pragma unroll
      for (int i = 0; i < NC; ++i) {
        v[i] *= sg;
        v2[i] *= sg2;
        if constexpr (DF) {
          if (sg < 0.f) l[i] ^= 0x8000u;           // BF16 sign flip
          if (sg2 < 0.f) l2[i] ^= 0x8000u;
        }
      }
    }
    if constexpr (NU) {
      // the e values were issued before the tile: waiting for them here
      // leaves the tile loads in flight
      const float gzc = a.gz[vzc / 4];       // taper at the clamped row (nonzero)
#pragma unroll
      for (int j = 0; j < W1; ++j) {
        const float g = gzc * gx1[j];
        ds1[j] += em1[j] / g - 2.f * e01[j] + g * ep1[j];
      }
    }
    // Step 2's own-row operands, issued now so that their latency hides
    // behind the tile load and step 1 (EARLY2; the multi-job kernel, short of
    // registers, loads them at step 2).  Clamped like step 1's; with a single
    // step the step-1 source stands in for the (absent) second one, so every
    // address is valid and no load sits behind a branch.
    if constexpr (EARLY2) load_step2_operands();
    if constexpr (DS) {
      const auto r_ds2 = rsrc((p.two ? p.dsrc2 : a.dsrc) + (long)s * a.dsrc_sstride, FB);
#pragma unroll
      for (int j = 0; j < W2; ++j) ds2[j] = ld(r_ds2, vzc, min(xs2 + j, NX - 1) * CB);
    }
    // Lanes 8..63 put their (zero) second value into this wave's own column
    // of the u^{n+1} tile, which step 1 overwrites after the barrier: a write
    // without a branch keeps the compiler from moving those loads into one.
    const bool lo8 = lane < 2 * kR;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      const int c = w + kWaves * i;
      sh.u0[c][lane] = v[i];
      *(lo8 ? &sh.u0[c][64 + lane] : &sh.u1[w][lane]) = v2[i];
      if constexpr (DF) {
        sh.l0[c][lane] = l[i];
        *(lo8 ? &sh.l0[c][64 + lane] : &sh.l1[w][lane]) = l2[i];
      }
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
  // the tile's rows z0-4 .. z0+59 reach the four rows above a free surface
  [[maybe_unused]] const bool fs_near = FS && a.fs >= 0 && z0 - kR <= a.fs - 1 && z0 + kTZ2 + kR - 1 >= a.fs - kR;
  // The low part of the extended-precision field is a rounding residual
  // (below 2^-24 of the field): its Laplacian needs only a few correct
  // digits, so it is summed directly, sum_k w_k (l(-k) + l(k)) + w_0 l, with
  // w_0 = -2 sum_k w_k, instead of in difference form.
  [[maybe_unused]] float c0l = 0.f;
  if constexpr (DF) {
#pragma unroll
    for (int k = 0; k < kR; ++k) c0l -= 2.f * (a.cz[k] + a.cx[k]);
  }
  // ---- step 1: u^{n+1} on the tile plus a 4-cell halo --------------------
  {
    fold_sources<W1>(a.inj, logical, w, lane, ds1);
    const auto r_out = rsrc(a.out + soff, FB);
    [[maybe_unused]] __amdgpu_buffer_rsrc_t r_t2, r_lout;
    if constexpr (T2) r_t2 = rsrc(a.t2 + (long)s * a.t2_sstride, FB);
    if constexpr (DF) r_lout = rsrc(p.lo_out + soff, FB / 2);
    // all 17 stencil operands come straight from LDS at fixed offsets from
    // one per-lane base (a register queue along x costs a move per operand)
    const float *base = &sh.u0[w * W1 + kR][lz];                   // u0 column of the wave's first column
    [[maybe_unused]] const unsigned short *basel = nullptr;
    if constexpr (DF) basel = &sh.l0[w * W1 + kR][lz];
    // forward x-differences d[k][j] = u(j + k) - u(j): the backward one of
    // column j, u(j - k) - u(j), is -d[k][j - k] (exact), so each difference
    // along x is formed once
    float dxf[kR][W1];
#pragma unroll
    for (int j = 0; j < W1; ++j) {
      const float *col = base + j * ROWS;
      const float c = col[0];
      float lap = 0.f;
      // extended precision: the neighbour differences (exact or nearly, in
      // FP32) are summed and weighted in FP64, so the Laplacian carries no
      // FP32 accumulation error into the update
      [[maybe_unused]] double lapd = 0.0;
#pragma unroll
      for (int k = 1; k <= kR; ++k) {
        dxf[k - 1][j] = col[k * ROWS] - c;
        const float back = j >= k ? -dxf[k - 1][j - k] : col[-k * ROWS] - c;
        if constexpr (DF) {
          lapd = fma((double)a.cz[k - 1], (double)(col[-k] - c) + (double)(col[k] - c), lapd);
          lapd = fma((double)a.cx[k - 1], (double)back + (double)dxf[k - 1][j], lapd);
        } else {
          lap += a.cz[k - 1] * ((col[-k] - c) + (col[k] - c));
          lap += a.cx[k - 1] * (back + dxf[k - 1][j]);
        }
      }
      float cl = 0.f;
      if constexpr (DF) {
        const unsigned short *cll = basel + j * ROWS;
        cl = bf16_f32(cll[0]);
        float lapl = c0l * cl;
#pragma unroll
        for (int k = 1; k <= kR; ++k) {
          lapl += a.cz[k - 1] * (bf16_f32(cll[-k]) + bf16_f32(cll[k]));
          lapl += a.cx[k - 1] * (bf16_f32(cll[-k * ROWS]) + bf16_f32(cll[k * ROWS]));
        }
        lapd += (double)lapl;
      }
      const int x = xs1 + j;
      const bool xin = x >= 0 && x < NX;     // wave-uniform
      // computed for every lane; cells outside the grid are set to zero
      const float g = gzv * gx1[j];
      [[maybe_unused]] double r64 = 0.0;
      if constexpr (DF) r64 = (double)vv1[j] * (lapd + (double)ds1[j]);
      const float r = DF ? (float)r64 : vv1[j] * (lap + ds1[j]);
      unsigned short u1l = 0;
      float u1;
      if constexpr (DF) u1 = df_update(g, c, cl, pv[j], pl[j], r64, u1l);
      else u1 = g * (2.f * c - g * pv[j] + r);
      if (!(xin && zin)) {
        u1 = 0.f;
        u1l = 0;
      }
      [[maybe_unused]] float rs = r;
      if constexpr (FS) {
        if (z <= a.fs) {                      // at and above the free surface
          u1 = rs = 0.f;
          u1l = 0;
        }
      }
      if constexpr (!EARLY2) {
        const bool xst = xin && x >= x0 && x < x0 + TX;             // wave-uniform
        st(rsrc(a.out + soff, xst ? FB : 0u), u1, vz_st, x * CB);
        if constexpr (DF) st16(rsrc(p.lo_out + soff, xst ? FB / 2 : 0u), u1l, vz16_st, x * (CB / 2));
        if constexpr (T2) st(rsrc(a.t2 + (long)s * a.t2_sstride, xst ? FB : 0u), FS ? rs : r, vz_st, x * CB);
      } else if (xin && x >= x0 && x < x0 + TX) {                   // wave-uniform
        if (zin && zown) {
          st(r_out, u1, vz, x * CB);
          if constexpr (DF) st16(r_lout, u1l, z * 2, x * (CB / 2));
          if constexpr (T2) st(r_t2, FS ? rs : r, vz, x * CB);
        }
      }
      float u1t = u1;
      [[maybe_unused]] unsigned short u1lt = u1l;
      if constexpr (FS) {
        // rows fs-4 .. fs-1 of the tile: the negated mirror row 2 fs - z,
        // held by lane 2 (fs - z0 + 4) - lane of this wavefront
        if (fs_near) {                        // workgroup-uniform
          const int src = ((2 * (a.fs - z0 + kR) - lane) & 63) << 2;
          const float m = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(src, __builtin_bit_cast(int, u1)));
          [[maybe_unused]] int ml = 0;
          if constexpr (DF) ml = __builtin_amdgcn_ds_bpermute(src, (int)u1l);
          if (fs_mirrored(z, a.fs)) {
            u1t = -m;
            if constexpr (DF) u1lt = (unsigned short)(ml ^ 0x8000);
          }
        }
      }
      sh.u1[w * W1 + j][lz] = u1t;
      if constexpr (DF) sh.l1[w * W1 + j][lz] = u1lt;
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
    if constexpr (!EARLY2) load_step2_operands();
    if constexpr (NU) {
      const long so = (long)s * a.nu.sstride;
      const auto rm2 = rsrc(p.nu2.em + so, FB), r02 = rsrc(p.nu2.e0 + so, FB), rp2 = rsrc(p.nu2.ep + so, FB);
      const float gzc = a.gz[vzc / 4];
#pragma unroll
      for (int j = 0; j < W2; ++j) {
        const int xc = min(xs2 + j, NX - 1);
        const float g = gzc * gx2[j];
        ds2[j] += ld(rm2, vzc, xc * CB) / g - 2.f * ld(r02, vzc, xc * CB) + g * ld(rp2, vzc, xc * CB);
      }
    }
    fold_sources<W2>(p.inj2, logical, w, lane, ds2);
    const auto r_out = rsrc(p.out2 + soff, FB);
    [[maybe_unused]] __amdgpu_buffer_rsrc_t r_t2, r_lout;
    if constexpr (T2) r_t2 = rsrc(p.t2b + (long)s * a.t2_sstride, FB);
    if constexpr (DF) r_lout = rsrc(p.lo_out2 + soff, FB / 2);
    const int cb = w * W2 + kR;              // u1 column of the wave's first column
    const float *base = &sh.u1[cb][lz];
    const float *base0 = &sh.u0[cb + kR][lz];                      // u^n at the wave's first column
    [[maybe_unused]] const unsigned short *basel = nullptr, *basel0 = nullptr;
    if constexpr (DF) {
      basel = &sh.l1[cb][lz];
      basel0 = &sh.l0[cb + kR][lz];
    }
    float dxf[kR][W2];                       // forward x-differences, as in step 1
#pragma unroll
    for (int j = 0; j < W2; ++j) {
      const float *col = base + j * ROWS;
      const float c = col[0];
      float lap = 0.f;
      // extended precision: the neighbour differences (exact or nearly, in
      // FP32) are summed and weighted in FP64, so the Laplacian carries no
      // FP32 accumulation error into the update
      [[maybe_unused]] double lapd = 0.0;
#pragma unroll
      for (int k = 1; k <= kR; ++k) {
        dxf[k - 1][j] = col[k * ROWS] - c;
        const float back = j >= k ? -dxf[k - 1][j - k] : col[-k * ROWS] - c;
        if constexpr (DF) {
          lapd = fma((double)a.cz[k - 1], (double)(col[-k] - c) + (double)(col[k] - c), lapd);
          lapd = fma((double)a.cx[k - 1], (double)back + (double)dxf[k - 1][j], lapd);
        } else {
          lap += a.cz[k - 1] * ((col[-k] - c) + (col[k] - c));
          lap += a.cx[k - 1] * (back + dxf[k - 1][j]);
        }
      }
      float cl = 0.f;
      if constexpr (DF) {
        const unsigned short *cll = basel + j * ROWS;
        cl = bf16_f32(cll[0]);
        float lapl = c0l * cl;
#pragma unroll
        for (int k = 1; k <= kR; ++k) {
          lapl += a.cz[k - 1] * (bf16_f32(cll[-k]) + bf16_f32(cll[k]));
          lapl += a.cx[k - 1] * (bf16_f32(cll[-k * ROWS]) + bf16_f32(cll[k * ROWS]));
        }
        lapd += (double)lapl;
      }
      const int x = xs2 + j;
      const bool xin = x < NX;               // wave-uniform
      const float g = gzv * gx2[j];
      const float un = base0[j * ROWS];
      [[maybe_unused]] double r64 = 0.0;
      if constexpr (DF) r64 = (double)vv2[j] * (lapd + (double)ds2[j]);
      const float r = DF ? (float)r64 : vv2[j] * (lap + ds2[j]);
      unsigned short u2l = 0;
      float u2;
      if constexpr (DF) u2 = df_update(g, c, cl, un, bf16_f32(basel0[j * ROWS]), r64, u2l);
      else u2 = g * (2.f * c - g * un + r);
      [[maybe_unused]] float rs = r;
      if constexpr (FS) {
        if (z <= a.fs) {                      // at and above the free surface
          u2 = rs = 0.f;
          u2l = 0;
        }
      }
      if constexpr (!EARLY2) {
        st(rsrc(p.out2 + soff, xin ? FB : 0u), u2, vz_st, x * CB);
        if constexpr (DF) st16(rsrc(p.lo_out2 + soff, xin ? FB / 2 : 0u), u2l, vz16_st, x * (CB / 2));
        if constexpr (T2) st(rsrc(p.t2b + (long)s * a.t2_sstride, xin ? FB : 0u), FS ? rs : r, vz_st, x * CB);
      } else if (xin) {
        if (zown && zin) {
          st(r_out, u2, vz, x * CB);
          if constexpr (DF) st16(r_lout, u2l, z * 2, x * (CB / 2));
          if constexpr (T2) st(r_t2, FS ? rs : r, vz, x * CB);
        }
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

// Workgroups per CU that the multi-job tile's LDS allows (at most 8).  The
// kernel is held to the registers of that many workgroups: without the
// bound, the branch-free stores let the compiler keep more operands live and
// cost a wavefront per SIMD.  Width 24 (LDS for 7) needs 73 registers, one
// more than 7 workgroups leave, so it is held to 6 rather than spill.
template <int TX>
constexpr int step2_multi_blocks() {
  constexpr int n = 163840 / (int)sizeof(Step2Tile<TX>);
  return TX == 24 ? 6 : n < 8 ? n : 8;
}

// Many jobs (grids, models, geometries) in one launch, two steps per launch.
// The time index of job j is n = step - t0_j, with step read from device
// memory (*step, advanced by 2 per launch under graph replay) or, when that
// pointer is null, the launch argument step_val.
// Job j's fields rotate through buf[0..3] (prev = buf[n % 4]).  At
// n = nt_j - 2 it takes one step and samples u^n and u^{n+1}; at n = nt_j - 1
// it only samples u^n; outside [0, nt_j - 1] it is idle.
template <int TX, int MODE>
__global__ void __launch_bounds__(256, step2_multi_blocks<TX>()) k_step2_multi(const BatchJob2 *jobs,
                                                                              const int *tile_job, int njobs,
                                                                              int total, const int *step,
                                                                              int step_val) {
  __shared__ Step2Tile<TX> sh;
  const int per = (total + 7) >> 3;
  const int b = blockIdx.x;
  const int logical = (b & 7) * per + (b >> 3);
  if (logical >= total) return;
  int lo = 0;                                       // last job with tile_begin <= logical
  if (tile_job) {
    lo = tile_job[logical];
  } else {
    int hi = njobs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (jobs[mid].tile_begin <= logical) lo = mid;
      else hi = mid - 1;
    }
  }
  const BatchJob2 &jb = jobs[lo];
  const int n = (step ? *step : step_val) - jb.t0;
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
  step2_body<TX, MODE, false>(p, logical - jb.tile_begin, sh, n == jb.nt - 1, true);
}

template <int TX>
static void launch_step2_multi_tx(dim3 grid, const BatchJob2 *jobs, const int *tile_job, int njobs, int total_tiles,
                                  const int *step, int step_val, bool fs, hipStream_t st) {
  if (fs) k_step2_multi<TX, kModeFS><<<grid, 256, 0, st>>>(jobs, tile_job, njobs, total_tiles, step, step_val);
  else k_step2_multi<TX, kModePlain><<<grid, 256, 0, st>>>(jobs, tile_job, njobs, total_tiles, step, step_val);
}

hipError_t launch_step2_multi(const BatchJob2 *jobs, const int *tile_job, int njobs, int total_tiles, const int *step,
                              int step_val, int tile_x, bool fs, hipStream_t st) {
  const long per = (total_tiles + 7) / 8;
  const dim3 grid((unsigned)(per * 8));
  switch (tile_x) {
    case 16: launch_step2_multi_tx<16>(grid, jobs, tile_job, njobs, total_tiles, step, step_val, fs, st); break;
    case 24: launch_step2_multi_tx<24>(grid, jobs, tile_job, njobs, total_tiles, step, step_val, fs, st); break;
    case 32: launch_step2_multi_tx<32>(grid, jobs, tile_job, njobs, total_tiles, step, step_val, fs, st); break;
    case 48: launch_step2_multi_tx<48>(grid, jobs, tile_job, njobs, total_tiles, step, step_val, fs, st); break;
    case 64: launch_step2_multi_tx<64>(grid, jobs, tile_job, njobs, total_tiles, step, step_val, fs, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int TX>
static hipError_t launch_step2_tx(const Step2Args &p, int mode, hipStream_t st) {
  const long total = (long)p.a.ntz * p.a.ntx * p.a.nshots;
  const dim3 grid((unsigned)((total + 7) / 8 * 8));
  if (p.a.fs >= 0) mode |= kModeFS;
  switch (mode) {
#define FW_STEP2_MODE(M)                                     \
  case M: k_step2<TX, M><<<grid, 256, 0, st>>>(p); break;    \
  case M | kModeFS: k_step2<TX, M | kModeFS><<<grid, 256, 0, st>>>(p); break;
    FW_STEP2_MODE(kModePlain)
    FW_STEP2_MODE(kModeT2)
    FW_STEP2_MODE(kModeDsrc)
    FW_STEP2_MODE(kModeT2 | kModeDsrc)
    FW_STEP2_MODE(kModeNu)
    FW_STEP2_MODE(kModeDF)
    FW_STEP2_MODE(kModeT2 | kModeDF)
    FW_STEP2_MODE(kModeDsrc | kModeDF)
#undef FW_STEP2_MODE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_step2(const Step2Args &p, int tile_x, int mode, hipStream_t st) {
  switch (tile_x) {
    case 16: return launch_step2_tx<16>(p, mode, st);
    case 24: return launch_step2_tx<24>(p, mode, st);
    case 32: return launch_step2_tx<32>(p, mode, st);
    case 48: return launch_step2_tx<48>(p, mode, st);
    case 64: return launch_step2_tx<64>(p, mode, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fw

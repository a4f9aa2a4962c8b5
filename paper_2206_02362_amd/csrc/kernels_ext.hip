// Horizontal subsurface-offset kernels (gfx950, wave64): the extended
// scattering source of B~, its transpose (the spread of the receiver-side
// field used by the tomographic gradient), the extended imaging condition of
// B~^T, the per-cell gradient accumulation and the small finalizers.
//
// In all of them lane = model-grid depth z, so every global access of a
// wavefront is one contiguous 256-byte run of a z-fastest column; offsets act
// along x only.  Time is handled in chunks: a kernel call consumes nk stored
// time slots at once, so the coefficient field (nh x model grid) and the
// image accumulator are touched once per chunk instead of once per step.
#include "internal.h"

#include <algorithm>
#include <cstdlib>
#include <string>

namespace fw {

// Raw buffer access: a load whose byte offset falls outside [0, bytes) of the
// resource returns 0 in hardware (negative offsets wrap to large unsigned
// values).  Window staging relies on this to drop the terms whose column lies
// outside the padded grid without any per-element test, so the whole offset
// goes in the vector operand: the scalar offset is not range-checked.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t slot_rsrc(const float *base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, int byte_off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}

// (shot, slot, ring position) of consecutive flat slot indices q = s nk + n,
// advanced without an integer division per slot.  ring == 0: position = n;
// otherwise position = (first + n) mod ring (slots n < nk <= ring).
struct SlotCursor {
  int s, n, r, nk, ring, f0;
  __device__ void init(int q, int nk_, int first, int ring_) {
    nk = nk_;
    ring = ring_;
    s = q / nk;
    n = q - s * nk;
    f0 = ring ? first % ring : 0;
    r = ring ? (f0 + n) % ring : n;
  }
  __device__ void next() {
    if (++n == nk) {
      n = 0;
      ++s;
      r = f0;
      return;
    }
    ++r;
    if (ring && r == ring) r = 0;
  }
};

// SlotCursor that also carries the element offset s sstride + r slot of its
// position, advanced by one add per slot (the products are formed once per
// shot only).
struct OffCursor {
  SlotCursor c;
  long off, slot, sstride;
  __device__ void init(int q, int nk, int first, int ring, long slot_, long sstride_) {
    c.init(q, nk, first, ring);
    slot = slot_;
    sstride = sstride_;
    off = (long)c.s * sstride + (long)c.r * slot;
  }
  __device__ void next() {
    const int s0 = c.s;
    c.next();
    if (c.s != s0) off = (long)c.s * sstride + (long)c.r * slot;
    else if (c.r == 0) off -= (long)(c.ring - 1) * slot;   // ring wrap (ring > 0)
    else off += slot;
  }
};

// ---------------------------------------------------------------------------
// c(z,y,h) = 2 p~(z,y,h) / (v(z,y)^3 dt^2), model grid, [nh][nx][nz]
// ---------------------------------------------------------------------------
__global__ void k_ext_coef(const float *pt, const float *vel, int nz, int nx, int nh, float dt, float *coef) {
  const long n = (long)nh * nx * nz;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const long cell = i % ((long)nx * nz);
    const float v = vel[cell];
    coef[i] = 2.f * pt[i] / (v * v * v * dt * dt);
  }
}

hipError_t launch_ext_coef(const float *ptilde, const float *vel, const ExtGeom &g, float dt, float *coef,
                           hipStream_t st) {
  const long n = (long)g.nh * g.nx * g.nz;
  long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  k_ext_coef<<<(unsigned)blocks, 256, 0, st>>>(ptilde, vel, g.nz, g.nx, g.nh, dt, coef);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scatter (sg = +1) / spread (sg = -1):
//   out_n(z, j) = sum_h c(z, j - sg h, h) in_n(z, j - 2 sg h)
//
// Weight-stationary: the offset weights of an output column are loaded once
// per launch into registers and reused for every time slot of every shot.
// Out-of-grid input columns read as zero and out-of-model weights are zero,
// which drops exactly the terms the operator drops.  Requires H <= HMAX (30);
// larger offset counts use the generic kernel further below.
// ---------------------------------------------------------------------------
struct ScatterArgs {
  const float *coef;
  const float *in;
  float *out;
  long in_slot, out_slot, sstride;
  int in_ring, in_first, out_ring, out_first;
  int nz, nx, nb, NX, LZ, nh, H, sg;
  int j0, nj;       // writable padded columns [j0, j0 + nj)
  int nzs;          // z strips
  int zpad;         // rows of the first strip above the model (direct-load kernel)
  int nk, nshots;
  int slots_per_block;
};

// Pipelined weight-stationary kernel, register-staged (k_ext_scatter_ws; the
// direct-load kernel further below is the default).  A workgroup of 8 wavefronts owns 16
// consecutive output columns of one 64-row depth strip; wavefront w holds the
// weights of two same-parity columns ja and ja + 2 in registers for every h.
// Input windows [jb - 2H, jb + 16 + 2H) of successive time slots flow through a
// 3-deep LDS ring: slot q is consumed while slot q + 1 is written from
// registers and the global loads of slot q + 2 are in flight, with one barrier
// per slot.  Each wavefront forms its two outputs with 2 nh multiply-adds from
// nh + 1 LDS reads.
constexpr int kScJB = 16;         // output columns per workgroup of the register-staged kernel
constexpr int kScThreads = 512;
constexpr int kScMaxSlots = 2048; // time slots per workgroup of the direct-load kernel (offset table in LDS)

// a value the whole wavefront read from the same LDS cell, as a scalar
__device__ __forceinline__ long wave_uniform(long v) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((unsigned long)v >> 32));
  return (long)(((unsigned long)hi << 32) | lo);
}

template <int HMAX, int SG>
__global__ void __launch_bounds__(kScThreads) k_ext_scatter_ws(const ScatterArgs a) {
  constexpr int NH = 2 * HMAX + 1;
  constexpr int WMAX = kScJB + 4 * HMAX;                          // staged columns
  constexpr int PER = (WMAX + 7) / 8;                             // staged rows per thread
  __shared__ float ring[3][WMAX * 64];

  // XCD-contiguous order: hardware workgroup b runs on XCD b % 8; give each
  // XCD a contiguous range of (strip, column block) tiles so the overlapping
  // input windows of neighbouring tiles are served by that XCD's L2.
  const int nblk_j = (a.nj + kScJB - 1) / kScJB;
  const int ntile = a.nzs * nblk_j;
  const int per = (ntile + 7) >> 3;
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= ntile) return;
  const int zs = tile % a.nzs;
  const int jbk = tile / a.nzs;
  const int jb = a.j0 + jbk * kScJB;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int z = zs * 64 + lane;
  const bool zin = z < a.nz;
  const int zp = a.nb + z;
  const int H = a.H;
  const int col0 = jb - 2 * HMAX;                       // padded column of ring row 0 (window sized for HMAX)
  const int ja = jb + (w & 1) + 4 * (w >> 1);
  const int jc = ja + 2;
  const int jend = a.j0 + a.nj;

  float ca[NH], cb[NH];
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    const int ih = k - HMAX;
    float va = 0.f, vb = 0.f;
    if (ih >= -H && ih <= H && zin) {
      const int ya = ja - SG * ih - a.nb, yc = jc - SG * ih - a.nb;
      const long hb = (long)(ih + H) * a.nx;
      if (ya >= 0 && ya < a.nx) va = a.coef[(hb + ya) * a.nz + z];
      if (yc >= 0 && yc < a.nx) vb = a.coef[(hb + yc) * a.nz + z];
    }
    ca[k] = va;
    cb[k] = vb;
  }

  const int total = a.nshots * a.nk;
  const int q0 = blockIdx.y * a.slots_per_block;
  const int q1 = min(total, q0 + a.slots_per_block);
  if (q0 >= q1) return;

  // thread (w, lane) stages ring rows w + 8 r (r < PER) at depth lane; columns
  // outside [0, NX) come back as zero from the bounds-checked buffer load
  const unsigned slot_bytes = (unsigned)((long)a.NX * a.LZ * 4);
  const int off0 = ((col0 + w) * a.LZ + zp) * 4;
  const int rstep = 8 * a.LZ * 4;
  // (slot indices are recomputed per slot here: cursors held in scalar
  // registers push this register-bound kernel into spills)
  auto fetch = [&](int q, float (&pre)[PER]) {
    if (q >= q1) return;
    const int s = q / a.nk, n = q - s * a.nk;
    const long sl = a.in_ring ? (long)((a.in_first + n) % a.in_ring) : (long)n;
    const auto rs = slot_rsrc(a.in + (long)s * a.sstride + sl * a.in_slot, slot_bytes);
#pragma unroll
    for (int r = 0; r < PER; ++r) pre[r] = bload(rs, off0 + r * rstep);
  };
  auto put = [&](int slot_buf, const float (&pre)[PER]) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int c = w + 8 * r;
      if (c < WMAX) ring[slot_buf][c * 64 + lane] = pre[r];
    }
  };
  auto consume = [&](int q, int rbuf) {
    const float *row = &ring[rbuf][(ja - col0) * 64 + lane];   // input column ja
    float oa = 0.f, ob = 0.f;
#pragma unroll
    for (int k = 0; k < NH; ++k) {
      const int ih = k - HMAX;
      // input column of (ja, ih) is ja - 2 sg ih; of (ja + 2, ih) two further.
      // Weights of |ih| > H are zero and their rows lie inside the window.
      oa += ca[k] * row[-2 * SG * ih * 64];
      ob += cb[k] * row[(2 - 2 * SG * ih) * 64];
    }
    const int s = q / a.nk, n = q - s * a.nk;
    const long sl = a.out_ring ? (long)((a.out_first + n) % a.out_ring) : (long)n;
    float *dst = a.out + (long)s * a.sstride + sl * a.out_slot;
    if (zin) {
      if (ja < jend) dst[(long)ja * a.LZ + zp] = oa;
      if (jc < jend) dst[(long)jc * a.LZ + zp] = ob;
    }
  };

  // ring[rb] holds slot q; pA / pB hold the two following slots
  float pA[PER], pB[PER];
  fetch(q0, pA);
  put(0, pA);
  fetch(q0 + 1, pA);
  fetch(q0 + 2, pB);
  __syncthreads();
  int rb = 0;
  for (int q = q0; q < q1; q += 2) {
    int nb1 = rb == 2 ? 0 : rb + 1;
    consume(q, rb);
    if (q + 1 < q1) put(nb1, pA);
    fetch(q + 3, pA);
    __syncthreads();
    rb = nb1;
    if (q + 1 >= q1) break;
    nb1 = rb == 2 ? 0 : rb + 1;
    consume(q + 1, rb);
    if (q + 2 < q1) put(nb1, pB);
    fetch(q + 4, pB);
    __syncthreads();
    rb = nb1;
  }
}

// Same operator, input windows brought in by direct global-to-LDS loads
// (buffer loads with the LDS as destination) into a 4-deep ring: three slots
// are in flight while one is consumed, and no registers are spent on
// staging.  Each load moves 16 bytes per lane (lane i fills LDS bytes
// [16 i, 16 i + 16) from M0), i.e. four 64-deep columns per instruction; a
// wavefront's padding loads, when the window's chunk count is not a multiple
// of 8, read past the end of the buffer (zeros, no memory traffic) into a
// sink.  Before the barrier that publishes slot q each wavefront waits until
// its own loads of slot q have landed; the loads of the two younger slots may
// still be outstanding (vector memory operations complete in order).  The
// barrier is a bare s_barrier: a fenced one would wait for every outstanding
// load.
//
// A workgroup owns the 24 output columns of one parity in a 48-column block;
// wavefront w holds the weights of three same-parity columns (ja, ja + 2,
// ja + 4) in registers, so each LDS read of the window feeds up to three
// multiply-adds.  The 64-row strips start a.zpad rows above the model, on a
// 64-byte boundary of the (256-byte aligned) padded column, so every 256-byte
// run a wavefront loads or stores covers whole 64-byte memory sectors.
constexpr int kScDmaJB = 24;      // outputs of one parity per workgroup of the direct-load kernel

typedef __attribute__((address_space(3))) void lds_void_t;

// s_waitcnt vmcnt(min(n, N)) for a wave-uniform n, other counters untouched
template <int N>
__device__ __forceinline__ void wait_vmcnt_at_most(int n) {
  if constexpr (N > 0) {
    if (n >= N) {
      __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
      return;
    }
    wait_vmcnt_at_most<N - 1>(n);
  } else {
    __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));
  }
}

template <int HMAX, int SG>
__global__ void __launch_bounds__(kScThreads) k_ext_scatter_dma(const ScatterArgs a) {
  constexpr int NH = 2 * HMAX + 1;
  constexpr int WMAX = kScDmaJB + 2 * HMAX;                       // staged same-parity columns
  constexpr int NCH = (WMAX + 3) / 4;                             // 4-column chunks per slot
  constexpr int PER = (NCH + 7) / 8;                              // chunk loads per wavefront and slot
  static_assert(2 * PER + 9 <= 63, "window");
  __shared__ float b0[NCH * 256], b1[NCH * 256], b2[NCH * 256], b3[NCH * 256];
  __shared__ float sink[256];                                     // destination of the padding loads

  // every input column the workgroup's outputs read has their parity, so
  // the window holds only those (m = 0 .. WMAX - 1 <-> padded column col0 + 2 m)
  const int nblk_j = (a.nj + 2 * kScDmaJB - 1) / (2 * kScDmaJB);
  const int ntile = a.nzs * nblk_j * 2;
  const int per = (ntile + 7) >> 3;
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (tile >= ntile) return;
  // column blocks fastest: the workgroups that run together on one XCD
  // cover a wide run of columns of one strip, whose overlapping windows
  // then come from that XCD's L2 rather than from HBM
  const int jbk = tile % nblk_j;
  const int par = (tile / nblk_j) & 1;
  const int zs = tile / nblk_j >> 1;
  const int jb = a.j0 + jbk * 2 * kScDmaJB + par;                 // first output column
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int z = zs * 64 + lane - a.zpad;                          // model row of this lane
  const bool zin = z >= 0 && z < a.nz;
  const int zp = a.nb + z;
  const int H = a.H;
  const int col0 = jb - 2 * HMAX;
  const int ja = jb + 6 * w;                                      // outputs k = 3 w .. 3 w + 2
  const int jc = ja + 2, je = ja + 4;
  const int jend = a.j0 + a.nj;

  float ca[NH], cb[NH], cc[NH];
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    const int ih = k - HMAX;
    float va = 0.f, vb = 0.f, vc = 0.f;
    if (ih >= -H && ih <= H && zin) {
      const int ya = ja - SG * ih - a.nb, yc = jc - SG * ih - a.nb, ye = je - SG * ih - a.nb;
      const long hb = (long)(ih + H) * a.nx;
      if (ya >= 0 && ya < a.nx) va = a.coef[(hb + ya) * a.nz + z];
      if (yc >= 0 && yc < a.nx) vb = a.coef[(hb + yc) * a.nz + z];
      if (ye >= 0 && ye < a.nx) vc = a.coef[(hb + ye) * a.nz + z];
    }
    ca[k] = va;
    cb[k] = vb;
    cc[k] = vc;
  }

  const int total = a.nshots * a.nk;
  const int q0 = blockIdx.y * a.slots_per_block;
  const int q1 = min(total, q0 + a.slots_per_block);
  if (q0 >= q1) return;
  const unsigned slot_bytes = (unsigned)((long)a.NX * a.LZ * 4);
  // lane i of a chunk load: window column m = 4 g + i / 16 (padded column
  // col0 + 2 m), rows 4 (i % 16) .. + 3 of the strip; columns left of the
  // grid give negative offsets, which wrap past the end of the buffer and
  // read as zero like those right of it
  const int off0 = (col0 * a.LZ + a.nb - a.zpad + zs * 64) * 4 + (2 * (lane >> 4) * a.LZ + 4 * (lane & 15)) * 4;
  const int gstep = 8 * a.LZ * 4;                                 // bytes per chunk of 4 window columns
  // cells not written go past the end of the buffer and are dropped
  const int oa_off = zin && ja < jend ? (ja * a.LZ + zp) * 4 : kOutOfRange;
  const int oc_off = zin && jc < jend ? (jc * a.LZ + zp) * 4 : kOutOfRange;
  const int oe_off = zin && je < jend ? (je * a.LZ + zp) * 4 : kOutOfRange;

  // element offsets of the workgroup's input and output slots, computed once
  // (slot q is shot s = q / nk, step n = q mod nk, at ring position
  // (first + n) mod ring, or n without a ring), so that the per-slot scalar
  // work is two table reads instead of two cursor updates with branches
  __shared__ long tin[kScMaxSlots], tout[kScMaxSlots];
  for (int i = tid; i < q1 - q0; i += kScThreads) {
    const int q = q0 + i;
    const int sh = q / a.nk, n = q - sh * a.nk;
    const int ri = a.in_ring ? (a.in_first % a.in_ring + n) % a.in_ring : n;
    const int ro = a.out_ring ? (a.out_first % a.out_ring + n) % a.out_ring : n;
    tin[i] = (long)sh * a.sstride + (long)ri * a.in_slot;
    tout[i] = (long)sh * a.sstride + (long)ro * a.out_slot;
  }
  __syncthreads();
  // wavefront w brings chunks g = w + 8 r (window columns 4 g .. 4 g + 3) of
  // slot q into buf, column-major with lane = row
  auto issue = [&](int q, float *buf) {
    if (q >= q1) return;
    const auto rs = slot_rsrc(a.in + wave_uniform(tin[q - q0]), slot_bytes);
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int g = w + 8 * r;
      const bool real = g < NCH;                                  // wave-uniform
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_t *)(real ? &buf[g * 256] : sink), 16,
                                                real ? off0 + g * gstep : kOutOfRange, 0, 0, 0);
    }
  };
  // This wavefront's loads of slot q have landed.  Issued after them and
  // possibly still outstanding: the loads of the y younger slots already
  // issued and the three stores of each of the c slots consumed since; vector
  // memory operations complete in order, so waiting until no more than
  // PER y + 3 c remain is exact.
  auto ready = [&](int q) {
    if (q + 2 < q1 && q - q0 >= 3) {      // steady state: y = 2, c = 3
      wait_vmcnt_at_most<2 * PER + 9>(2 * PER + 9);
      return;
    }
    const int y = min(2, q1 - 1 - q);
    const int c = min(3, q - q0);
    wait_vmcnt_at_most<2 * PER + 9>(PER * y + 3 * c);
  };
  auto consume = [&](int q, const float *buf) {
    // output k reads window column m = k - SG ih + HMAX; based at m = 3 w so
    // that every LDS offset is a non-negative immediate
    const float *row = &buf[3 * w * 64 + lane];
    float oa = 0.f, ob = 0.f, oc = 0.f;
#pragma unroll
    for (int k = 0; k < NH; ++k) {
      const int ih = k - HMAX;
      oa += ca[k] * row[(HMAX - SG * ih) * 64];
      ob += cb[k] * row[(HMAX + 1 - SG * ih) * 64];
      oc += cc[k] * row[(HMAX + 2 - SG * ih) * 64];
    }
    // always three store instructions, so that ready() can count them
    const auto ro = slot_rsrc(a.out + wave_uniform(tout[q - q0]), slot_bytes);
    st(ro, oa, oa_off, 0);
    st(ro, ob, oc_off, 0);
    st(ro, oc, oe_off, 0);
  };
  // slot q sits in buffer q mod 4; the slot loaded in its place is q + 3,
  // whose buffer held slot q - 1 (everyone is past it once the barrier passed)
  auto step = [&](int q, const float *cur, float *nxt) {
    asm volatile("" ::: "memory");        // the barrier is no memory operation to the compiler:
    ready(q);                             // keep LDS accesses on their side of it
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    issue(q + 3, nxt);
    consume(q, cur);
  };
  issue(q0, b0);
  issue(q0 + 1, b1);
  issue(q0 + 2, b2);
  for (int q = q0; q < q1; q += 4) {
    step(q, b0, b3);
    if (q + 1 >= q1) break;
    step(q + 1, b1, b0);
    if (q + 2 >= q1) break;
    step(q + 2, b2, b1);
    if (q + 3 >= q1) break;
    step(q + 3, b3, b2);
  }
}

// Generic fallback (any H): one thread per (z, j), coefficient reused over up
// to kScatterKC slots held in registers.
constexpr int kScatterKC = 16;

__global__ void __launch_bounds__(256) k_ext_scatter(const ScatterArgs a) {
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int per_shot = a.nzs * a.nj;
  const int s = wave / per_shot;
  if (s >= a.nshots) return;
  const int rem = wave - s * per_shot;
  const int jj = rem / a.nzs;
  const int zs = rem - jj * a.nzs;
  const int j = __builtin_amdgcn_readfirstlane(a.j0 + jj);
  const int z = zs * 64 + lane;
  const bool zin = z < a.nz;
  const int zp = a.nb + z;
  const long sb = (long)s * a.sstride;

  for (int n0 = 0; n0 < a.nk; n0 += kScatterKC) {
    float acc[kScatterKC];
#pragma unroll
    for (int m = 0; m < kScatterKC; ++m) acc[m] = 0.f;
    const int nn = min(kScatterKC, a.nk - n0);
    for (int ih = -a.H; ih <= a.H; ++ih) {
      const int y = j - a.sg * ih - a.nb;
      const int i = j - 2 * a.sg * ih;
      if (y < 0 || y >= a.nx || i < 0 || i >= a.NX) continue;   // wave-uniform
      const float c = zin ? a.coef[((long)(ih + a.H) * a.nx + y) * a.nz + z] : 0.f;
      const long off = sb + (long)i * a.LZ + zp;
#pragma unroll
      for (int m = 0; m < kScatterKC; ++m) {
        if (m < nn) {
          const int n = n0 + m;
          const long slot = a.in_ring ? (long)((a.in_first + n) % a.in_ring) : (long)n;
          const float v = zin ? a.in[off + slot * a.in_slot] : 0.f;
          acc[m] += c * v;
        }
      }
    }
    if (zin) {
      const long off = sb + (long)j * a.LZ + zp;
#pragma unroll
      for (int m = 0; m < kScatterKC; ++m) {
        if (m < nn) {
          const int n = n0 + m;
          const long slot = a.out_ring ? (long)((a.out_first + n) % a.out_ring) : (long)n;
          a.out[off + slot * a.out_slot] = acc[m];
        }
      }
    }
  }
}

// Rows above the model at which the 64-row strips of the direct-load offset
// kernels start: the first strip begins on a 64-byte boundary of the padded
// column (256-byte aligned), so each wavefront's 256-byte runs cover whole
// 64-byte memory sectors; 0 where that would take one more strip.
static int strip_pad(int nz, int nb) {
  const int pad = nb % 16;
  return (nz + pad + 63) / 64 == (nz + 63) / 64 ? pad : 0;
}

hipError_t launch_ext_scatter(const float *coef, const ExtGeom &g, int sg, const float *in, long in_slot,
                              float *out, long out_slot, long sstride, int nshots, int nk, hipStream_t st,
                              int in_ring, int in_first, int out_ring, int out_first) {
  if (nk <= 0 || nshots <= 0) return hipSuccess;
  ScatterArgs a;
  a.coef = coef;
  a.in = in;
  a.out = out;
  a.in_slot = in_slot;
  a.out_slot = out_slot;
  a.sstride = sstride;
  a.in_ring = in_ring;
  a.in_first = in_first;
  a.out_ring = out_ring;
  a.out_first = out_first;
  a.nz = g.nz;
  a.nx = g.nx;
  a.nb = g.nb;
  a.NX = g.NX;
  a.LZ = g.LZ;
  a.nh = g.nh;
  a.H = g.H;
  a.sg = sg;
  // columns that can receive a nonzero value: j = nb + y + sg h
  a.j0 = max(0, g.nb - g.H);
  const int j1 = min(g.NX, g.nb + g.nx + g.H);
  a.nj = j1 - a.j0;
  a.nzs = (g.nz + 63) / 64;
  a.zpad = 0;
  a.nk = nk;
  a.nshots = nshots;
  const int total = nshots * nk;
  // FWIME_SCATTER_KERNEL=ws selects the register-staged ring for
  // comparisons (read per launch); the default is the ring fed by direct
  // global-to-LDS loads
  const char *sel = std::getenv("FWIME_SCATTER_KERNEL");
  const bool staged = sel && std::string(sel) == "ws";
#define FW_SCATTER(K, GRID, THREADS)                                                                    \
  if (g.H <= 8)                                                                                         \
    sg > 0 ? K<8, 1><<<GRID, THREADS, 0, st>>>(a) : K<8, -1><<<GRID, THREADS, 0, st>>>(a);              \
  else if (g.H <= 16)                                                                                   \
    sg > 0 ? K<16, 1><<<GRID, THREADS, 0, st>>>(a) : K<16, -1><<<GRID, THREADS, 0, st>>>(a);            \
  else if (g.H <= 24)                                                                                   \
    sg > 0 ? K<24, 1><<<GRID, THREADS, 0, st>>>(a) : K<24, -1><<<GRID, THREADS, 0, st>>>(a);            \
  else                                                                                                  \
    sg > 0 ? K<30, 1><<<GRID, THREADS, 0, st>>>(a) : K<30, -1><<<GRID, THREADS, 0, st>>>(a);
  if (g.H <= 30) {
    // spread the slots over enough workgroups to fill the device (the
    // direct-load kernel tiles 48-column blocks once per column parity)
    if (!staged) a.zpad = strip_pad(g.nz, g.nb);
    a.nzs = (g.nz + a.zpad + 63) / 64;
    const int ntile = staged ? a.nzs * ((a.nj + kScJB - 1) / kScJB)
                             : a.nzs * ((a.nj + 2 * kScDmaJB - 1) / (2 * kScDmaJB)) * 2;
    const int nblk = (ntile + 7) / 8 * 8;
    int groups = std::max(1, std::min(total, (2048 + nblk - 1) / nblk));
    if (!staged) groups = std::max(groups, (total + kScMaxSlots - 1) / kScMaxSlots);
    a.slots_per_block = (total + groups - 1) / groups;
    groups = (total + a.slots_per_block - 1) / a.slots_per_block;
    const dim3 grid((unsigned)nblk, (unsigned)groups);
    if (staged) {
      FW_SCATTER(k_ext_scatter_ws, grid, kScThreads)
    } else {
      FW_SCATTER(k_ext_scatter_dma, grid, kScThreads)
    }
    return hipGetLastError();
  }
#undef FW_SCATTER
  const long waves = (long)nshots * a.nzs * a.nj;
  k_ext_scatter<<<(unsigned)((waves + 3) / 4), 256, 0, st>>>(a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Extended imaging condition:
//   acc(z, y, h) += sum_s sum_n a_n(z, y - h) b_n(z, y + h)
// A wavefront owns a YT x HT tile of (y, h) for 64 depths; per time slot it
// reads YT + HT - 1 source-side and receiver-side columns and performs
// YT * HT multiply-adds.
// ---------------------------------------------------------------------------
constexpr int kImgYT = 8;
constexpr int kImgHT = 8;

// Each wavefront sums its tile in FP32 registers over the slots of its
// group, then stores the sums into its group's partial image; a second
// kernel adds the partials to the FP64 accumulator in group order.  The launch splits its slots into enough
// groups that no group sums more than kImgChain of them, which bounds the
// FP32 chain's rounding to about 1e-6 of a sum of random-sign terms,
// whatever the number of shots and steps of the launch.
constexpr int kImgChain = 512;

struct ImageArgs {
  const float *a;
  const float *b;
  double *acc;
  float *parts;        // partial images, one per slot group
  long a_slot, b_slot, a_sstride, b_sstride;
  int b_ring, b_first;
  int nshots, nk;
  int nz, nx, nb, NX, LZ, nh, H;
  int nzs, nyt, nht;
  int zpad;            // rows of the first strip above the model (direct-load kernel)
  int nhb;             // offset blocks (blockIdx.x: tile and offset block, offset block fastest)
  int groups, slots_per_group;
};

// Stores a wavefront's FP32 tile sums into its group's partial image.  Every
// cell of a group's image is owned by one wavefront.
__device__ __forceinline__ void image_store(const ImageArgs &p, const float (&acc)[kImgYT][kImgHT], int grp, int y0,
                                            int h0, int hhi, int z) {
#pragma unroll
  for (int yy = 0; yy < kImgYT; ++yy) {
    const int y = y0 + yy;
    if (y >= p.nx) continue;
#pragma unroll
    for (int hh = 0; hh < kImgHT; ++hh) {
      const int ih = h0 + hh;
      if (ih > hhi) continue;
      const long o = ((long)(ih + p.H) * p.nx + y) * p.nz + z;
      p.parts[(long)grp * p.nh * p.nx * p.nz + o] = acc[yy][hh];
    }
  }
}

// LDS-staged, pipelined version.  A workgroup of 16 wavefronts covers one
// depth strip, YB = 8 NYT model columns and one block of 8 NHT offsets, for
// the slots of group blockIdx.y; the wavefronts tile (y, h) as NYT x NHT tiles of 8 x 8
// (NYT NHT = 16).  Per time slot the source-side window (y - h) and the
// receiver-side window (y + h), each YB + 8 NHT - 1 columns wide, are staged in
// a 3-deep LDS ring: slot q is consumed while slot q + 1 is written from
// registers and the loads of slots q + 2 and q + 3 are in flight (one barrier
// per slot).  With several slot groups (enough workgroups to fill the device when the
// tiles alone do not), group g stores its partial image and a second kernel
// adds the partials to the accumulator in group order, so the result does not
// depend on scheduling.
template <int NYT, int NHT>
__global__ void __launch_bounds__(1024) k_ext_image_lds(const ImageArgs p) {
  constexpr int NA = kImgYT + kImgHT - 1;
  constexpr int YB = 8 * NYT;
  constexpr int HSPAN = 8 * NHT;
  constexpr int WW = YB + HSPAN - 1;
  constexpr int ROWS = 2 * WW;                  // a-window rows then b-window rows
  constexpr int PER = (ROWS + 15) / 16;         // rows staged per thread
  __shared__ float ring[3][ROWS * 64];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  // (tile, offset block) pairs in XCD-contiguous ranges, offset block
  // fastest: the offset blocks of a tile read the same slots at the same
  // time and share them through the XCD's L2
  const int npair = p.nzs * ((p.nx + YB - 1) / YB) * p.nhb;
  const int per = (npair + 7) >> 3;
  const int pair = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (pair >= npair) return;
  const int tile = pair / p.nhb;
  const int zs = tile % p.nzs;
  const int yblk = tile / p.nzs;
  const int yb = yblk * YB;
  const int grp = blockIdx.y;
  const int hlo = -p.H + HSPAN * (pair - tile * p.nhb);
  const int hhi = min(p.H, hlo + HSPAN - 1);
  const int z = zs * 64 + lane;
  const bool zin = z < p.nz;
  const int zp = p.nb + z;
  const int yt = w % NYT, ht = w / NYT;
  const int y0 = yb + 8 * yt;
  const int h0 = hlo + 8 * ht;
  const bool active = h0 <= hhi && y0 < p.nx;
  // window origins (padded columns)
  const int xa0 = p.nb + yb - (hlo + HSPAN - 1);
  const int xb0 = p.nb + yb + hlo;
  const int ia = 8 * yt + (HSPAN - 8 - 8 * ht);  // a-window row of A[0]
  const int ib = WW + 8 * yt + 8 * ht;           // b-window row of B[0]

  float acc[kImgYT][kImgHT];
#pragma unroll
  for (int yy = 0; yy < kImgYT; ++yy)
#pragma unroll
    for (int hh = 0; hh < kImgHT; ++hh) acc[yy][hh] = 0.f;

  const int q0 = grp * p.slots_per_group;
  const int total = min(p.nshots * p.nk, q0 + p.slots_per_group);
  // thread (w, lane) stages rows w + 16 r at depth lane; out-of-grid columns
  // read as zero through the bounds-checked buffer loads
  const unsigned slot_bytes = (unsigned)((long)p.NX * p.LZ * 4);
  const int zoff = zp * 4;                          // per lane
  const int CBy = p.LZ * 4;                         // bytes per column
  SlotCursor fc;                                    // fetch walks q0, q0 + 1, ... once, in order
  fc.init(q0, p.nk, p.b_first, p.b_ring);
  auto fetch = [&](int q, float (&pre)[PER]) {
    if (q >= total) return;
    const auto ra = slot_rsrc(p.a + (long)fc.s * p.a_sstride + (long)fc.n * p.a_slot, slot_bytes);
    const auto rbb = slot_rsrc(p.b + (long)fc.s * p.b_sstride + (long)fc.r * p.b_slot, slot_bytes);
    fc.next();
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int c = w + 16 * r;
      if (c < WW)
        pre[r] = bload(ra, zoff + (xa0 + c) * CBy);
      else
        pre[r] = bload(rbb, zoff + (xb0 + c - WW) * CBy);
    }
  };
  auto put = [&](int rbuf, const float (&pre)[PER]) {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int c = w + 16 * r;
      if (c < ROWS) ring[rbuf][c * 64 + lane] = pre[r];
    }
  };
  auto consume = [&](int rbuf) {
    if (!active) return;
    const float *win = ring[rbuf];
    float va[NA], vb[NA];
#pragma unroll
    for (int m = 0; m < NA; ++m) {
      va[m] = win[(ia + m) * 64 + lane];
      vb[m] = win[(ib + m) * 64 + lane];
    }
#pragma unroll
    for (int yy = 0; yy < kImgYT; ++yy)
#pragma unroll
      for (int hh = 0; hh < kImgHT; ++hh) acc[yy][hh] += va[yy - hh + kImgHT - 1] * vb[yy + hh];
  };
  // ring[rb] holds slot q; pA / pB hold the two following slots (unrolled by
  // two so the staging registers alternate instead of being copied)
  float pA[PER], pB[PER];
  fetch(q0, pA);
  put(0, pA);
  fetch(q0 + 1, pA);
  fetch(q0 + 2, pB);
  __syncthreads();
  int rb = 0;
  int q = q0;
  for (; q + 1 < total; q += 2) {   // pairs of slots; no exit in between
    int nb1 = rb == 2 ? 0 : rb + 1;
    consume(rb);
    put(nb1, pA);
    fetch(q + 3, pA);
    __syncthreads();
    rb = nb1;
    nb1 = rb == 2 ? 0 : rb + 1;
    consume(rb);
    if (q + 2 < total) put(nb1, pB);
    fetch(q + 4, pB);
    __syncthreads();
    rb = nb1;
  }
  if (q < total) consume(rb);       // odd last slot, already staged
  if (!active || !zin) return;
  image_store(p, acc, grp, y0, h0, hhi, z);
}

// Wide-offset variant with the windows brought in by 16-byte direct
// global-to-LDS loads into a 4-deep ring (as in k_ext_scatter_dma): three
// slots in flight while one is consumed, no staging registers.  Each window is
// padded to 64 columns, 16 chunks of four 64-deep columns, so wavefront w
// loads chunk w of the source-side and of the receiver-side window; columns
// outside the grid read as zero through the range check.  Slots are consumed
// in the same order as in k_ext_image_lds, so both give the same bits.  As in
// the scatter, the 64-row strips start on a 64-byte boundary of the column
// (p.zpad rows above the model).
template <int NYT, int NHT>
__global__ void __launch_bounds__(1024) k_ext_image_dma(const ImageArgs p) {
  constexpr int NA = kImgYT + kImgHT - 1;
  constexpr int YB = 8 * NYT;
  constexpr int HSPAN = 8 * NHT;
  constexpr int WW = YB + HSPAN - 1;
  constexpr int WWP = (WW + 3) / 4 * 4;          // window columns in LDS
  static_assert(WWP / 4 == 16, "one chunk of each window per wavefront");
  constexpr int BUF = 2 * WWP * 64;              // a-window columns, then b-window columns
  __shared__ float b0[BUF], b1[BUF], b2[BUF], b3[BUF];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  // (tile, offset block) pairs in XCD-contiguous ranges, offset block
  // fastest, then column blocks, as in the scatter: the offset blocks of a
  // tile and the neighbouring windows of one strip are read together and
  // come from the XCD's L2
  const int nyb = (p.nx + YB - 1) / YB;
  const int npair = p.nzs * nyb * p.nhb;
  const int per = (npair + 7) >> 3;
  const int pair = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (pair >= npair) return;
  const int tile = pair / p.nhb;
  const int yblk = tile % nyb;
  const int zs = tile / nyb;
  const int yb = yblk * YB;
  const int grp = blockIdx.y;
  const int hlo = -p.H + HSPAN * (pair - tile * p.nhb);
  const int hhi = min(p.H, hlo + HSPAN - 1);
  const int z = zs * 64 + lane - p.zpad;           // model row of this lane
  const bool zin = z >= 0 && z < p.nz;
  const int yt = w % NYT, ht = w / NYT;
  const int y0 = yb + 8 * yt;
  const int h0 = hlo + 8 * ht;
  const bool active = h0 <= hhi && y0 < p.nx;
  const int xa0 = p.nb + yb - (hlo + HSPAN - 1);
  const int xb0 = p.nb + yb + hlo;
  const int ia = 8 * yt + (HSPAN - 8 - 8 * ht);  // a-window column of A[0]
  const int ib = WWP + 8 * yt + 8 * ht;          // b-window column of B[0]

  float acc[kImgYT][kImgHT];
#pragma unroll
  for (int yy = 0; yy < kImgYT; ++yy)
#pragma unroll
    for (int hh = 0; hh < kImgHT; ++hh) acc[yy][hh] = 0.f;

  const int q0 = grp * p.slots_per_group;
  const int total = min(p.nshots * p.nk, q0 + p.slots_per_group);
  const unsigned slot_bytes = (unsigned)((long)p.NX * p.LZ * 4);
  const int CBy = p.LZ * 4;
  // lane i of a chunk: column 4 w + i / 16 of the window, depths 4 (i % 16) .. + 3
  const int lane_off = (p.nb - p.zpad + zs * 64 + 4 * (lane & 15)) * 4 + (lane >> 4) * CBy;
  const int offa = lane_off + (xa0 + 4 * w) * CBy;
  const int offb = lane_off + (xb0 + 4 * w) * CBy;
  OffCursor fa, fb;                              // issue walks q0, q0 + 1, ... once, in order
  fa.init(q0, p.nk, 0, 0, p.a_slot, p.a_sstride);
  fb.init(q0, p.nk, p.b_first, p.b_ring, p.b_slot, p.b_sstride);
  auto issue = [&](int q, float *buf) {
    if (q >= total) return;
    const auto ra = slot_rsrc(p.a + fa.off, slot_bytes);
    const auto rbb = slot_rsrc(p.b + fb.off, slot_bytes);
    fa.next();
    fb.next();
    __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_void_t *)&buf[w * 256], 16, offa, 0, 0, 0);
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rbb, (lds_void_t *)&buf[WWP * 64 + w * 256], 16, offb, 0, 0, 0);
  };
  // this wavefront's two loads of slot q have landed; younger slots may be in flight
  auto ready = [&](int q) {
    constexpr int kExpLgkm = (7 << 4) | (15 << 8);
    if (q + 2 < total) __builtin_amdgcn_s_waitcnt(4 | kExpLgkm);
    else if (q + 1 < total) __builtin_amdgcn_s_waitcnt(2 | kExpLgkm);
    else __builtin_amdgcn_s_waitcnt(kExpLgkm);
  };
  // every wavefront consumes (an inactive one's sums are never stored): a
  // branch here makes the compiler wait for all outstanding loads first
  auto consume = [&](const float *win) {
    float va[NA], vb[NA];
#pragma unroll
    for (int m = 0; m < NA; ++m) {
      va[m] = win[(ia + m) * 64 + lane];
      vb[m] = win[(ib + m) * 64 + lane];
    }
#pragma unroll
    for (int yy = 0; yy < kImgYT; ++yy)
#pragma unroll
      for (int hh = 0; hh < kImgHT; ++hh) acc[yy][hh] += va[yy - hh + kImgHT - 1] * vb[yy + hh];
  };
  // slot q sits in buffer q mod 4; the slot loaded in its place is q + 3,
  // whose buffer held slot q - 1 (everyone is past it once the barrier passed)
  auto step = [&](int q, const float *cur, float *nxt) {
    asm volatile("" ::: "memory");
    ready(q);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    consume(cur);
    issue(q + 3, nxt);
  };
  issue(q0, b0);
  issue(q0 + 1, b1);
  issue(q0 + 2, b2);
  for (int q = q0; q < total; q += 4) {
    step(q, b0, b3);
    if (q + 1 >= total) break;
    step(q + 1, b1, b0);
    if (q + 2 >= total) break;
    step(q + 2, b2, b1);
    if (q + 3 >= total) break;
    step(q + 3, b3, b2);
  }
  if (!active || !zin) return;
  image_store(p, acc, grp, y0, h0, hhi, z);
}

// acc += sum over g of parts[g], in group order (FP64)
__global__ void k_image_reduce(double *acc, const float *parts, long n, int groups) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double s = parts[i];
    for (int g = 1; g < groups; ++g) s += (double)parts[(long)g * n + i];
    acc[i] += s;
  }
}

hipError_t launch_ext_image(const float *a, long a_slot, long a_sstride, const float *b, long b_slot, long b_sstride,
                            int b_ring, int b_first, int nshots, int nk, const ExtGeom &g, double *acc,
                            float *parts, hipStream_t st) {
  if (nk <= 0 || nshots <= 0) return hipSuccess;
  ImageArgs p;
  p.a = a;
  p.b = b;
  p.acc = acc;
  p.parts = parts;
  p.a_slot = a_slot;
  p.b_slot = b_slot;
  p.a_sstride = a_sstride;
  p.b_sstride = b_sstride;
  p.b_ring = b_ring;
  p.b_first = b_first;
  p.nshots = nshots;
  p.nk = nk;
  p.nz = g.nz;
  p.nx = g.nx;
  p.nb = g.nb;
  p.NX = g.NX;
  p.LZ = g.LZ;
  p.nh = g.nh;
  p.H = g.H;
  const bool wide = g.nh > 16;
  // FWIME_IMAGE_KERNEL=lds selects the register-staged ring for the wide
  // tiles too (for comparisons; read per launch)
  const char *sel = std::getenv("FWIME_IMAGE_KERNEL");
  const bool staged = sel && std::string(sel) == "lds";
  p.zpad = wide && !staged ? strip_pad(g.nz, g.nb) : 0;
  p.nzs = (g.nz + p.zpad + 63) / 64;
  p.nhb = wide ? (g.nh + 31) / 32 : 1;
  const int npair = p.nzs * ((g.nx + (wide ? 31 : 63)) / (wide ? 32 : 64)) * p.nhb;
  const int nblk = (npair + 7) / 8 * 8;
  // one workgroup fits a CU: split the slots into groups until there are
  // about eight workgroups per CU, so the last round of workgroups leaves
  // little of the device idle, and until no group sums more than kImgChain
  // slots (at most kImageGroups partial images)
  const int total = nshots * nk;
  const int want = std::max((2048 + nblk - 1) / nblk, (total + kImgChain - 1) / kImgChain);
  int groups = std::min(kImageGroups, std::max(1, want));
  groups = std::min(groups, total);
  p.slots_per_group = (total + groups - 1) / groups;
  p.groups = (total + p.slots_per_group - 1) / p.slots_per_group;
  const dim3 grid((unsigned)nblk, (unsigned)p.groups);
  if (wide && !staged) k_ext_image_dma<4, 4><<<grid, 1024, 0, st>>>(p);
  else if (wide) k_ext_image_lds<4, 4><<<grid, 1024, 0, st>>>(p);
  else k_ext_image_lds<8, 2><<<grid, 1024, 0, st>>>(p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long n = (long)g.nh * g.nx * g.nz;
  long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  k_image_reduce<<<(unsigned)blocks, 256, 0, st>>>(acc, parts, n, p.groups);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Time-lag extension (lags tau_k = k L dt, k = -K .. K; the other extension of
// Section 2).  A model cell's scattering source at step n takes the
// background's T2 term at steps n - 2kL, and its image at lag k correlates
// that term with the adjoint field along time.  One thread per model cell
// and shot (scatter) or per model cell and lag (image), cells z-fastest so
// every access of a wavefront is one column run; the terms are summed in the
// order k = -K .. K, and over shots then steps.
// ---------------------------------------------------------------------------
__global__ void k_tau_scatter(const float *coef, const float *in, float *out, long slot, long sstride, int nslots,
                              int K, int L, int nz, int nx, int nb, int LZ, int nshots) {
  const long ncell = (long)nx * nz;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < ncell * nshots;
       i += (long)gridDim.x * blockDim.x) {
    const int s = (int)(i / ncell);
    const long cell = i - (long)s * ncell;
    const int y = (int)(cell / nz), z = (int)(cell - (long)y * nz);
    const long off = (long)s * sstride + (long)(y + nb) * LZ + (z + nb);
    for (int n = 0; n < nslots; ++n) {
      float acc = 0.f;
      for (int k = -K; k <= K; ++k) {
        const int m = n - 2 * k * L;
        if (m >= 0 && m < nslots) acc = fmaf(coef[((long)(k + K) * nx + y) * nz + z], in[off + (long)m * slot], acc);
      }
      out[off + (long)n * slot] = acc;
    }
  }
}

__global__ void k_tau_image(const float *in, long in_slot, long in_sstride, const float *lam, long lam_slot,
                            long lam_sstride, int nslots, int nshots, int K, int L, int nz, int nx, int nb, int LZ,
                            const float *vel, float dt, float *acc) {
  const long ncell = (long)nx * nz;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < ncell * (2 * K + 1);
       i += (long)gridDim.x * blockDim.x) {
    const int ik = (int)(i / ncell);
    const long cell = i - (long)ik * ncell;
    const int y = (int)(cell / nz), z = (int)(cell - (long)y * nz);
    const long pc = (long)(y + nb) * LZ + (z + nb);
    const int sh = 2 * (ik - K) * L;
    float sum = 0.f;
    for (int s = 0; s < nshots; ++s) {
      const float *a = in + (long)s * in_sstride + pc;
      const float *b = lam + (long)s * lam_sstride + pc;
      for (int n = max(0, sh); n < min(nslots, nslots + sh); ++n)   // 0 <= n - sh < nslots
        sum = fmaf(a[(long)(n - sh) * in_slot], b[(long)n * lam_slot], sum);
    }
    const float v = vel[cell];
    acc[i] += 2.f / (v * v * v * dt * dt) * sum;
  }
}

// Residue form.  With n = P q + r (P = 2L, 0 <= r < P) the lag terms only
// connect steps of one residue: out_r[q] = sum_k c_k in_r[q - k], image_k =
// sum_q in_r[q - k] lam_r[q], with x_r[q] = x_{Pq + r}.  A workgroup stages
// the Q_r samples of a residue for 64 model cells (lane = cell) in LDS, so
// each history sample is read from HBM once instead of once per lag.
constexpr int kTauQMax = 128;                 // samples per residue held in LDS
constexpr int kTauImgWaves = 8;               // wavefronts per workgroup of the lag imaging kernel

// Scatter: workgroup = (64-cell block, shot), walking the shot's residues;
// weights of the lane's cell in registers (zero beyond K); every output adds
// the same terms in the same order as in k_tau_scatter, so both give the
// same bits.
template <int KMAX>
__global__ void __launch_bounds__(256) k_tau_scatter_lds(const float *coef, const float *in, float *out, long slot,
                                                         long sstride, int nslots, int K, int L, int nz, int nx,
                                                         int nb, int LZ, int nshots, int ncb) {
  constexpr int PQ = kTauQMax / 4;             // samples per wavefront and residue
  __shared__ float win[kTauQMax * 64];
  const int P = 2 * L;
  // shot fastest, then cell block, in XCD-contiguous ranges: the workgroups
  // of one cell block run together on one XCD and share its lag weights in
  // that XCD's L2; a workgroup walks every residue of its shot
  const int total = ncb * nshots;
  const int per = (total + 7) >> 3;
  const int b = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (b >= total) return;
  const int s = b % nshots;
  const int cbk = b / nshots;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const long ncell = (long)nx * nz;
  const long cell = (long)cbk * 64 + lane;
  const bool cin = cell < ncell;
  const int y = cin ? (int)(cell / nz) : 0, z = cin ? (int)(cell - (long)y * nz) : 0;
  const long pc = (long)(y + nb) * LZ + (z + nb);
  const long off = (long)s * sstride + pc;
  // Samples q = w + 4 i of residue r: loaded into registers (a buffer
  // resource on the wave's slot plus one per-lane offset, clamped to a valid
  // slot, no branch) while the previous residue is summed, zeroed past the
  // residue's Q steps or outside the model when written to LDS.
  float pw[PQ];
  const int pcb = (int)pc * 4;
  auto fetch = [&](int r) {
#pragma unroll
    for (int i = 0; i < PQ; ++i) {
      const long n = min(P * (w + 4 * i) + r, nslots - 1);
      pw[i] = bload(slot_rsrc(in + (long)s * sstride + n * slot, (unsigned)(slot * 4)), pcb);
    }
  };
  fetch(0);
  float c[2 * KMAX + 1];
#pragma unroll
  for (int k = -KMAX; k <= KMAX; ++k)
    c[k + KMAX] = (cin && k >= -K && k <= K) ? coef[((long)(k + K) * nx + y) * nz + z] : 0.f;
  for (int r = 0; r < P; ++r) {
    const int Q = (nslots - r + P - 1) / P;   // steps P q + r < nslots
    __syncthreads();                         // the previous residue's reads are done
#pragma unroll
    for (int i = 0; i < PQ; ++i) win[(w + 4 * i) * 64 + lane] = cin && w + 4 * i < Q ? pw[i] : 0.f;
    __syncthreads();
    if (r + 1 < P) fetch(r + 1);
    // eight consecutive outputs q0 .. q0 + 7 per pass, so that each LDS read
    // feeds up to eight multiply-adds; inputs j = q0 + t are taken from the
    // highest down, which adds every output's terms in ascending k
    for (int q0 = 8 * w; q0 < Q; q0 += 32) {
      float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 7 + KMAX; t >= -KMAX; --t) {
        const int j = q0 + t;                  // wave-uniform
        if (j < 0 || j >= Q) continue;
        const float x = win[j * 64 + lane];
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
          const int k = jj - t;                // output q0 + jj takes lag k from input j
          if (k >= -KMAX && k <= KMAX) acc[jj] = fmaf(c[k + KMAX], x, acc[jj]);
        }
      }
#pragma unroll
      for (int jj = 0; jj < 8; ++jj)
        if (cin && q0 + jj < Q) out[off + (long)(P * (q0 + jj) + r) * slot] = acc[jj];
    }
  }
}

// Image: workgroup = 64-cell block of kTauImgWaves wavefronts; it walks every
// shot and residue, staging the history and adjoint samples.  Lags come in
// groups of four consecutive ones, group G = w + kTauImgWaves g to wavefront w
// (at most KPW lags per wavefront, accumulated in registers): one adjoint
// sample and a window of four history samples feed four multiply-adds.  Each lag sums its products in ascending
// q, where every lag of the group is in range without a test and at the two
// edges with one.
template <int KPW>
__global__ void __launch_bounds__(kTauImgWaves * 64) k_tau_image_lds(const float *in, long in_slot, long in_sstride,
                                                       const float *lam, long lam_slot, long lam_sstride, int nslots,
                                                       int nshots, int K, int L, int nz, int nx, int nb, int LZ,
                                                       const float *vel, float dt, float *acc) {
  constexpr int NW = kTauImgWaves;
  constexpr int PQ = kTauQMax / NW;            // samples per wavefront and residue
  __shared__ float ta[kTauQMax * 64], tb[kTauQMax * 64];
  const int P = 2 * L;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const long ncell = (long)nx * nz;
  const long cell = (long)blockIdx.x * 64 + lane;
  const bool cin = cell < ncell;
  const int y = cin ? (int)(cell / nz) : 0, z = cin ? (int)(cell - (long)y * nz) : 0;
  const long pc = (long)(y + nb) * LZ + (z + nb);
  float sum[KPW];
#pragma unroll
  for (int i = 0; i < KPW; ++i) sum[i] = 0.f;
  // Samples q = w + NW i of residue r of shot s (history and adjoint field).
  // Every load reads a valid slot (clamped) and none sits behind a branch or
  // feeds an instruction before the next residue's LDS writes, so the loads
  // stay in flight while the current residue is summed; samples past the
  // residue's Q steps or outside the model are zeroed when written to LDS.
  // The slot is the same for the whole wavefront: each load is a buffer
  // resource on that slot (scalar registers) plus one per-lane byte offset.
  float pa[PQ], pb[PQ];
  const int pcb = (int)pc * 4;
  auto fetch = [&](int s, int r) {
#pragma unroll
    for (int i = 0; i < PQ; ++i) {
      const long n = min(P * (w + NW * i) + r, nslots - 1);
      pa[i] = bload(slot_rsrc(in + (long)s * in_sstride + n * in_slot, (unsigned)(in_slot * 4)), pcb);
      pb[i] = bload(slot_rsrc(lam + (long)s * lam_sstride + n * lam_slot, (unsigned)(lam_slot * 4)), pcb);
    }
  };
  fetch(0, 0);
  for (int s = 0; s < nshots; ++s) {
    for (int r = 0; r < P; ++r) {
      const int Q = (nslots - r + P - 1) / P;
      __syncthreads();                         // the previous residue's reads are done
#pragma unroll
      for (int i = 0; i < PQ; ++i) {
        const bool ok = cin && w + NW * i < Q;
        ta[(w + NW * i) * 64 + lane] = ok ? pa[i] : 0.f;
        tb[(w + NW * i) * 64 + lane] = ok ? pb[i] : 0.f;
      }
      __syncthreads();
      const int s2 = r + 1 < P ? s : s + 1;    // the next residue
      if (s2 < nshots) fetch(s2, r + 1 < P ? r + 1 : 0);
#pragma unroll
      for (int g = 0; g < KPW / 4; ++g) {
        const int k0 = -K + 4 * (w + NW * g);  // lags k0 .. k0 + 3, wave-uniform
        if (k0 > K) break;
        float t[4] = {0.f, 0.f, 0.f, 0.f};
        // lag k takes q in [max(0, k), min(Q, Q + k)); all four in [qlo, qhi)
        const int qlo = max(0, k0 + 3), qhi = min(Q, Q + k0);
        const int e0 = max(0, k0), e1 = min(qlo, Q);
        for (int q = e0; q < e1; ++q) {
          const float x = tb[q * 64 + lane];
#pragma unroll
          for (int jj = 0; jj < 4; ++jj)
            if (q >= k0 + jj && q < Q + k0 + jj) t[jj] = fmaf(ta[(q - k0 - jj) * 64 + lane], x, t[jj]);
        }
        // the four history samples of step q are those of step q - 1 moved
        // by one lag plus one new one: they stay in registers (w0..w3 =
        // history at q - k0 .. q - k0 - 3 when four steps start), one new
        // LDS read per step instead of four; each lag still sums in
        // ascending q, as the per-step form does
        if (qlo < qhi) {
          const float *hq = &ta[(qlo - k0) * 64 + lane];
          float w0 = hq[0], w1 = hq[-64], w2 = hq[-128], w3 = hq[-192];
          int q = qlo;
          for (; q + 4 <= qhi; q += 4) {
            const float *tq = &tb[q * 64 + lane];
            const float *hn = &ta[(q - k0) * 64 + lane];
            float x = tq[0];
            t[0] = fmaf(w0, x, t[0]); t[1] = fmaf(w1, x, t[1]); t[2] = fmaf(w2, x, t[2]); t[3] = fmaf(w3, x, t[3]);
            w3 = hn[64];
            x = tq[64];
            t[0] = fmaf(w3, x, t[0]); t[1] = fmaf(w0, x, t[1]); t[2] = fmaf(w1, x, t[2]); t[3] = fmaf(w2, x, t[3]);
            w2 = hn[128];
            x = tq[128];
            t[0] = fmaf(w2, x, t[0]); t[1] = fmaf(w3, x, t[1]); t[2] = fmaf(w0, x, t[2]); t[3] = fmaf(w1, x, t[3]);
            w1 = hn[192];
            x = tq[192];
            t[0] = fmaf(w1, x, t[0]); t[1] = fmaf(w2, x, t[1]); t[2] = fmaf(w3, x, t[2]); t[3] = fmaf(w0, x, t[3]);
            // w1, w2, w3 now hold the history at q + 3, q + 2, q + 1 (- k0):
            // the next four steps need only q + 4
            if (q + 8 <= qhi) w0 = hn[256];
          }
          for (; q < qhi; ++q) {
            const float x = tb[q * 64 + lane];
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) t[jj] = fmaf(ta[(q - k0 - jj) * 64 + lane], x, t[jj]);
          }
        }
        const int h0 = max(qhi, qlo), h1 = min(Q, Q + k0 + 3);
        for (int q = h0; q < h1; ++q) {
          const float x = tb[q * 64 + lane];
#pragma unroll
          for (int jj = 0; jj < 4; ++jj)
            if (q >= k0 + jj && q < Q + k0 + jj) t[jj] = fmaf(ta[(q - k0 - jj) * 64 + lane], x, t[jj]);
        }
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) sum[4 * g + jj] += t[jj];
      }
    }
  }
  if (!cin) return;
  const float v = vel[cell];
  const float sc = 2.f / (v * v * v * dt * dt);
#pragma unroll
  for (int g = 0; g < KPW / 4; ++g) {
    const int k0 = -K + 4 * (w + NW * g);
    if (k0 > K) break;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
      if (k0 + jj <= K) acc[(long)(k0 + jj + K) * ncell + cell] += sc * sum[4 * g + jj];
  }
}

static unsigned tau_blocks(long n) {
  const long b = (n + 255) / 256;
  return (unsigned)(b < 16384 ? (b > 0 ? b : 1) : 16384);
}

hipError_t launch_tau_scatter(const float *coef, const ExtGeom &g, int L, const float *in, float *out, long slot,
                              long sstride, int nslots, int nshots, hipStream_t st) {
  if (nslots <= 0 || nshots <= 0) return hipSuccess;
  const int P = 2 * L;
  const long ncell = (long)g.nx * g.nz;
  const int ncb = (int)((ncell + 63) / 64);
  const long nblk = (long)ncb * nshots;
  if ((nslots + P - 1) / P > kTauQMax || g.H > 64 || nblk + 8 >= (1L << 31) || (long)slot * 4 >= (1L << 32)) {
    k_tau_scatter<<<tau_blocks(ncell * nshots), 256, 0, st>>>(coef, in, out, slot, sstride, nslots, g.H, L, g.nz,
                                                              g.nx, g.nb, g.LZ, nshots);
    return hipGetLastError();
  }
  const dim3 grid((unsigned)((nblk + 7) / 8 * 8));
#define FW_TAU_S(KM)                                                                                     \
  k_tau_scatter_lds<KM><<<grid, 256, 0, st>>>(coef, in, out, slot, sstride, nslots, g.H, L, g.nz, g.nx, g.nb, \
                                              g.LZ, nshots, ncb)
  // every pass multiplies 2 KMAX + 1 weights, those beyond K being zero:
  // buckets of 8 lags keep that waste small for the wide lag ranges
  if (g.H <= 8) FW_TAU_S(8);
  else if (g.H <= 16) FW_TAU_S(16);
  else if (g.H <= 32) FW_TAU_S(32);
  else if (g.H <= 40) FW_TAU_S(40);
  else if (g.H <= 48) FW_TAU_S(48);
  else if (g.H <= 56) FW_TAU_S(56);
  else FW_TAU_S(64);
#undef FW_TAU_S
  return hipGetLastError();
}

hipError_t launch_tau_image(const float *in, long in_slot, long in_sstride, const float *lam, long lam_slot,
                            long lam_sstride, int nslots, int nshots, const ExtGeom &g, int L, const float *vel,
                            float dt, float *acc, hipStream_t st) {
  if (nslots <= 0 || nshots <= 0) return hipSuccess;
  const int P = 2 * L;
  const long ncell = (long)g.nx * g.nz;
  // lags per wavefront, whole groups of four dealt round-robin over the
  // workgroup's wavefronts
  const int kpw = 4 * (((g.nh + 3) / 4 + kTauImgWaves - 1) / kTauImgWaves);
  if ((nslots + P - 1) / P > kTauQMax || kpw > 16) {
    k_tau_image<<<tau_blocks(ncell * g.nh), 256, 0, st>>>(in, in_slot, in_sstride, lam, lam_slot, lam_sstride,
                                                          nslots, nshots, g.H, L, g.nz, g.nx, g.nb, g.LZ, vel, dt,
                                                          acc);
    return hipGetLastError();
  }
  const dim3 grid((unsigned)((ncell + 63) / 64));
#define FW_TAU_I(KP)                                                                                              \
  k_tau_image_lds<KP><<<grid, kTauImgWaves * 64, 0, st>>>(in, in_slot, in_sstride, lam, lam_slot, lam_sstride,  \
                                                          nslots, nshots, g.H, L, g.nz, g.nx, g.nb, g.LZ, vel, dt, \
                                                          acc)
  if (kpw <= 4) FW_TAU_I(4);
  else if (kpw <= 8) FW_TAU_I(8);
  else FW_TAU_I(16);
#undef FW_TAU_I
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// gacc(x, z) += sum_s sum_n (t2u_n + t2d_n) lam_n + t2u_n rho_n   (padded grid)
// ---------------------------------------------------------------------------
__global__ void k_grad_accum(const float *t2u, const float *t2d, long slot, long seg_sstride, const float *lam,
                             long ring_slot, long ring_sstride, int ring, int first, const float *rho,
                             long rho_slot, long rho_sstride, int rho_ring, int rho_first, int nshots, int nk,
                             int NZ, long ncell, int LZ, float *gacc) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncell) return;
  const int z = (int)(i % LZ);
  if (z >= NZ) return;
  float g = 0.f;
  for (int s = 0; s < nshots; ++s) {
    const long sa = (long)s * seg_sstride + i;
    const long sr = (long)s * ring_sstride + i;
    const long sp = (long)s * rho_sstride + i;
    for (int n = 0; n < nk; ++n) {
      const long rs = (long)((first + n) % ring) * ring_slot;
      const long ps = (long)((rho_first + n) % rho_ring) * rho_slot;
      const float u = t2u[sa + n * slot];
      const float d = t2d[sa + n * slot];
      g += (u + d) * lam[sr + rs] + u * rho[sp + ps];
    }
  }
  gacc[i] += g;
}

hipError_t launch_grad_accum(const float *t2u, const float *t2d, long slot, long seg_sstride, const float *lam,
                             const float *rho, long ring_slot, long ring_sstride, int ring, int first, int nshots,
                             int nk, int NZ, int NX, int LZ, float *gacc, hipStream_t st) {
  return launch_grad_accum2(t2u, t2d, slot, seg_sstride, lam, ring_slot, ring_sstride, ring, first, rho, ring_slot,
                            ring_sstride, ring, first, nshots, nk, NZ, NX, LZ, gacc, st);
}

hipError_t launch_grad_accum2(const float *t2u, const float *t2d, long slot, long seg_sstride, const float *lam,
                              long lam_slot, long lam_sstride, int lam_ring, int lam_first, const float *rho,
                              long rho_slot, long rho_sstride, int rho_ring, int rho_first, int nshots, int nk,
                              int NZ, int NX, int LZ, float *gacc, hipStream_t st) {
  if (nk <= 0 || nshots <= 0) return hipSuccess;
  const long ncell = (long)NX * LZ;
  k_grad_accum<<<(unsigned)((ncell + 255) / 256), 256, 0, st>>>(t2u, t2d, slot, seg_sstride, lam, lam_slot,
                                                                 lam_sstride, lam_ring, lam_first, rho, rho_slot,
                                                                 rho_sstride, rho_ring, rho_first, nshots, nk, NZ,
                                                                 ncell, LZ, gacc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Residual and sum of squares (FP64 accumulation in a fixed order: each of
// kRedBlocks workgroups reduces its strided share by a tree, and one
// workgroup adds the partials by a tree, so the result does not depend on
// scheduling and repeats bit for bit).
// ---------------------------------------------------------------------------
constexpr int kRedBlocks = 1024;
constexpr int kRedThreads = 256;

int red_partials() { return kRedBlocks; }

__device__ __forceinline__ double block_tree_sum(double acc, double *red) {
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kRedThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  return red[0];
}

__global__ void __launch_bounds__(kRedThreads) k_residual(float *du, const float *ddu, const float *dobs, long n,
                                                          double *part) {
  __shared__ double red[kRedThreads];
  double acc = 0.0;
  for (long i = (long)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (long)kRedBlocks * kRedThreads) {
    const float r = du[i] + ddu[i] - dobs[i];
    du[i] = r;
    acc += (double)r * (double)r;
  }
  const double s = block_tree_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// *target = base (or *target when base is null) + scale * sum of the partials
__global__ void __launch_bounds__(kRedThreads) k_red_final(const double *part, double *target, const double *base,
                                                           double scale, double base_scale) {
  __shared__ double red[kRedThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < kRedBlocks; i += kRedThreads) acc += part[i];
  const double s = block_tree_sum(acc, red);
  if (threadIdx.x == 0) *target = base_scale * (base ? *base : *target) + scale * s;
}

hipError_t launch_residual(float *du, const float *ddu, const float *dobs, long n, double *part, double *sumsq,
                           hipStream_t st) {
  k_residual<<<kRedBlocks, kRedThreads, 0, st>>>(du, ddu, dobs, n, part);
  k_red_final<<<1, kRedThreads, 0, st>>>(part, sumsq, nullptr, 1.0, 1.0);
  return hipGetLastError();
}

__global__ void k_fill_d(double *a, long n, double v) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) a[i] = v;
}

hipError_t launch_zero_d(double *a, long n, hipStream_t st) {
  long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  k_fill_d<<<(unsigned)blocks, 256, 0, st>>>(a, n, 0.0);
  return hipGetLastError();
}

__global__ void k_sum2(float *out, const float *a, const float *b, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    out[i] = a[i] + b[i];
}

hipError_t launch_residual_sum(float *out, const float *a, const float *b, long n, hipStream_t st) {
  long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  k_sum2<<<(unsigned)blocks, 256, 0, st>>>(out, a, b, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Finalizers
// ---------------------------------------------------------------------------
__global__ void k_ext_finalize(const double *acc, const float *vel, int nz, int nx, int nh, float dt,
                               const float *pt, const float *e2d2, float *out) {
  const long n = (long)nh * nx * nz;
  const long plane = (long)nx * nz;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float v = vel[i % plane];
    float r = (float)(2.0 * acc[i] / (double)(v * v * v * dt * dt));
    if (pt != nullptr) r += e2d2[i / plane] * pt[i];
    out[i] = r;
  }
}

hipError_t launch_ext_finalize(const double *acc, const float *vel, const ExtGeom &g, float dt,
                               const float *ptilde, const float *dso2eps2, float *out, hipStream_t st) {
  const long n = (long)g.nh * g.nx * g.nz;
  long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  k_ext_finalize<<<(unsigned)blocks, 256, 0, st>>>(acc, vel, g.nz, g.nx, g.nh, dt, ptilde, dso2eps2, out);
  return hipGetLastError();
}

// grad(y, z) = 2/(v^3 dt^2) sum_{padded cells copied from (y,z)} gacc - 3/v sum_h p~ img
__global__ void k_grad_finalize(const float *gacc, const float *vel, int nz, int nx, int nb, int NZ, int NX, int LZ,
                                int nh, float dt, const float *pt, const float *img, float *grad) {
  const long plane = (long)nx * nz;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= plane) return;
  const int y = (int)(i / nz);
  const int z = (int)(i - (long)y * nz);
  const int x0 = (y == 0) ? 0 : nb + y;
  const int x1 = (y == nx - 1) ? NX - 1 : nb + y;
  const int z0 = (z == 0) ? 0 : nb + z;
  const int z1 = (z == nz - 1) ? NZ - 1 : nb + z;
  float sum = 0.f;
  for (int x = x0; x <= x1; ++x)
    for (int zz = z0; zz <= z1; ++zz) sum += gacc[(long)x * LZ + zz];
  const float v = vel[i];
  float g = 2.f * sum / (v * v * v * dt * dt);
  if (pt != nullptr) {
    float t = 0.f;
    for (int h = 0; h < nh; ++h) t += pt[h * plane + i] * img[h * plane + i];
    g -= 3.f * t / v;
  }
  grad[i] = g;
}

hipError_t launch_grad_finalize(const float *gacc, const float *V, const float *vel, const ExtGeom &g, float dt,
                                const float *ptilde, const float *img, float *grad, hipStream_t st) {
  (void)V;
  const long plane = (long)g.nx * g.nz;
  k_grad_finalize<<<(unsigned)((plane + 255) / 256), 256, 0, st>>>(gacc, vel, g.nz, g.nx, g.nb, g.NZ, g.NX, g.LZ,
                                                                    g.nh, dt, ptilde, img, grad);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kRedThreads) k_obj_reg(const float *pt, const float *e2d2, long plane, int nh,
                                                         double *part) {
  __shared__ double red[kRedThreads];
  double acc = 0.0;
  const long n = plane * nh;
  for (long i = (long)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += (long)kRedBlocks * kRedThreads) {
    const double p = pt[i];
    acc += (double)e2d2[i / plane] * p * p;
  }
  const double s = block_tree_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

hipError_t launch_objective(const double *sumsq, const float *ptilde, const float *eps2d2, const ExtGeom &g,
                            double *part, double *obj, hipStream_t st) {
  const long plane = (long)g.nx * g.nz;
  k_obj_reg<<<kRedBlocks, kRedThreads, 0, st>>>(ptilde, eps2d2, plane, g.nh, part);
  // obj = 0.5 sumsq + 0.5 sum_h eps^2 d_h^2 ||p~_h||^2
  k_red_final<<<1, kRedThreads, 0, st>>>(part, obj, sumsq, 0.5, 0.5);
  return hipGetLastError();
}

}  // namespace fw

// Internal declarations shared by the kernel and runtime translation units.
// Not part of the public ABI (include/fwime.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace fw {

constexpr int kTZ = 64;        // rows (z) per tile: one wavefront, lane = z
constexpr int kR = 4;          // stencil radius (8th-order second derivative)
constexpr int kWaves = 4;      // wavefronts per stencil workgroup
constexpr int kTZ2 = 56;       // output rows per tile of the two-step kernel (64 lanes = rows z0-4 .. z0+59)

// Raw buffer access: per-lane 32-bit byte offset (the row) plus a wave-uniform
// byte offset (the column) that lives in a scalar register, so no 64-bit
// address arithmetic is spent per access.  The hardware range check covers
// the per-lane offset only (offset >= the buffer's byte size reads as zero and
// drops a store), not the scalar one: an access whose column comes in the
// scalar offset is guarded, or clamped into the grid; one that folds the
// column into the per-lane offset can instead be sent past the end with
// kOutOfRange to read zero without a branch.
constexpr int kOutOfRange = (int)0x80000000u;   // beyond any field (fields are < 2 GiB)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, float v, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}
__device__ __forceinline__ unsigned short ld16(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
}
__device__ __forceinline__ void st16(__amdgpu_buffer_rsrc_t r, unsigned short v, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b16(v, r, voff, soff, 0);
}

// Order of the stencil tiles of one launch (S shots, ntz x ntx tiles each).
// Columns of tiles are taken kTileGroupX x-strips at a time; inside a group
// one shot's tiles come together (z fastest), then the next shot's tiles of
// the same group.  Consecutive workgroups are thus spatial neighbours of one
// shot (their shared halo columns and rows are still in L2) and the velocity
// tile of the group is reused by every shot while it is cached.
constexpr int kTileGroupX = 4;

__host__ __device__ inline long tile_index(int txi, int tzi, int s, int ntz, int ntx, int S) {
  const int xg = txi / kTileGroupX, txl = txi - xg * kTileGroupX;
  const int ngx = min(kTileGroupX, ntx - xg * kTileGroupX);
  return (long)xg * kTileGroupX * ntz * S + ((long)s * ngx + txl) * ntz + tzi;
}

__host__ __device__ inline void tile_coords(int logical, int ntz, int ntx, int S, int &txi, int &tzi, int &s) {
  const int per_group = kTileGroupX * ntz * S;
  const int xg = logical / per_group;
  const int rem = logical - xg * per_group;
  const int ngx = min(kTileGroupX, ntx - xg * kTileGroupX);
  s = rem / (ngx * ntz);
  const int r2 = rem - s * ngx * ntz;
  const int txl = r2 / ntz;
  tzi = r2 - txl * ntz;
  txi = xg * kTileGroupX + txl;
}

// Per-tile injection list (compressed rows over tile*kWaves + wave).
// An entry {(j << 6) | lz, idx} adds  val[idx * stride_idx + t] * scale  to the
// source term of the cell in column j (of the wave's columns) and row lz.
struct Inject {
  const int *ptr = nullptr;     // [ntiles_total * kWaves + 1]
  const int2 *ent = nullptr;
  const float *val = nullptr;
  long stride_idx = 0;
  int t = 0;
  float scale = 1.f;
};

// Per-tile extraction list (compressed rows over tiles).  An entry
// {(lx << 6) | lz, idx} stores the INPUT field's value of that interior tile
// cell to out[idx * stride_idx + t].
struct Extract {
  const int *ptr = nullptr;     // [ntiles_total + 1]
  const int2 *ent = nullptr;
  float *out = nullptr;
  long stride_idx = 0;
  int t = 0;
};

// Dense source term read from three time slots of a field ring (the
// transposed second time difference e_{k-1}/g - 2 e_k + g e_{k+1}).
struct NuSource {
  const float *em = nullptr, *e0 = nullptr, *ep = nullptr;   // shot 0 slot pointers
  long sstride = 0;                                          // per-shot stride
};

struct StepArgs {
  const float *cur = nullptr;   // field at the current time, [S][NX][LZ]
  const float *prev = nullptr;  // field one step behind (read)
  float *out = nullptr;         // next field (may alias prev)
  const float *V = nullptr;     // v^2 dt^2, [NX][LZ]
  const float *gz = nullptr;    // taper along z, [LZ]
  const float *gx = nullptr;    // taper along x, [NX]
  float *t2 = nullptr;          // optional V (L cur + src) output, [S] x t2_sstride
  long t2_sstride = 0;
  const float *dsrc = nullptr;  // optional dense source, [S] x dsrc_sstride
  long dsrc_sstride = 0;
  NuSource nu;
  Inject inj;
  Extract ext;
  int NZ = 0, NX = 0, LZ = 0;
  int nshots = 0, ntz = 0, ntx = 0;
  long sstride = 0;             // elements between shots in cur/prev/out
  float cz[kR] = {};            // w_k / dz^2
  float cx[kR] = {};            // w_k / dx^2
  int fs = -1;                  // padded row of a free surface (mode kModeFS), -1: none
};

enum StepMode : int {
  kModePlain = 0,
  kModeT2 = 1,       // also write V (L cur + src)
  kModeDsrc = 2,     // add a dense source field
  kModeNu = 4,       // add the e-ring second time difference as a dense source
  kModeDF = 8,       // two-step kernel only: fields carried as FP32 hi + BF16 lo
  // Free surface on row fs (image method): the field is zero at and above
  // row fs, and the Laplacian of the rows below reads the field mirrored with
  // opposite sign above it, u(fs - k) = -u(fs + k).  The launch functions add
  // this bit themselves when StepArgs::fs >= 0; with fs = -1 the FS kernels
  // compute exactly what the plain ones do.
  kModeFS = 16,
};

// Rows fs-kR .. fs-1 above a free surface on row fs (none when fs < 0: a job
// without a free surface served by a free-surface multi-job launch).
__device__ __forceinline__ bool fs_mirrored(int z, int fs) { return fs >= 0 && z >= fs - kR && z < fs; }

// Row read for the stencil operand of padded row z under a free surface on
// row fs: rows fs-kR .. fs-1 read the mirrored row 2 fs - z with opposite sign.
__device__ __forceinline__ int fs_mirror_row(int z, int fs, float &sign) {
  const bool m = fs_mirrored(z, fs);
  sign = m ? -1.f : 1.f;
  return m ? 2 * fs - z : z;
}

// One job of a multi-job launch: its step arguments (cur/prev/out are chosen
// per step from bufA/bufB by the parity of the job's time index), the job's
// first tile in the launch, its time origin and length.
struct BatchJob {
  StepArgs a;
  float *bufA = nullptr, *bufB = nullptr;
  int tile_begin = 0;    // prefix of (tiles x shots) over the preceding jobs
  int t0 = 0;            // global step at which the job's time index is 0
  int nt = 0;
};

// Two time steps per launch (see kernels_step2.hip).  a.prev = u^{n-1} and
// a.cur = u^n (both read with halos), a.out = u^{n+1}, out2 = u^{n+2}: four
// distinct buffers.  a.inj lists the step-1 sources per (tile, wave) over the
// tile plus a 4-cell halo (time a.inj.t = n), inj2 the step-2 sources on the
// tile (time n + 1).  a.ext samples u^n at a.ext.t and u^{n+1} at a.ext.t + 1.
// a.t2 / t2b receive V (L u + f) of the two steps (mode kModeT2); a.dsrc /
// dsrc2 are dense sources of the two steps (mode kModeDsrc, a.dsrc read on
// the halo: it must not alias a.t2).  a.ntz counts 56-row tiles.  two == 0:
// one step only (no out2, t2b, dsrc2, inj2, second sample).
struct Step2Args {
  StepArgs a;
  float *out2 = nullptr;
  float *t2b = nullptr;
  const float *dsrc2 = nullptr;
  NuSource nu2;                 // mode kModeNu: slots of the second step (a.nu: first)
  Inject inj2;
  // mode kModeDF: BF16 low parts of prev / cur / out / out2 (same layout and
  // shot stride as the FP32 fields)
  const unsigned short *lo_prev = nullptr, *lo_cur = nullptr;
  unsigned short *lo_out = nullptr, *lo_out2 = nullptr;
  int two = 1;
};

// mode: kModePlain, kModeT2, kModeDsrc, kModeT2 | kModeDsrc (a.t2 and a.dsrc in
// distinct buffers), kModeNu, kModeDF, kModeT2 | kModeDF or kModeDsrc | kModeDF
// (plus kModeFS, added when p.a.fs >= 0)
hipError_t launch_step2(const Step2Args &p, int tile_x, int mode, hipStream_t st);

// One job of a two-step multi-job launch: its step arguments (fields, times
// and the step flag are filled in per launch from buf and the step counter),
// four field buffers, first tile in the launch, time origin and length.
struct BatchJob2 {
  Step2Args p;
  float *buf[4] = {nullptr, nullptr, nullptr, nullptr};
  int tile_begin = 0;
  int t0 = 0;
  int nt = 0;
};

// The global step is *step when `step` is non-null (a device counter that
// graph replays advance with launch_bump), else step_val.  fs: some job has
// a free surface (the FS kernel then serves every job of the launch).
// tile_job: job of every tile of the launch, or null (binary search over the
// jobs' tile_begin).
hipError_t launch_step2_multi(const BatchJob2 *jobs, const int *tile_job, int njobs, int total_tiles, const int *step,
                              int step_val, int tile_x, bool fs, hipStream_t st);

hipError_t launch_step_multi(const BatchJob *jobs, int njobs, int total_tiles, const int *step, int step_val,
                             int tile_x, bool fs, hipStream_t st);
hipError_t launch_bump(int *step, int by, hipStream_t st);

// Tile width in x of the stencil kernel (columns per workgroup).
int step_tile_x_supported(int tx);
hipError_t launch_step(const StepArgs &a, int tile_x, int mode, hipStream_t st);

// out[s][r][t] = field[s][cell[s][r]] (cell = padded x * LZ + z)
hipError_t launch_gather(const float *field, long sstride, const int *cells, int nshots, int nrec,
                         float *out, long stride_r, int t, hipStream_t st);

// V = vpad^2 dt^2 on the padded grid (edge replication) and model-grid coefficient fields.
hipError_t launch_prep(const float *vel, int nz, int nx, int nb, int NZ, int NX, int LZ, float dt,
                       float *V, hipStream_t st);

// min, max and non-finite count of a device array (result in a device buffer of 3 doubles)
hipError_t launch_minmax(const float *a, long n, double *res, hipStream_t st);

// Fill a float array with zeros (kernel, usable under graph capture).
hipError_t launch_zero(float *a, long n, hipStream_t st);

// dst[s * dst_sstride + i] = src[s * src_sstride + i], i < n, s < S
hipError_t launch_copy_fields(float *dst, long dst_sstride, const float *src, long src_sstride, int S, long n,
                              hipStream_t st);

// ---------------------------------------------------------------------------
// Subsurface-offset kernels.  Coefficient field c(z,y,h) = 2 p~ / (v^3 dt^2)
// lives on the model grid as [nh][nx][nz].  Fields are padded [NX][LZ].
// ---------------------------------------------------------------------------
struct ExtGeom {
  int nz = 0, nx = 0, nb = 0, NZ = 0, NX = 0, LZ = 0, nh = 0, H = 0;
};

// c = 2 p~ / (v^3 dt^2)
hipError_t launch_ext_coef(const float *ptilde, const float *vel, const ExtGeom &g, float dt, float *coef,
                           hipStream_t st);

// For n < nk and every shot: out_n(z, j) = sum_h c(z, j - sg h, h) in_n(z, j - 2 sg h)
// (sg = +1: extended scattering source; sg = -1: its transpose, the spread of
// the receiver-side field).  in/out slot n of shot s at base + s*sstride + n*slot.
hipError_t launch_ext_scatter(const float *coef, const ExtGeom &g, int sg, const float *in, long in_slot,
                              float *out, long out_slot, long sstride, int nshots, int nk, hipStream_t st,
                              int in_ring = 0, int in_first = 0, int out_ring = 0, int out_first = 0);

// acc(z,y,h) += sum_s sum_{n<nk} a_n(z, y-h) b_n(z, y+h) (FP64 accumulator;
// products summed in FP32 over at most 512 slots of a slot group while there
// are at most kImageGroups groups).  Slot n of a is a + n*a_slot; slot of b
// is ring index (b_first + n) % b_ring.  parts: scratch for up to kImageGroups
// FP32 partial images ([kImageGroups][nh][nx][nz]), one per slot group.
constexpr int kImageGroups = 16;
hipError_t launch_ext_image(const float *a, long a_slot, long a_sstride, const float *b, long b_slot, long b_sstride,
                            int b_ring, int b_first, int nshots, int nk, const ExtGeom &g, double *acc,
                            float *parts, hipStream_t st);

// Time-lag extension, lags tau_k = k L dt, k in [-K, K] (g.nh = 2K+1, g.H = K).
// Slots hold one padded field per time step, slot n of shot s at
// base + s*sstride + n*slot; nslots = nt - 1 steps.
//   scatter: out_n(z, y) = sum_k c(z, y, k) in_{n-2kL}(z, y) on the model grid
//            (terms with n - 2kL outside [0, nslots) dropped; cells outside the
//            model grid are not written)
//   image:   acc(z, y, k) += 2 / (v(z,y)^3 dt^2) sum_s sum_n in_{n-2kL}(z, y) lam_n(z, y)
hipError_t launch_tau_scatter(const float *coef, const ExtGeom &g, int L, const float *in, float *out, long slot,
                              long sstride, int nslots, int nshots, hipStream_t st);
hipError_t launch_tau_image(const float *in, long in_slot, long in_sstride, const float *lam, long lam_slot,
                            long lam_sstride, int nslots, int nshots, const ExtGeom &g, int L, const float *vel,
                            float dt, float *acc, hipStream_t st);

// gacc(x,z) += sum_s sum_{n<nk} (t2u_n + t2d_n) lam_n + t2u_n rho_n
// (lam and rho in rings of the same shape)
hipError_t launch_grad_accum(const float *t2u, const float *t2d, long slot, long seg_sstride, const float *lam,
                             const float *rho, long ring_slot, long ring_sstride, int ring, int first, int nshots,
                             int nk, int NZ, int NX, int LZ, float *gacc, hipStream_t st);
// the same with lam and rho in rings of their own shapes
hipError_t launch_grad_accum2(const float *t2u, const float *t2d, long slot, long seg_sstride, const float *lam,
                              long lam_slot, long lam_sstride, int lam_ring, int lam_first, const float *rho,
                              long rho_slot, long rho_sstride, int rho_ring, int rho_first, int nshots, int nk,
                              int NZ, int NX, int LZ, float *gacc, hipStream_t st);

// r = du + ddu - dobs (in place into du), sum r^2 ADDED to *sumsq (double);
// part: red_partials() doubles of scratch.  The sum is taken in a fixed order.
hipError_t launch_residual(float *du, const float *ddu, const float *dobs, long n, double *part, double *sumsq,
                           hipStream_t st);
int red_partials();
// a[0 .. n) = 0 (a kernel, usable under graph capture)
hipError_t launch_zero_d(double *a, long n, hipStream_t st);

// out = a + b (receiver data of u and du~)
hipError_t launch_residual_sum(float *out, const float *a, const float *b, long n, hipStream_t st);

// ptilde_out = 2/(v^3 dt^2) acc  (+ eps^2 d_h^2 p~ when ptilde != null)
hipError_t launch_ext_finalize(const double *acc, const float *vel, const ExtGeom &g, float dt,
                               const float *ptilde, const float *dso2eps2, float *out, hipStream_t st);

// grad_vel = P^T (2/(v^3 dt^2) gacc) - 3/v sum_h p~ img   (img already scaled)
hipError_t launch_grad_finalize(const float *gacc, const float *V, const float *vel, const ExtGeom &g,
                                float dt, const float *ptilde, const float *img, float *grad, hipStream_t st);

// obj = 0.5 * sumsq + 0.5 * sum_h eps2d2[h] ||p~_h||^2 (fixed summation order;
// part: red_partials() doubles of scratch)
hipError_t launch_objective(const double *sumsq, const float *ptilde, const float *eps2d2, const ExtGeom &g,
                            double *part, double *obj, hipStream_t st);

// Vector kernels of the variable-projection solver (kernels_vec.hip).
// out = a - b
hipError_t launch_sub(const float *a, const float *b, float *out, long n, hipStream_t st);
// *out = sum_i x[i] y[i] in FP64, fixed reduction order; part holds dot_partials() doubles
hipError_t launch_dot(const float *x, const float *y, long n, double *part, double *out, hipStream_t st);
int dot_partials();
// p += alpha s, r -= alpha q
hipError_t launch_cg_step(float *p, float *r, const float *s, const float *q, float alpha, long n, hipStream_t st);
// s = r + beta s
hipError_t launch_cg_dir(float *s, const float *r, float beta, long n, hipStream_t st);
// q[h] += e2d2[h] s[h] per offset plane of `plane` cells
hipError_t launch_add_diag(float *q, const float *s, const float *e2d2, long plane, int nh, hipStream_t st);

}  // namespace fw

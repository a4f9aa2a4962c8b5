// Host runtime of the FWIME hot-path library: the C ABI of include/fwime.h.
//
// Responsibilities: input validation (including the CFL test, which needs the
// velocity range and therefore one small device reduction), the context's
// device-memory arena under an HBM budget, the per-tile source/receiver tables
// consumed by the stencil kernel, shot batching, and the time loops with
// sqrt(nt) wavefield checkpointing for the adjoint-state operators.
//
// Time bookkeeping (equation n = 0 .. nt-2 advances u^n -> u^{n+1}):
//   - forward: the kernel of equation n reads u^n, u^{n-1}, writes u^{n+1},
//     injects f^n and records u^n at the receivers; u^{nt-1} is gathered after
//     the loop;
//   - adjoint: the kernel of index k = nt-1 .. 1 reads lambda_k, lambda_{k+1},
//     writes lambda_{k-1} and injects the adjoint source of time k;
//   - segments of K = ceil(sqrt(nt - 1)) equations: the forward pass stores
//     (u^{n0-1}, u^{n0}) at each segment start n0; the backward pass recomputes
//     one segment from its checkpoint, keeping T2u_n = V (L u^n + f^n) for the
//     segment, while the adjoint fields live in rings of K + 2 time slots.
#include "../../include/fwime.h"
#include "internal.h"
#include "line_search.h"

#include <algorithm>
#include <cstdint>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using namespace fw;

struct fwime_ctx {
  int device = 0;
  size_t budget = 0;
  std::string err;
  void *arena = nullptr;
  size_t arena_bytes = 0;
  double *host_red = nullptr;   // pinned: reduction results
  size_t host_red_n = 0;        // doubles it holds
  int tile_x = 32;
  bool two_step = true;         // plain propagation two time steps per launch
  size_t tape_bytes = 0;        // device memory held by live tapes
  size_t last_arena_request = 0;
  hipStream_t capture = nullptr;          // private stream used only to record graphs
  std::map<std::string, int> tuned;       // batch signature -> tile width
  int last_batch_tile = 0;
  int graph_steps = 64;                   // steps per captured graph
  hipGraph_t graph = nullptr;             // last batch graph, released after the
  hipGraphExec_t graph_exec = nullptr;    // next stream synchronization
  void *vp = nullptr;                     // variable-projection solver vectors
  size_t vp_bytes = 0;
  // optional timing of the stencil launch loop of the modeling calls: two
  // events recorded on the call's stream around its launches
  bool timing = false;
  hipEvent_t tev[2] = {nullptr, nullptr};
  long timed_launches = -1;               // launches between the events of the last timed call
  // while set, the call's scratch is carved from this fixed device buffer
  // instead of the arena, and nothing is allocated (fwime_model_static)
  char *fixed = nullptr;
  size_t fixed_bytes = 0;
  char *static_scratch = nullptr;         // device address of the static scratch array on `device`
};

static void release_graph(fwime_ctx_t *ctx) {
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  ctx->graph_exec = nullptr;
  ctx->graph = nullptr;
}

namespace {

constexpr int kSplineMaxNodes = 1 << 24;  // spline nodes per axis
constexpr int kLbfgsMaxPairs = 256;    // L-BFGS pairs accepted by fwime_lbfgs_direction
constexpr int kGxPad = 64;              // zero taper entries past NX read by the last x-tile
constexpr int kGraphMaxTiles = 16384;   // batches above this many tiles launch directly
constexpr double kW[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};

int set_err(fwime_ctx_t *ctx, int code, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return code;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return set_err(ctx, FWIME_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Events around a call's stencil launch loop (fwime_ctx_set_timing).
hipError_t timing_begin(fwime_ctx_t *ctx, hipStream_t st) {
  if (!ctx->timing) return hipSuccess;
  ctx->timed_launches = -1;
  return hipEventRecord(ctx->tev[0], st);
}
hipError_t timing_end(fwime_ctx_t *ctx, hipStream_t st, long launches) {
  if (!ctx->timing) return hipSuccess;
  hipError_t e = hipEventRecord(ctx->tev[1], st);
  if (e == hipSuccess) ctx->timed_launches = launches;
  return e;
}

double cfl_limit(double dz, double dx) {
  double nyq = -(kW[0] + 2.0 * (-kW[1] + kW[2] - kW[3] + kW[4]));
  return 2.0 / std::sqrt(nyq * (1.0 / (dz * dz) + 1.0 / (dx * dx)));
}

struct Dims {
  int nz, nx, nb, nt, NZ, NX, LZ, ntz, ntx, TX;
  int ntz2;     // 56-row tiles of the two-step kernel
  long field;   // NX * LZ
};

Dims make_dims(const fwime_grid_t *g, int tx) {
  Dims d;
  d.nz = g->nz;
  d.nx = g->nx;
  d.nb = g->nb;
  d.nt = g->nt;
  d.NZ = g->nz + 2 * g->nb;
  d.NX = g->nx + 2 * g->nb;
  d.LZ = (d.NZ + 4 + 63) / 64 * 64;   // >= 4 zero rows below the grid in every column
  d.TX = tx;
  d.ntz = (d.NZ + kTZ - 1) / kTZ;
  d.ntz2 = (d.NZ + kTZ2 - 1) / kTZ2;
  d.ntx = (d.NX + tx - 1) / tx;
  d.field = (long)d.NX * d.LZ;
  return d;
}

// ---------------------------------------------------------------------------
// Arena: one device allocation carved into aligned pieces for one call.
// ---------------------------------------------------------------------------
struct Carve {
  std::vector<std::pair<void **, size_t>> items;
  size_t total = 0;
  template <class T>
  void add(T **p, size_t count) {
    size_t bytes = (count * sizeof(T) + 255) / 256 * 256;
    items.push_back({(void **)p, bytes});
    total += bytes;
  }
  // point every piece into `base` (at least `total` bytes)
  void assign(void *base) const {
    char *p = (char *)base;
    for (const auto &it : items) {
      *it.first = p;
      p += it.second;
    }
  }
};

int arena_get(fwime_ctx_t *ctx, Carve &cv) {
  if (ctx->fixed) {
    if (cv.total > ctx->fixed_bytes)
      return set_err(ctx, FWIME_ENOMEM, "the call needs " + std::to_string(cv.total) +
                                            " bytes of scratch; the static scratch array holds " +
                                            std::to_string(ctx->fixed_bytes));
    cv.assign(ctx->fixed);
    return FWIME_OK;
  }
  if (cv.total > ctx->arena_bytes) {
    if (ctx->budget && cv.total > ctx->budget)
      return set_err(ctx, FWIME_ENOMEM, "request of " + std::to_string(cv.total) + " bytes exceeds the HBM budget");
    if (ctx->arena) {
      // the context's work runs on one stream, which every call synchronizes
      // during its input checks: the old arena is idle here
      HIPCHK(hipFree(ctx->arena));
      ctx->arena = nullptr;
      ctx->arena_bytes = 0;
    }
    // grow geometrically (within the budget) so that a sequence of slightly
    // larger calls does not reallocate every time
    size_t want = std::max(cv.total, ctx->last_arena_request + ctx->last_arena_request / 2);
    if (ctx->budget) want = std::min(want, ctx->budget);
    want = std::max(want, cv.total);
    hipError_t e = hipMalloc(&ctx->arena, want);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      want = cv.total;
      e = hipMalloc(&ctx->arena, want);
    }
    if (e != hipSuccess) {
      ctx->arena = nullptr;
      (void)hipGetLastError();
      return set_err(ctx, FWIME_ENOMEM, "hipMalloc of " + std::to_string(cv.total) + " bytes failed");
    }
    ctx->arena_bytes = want;
  }
  ctx->last_arena_request = std::max(ctx->last_arena_request, cv.total);
  char *p = (char *)ctx->arena;
  for (auto &it : cv.items) {
    *it.first = p;
    p += it.second;
  }
  return FWIME_OK;
}

// ---------------------------------------------------------------------------
// Validation
// ---------------------------------------------------------------------------
int check_grid(fwime_ctx_t *ctx, const fwime_grid_t *g) {
  if (!g) return set_err(ctx, FWIME_EINVAL, "grid is null");
  if (g->nz < 1 || g->nx < 1 || g->nb < 0 || g->nt < 2)
    return set_err(ctx, FWIME_EINVAL, "grid needs nz, nx >= 1, nb >= 0, nt >= 2");
  if (!(g->dz > 0 && g->dx > 0 && g->dt > 0) || !std::isfinite(g->dz) || !std::isfinite(g->dx) ||
      !std::isfinite(g->dt))
    return set_err(ctx, FWIME_EINVAL, "dz, dx, dt must be positive and finite");
  if (!(g->sponge_alpha >= 0) || !std::isfinite(g->sponge_alpha))
    return set_err(ctx, FWIME_EINVAL, "sponge_alpha must be >= 0");
  if (g->free_surface && g->nb < kR)
    return set_err(ctx, FWIME_EINVAL, "a free surface needs nb >= 4 (the mirrored stencil rows)");
  const long NZ = (long)g->nz + 2L * g->nb, NX = (long)g->nx + 2L * g->nb;
  const long LZ = (NZ + 4 + 63) / 64 * 64;
  // kernels address one shot's field with 32-bit byte offsets
  if ((NX + 256) * LZ * 4 >= (1L << 31)) return set_err(ctx, FWIME_EINVAL, "padded grid too large");
  return FWIME_OK;
}

int check_geom(fwime_ctx_t *ctx, const fwime_grid_t *g, const fwime_geom_t *geo) {
  if (!geo) return set_err(ctx, FWIME_EINVAL, "geometry is null");
  if (geo->nshots < 1 || geo->nrec < 1) return set_err(ctx, FWIME_EINVAL, "need nshots >= 1 and nrec >= 1");
  if (!geo->src_iz || !geo->src_ix || !geo->rec_iz || !geo->rec_ix || !geo->wavelet)
    return set_err(ctx, FWIME_EINVAL, "geometry pointer is null");
  for (int s = 0; s < geo->nshots; ++s) {
    if (geo->src_iz[s] < 0 || geo->src_iz[s] >= g->nz || geo->src_ix[s] < 0 || geo->src_ix[s] >= g->nx)
      return set_err(ctx, FWIME_EINVAL, "source " + std::to_string(s) + " outside the model grid");
  }
  const long n = (long)geo->nshots * geo->nrec;
  for (long i = 0; i < n; ++i) {
    if (geo->rec_iz[i] < 0 || geo->rec_iz[i] >= g->nz || geo->rec_ix[i] < 0 || geo->rec_ix[i] >= g->nx)
      return set_err(ctx, FWIME_EINVAL, "receiver " + std::to_string(i) + " outside the model grid");
  }
  return FWIME_OK;
}

int check_nh(fwime_ctx_t *ctx, const fwime_grid_t *g, int nh) {
  if (nh < 1 || nh % 2 == 0 || nh > 2 * g->nx - 1)
    return set_err(ctx, FWIME_EINVAL, "nh must be odd with 1 <= nh <= 2 nx - 1");
  return FWIME_OK;
}

// Pinned host space for at least n doubles of reduction results.
int host_red_reserve(fwime_ctx_t *ctx, size_t n) {
  if (n <= ctx->host_red_n) return FWIME_OK;
  if (ctx->fixed) return set_err(ctx, FWIME_ENOMEM, "too many arrays to validate without allocating");
  if (ctx->host_red) HIPCHK(hipHostFree(ctx->host_red));
  ctx->host_red = nullptr;
  ctx->host_red_n = 0;
  const size_t want = std::max<size_t>(n, 64);
  HIPCHK(hipHostMalloc((void **)&ctx->host_red, want * sizeof(double), hipHostMallocDefault));
  ctx->host_red_n = want;
  return FWIME_OK;
}

// min / max / non-finite count of several device arrays: one reduction per
// array into consecutive triples of a scratch buffer at the front of the
// arena, one copy to pinned host memory and one stream synchronization for
// all of them.  out[3 k .. 3 k + 2] describe array k.
int device_ranges(fwime_ctx_t *ctx, const std::vector<std::pair<const float *, long>> &arrays, hipStream_t st,
                  std::vector<double> &out) {
  const size_t n = arrays.size();
  double *scratch = nullptr;
  Carve cv;
  cv.add(&scratch, 3 * n);
  // later carves of the same call reuse this memory: the reductions are
  // complete once this function returns
  int rc = arena_get(ctx, cv);
  if (rc) return rc;
  if ((rc = host_red_reserve(ctx, 3 * n))) return rc;
  for (size_t k = 0; k < n; ++k) {
    if (!arrays[k].first) return set_err(ctx, FWIME_EINVAL, "input pointer is null");
    HIPCHK(launch_minmax(arrays[k].first, arrays[k].second, scratch + 3 * k, st));
  }
  HIPCHK(hipMemcpyAsync(ctx->host_red, scratch, 3 * n * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  out.assign(ctx->host_red, ctx->host_red + 3 * n);
  return FWIME_OK;
}

// Velocity range (positive, finite, CFL) from its min / max / non-finite triple.
int check_velocity_range(fwime_ctx_t *ctx, const fwime_grid_t *g, const double *r) {
  if (r[2] > 0) return set_err(ctx, FWIME_ENONFINITE, "vel has non-finite values");
  if (!(r[0] > 0)) return set_err(ctx, FWIME_EINVAL, "velocity must be positive");
  if (r[1] * g->dt > cfl_limit(g->dz, g->dx) * (1 + 1e-12))
    return set_err(ctx, FWIME_EINVAL, "CFL condition violated: v_max dt = " + std::to_string(r[1] * g->dt) +
                                          " > " + std::to_string(cfl_limit(g->dz, g->dx)));
  return FWIME_OK;
}

// Common prologue: validates velocity (positive, finite, CFL), the wavelets
// and the other float inputs in one device pass and one synchronization;
// runs before any output is touched.
int check_inputs(fwime_ctx_t *ctx, const fwime_grid_t *g, const float *vel, const fwime_geom_t *geo,
                 std::vector<std::pair<const float *, long>> extra, hipStream_t st) {
  if (!vel) return set_err(ctx, FWIME_EINVAL, "vel is null");
  std::vector<std::pair<const float *, long>> arrays{{vel, (long)g->nx * g->nz},
                                                     {geo->wavelet, (long)geo->nshots * g->nt}};
  arrays.insert(arrays.end(), extra.begin(), extra.end());
  std::vector<double> r;
  int rc = device_ranges(ctx, arrays, st, r);
  if (rc) return rc;
  if ((rc = check_velocity_range(ctx, g, r.data()))) return rc;
  for (size_t k = 1; k < arrays.size(); ++k)
    if (r[3 * k + 2] > 0) return set_err(ctx, FWIME_ENONFINITE, "input array has non-finite values");
  return FWIME_OK;
}

// ---------------------------------------------------------------------------
// Geometry tables for one batch of shots [s0, s0 + S).  Indices stored in the
// tables are batch-local (shot s, receiver s * nrec + r); callers offset the
// wavelet and data pointers to the batch start.
// ---------------------------------------------------------------------------
// One-step tiling (64-row tiles): src / rinj lists per (tile, wave) on the
// tile, rext per tile.  Two-step tiling (56-row tiles): src / rinj are the
// step-2 lists on the tile, src1 / rinj1 the step-1 lists over the tile plus
// a 4-cell halo, rext per tile.
struct HostTables {
  std::vector<int> src_ptr, rext_ptr, rinj_ptr, cells, src1_ptr, rinj1_ptr;
  std::vector<int2> src_ent, rext_ent, rinj_ent, src1_ent, rinj1_ent;
};

struct DevTables {
  int *src_ptr, *rext_ptr, *rinj_ptr, *cells, *src1_ptr, *rinj1_ptr;
  int2 *src_ent, *rext_ent, *rinj_ent, *src1_ent, *rinj1_ent;
};

void csr_build(std::vector<int> &ptr, std::vector<int2> &ent, long nbucket,
               const std::vector<std::pair<long, int2>> &items) {
  ptr.assign(nbucket + 1, 0);
  for (auto &it : items) ptr[it.first + 1]++;
  for (long b = 0; b < nbucket; ++b) ptr[b + 1] += ptr[b];
  ent.resize(items.size());
  std::vector<int> fill(ptr.begin(), ptr.end() - 1);
  for (auto &it : items) ent[fill[it.first]++] = it.second;
  // inject lists are consumed in column order by each wave
  for (long b = 0; b < nbucket; ++b)
    std::stable_sort(ent.begin() + ptr[b], ent.begin() + ptr[b + 1],
                     [](const int2 &a, const int2 &c) { return (a.x >> 6) < (c.x >> 6); });
}

HostTables build_tables(const Dims &d, const fwime_geom_t *geo, int s0, int S) {
  HostTables t;
  const int CPW = d.TX / kWaves;
  const long ntiles = (long)d.ntz * d.ntx * S;
  auto locate = [&](int s, int px, int pz, long &tile, int &lx, int &lz) {
    const int txi = px / d.TX, tzi = pz / kTZ;
    tile = tile_index(txi, tzi, s, d.ntz, d.ntx, S);
    lx = px - txi * d.TX;
    lz = pz - tzi * kTZ;
  };
  std::vector<std::pair<long, int2>> src, rext, rinj;
  for (int s = 0; s < S; ++s) {
    const int sg = s0 + s;
    long tile;
    int lx, lz;
    locate(s, geo->src_ix[sg] + d.nb, geo->src_iz[sg] + d.nb, tile, lx, lz);
    src.push_back({tile * kWaves + lx / CPW, make_int2(((lx % CPW) << 6) | lz, s)});
    for (int r = 0; r < geo->nrec; ++r) {
      const long ir = (long)sg * geo->nrec + r;      // global receiver (geometry lookup)
      const int il = s * geo->nrec + r;              // batch-local receiver (table index)
      const int px = geo->rec_ix[ir] + d.nb, pz = geo->rec_iz[ir] + d.nb;
      locate(s, px, pz, tile, lx, lz);
      rext.push_back({tile, make_int2((lx << 6) | lz, il)});
      rinj.push_back({tile * kWaves + lx / CPW, make_int2(((lx % CPW) << 6) | lz, il)});
      t.cells.push_back(px * d.LZ + pz);
    }
  }
  csr_build(t.src_ptr, t.src_ent, ntiles * kWaves, src);
  csr_build(t.rext_ptr, t.rext_ent, ntiles, rext);
  csr_build(t.rinj_ptr, t.rinj_ent, ntiles * kWaves, rinj);
  return t;
}

// Two-step tiling: a cell (px, pz) lies on the tile (txi, tzi) with
// txi = px / TX, tzi = pz / 56, and in the step-1 region (tile plus 4-cell
// halo) of every tile whose [x0 - 4, x0 + TX + 4) x [z0 - 4, z0 + 60) holds it.
HostTables build_tables2(const Dims &d, const fwime_geom_t *geo, int s0, int S) {
  HostTables t;
  const int W1 = (d.TX + 2 * kR) / kWaves, W2 = d.TX / kWaves;
  const long ntiles = (long)d.ntz2 * d.ntx * S;
  auto tile_of = [&](int s, int txi, int tzi) { return tile_index(txi, tzi, s, d.ntz2, d.ntx, S); };
  std::vector<std::pair<long, int2>> src1, src2, rext, rinj1, rinj2;
  auto add_inject = [&](int s, int px, int pz, int idx, std::vector<std::pair<long, int2>> &l1,
                        std::vector<std::pair<long, int2>> &l2) {
    const int txi = px / d.TX, tzi = pz / kTZ2;
    {
      const int lx = px - txi * d.TX, lane = pz - tzi * kTZ2 + kR;
      l2.push_back({tile_of(s, txi, tzi) * kWaves + lx / W2, make_int2(((lx % W2) << 6) | lane, idx)});
    }
    // candidate neighbours: the own tile and the ones before / after it
    for (int tx = std::max(0, txi - 1); tx <= std::min(d.ntx - 1, txi + 1); ++tx)
      for (int tz = std::max(0, tzi - 1); tz <= std::min(d.ntz2 - 1, tzi + 1); ++tz) {
        const int jj = px - (tx * d.TX - kR), lane = pz - (tz * kTZ2 - kR);
        if (jj < 0 || jj >= d.TX + 2 * kR || lane < 0 || lane >= 64) continue;
        l1.push_back({tile_of(s, tx, tz) * kWaves + jj / W1, make_int2(((jj % W1) << 6) | lane, idx)});
      }
  };
  for (int s = 0; s < S; ++s) {
    const int sg = s0 + s;
    add_inject(s, geo->src_ix[sg] + d.nb, geo->src_iz[sg] + d.nb, s, src1, src2);
    for (int r = 0; r < geo->nrec; ++r) {
      const long ir = (long)sg * geo->nrec + r;
      const int il = s * geo->nrec + r;
      const int px = geo->rec_ix[ir] + d.nb, pz = geo->rec_iz[ir] + d.nb;
      const int txi = px / d.TX, tzi = pz / kTZ2;
      rext.push_back({tile_of(s, txi, tzi), make_int2(((px - txi * d.TX) << 6) | (pz - tzi * kTZ2), il)});
      add_inject(s, px, pz, il, rinj1, rinj2);
      t.cells.push_back(px * d.LZ + pz);
    }
  }
  csr_build(t.src1_ptr, t.src1_ent, ntiles * kWaves, src1);
  csr_build(t.src_ptr, t.src_ent, ntiles * kWaves, src2);
  csr_build(t.rext_ptr, t.rext_ent, ntiles, rext);
  csr_build(t.rinj1_ptr, t.rinj1_ent, ntiles * kWaves, rinj1);
  csr_build(t.rinj_ptr, t.rinj_ent, ntiles * kWaves, rinj2);
  return t;
}

size_t tables_ints(const HostTables &t) {
  return t.src_ptr.size() + t.rext_ptr.size() + t.rinj_ptr.size() + t.cells.size() + t.src1_ptr.size() +
         t.rinj1_ptr.size() +
         2 * (t.src_ent.size() + t.rext_ent.size() + t.rinj_ent.size() + t.src1_ent.size() + t.rinj1_ent.size()) +
         11 * 64;
}

// Lay out all batch tables into one host blob and one device buffer.
struct TableSet {
  std::vector<HostTables> host;
  std::vector<DevTables> dev;
  std::vector<int> blob;
};

TableSet build_table_set(const Dims &d, const fwime_geom_t *geo, const std::vector<std::pair<int, int>> &batches,
                         bool two_step = false) {
  TableSet ts;
  for (auto &b : batches)
    ts.host.push_back(two_step ? build_tables2(d, geo, b.first, b.second) : build_tables(d, geo, b.first, b.second));
  return ts;
}

size_t table_set_ints(const TableSet &ts) {
  size_t n = 0;
  for (auto &t : ts.host) n += tables_ints(t);
  return n;
}

// sync = false: the copy may still read ts.blob after the call returns, so
// the caller keeps ts alive until the stream has passed the copy.
int upload_tables(fwime_ctx_t *ctx, TableSet &ts, int *dev, hipStream_t st, bool sync = true) {
  ts.blob.clear();
  ts.dev.clear();
  auto put = [&](const void *src, size_t nint) -> size_t {
    size_t off = (ts.blob.size() + 63) / 64 * 64;
    ts.blob.resize(off + nint);
    if (nint) std::memcpy(ts.blob.data() + off, src, nint * sizeof(int));
    return off;
  };
  std::vector<std::vector<size_t>> offs;
  for (auto &t : ts.host) {
    std::vector<size_t> o;
    o.push_back(put(t.src_ptr.data(), t.src_ptr.size()));
    o.push_back(put(t.rext_ptr.data(), t.rext_ptr.size()));
    o.push_back(put(t.rinj_ptr.data(), t.rinj_ptr.size()));
    o.push_back(put(t.cells.data(), t.cells.size()));
    o.push_back(put(t.src_ent.data(), 2 * t.src_ent.size()));
    o.push_back(put(t.rext_ent.data(), 2 * t.rext_ent.size()));
    o.push_back(put(t.rinj_ent.data(), 2 * t.rinj_ent.size()));
    o.push_back(put(t.src1_ptr.data(), t.src1_ptr.size()));
    o.push_back(put(t.src1_ent.data(), 2 * t.src1_ent.size()));
    o.push_back(put(t.rinj1_ptr.data(), t.rinj1_ptr.size()));
    o.push_back(put(t.rinj1_ent.data(), 2 * t.rinj1_ent.size()));
    offs.push_back(o);
  }
  for (auto &o : offs) {
    DevTables dt;
    dt.src_ptr = dev + o[0];
    dt.rext_ptr = dev + o[1];
    dt.rinj_ptr = dev + o[2];
    dt.cells = dev + o[3];
    dt.src_ent = (int2 *)(dev + o[4]);
    dt.rext_ent = (int2 *)(dev + o[5]);
    dt.rinj_ent = (int2 *)(dev + o[6]);
    dt.src1_ptr = dev + o[7];
    dt.src1_ent = (int2 *)(dev + o[8]);
    dt.rinj1_ptr = dev + o[9];
    dt.rinj1_ent = (int2 *)(dev + o[10]);
    ts.dev.push_back(dt);
  }
  // With sync the blob is copied synchronously (pageable memory): the call
  // owns no host staging that could outlive it.
  HIPCHK(hipMemcpyAsync(dev, ts.blob.data(), ts.blob.size() * sizeof(int), hipMemcpyHostToDevice, st));
  if (sync) HIPCHK(hipStreamSynchronize(st));
  return FWIME_OK;
}

// ---------------------------------------------------------------------------
// Shared per-call state
// ---------------------------------------------------------------------------
struct Common {
  Dims d;
  float *V = nullptr, *gz = nullptr, *gx = nullptr;
  int *tables = nullptr;
  StepArgs base;
};

void taper_host(int n, int nb, double alpha, int len, std::vector<float> &out) {
  out.assign(len, 0.f);
  for (int i = 0; i < n + 2 * nb; ++i) {
    int k = 0;
    if (i < nb) k = nb - i;
    else if (i >= nb + n) k = i - (nb + n - 1);
    const double a = nb > 0 ? alpha * k / nb : 0.0;
    out[i] = (float)std::exp(-a * a);
  }
}

int setup_common(fwime_ctx_t *ctx, Common &c, const fwime_grid_t *g, const float *vel, hipStream_t st) {
  const Dims &d = c.d;
  HIPCHK(launch_prep(vel, d.nz, d.nx, d.nb, d.NZ, d.NX, d.LZ, (float)g->dt, c.V, st));
  std::vector<float> gz, gx;
  taper_host(d.nz, d.nb, g->sponge_alpha, d.LZ, gz);
  taper_host(d.nx, d.nb, g->sponge_alpha, d.NX + kGxPad, gx);
  HIPCHK(hipMemcpyAsync(c.gz, gz.data(), gz.size() * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(c.gx, gx.data(), gx.size() * sizeof(float), hipMemcpyHostToDevice, st));
  StepArgs &a = c.base;
  a = StepArgs();
  a.V = c.V;
  a.gz = c.gz;
  a.gx = c.gx;
  a.NZ = d.NZ;
  a.NX = d.NX;
  a.LZ = d.LZ;
  a.ntz = d.ntz;
  a.ntx = d.ntx;
  a.fs = g->free_surface ? d.nb : -1;
  const double idz2 = 1.0 / (g->dz * g->dz), idx2 = 1.0 / (g->dx * g->dx);
  for (int k = 0; k < kR; ++k) {
    a.cz[k] = (float)(kW[k + 1] * idz2);
    a.cx[k] = (float)(kW[k + 1] * idx2);
  }
  return FWIME_OK;
}

// Step-argument helpers for one batch.
StepArgs batch_args(const Common &c, int S, long sstride) {
  StepArgs a = c.base;
  a.nshots = S;
  a.sstride = sstride;
  return a;
}

void with_src_w(StepArgs &a, const DevTables &t, const float *wav_b, const fwime_grid_t *g, int n) {
  a.inj.ptr = t.src_ptr;
  a.inj.ent = t.src_ent;
  a.inj.val = wav_b;
  a.inj.stride_idx = g->nt;
  a.inj.t = n;
  a.inj.scale = (float)(1.0 / (g->dx * g->dz));
}

void with_src(StepArgs &a, const DevTables &t, const fwime_geom_t *geo, const fwime_grid_t *g, int s0, int n) {
  with_src_w(a, t, geo->wavelet + (long)s0 * g->nt, g, n);
}

void with_rec_inject(StepArgs &a, const DevTables &t, const float *data, int nt, int k) {
  a.inj.ptr = t.rinj_ptr;
  a.inj.ent = t.rinj_ent;
  a.inj.val = data;
  a.inj.stride_idx = nt;
  a.inj.t = k;
  a.inj.scale = 1.f;
}

void with_rec_extract(StepArgs &a, const DevTables &t, float *data, int nt, int n) {
  a.ext.ptr = t.rext_ptr;
  a.ext.ent = t.rext_ent;
  a.ext.out = data;
  a.ext.stride_idx = nt;
  a.ext.t = n;
}

// Four field buffers of one batch for the two-step kernel: prev = f[i],
// cur = f[i + 1]; a launch of k steps writes f[i + 2] (and f[i + 3]) and
// advances i by k.  Neither output buffer is read by that launch, and after
// it u^{n-1}, u^n, u^{n+1}, u^{n+2} are all still in memory.
template <class T>
struct Ring4T {
  T *f[4];
  int i = 0;
  Ring4T(T *base, long stride) {
    for (int k = 0; k < 4; ++k) f[k] = base + k * stride;
  }
  T *at(int k) const { return f[(i + k) & 3]; }
  T *prev() const { return at(0); }
  T *cur() const { return at(1); }
  void advance(int k) { i += k; }
};
using Ring4 = Ring4T<float>;
using Ring4L = Ring4T<unsigned short>;   // BF16 low parts of an extended-precision field

Step2Args step2_args(const Common &c, const Ring4 &f, int S, long sstride, int k) {
  Step2Args p;
  p.a = batch_args(c, S, sstride);
  p.a.ntz = c.d.ntz2;
  p.a.prev = f.prev();
  p.a.cur = f.cur();
  p.a.out = f.at(2);
  p.out2 = k == 2 ? f.at(3) : nullptr;
  p.two = k == 2;
  return p;
}

// point sources: step-1 list at time n, step-2 list at time n + 1
void with_src2(Step2Args &p, const DevTables &t, const float *wav_b, const fwime_grid_t *g, int n) {
  with_src_w(p.a, t, wav_b, g, n);
  p.a.inj.ptr = t.src1_ptr;
  p.a.inj.ent = t.src1_ent;
  p.inj2 = p.a.inj;
  p.inj2.ptr = t.src_ptr;
  p.inj2.ent = t.src_ent;
  p.inj2.t = n + 1;
}

// receiver injection (adjoint sources): time k1 of `data` in step 1, k2 in
// step 2 (k2 = k1 - 1 when the recursion runs backwards in time)
void with_rec_inject2(Step2Args &p, const DevTables &t, const float *data, int nt, int k1, int k2) {
  with_rec_inject(p.a, t, data, nt, k1);
  p.a.inj.ptr = t.rinj1_ptr;
  p.a.inj.ent = t.rinj1_ent;
  p.inj2 = p.a.inj;
  p.inj2.ptr = t.rinj_ptr;
  p.inj2.ent = t.rinj_ent;
  p.inj2.t = k2;
}

// Advances ring f over the steps n0 .. n1 - 1 forward in time: two steps per
// launch, one in the last launch when the count is odd.  setup(p, n, k) adds
// the step-specific arguments of the launch that starts at step n.
// With lo != nullptr the field is carried in extended precision (mode gets
// kModeDF) and lo rotates with f.
template <class Setup>
int march2(fwime_ctx_t *ctx, const Common &c, Ring4 &f, int S, int n0, int n1, int mode, Setup setup,
           hipStream_t st, Ring4L *lo = nullptr) {
  for (int n = n0; n < n1;) {
    const int k = std::min(2, n1 - n);
    Step2Args p = step2_args(c, f, S, c.d.field, k);
    if (lo) {
      p.lo_prev = lo->prev();
      p.lo_cur = lo->cur();
      p.lo_out = lo->at(2);
      p.lo_out2 = k == 2 ? lo->at(3) : nullptr;
    }
    setup(p, n, k);
    HIPCHK(launch_step2(p, c.d.TX, lo ? (mode | kModeDF) : mode, st));
    f.advance(k);
    if (lo) lo->advance(k);
    n += k;
  }
  return FWIME_OK;
}

// dense source of a two-step launch: slot `first` for its first step, the
// next slot (`slot` elements on) for its second; per-shot stride sstride
void with_dsrc2(Step2Args &p, const float *first, long slot, int k, long sstride) {
  p.a.dsrc = first;
  p.dsrc2 = k == 2 ? first + slot : nullptr;
  p.a.dsrc_sstride = sstride;
}

// BF16 arrays copied as 32-bit words (fields hold an even number of cells)
hipError_t copy_lo(unsigned short *dst, long dst_sstride, const unsigned short *src, long src_sstride, int S, long n,
                   hipStream_t st) {
  return launch_copy_fields((float *)dst, dst_sstride / 2, (const float *)src, src_sstride / 2, S, n / 2, st);
}

// Adjoint recursion over a ring of R field slots (slot of time k: k % R),
// from time k = k1 down to k0 + 1, producing the fields of times k1 - 1 ..
// k0: two steps per launch.  setup(p, k, kk) adds the sources of the launch
// that starts at time k.
// With lo != nullptr (a BF16 ring of the same shape) the field is carried in
// extended precision (mode gets kModeDF).
template <class Setup>
int march2_back_ring(fwime_ctx_t *ctx, const Common &c, float *ring, long ring_stride, int R, int S, int k0, int k1,
                     int mode, Setup setup, hipStream_t st, unsigned short *lo = nullptr) {
  const long F = c.d.field;
  for (int k = k1; k >= k0 + 1;) {
    const int kk = (k - 2 >= k0) ? 2 : 1;
    Step2Args p;
    p.a = batch_args(c, S, ring_stride);
    p.a.ntz = c.d.ntz2;
    p.a.cur = ring + (long)(k % R) * F;
    p.a.prev = ring + (long)((k + 1) % R) * F;
    p.a.out = ring + (long)((k - 1) % R) * F;
    p.out2 = kk == 2 ? ring + (long)((k - 2) % R) * F : nullptr;
    p.two = kk == 2;
    if (lo) {
      p.lo_cur = lo + (long)(k % R) * F;
      p.lo_prev = lo + (long)((k + 1) % R) * F;
      p.lo_out = lo + (long)((k - 1) % R) * F;
      p.lo_out2 = kk == 2 ? lo + (long)((k - 2) % R) * F : nullptr;
    }
    setup(p, k, kk);
    HIPCHK(launch_step2(p, c.d.TX, lo ? (mode | kModeDF) : mode, st));
    k -= kk;
  }
  return FWIME_OK;
}

// lambda: receiver injection of `data` at the current time
int march2_back_lambda(fwime_ctx_t *ctx, const Common &c, float *ring, long ring_stride, int R, int S, int k0,
                       int k1, const DevTables &t, const float *data, int nt, hipStream_t st,
                       unsigned short *lo = nullptr) {
  return march2_back_ring(ctx, c, ring, ring_stride, R, S, k0, k1, kModePlain,
                          [&](Step2Args &p, int k, int) { with_rec_inject2(p, t, data, nt, k, k - 1); }, st, lo);
}

int choose_batch(fwime_ctx_t *ctx, long per_shot_bytes, size_t fixed_bytes, int nshots) {
  size_t cap = 0;
  if (ctx->fixed) {
    cap = ctx->fixed_bytes;                // the static scratch array is all there is
  } else {
    size_t avail = 0, total = 0;
    if (hipMemGetInfo(&avail, &total) != hipSuccess) avail = 0;
    avail += ctx->arena_bytes;             // the arena can be reused
    cap = (size_t)(avail * 0.85);
    if (ctx->budget && ctx->budget < cap) cap = ctx->budget;
  }
  if (cap <= fixed_bytes) return 1;
  long S = (long)((cap - fixed_bytes) / std::max<long>(per_shot_bytes, 1));
  S = std::max<long>(1, std::min<long>(S, nshots));
  return (int)S;
}

std::vector<std::pair<int, int>> split_batches(int nshots, int S) {
  std::vector<std::pair<int, int>> b;
  const int nb = (nshots + S - 1) / S;
  const int base = nshots / nb, extra = nshots % nb;   // balanced batch sizes
  int s0 = 0;
  for (int i = 0; i < nb; ++i) {
    const int n = base + (i < extra ? 1 : 0);
    b.push_back({s0, n});
    s0 += n;
  }
  return b;
}

// Segment length of the sqrt(nt) checkpointing, rounded up to an even count
// so two-step launches never straddle a segment start.
int seg_len(int nt) {
  int K = (int)std::ceil(std::sqrt((double)(nt - 1)));
  K = std::max(K, 1);
  return K + (K & 1);
}


}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *fwime_strerror(int code) {
  switch (code) {
    case FWIME_OK: return "ok";
    case FWIME_EINVAL: return "invalid argument";
    case FWIME_ENOMEM: return "out of device memory or HBM budget";
    case FWIME_EHIP: return "HIP runtime error";
    case FWIME_ENONFINITE: return "non-finite input";
    default: return "unknown error";
  }
}

const char *fwime_last_error(const fwime_ctx_t *ctx) { return ctx ? ctx->err.c_str() : ""; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Static scratch for the allocation-free entry point (fwime_model_static).
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is looked up once per device (fwime_ctx_create, with that
// device current) and only that address is ever passed to kernels or copies.
// Every call on a device shares its array.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[FWIME_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (the current device).
int static_scratch_address(int device, char **out) {
  if (device < 0 || device >= kMaxDevices) return FWIME_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return FWIME_EHIP;
    }
    g_scratch_ptr[device] = (char *)p;
  }
  *out = g_scratch_ptr[device];
  return FWIME_OK;
}
}  // namespace

extern "C" {


int fwime_ctx_create(int device, size_t hbm_budget_bytes, fwime_ctx_t **out) {
  if (!out) return FWIME_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FWIME_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return FWIME_EHIP;
  fwime_ctx_t *ctx = new fwime_ctx_t();
  ctx->device = device;
  ctx->budget = hbm_budget_bytes;
  if (host_red_reserve(ctx, 64) != FWIME_OK) {
    delete ctx;
    return FWIME_EHIP;
  }
  if (static_scratch_address(device, &ctx->static_scratch) != FWIME_OK) {
    (void)hipHostFree(ctx->host_red);
    delete ctx;
    return FWIME_EHIP;
  }
  const char *tx = std::getenv("FWIME_TILE_X");
  if (tx && step_tile_x_supported(std::atoi(tx))) ctx->tile_x = std::atoi(tx);
  // FWIME_STEP1=1: one time step per launch everywhere (same results, bit for bit)
  const char *s1 = std::getenv("FWIME_STEP1");
  if (s1 && std::atoi(s1) != 0) ctx->two_step = false;
  *out = ctx;
  return FWIME_OK;
}

int fwime_ctx_trim(fwime_ctx_t *ctx, void *stream) {
  if (!ctx) return FWIME_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return FWIME_EHIP;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return FWIME_EHIP;
  release_graph(ctx);
  if (ctx->arena && hipFree(ctx->arena) != hipSuccess) return FWIME_EHIP;
  ctx->arena = nullptr;
  ctx->arena_bytes = 0;
  ctx->last_arena_request = 0;
  if (ctx->vp && hipFree(ctx->vp) != hipSuccess) return FWIME_EHIP;
  ctx->vp = nullptr;
  ctx->vp_bytes = 0;
  return FWIME_OK;
}

int fwime_ctx_info(const fwime_ctx_t *ctx, fwime_info_t *out) {
  if (!ctx || !out) return FWIME_EINVAL;
  out->arena_bytes = ctx->arena_bytes;
  out->tape_bytes = ctx->tape_bytes;
  out->tile_x = ctx->tile_x;
  out->last_batch_tile_x = ctx->last_batch_tile;
  out->tuned_signatures = (int32_t)ctx->tuned.size();
  out->last_stencil_launches = -1;
  out->last_stencil_ms = 0.0;
  if (ctx->timing && ctx->timed_launches >= 0) {
    if (hipSetDevice(ctx->device) != hipSuccess || hipEventSynchronize(ctx->tev[1]) != hipSuccess) return FWIME_EHIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->tev[0], ctx->tev[1]) != hipSuccess) return FWIME_EHIP;
    out->last_stencil_launches = ctx->timed_launches;
    out->last_stencil_ms = ms;
  }
  return FWIME_OK;
}

int fwime_ctx_set_timing(fwime_ctx_t *ctx, int32_t on) {
  if (!ctx) return FWIME_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return FWIME_EHIP;
  if (on && !ctx->tev[0]) {
    for (auto &e : ctx->tev)
      if (hipEventCreate(&e) != hipSuccess) return set_err(ctx, FWIME_EHIP, "hipEventCreate failed");
  }
  ctx->timing = on != 0;
  ctx->timed_launches = -1;
  return FWIME_OK;
}

void fwime_ctx_destroy(fwime_ctx_t *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  release_graph(ctx);
  if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
  if (ctx->arena) (void)hipFree(ctx->arena);
  if (ctx->vp) (void)hipFree(ctx->vp);
  if (ctx->host_red) (void)hipHostFree(ctx->host_red);
  for (auto &e : ctx->tev)
    if (e) (void)hipEventDestroy(e);
  delete ctx;
}

// ---------------------------------------------------------------------------
int fwime_model(fwime_ctx_t *ctx, const fwime_grid_t *g, const float *vel, const fwime_geom_t *geo, float *data,
                void *stream) {
  if (!ctx) return FWIME_EINVAL;
  ctx->err.clear();
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if ((rc = check_grid(ctx, g)) || (rc = check_geom(ctx, g, geo))) return rc;
  if (!data) return set_err(ctx, FWIME_EINVAL, "data is null");
  HIPCHK(hipSetDevice(ctx->device));
  if ((rc = check_inputs(ctx, g, vel, geo, {}, st))) return rc;

  Common c;
  c.d = make_dims(g, ctx->tile_x);
  const Dims &d = c.d;
  const bool two = ctx->two_step;
  const int nf = two ? 4 : 2;                 // field buffers per shot
  const long per_shot = nf * d.field * 4 + (long)geo->nrec * 64;
  const int S = choose_batch(ctx, per_shot, (size_t)d.field * 8, geo->nshots);
  auto batches = split_batches(geo->nshots, S);
  TableSet ts = build_table_set(d, geo, batches, two);

  float *fields = nullptr;
  Carve cv;
  cv.add(&c.V, d.field);
  cv.add(&c.gz, d.LZ);
  cv.add(&c.gx, d.NX + kGxPad);
  cv.add(&c.tables, table_set_ints(ts) + 64 * batches.size() * 8);
  cv.add(&fields, nf * d.field * S);
  if ((rc = arena_get(ctx, cv))) return rc;
  if ((rc = upload_tables(ctx, ts, c.tables, st))) return rc;
  if ((rc = setup_common(ctx, c, g, vel, st))) return rc;

  HIPCHK(timing_begin(ctx, st));
  long launches = 0;
  for (size_t bi = 0; bi < batches.size(); ++bi) {
    const int s0 = batches[bi].first, Sb = batches[bi].second;
    const DevTables &t = ts.dev[bi];
    float *out_b = data + (long)s0 * geo->nrec * g->nt;
    launches += two ? g->nt / 2 : g->nt - 1;
    if (two) {
      HIPCHK(launch_zero(fields, 4 * d.field * Sb, st));
      Ring4 f(fields, d.field * Sb);
      for (int n = 0; n < g->nt - 1;) {
        const int k = std::min(2, g->nt - 1 - n);
        Step2Args p = step2_args(c, f, Sb, d.field, k);
        with_src2(p, t, geo->wavelet + (long)s0 * g->nt, g, n);
        with_rec_extract(p.a, t, out_b, g->nt, n);
        HIPCHK(launch_step2(p, d.TX, kModePlain, st));
        f.advance(k);
        n += k;
      }
      HIPCHK(launch_gather(f.cur(), d.field, t.cells, Sb, geo->nrec, out_b, g->nt, g->nt - 1, st));
      continue;
    }
    float *A = fields, *B = fields + d.field * Sb;
    HIPCHK(launch_zero(fields, 2 * d.field * Sb, st));
    float *cur = A, *prev = B;
    for (int n = 0; n < g->nt - 1; ++n) {
      StepArgs a = batch_args(c, Sb, d.field);
      a.cur = cur;
      a.prev = prev;
      a.out = prev;
      with_src(a, t, geo, g, s0, n);
      with_rec_extract(a, t, out_b, g->nt, n);
      HIPCHK(launch_step(a, d.TX, kModePlain, st));
      std::swap(cur, prev);
    }
    HIPCHK(launch_gather(cur, d.field, t.cells, Sb, geo->nrec, out_b, g->nt, g->nt - 1, st));
  }
  HIPCHK(timing_end(ctx, st, launches));
  return FWIME_OK;
}

// ---------------------------------------------------------------------------
int fwime_model_static(fwime_ctx_t *ctx, const fwime_grid_t *g, const float *vel, const fwime_geom_t *geo,
                       float *data, void *stream) {
  if (!ctx) return FWIME_EINVAL;
  if (!ctx->static_scratch) return set_err(ctx, FWIME_EHIP, "the static scratch array has no device address");
  // every piece of scratch (validation partials, padded velocity, tapers,
  // geometry tables, wavefields) comes from the static array; shots run in as
  // many batches as it needs, and a call that cannot fit one shot fails
  // with FWIME_ENOMEM before anything is written
  ctx->fixed = ctx->static_scratch;
  ctx->fixed_bytes = FWIME_STATIC_SCRATCH_BYTES;
  const int rc = fwime_model(ctx, g, vel, geo, data, stream);
  ctx->fixed = nullptr;
  ctx->fixed_bytes = 0;
  return rc;
}

// ---------------------------------------------------------------------------
int fwime_born_ext_fwd(fwime_ctx_t *ctx, const fwime_grid_t *g, const float *vel, const fwime_geom_t *geo,
                       int32_t nh, const float *ptilde, float *data, void *stream) {
  if (!ctx) return FWIME_EINVAL;
  ctx->err.clear();
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if ((rc = check_grid(ctx, g)) || (rc = check_geom(ctx, g, geo)) || (rc = check_nh(ctx, g, nh))) return rc;
  if (!data || !ptilde) return set_err(ctx, FWIME_EINVAL, "data or ptilde is null");
  HIPCHK(hipSetDevice(ctx->device));
  if ((rc = check_inputs(ctx, g, vel, geo, {{ptilde, (long)nh * g->nx * g->nz}}, st))) return rc;

  Common c;
  c.d = make_dims(g, ctx->tile_x);
  const Dims &d = c.d;
  ExtGeom eg{d.nz, d.nx, d.nb, d.NZ, d.NX, d.LZ, nh, (nh - 1) / 2};
  const int KC = 16;
  const bool two = ctx->two_step;
  const int nf = two ? 8 : 4;                  // u and du~ field buffers per shot
  // two-step path: both fields also carry four BF16 low-part fields each
  const long per_shot = (nf + 2L * KC + (two ? 4 : 0)) * d.field * 4 + (long)geo->nrec * 64;
  const size_t fixed = (size_t)d.field * 8 + (size_t)nh * d.nx * d.nz * 4;
  const int S = choose_batch(ctx, per_shot, fixed, geo->nshots);
  auto batches = split_batches(geo->nshots, S);
  TableSet ts = build_table_set(d, geo, batches, two);

  float *coef = nullptr, *pairs = nullptr, *t2 = nullptr, *sc = nullptr;
  unsigned short *lows = nullptr;
  Carve cv;
  cv.add(&c.V, d.field);
  cv.add(&c.gz, d.LZ);
  cv.add(&c.gx, d.NX + kGxPad);
  cv.add(&c.tables, table_set_ints(ts) + 64 * batches.size() * 8);
  cv.add(&coef, (long)nh * d.nx * d.nz);
  cv.add(&pairs, nf * d.field * S);
  if (two) cv.add(&lows, 8 * d.field * S);
  cv.add(&t2, (long)KC * d.field * S);
  cv.add(&sc, (long)KC * d.field * S);
  if ((rc = arena_get(ctx, cv))) return rc;
  if ((rc = upload_tables(ctx, ts, c.tables, st))) return rc;
  if ((rc = setup_common(ctx, c, g, vel, st))) return rc;
  HIPCHK(launch_ext_coef(ptilde, vel, eg, (float)g->dt, coef, st));

  const long chunk_stride = (long)KC * d.field;   // per shot in t2 / sc
  for (size_t bi = 0; bi < batches.size(); ++bi) {
    const int s0 = batches[bi].first, Sb = batches[bi].second;
    const DevTables &t = ts.dev[bi];
    float *out_b = data + (long)s0 * geo->nrec * g->nt;
    if (two) {
      HIPCHK(launch_zero(pairs, 8 * d.field * Sb, st));
      HIPCHK(launch_zero((float *)lows, 4 * d.field * Sb, st));
      HIPCHK(launch_zero(sc, chunk_stride * Sb, st));
      Ring4 fu(pairs, d.field * Sb), fw(pairs + 4 * d.field * Sb, d.field * Sb);
      Ring4L lu(lows, d.field * Sb), lw(lows + 4 * d.field * Sb, d.field * Sb);
      const float *wav_b = geo->wavelet + (long)s0 * g->nt;
      for (int c0 = 0; c0 < g->nt - 1; c0 += KC) {
        const int nk = std::min(KC, g->nt - 1 - c0);
        // background in extended precision: its T2 term is the scattering source
        rc = march2(ctx, c, fu, Sb, c0, c0 + nk, kModeT2, [&](Step2Args &p, int n, int k) {
          p.a.t2 = t2 + (long)(n - c0) * d.field;
          p.t2b = k == 2 ? t2 + (long)(n - c0 + 1) * d.field : nullptr;
          p.a.t2_sstride = chunk_stride;
          with_src2(p, t, wav_b, g, n);
        }, st, &lu);
        if (rc) return rc;
        HIPCHK(launch_ext_scatter(coef, eg, +1, t2, d.field, sc, d.field, chunk_stride, Sb, nk, st));
        // the scattered field in extended precision too: its FP32 rounding
        // would otherwise dominate the inconsistency of the B~ / B~^T pair
        rc = march2(ctx, c, fw, Sb, c0, c0 + nk, kModeDsrc, [&](Step2Args &p, int n, int k) {
          with_dsrc2(p, sc + (long)(n - c0) * d.field, d.field, k, chunk_stride);
          with_rec_extract(p.a, t, out_b, g->nt, n);
        }, st, &lw);
        if (rc) return rc;
      }
      HIPCHK(launch_gather(fw.cur(), d.field, t.cells, Sb, geo->nrec, out_b, g->nt, g->nt - 1, st));
      continue;
    }
    float *u0 = pairs, *u1 = pairs + d.field * Sb;
    float *w0 = pairs + 2 * d.field * Sb, *w1 = pairs + 3 * d.field * Sb;
    HIPCHK(launch_zero(pairs, 4 * d.field * Sb, st));
    HIPCHK(launch_zero(sc, chunk_stride * Sb, st));
    float *ucur = u0, *uprev = u1, *wcur = w0, *wprev = w1;
    for (int c0 = 0; c0 < g->nt - 1; c0 += KC) {
      const int nk = std::min(KC, g->nt - 1 - c0);
      for (int m = 0; m < nk; ++m) {
        StepArgs a = batch_args(c, Sb, d.field);
        a.cur = ucur;
        a.prev = uprev;
        a.out = uprev;
        a.t2 = t2 + m * d.field;
        a.t2_sstride = chunk_stride;
        with_src(a, t, geo, g, s0, c0 + m);
        HIPCHK(launch_step(a, d.TX, kModeT2, st));
        std::swap(ucur, uprev);
      }
      HIPCHK(launch_ext_scatter(coef, eg, +1, t2, d.field, sc, d.field, chunk_stride, Sb, nk, st));
      for (int m = 0; m < nk; ++m) {
        StepArgs a = batch_args(c, Sb, d.field);
        a.cur = wcur;
        a.prev = wprev;
        a.out = wprev;
        a.dsrc = sc + m * d.field;
        a.dsrc_sstride = chunk_stride;
        with_rec_extract(a, t, out_b, g->nt, c0 + m);
        HIPCHK(launch_step(a, d.TX, kModeDsrc, st));
        std::swap(wcur, wprev);
      }
    }
    HIPCHK(launch_gather(wcur, d.field, t.cells, Sb, geo->nrec, out_b, g->nt, g->nt - 1, st));
  }
  return FWIME_OK;
}

// ---------------------------------------------------------------------------
// Extended Born with time lags (lags tau_k = k L dt, k = -K .. K) and its
// adjoint.  The scattering source at step n takes the background's T2 term at
// steps n - 2kL, after n as well as before it, so the background's T2 history
// of a shot batch is kept whole (nt - 1 fields per shot); the batch size
// follows from that.  The background is carried in extended precision, as in
// the offset operators.
// ---------------------------------------------------------------------------
static int check_tau(fwime_ctx_t *ctx, const fwime_grid_t *g, int ntau, int lag) {
  if (ntau < 1 || ntau % 2 == 0 || ntau > 1023) return set_err(ctx, FWIME_EINVAL, "ntau must be odd, 1 <= ntau <= 1023");
  if (lag < 1 || (long)lag * (ntau - 1) > 4L * g->nt)
    return set_err(ctx, FWIME_EINVAL, "lag must be >= 1 with lag (ntau - 1) <= 4 nt");
  return FWIME_OK;
}

// Background T2 history of a shot batch: march all nt - 1 steps, T2 of step n
// into slot n of hist (per-shot stride hstride).
// Background of a shot batch in extended precision, keeping the T2 term of
// every step (slot n of shot s at hist + s hstride + n field); with rec_out
// (batch-local [Sb][nrec][nt]) it also records the receivers.
static int tau_background(fwime_ctx_t *ctx, const Common &c, const fwime_grid_t *g, const fwime_geom_t *geo,
                          int s0, int Sb, const DevTables &t, float *pairs, unsigned short *lows, float *hist,
                          long hstride, hipStream_t st, float *rec_out = nullptr) {
  const Dims &d = c.d;
  HIPCHK(launch_zero(pairs, 4 * d.field * Sb, st));
  HIPCHK(launch_zero((float *)lows, 2 * d.field * Sb, st));
  Ring4 fu(pairs, d.field * Sb);
  Ring4L lu(lows, d.field * Sb);
  const float *wav_b = geo->wavelet + (long)s0 * g->nt;
  int rc = march2(ctx, c, fu, Sb, 0, g->nt - 1, kModeT2, [&](Step2Args &p, int n, int k) {
    p.a.t2 = hist + (long)n * d.field;
    p.t2b = k == 2 ? hist + (long)(n + 1) * d.field : nullptr;
    p.a.t2_sstride = hstride;
    with_src2(p, t, wav_b, g, n);
    if (rec_out) with_rec_extract(p.a, t, rec_out, g->nt, n);
  }, st, &lu);
  if (rc || !rec_out) return rc;
  HIPCHK(launch_gather(fu.cur(), d.field, t.cells, Sb, geo->nrec, rec_out, g->nt, g->nt - 1, st));
  return FWIME_OK;
}

int fwime_born_ext_tau_fwd(fwime_ctx_t *ctx, const fwime_grid_t *g, const float *vel, const fwime_geom_t *geo,
                           int32_t ntau, int32_t lag, const float *ptau, float *data, void *stream) {
  if (!ctx) return FWIME_EINVAL;
  ctx->err.clear();
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if ((rc = check_grid(ctx, g)) || (rc = check_geom(ctx, g, geo)) || (rc = check_tau(ctx, g, ntau, lag))) return rc;
  if (!data || !ptau) return set_err(ctx, FWIME_EINVAL, "data or ptau is null");
  HIPCHK(hipSetDevice(ctx->device));
  if ((rc = check_inputs(ctx, g, vel, geo, {{ptau, (long)ntau * g->nx * g->nz}}, st))) return rc;

  Common c;
  c.d = make_dims(g, ctx->tile_x);
  const Dims &d = c.d;
  ExtGeom eg{d.nz, d.nx, d.nb, d.NZ, d.NX, d.LZ, ntau, (ntau - 1) / 2};
  const int ns = g->nt - 1;                        // time steps (equations)
  // per shot: T2 history and source history (ns fields each), the two
  // wavefields' rings (8 fields) and the background's BF16 low parts (2)
  const long per_shot = (2L * ns + 10) * d.field * 4 + (long)geo->nrec * 64;
  const size_t fixed = (size_t)d.field * 8 + (size_t)ntau * d.nx * d.nz * 4;
  const int S = choose_batch(ctx, per_shot, fixed, geo->nshots);
  auto batches = split_batches(geo->nshots, S);
  TableSet ts = build_table_set(d, geo, batches, true);

  float *coef = nullptr, *pairs = nullptr, *hist = nullptr, *sc = nullptr;
  unsigned short *lows = nullptr;
  Carve cv;
  cv.add(&c.V, d.field);
  cv.add(&c.gz, d.LZ);
  cv.add(&c.gx, d.NX + kGxPad);
  cv.add(&c.tables, table_set_ints(ts) + 64 * batches.size() * 8);
  cv.add(&coef, (long)ntau * d.nx * d.nz);
  cv.add(&pairs, 8 * d.field * S);
  cv.add(&lows, 4 * d.field * S);
  cv.add(&hist, (long)ns * d.field * S);
  cv.add(&sc, (long)ns * d.field * S);
  if ((rc = arena_get(ctx, cv))) return rc;
  if ((rc = upload_tables(ctx, ts, c.tables, st))) return rc;
  if ((rc = setup_common(ctx, c, g, vel, st))) return rc;
  HIPCHK(launch_ext_coef(ptau, vel, eg, (float)g->dt, coef, st));

  const long hstride = (long)ns * d.field;         // per shot in hist / sc
  for (size_t bi = 0; bi < batches.size(); ++bi) {
    const int s0 = batches[bi].first, Sb = batches[bi].second;
    const DevTables &t = ts.dev[bi];
    float *out_b = data + (long)s0 * geo->nrec * g->nt;
    if ((rc = tau_background(ctx, c, g, geo, s0, Sb, t, pairs, lows, hist, hstride, st))) return rc;
    HIPCHK(launch_zero(sc, hstride * Sb, st));
    HIPCHK(launch_tau_scatter(coef, eg, lag, hist, sc, d.field, hstride, ns, Sb, st));
    float *wp = pairs + 4 * d.field * Sb;
    HIPCHK(launch_zero(wp, 4 * d.field * Sb, st));
    Ring4 fw(wp, d.field * Sb);
    rc = march2(ctx, c, fw, Sb, 0, ns, kModeDsrc, [&](Step2Args &p, int n, int k) {
      with_dsrc2(p, sc + (long)n * d.field, d.field, k, hstride);
      with_rec_extract(p.a, t, out_b, g->nt, n);
    }, st);
    if (rc) return rc;
    HIPCHK(launch_gather(fw.cur(), d.field, t.cells, Sb, geo->nrec, out_b, g->nt, g->nt - 1, st));
  }
  return FWIME_OK;
}

int fwime_born_ext_tau_adj(fwime_ctx_t *ctx, const fwime_grid_t *g, const float *vel, const fwime_geom_t *geo,
                           int32_t ntau, int32_t lag, const float *data, float *ptau_out, void *stream) {
  if (!ctx) return FWIME_EINVAL;
  ctx->err.clear();
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if ((rc = check_grid(ctx, g)) || (rc = check_geom(ctx, g, geo)) || (rc = check_tau(ctx, g, ntau, lag))) return rc;
  if (!data || !ptau_out) return set_err(ctx, FWIME_EINVAL, "data or ptau_out is null");
  HIPCHK(hipSetDevice(ctx->device));
  if ((rc = check_inputs(ctx, g, vel, geo, {{data, (long)geo->nshots * geo->nrec * g->nt}}, st))) return rc;

  Common c;
  c.d = make_dims(g, ctx->tile_x);
  const Dims &d = c.d;
  ExtGeom eg{d.nz, d.nx, d.nb, d.NZ, d.NX, d.LZ, ntau, (ntau - 1) / 2};
  const int ns = g->nt - 1;
  const int R = g->nt + 1;                         // adjoint field of every time 0 .. nt
  // per shot: T2 history (ns fields), adjoint history (R), background ring (4), low parts (2)
  const long per_shot = ((long)ns + R + 6) * d.field * 4 + (long)geo->nrec * 64;
  const size_t fixed = (size_t)d.field * 8;
  const int S = choose_batch(ctx, per_shot, fixed, geo->nshots);
  auto batches = split_batches(geo->nshots, S);
  TableSet ts = build_table_set(d, geo, batches, true);

  float *pairs = nullptr, *hist = nullptr, *lam = nullptr;
  unsigned short *lows = nullptr;
  Carve cv;
  cv.add(&c.V, d.field);
  cv.add(&c.gz, d.LZ);
  cv.add(&c.gx, d.NX + kGxPad);
  cv.add(&c.tables, table_set_ints(ts) + 64 * batches.size() * 8);
  cv.add(&pairs, 4 * d.field * S);
  cv.add(&lows, 4 * d.field * S);
  cv.add(&hist, (long)ns * d.field * S);
  cv.add(&lam, (long)R * d.field * S);
  if ((rc = arena_get(ctx, cv))) return rc;
  if ((rc = upload_tables(ctx, ts, c.tables, st))) return rc;
  if ((rc = setup_common(ctx, c, g, vel, st))) return rc;
  HIPCHK(launch_zero(ptau_out, (long)ntau * d.nx * d.nz, st));

  const long hstride = (long)ns * d.field, lstride = (long)R * d.field;
  for (size_t bi = 0; bi < batches.size(); ++bi) {
    const int s0 = batches[bi].first, Sb = batches[bi].second;
    const DevTables &t = ts.dev[bi];
    const float *data_b = data + (long)s0 * geo->nrec * g->nt;
    if ((rc = tau_background(ctx, c, g, geo, s0, Sb, t, pairs, lows, hist, hstride, st))) return rc;
    HIPCHK(launch_zero(lam, lstride * Sb, st));
    if ((rc = march2_back_lambda(ctx, c, lam, lstride, R, Sb, 0, g->nt - 1, t, data_b, g->nt, st))) return rc;
    HIPCHK(launch_tau_image(hist, d.field, hstride, lam, d.field, lstride, ns, Sb, eg, lag, vel, (float)g->dt,
                            ptau_out, st));
  }
  return FWIME_OK;
}

// ---------------------------------------------------------------------------
// Background checkpoints of the extended-precision adjoint kept across calls
// with the same model and shots (the variable-projection step): per shot
// 2 nseg fields (FP32 and BF16 low parts) in shot order.  `valid` once a call
// has filled them; later calls skip their forward pass.
struct AdjCache {
  float *ckpt = nullptr;
  unsigned short *ckpt_lo = nullptr;
  bool valid = false;
};

static int born_ext_adj_run(fwime_ctx_t *ctx, const fwime_grid_t *g, const float *vel, const fwime_geom_t *geo,
                            int32_t nh, const float *data, float *ptilde_out, void *stream, AdjCache *cache);

int fwime_born_ext_adj(fwime_ctx_t *ctx, const fwime_grid_t *g, const float *vel, const fwime_geom_t *geo,
                       int32_t nh, const float *data, float *ptilde_out, void *stream) {
  return born_ext_adj_run(ctx, g, vel, geo, nh, data, ptilde_out, stream, nullptr);
}

static int born_ext_adj_run(fwime_ctx_t *ctx, const fwime_grid_t *g, const float *vel, const fwime_geom_t *geo,
                            int32_t nh, const float *data, float *ptilde_out, void *stream, AdjCache *cache) {
  if (!ctx) return FWIME_EINVAL;
  ctx->err.clear();
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if ((rc = check_grid(ctx, g)) || (rc = check_geom(ctx, g, geo)) || (rc = check_nh(ctx, g, nh))) return rc;
  if (!data || !ptilde_out) return set_err(ctx, FWIME_EINVAL, "data or ptilde_out is null");
  HIPCHK(hipSetDevice(ctx->device));
  if ((rc = check_inputs(ctx, g, vel, geo, {{data, (long)geo->nshots * geo->nrec * g->nt}}, st))) return rc;

  Common c;
  c.d = make_dims(g, ctx->tile_x);
  const Dims &d = c.d;
  ExtGeom eg{d.nz, d.nx, d.nb, d.NZ, d.NX, d.LZ, nh, (nh - 1) / 2};
  const int K = seg_len(g->nt);
  const int nseg = (g->nt - 1 + K - 1) / K;
  const int R = K + 2;
  const bool two = ctx->two_step;
  const int nf = two ? 4 : 2;
  if (!two) cache = nullptr;                    // the one-step path recomputes inside its checkpoints
  // two-step path: BF16 low parts of the four work fields and the checkpoints
  // (cached checkpoints live outside the arena)
  const long ck_fields = cache ? 0L : 2L * nseg + (two ? nseg : 0L);
  // (two-step path: the adjoint ring's BF16 low parts add R / 2 fields)
  const long per_shot = (nf + K + R + (two ? 2L + (R + 1) / 2 : 0L) + ck_fields) * d.field * 4 + (long)geo->nrec * 64;
  const long img = (long)nh * d.nx * d.nz;
  const size_t fixed = (size_t)d.field * 8 + (size_t)img * (8 + 4 * kImageGroups);   // FP64 image + partials
  const int S = choose_batch(ctx, per_shot, fixed, geo->nshots);
  auto batches = split_batches(geo->nshots, S);
  TableSet ts = build_table_set(d, geo, batches, two);

  float *pairs = nullptr, *ckpt = nullptr, *t2 = nullptr, *ring = nullptr;
  double *acc = nullptr;
  Carve cv;
  cv.add(&c.V, d.field);
  cv.add(&c.gz, d.LZ);
  cv.add(&c.gx, d.NX + kGxPad);
  cv.add(&c.tables, table_set_ints(ts) + 64 * batches.size() * 8);
  unsigned short *lows = nullptr, *ckpt_lo = nullptr, *ring_lo = nullptr;
  float *parts = nullptr;
  cv.add(&acc, img);
  cv.add(&parts, kImageGroups * img);
  cv.add(&pairs, nf * d.field * S);
  if (!cache) cv.add(&ckpt, 2L * nseg * d.field * S);
  if (two) {
    cv.add(&lows, 4 * d.field * S);
    cv.add(&ring_lo, (long)R * d.field * S);
    if (!cache) cv.add(&ckpt_lo, 2L * nseg * d.field * S);
  }
  cv.add(&t2, (long)K * d.field * S);
  cv.add(&ring, (long)R * d.field * S);
  if ((rc = arena_get(ctx, cv))) return rc;
  if ((rc = upload_tables(ctx, ts, c.tables, st))) return rc;
  if ((rc = setup_common(ctx, c, g, vel, st))) return rc;
  HIPCHK(launch_zero_d(acc, img, st));

  const long ck_stride = 2L * nseg * d.field;   // per shot
  const long t2_stride = (long)K * d.field;
  const long ring_stride = (long)R * d.field;
  for (size_t bi = 0; bi < batches.size(); ++bi) {
    const int s0 = batches[bi].first, Sb = batches[bi].second;
    const DevTables &t = ts.dev[bi];
    const float *data_b = data + (long)s0 * geo->nrec * g->nt;
    if (two) {
      const float *wav_b = geo->wavelet + (long)s0 * g->nt;
      auto src = [&](Step2Args &p, int n, int) { with_src2(p, t, wav_b, g, n); };
      if (cache) {                              // this batch's shots in the cached checkpoints
        ckpt = cache->ckpt + (long)s0 * ck_stride;
        ckpt_lo = cache->ckpt_lo + (long)s0 * ck_stride;
      }
      // forward pass (extended precision) storing (u^{n0-1}, u^{n0}) at every
      // segment start, unless the cached checkpoints already hold them
      HIPCHK(launch_zero(pairs, 4 * d.field * Sb, st));
      HIPCHK(launch_zero((float *)lows, 2 * d.field * Sb, st));
      Ring4 fu(pairs, d.field * Sb);
      Ring4L lu(lows, d.field * Sb);
      for (int j = 0; j < nseg && !(cache && cache->valid); ++j) {
        const int n0 = j * K, n1 = std::min(n0 + K, g->nt - 1);
        HIPCHK(launch_copy_fields(ckpt + (2L * j) * d.field, ck_stride, fu.prev(), d.field, Sb, d.field, st));
        HIPCHK(launch_copy_fields(ckpt + (2L * j + 1) * d.field, ck_stride, fu.cur(), d.field, Sb, d.field, st));
        HIPCHK(copy_lo(ckpt_lo + (2L * j) * d.field, ck_stride, lu.prev(), d.field, Sb, d.field, st));
        HIPCHK(copy_lo(ckpt_lo + (2L * j + 1) * d.field, ck_stride, lu.cur(), d.field, Sb, d.field, st));
        if (j == nseg - 1) break;   // the last segment is recomputed anyway
        if ((rc = march2(ctx, c, fu, Sb, n0, n1, kModePlain, src, st, &lu))) return rc;
      }
      // backward pass: recompute the segment from its checkpoint (keeping
      // T2 u_n), march lambda through the segment (in extended precision as
      // well), image
      HIPCHK(launch_zero(ring, ring_stride * Sb, st));
      HIPCHK(launch_zero((float *)ring_lo, ring_stride * Sb / 2, st));
      for (int j = nseg - 1; j >= 0; --j) {
        const int n0 = j * K, n1 = std::min(n0 + K, g->nt - 1), nk = n1 - n0;
        Ring4 wu(pairs, d.field * Sb);
        Ring4L wl(lows, d.field * Sb);
        HIPCHK(launch_copy_fields(wu.prev(), d.field, ckpt + (2L * j) * d.field, ck_stride, Sb, d.field, st));
        HIPCHK(launch_copy_fields(wu.cur(), d.field, ckpt + (2L * j + 1) * d.field, ck_stride, Sb, d.field, st));
        HIPCHK(copy_lo(wl.prev(), d.field, ckpt_lo + (2L * j) * d.field, ck_stride, Sb, d.field, st));
        HIPCHK(copy_lo(wl.cur(), d.field, ckpt_lo + (2L * j + 1) * d.field, ck_stride, Sb, d.field, st));
        rc = march2(ctx, c, wu, Sb, n0, n1, kModeT2, [&](Step2Args &p, int n, int k) {
          p.a.t2 = t2 + (long)(n - n0) * d.field;
          p.t2b = k == 2 ? t2 + (long)(n - n0 + 1) * d.field : nullptr;
          p.a.t2_sstride = t2_stride;
          with_src2(p, t, wav_b, g, n);
        }, st, &wl);
        if (rc) return rc;
        if ((rc = march2_back_lambda(ctx, c, ring, ring_stride, R, Sb, n0, n1, t, data_b, g->nt, st, ring_lo)))
          return rc;
        HIPCHK(launch_ext_image(t2, d.field, t2_stride, ring, d.field, ring_stride, R, n0, Sb, nk, eg, acc, parts, st));
      }
      continue;
    }
    // forward pass storing (u^{n0-1}, u^{n0}) at every segment start
    float *p0 = pairs, *p1 = pairs + d.field * Sb;
    HIPCHK(launch_zero(pairs, 2 * d.field * Sb, st));
    float *cur = p0, *prev = p1;
    for (int j = 0; j < nseg; ++j) {
      const int n0 = j * K, n1 = std::min(n0 + K, g->nt - 1);
      HIPCHK(launch_copy_fields(ckpt + (2L * j) * d.field, ck_stride, prev, d.field, Sb, d.field, st));
      HIPCHK(launch_copy_fields(ckpt + (2L * j + 1) * d.field, ck_stride, cur, d.field, Sb, d.field, st));
      if (j == nseg - 1) break;   // the last segment is recomputed anyway
      for (int n = n0; n < n1; ++n) {
        StepArgs a = batch_args(c, Sb, d.field);
        a.cur = cur;
        a.prev = prev;
        a.out = prev;
        with_src(a, t, geo, g, s0, n);
        HIPCHK(launch_step(a, d.TX, kModePlain, st));
        std::swap(cur, prev);
      }
    }
    // backward pass
    HIPCHK(launch_zero(ring, ring_stride * Sb, st));
    for (int j = nseg - 1; j >= 0; --j) {
      const int n0 = j * K, n1 = std::min(n0 + K, g->nt - 1), nk = n1 - n0;
      float *ccur = ckpt + (2L * j + 1) * d.field, *cprev = ckpt + (2L * j) * d.field;
      for (int n = n0; n < n1; ++n) {
        StepArgs a = batch_args(c, Sb, ck_stride);
        a.cur = ccur;
        a.prev = cprev;
        a.out = cprev;
        a.t2 = t2 + (long)(n - n0) * d.field;
        a.t2_sstride = t2_stride;
        with_src(a, t, geo, g, s0, n);
        HIPCHK(launch_step(a, d.TX, kModeT2, st));
        std::swap(ccur, cprev);
      }
      for (int k = n1; k >= n0 + 1; --k) {
        StepArgs a = batch_args(c, Sb, ring_stride);
        a.cur = ring + (long)(k % R) * d.field;
        a.prev = ring + (long)((k + 1) % R) * d.field;
        a.out = ring + (long)((k - 1) % R) * d.field;
        with_rec_inject(a, t, data_b, g->nt, k);
        HIPCHK(launch_step(a, d.TX, kModePlain, st));
      }
      HIPCHK(launch_ext_image(t2, d.field, t2_stride, ring, d.field, ring_stride, R, n0, Sb, nk, eg, acc, parts, st));
    }
  }
  HIPCHK(launch_ext_finalize(acc, vel, eg, (float)g->dt, nullptr, nullptr, ptilde_out, st));
  if (cache) cache->valid = true;
  return FWIME_OK;
}

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// FWIME gradient building blocks, shared by fwime_gradient and the tape API.
//
// Forward (one batch): u and du~ together, segment by segment; at each segment
// start the pairs (u^{n0-1}, u^{n0}) and (du~^{n0-1}, du~^{n0}) are stored, the
// segment's T2u_n feeds the extended scatter whose output drives du~, and the
// receivers of u and du~ are recorded separately.
// Backward (one batch, adjoint source r at the receivers): per segment, from
// last to first, recompute u (keeping T2u_n) and du~ (keeping T2du~_n), march
// lambda (source r), spread lambda into the e ring, march rho (source the
// transposed second time difference of e), then accumulate the extended image
// sum T2u(y-h) lambda(y+h) and the per-cell sum (T2u + T2du~) lambda + T2u rho.
// ---------------------------------------------------------------------------
struct GradPlan {
  int K, nseg, R;
  long ck_stride, seg_stride, ring_stride;
};

GradPlan grad_plan(const Dims &d, int nt) {
  GradPlan p;
  p.K = seg_len(nt);
  p.nseg = (nt - 1 + p.K - 1) / p.K;
  p.R = p.K + 2;
  p.ck_stride = 2L * p.nseg * d.field;
  p.seg_stride = (long)p.K * d.field;
  p.ring_stride = (long)p.R * d.field;
  return p;
}

struct GradWork {       // per-batch working fields (+ partial images of the imaging kernel)
  float *pairs, *t2u, *t2d, *lam, *er, *rho;
  float *parts = nullptr;
};

int grad_forward_batch(fwime_ctx_t *ctx, const Common &c, const ExtGeom &eg, const GradPlan &pl,
                       const fwime_grid_t *g, int Sb, const DevTables &t, const float *wav_b, const float *coef,
                       float *uck, float *dck, const GradWork &wk, float *drec, float *ddrec, int nrec,
                       hipStream_t st) {
  const Dims &d = c.d;
  int rc;
  if (ctx->two_step) {
    HIPCHK(launch_zero(wk.pairs, 8 * d.field * Sb, st));
    HIPCHK(launch_zero(wk.t2d, pl.seg_stride * Sb, st));
    Ring4 fu(wk.pairs, d.field * Sb), fw(wk.pairs + 4 * d.field * Sb, d.field * Sb);
    for (int j = 0; j < pl.nseg; ++j) {
      const int n0 = j * pl.K, n1 = std::min(n0 + pl.K, g->nt - 1), nk = n1 - n0;
      HIPCHK(launch_copy_fields(uck + (2L * j) * d.field, pl.ck_stride, fu.prev(), d.field, Sb, d.field, st));
      HIPCHK(launch_copy_fields(uck + (2L * j + 1) * d.field, pl.ck_stride, fu.cur(), d.field, Sb, d.field, st));
      HIPCHK(launch_copy_fields(dck + (2L * j) * d.field, pl.ck_stride, fw.prev(), d.field, Sb, d.field, st));
      HIPCHK(launch_copy_fields(dck + (2L * j + 1) * d.field, pl.ck_stride, fw.cur(), d.field, Sb, d.field, st));
      rc = march2(ctx, c, fu, Sb, n0, n1, kModeT2, [&](Step2Args &p, int n, int k) {
        p.a.t2 = wk.t2u + (long)(n - n0) * d.field;
        p.t2b = k == 2 ? wk.t2u + (long)(n - n0 + 1) * d.field : nullptr;
        p.a.t2_sstride = pl.seg_stride;
        with_src2(p, t, wav_b, g, n);
        with_rec_extract(p.a, t, drec, g->nt, n);
      }, st);
      if (rc) return rc;
      HIPCHK(launch_ext_scatter(coef, eg, +1, wk.t2u, d.field, wk.t2d, d.field, pl.seg_stride, Sb, nk, st));
      rc = march2(ctx, c, fw, Sb, n0, n1, kModeDsrc, [&](Step2Args &p, int n, int k) {
        with_dsrc2(p, wk.t2d + (long)(n - n0) * d.field, d.field, k, pl.seg_stride);
        with_rec_extract(p.a, t, ddrec, g->nt, n);
      }, st);
      if (rc) return rc;
    }
    HIPCHK(launch_gather(fu.cur(), d.field, t.cells, Sb, nrec, drec, g->nt, g->nt - 1, st));
    HIPCHK(launch_gather(fw.cur(), d.field, t.cells, Sb, nrec, ddrec, g->nt, g->nt - 1, st));
    return FWIME_OK;
  }
  float *u0 = wk.pairs, *u1 = wk.pairs + d.field * Sb, *w0 = wk.pairs + 2 * d.field * Sb,
        *w1 = wk.pairs + 3 * d.field * Sb;
  HIPCHK(launch_zero(wk.pairs, 4 * d.field * Sb, st));
  HIPCHK(launch_zero(wk.t2d, pl.seg_stride * Sb, st));
  float *ucur = u0, *uprev = u1, *wcur = w0, *wprev = w1;
  for (int j = 0; j < pl.nseg; ++j) {
    const int n0 = j * pl.K, n1 = std::min(n0 + pl.K, g->nt - 1), nk = n1 - n0;
    HIPCHK(launch_copy_fields(uck + (2L * j) * d.field, pl.ck_stride, uprev, d.field, Sb, d.field, st));
    HIPCHK(launch_copy_fields(uck + (2L * j + 1) * d.field, pl.ck_stride, ucur, d.field, Sb, d.field, st));
    HIPCHK(launch_copy_fields(dck + (2L * j) * d.field, pl.ck_stride, wprev, d.field, Sb, d.field, st));
    HIPCHK(launch_copy_fields(dck + (2L * j + 1) * d.field, pl.ck_stride, wcur, d.field, Sb, d.field, st));
    for (int n = n0; n < n1; ++n) {
      StepArgs a = batch_args(c, Sb, d.field);
      a.cur = ucur;
      a.prev = uprev;
      a.out = uprev;
      a.t2 = wk.t2u + (long)(n - n0) * d.field;
      a.t2_sstride = pl.seg_stride;
      with_src_w(a, t, wav_b, g, n);
      with_rec_extract(a, t, drec, g->nt, n);
      HIPCHK(launch_step(a, d.TX, kModeT2, st));
      std::swap(ucur, uprev);
    }
    HIPCHK(launch_ext_scatter(coef, eg, +1, wk.t2u, d.field, wk.t2d, d.field, pl.seg_stride, Sb, nk, st));
    for (int n = n0; n < n1; ++n) {
      StepArgs a = batch_args(c, Sb, d.field);
      a.cur = wcur;
      a.prev = wprev;
      a.out = wprev;
      a.dsrc = wk.t2d + (long)(n - n0) * d.field;
      a.dsrc_sstride = pl.seg_stride;
      with_rec_extract(a, t, ddrec, g->nt, n);
      HIPCHK(launch_step(a, d.TX, kModeDsrc, st));
      std::swap(wcur, wprev);
    }
  }
  HIPCHK(launch_gather(ucur, d.field, t.cells, Sb, nrec, drec, g->nt, g->nt - 1, st));
  HIPCHK(launch_gather(wcur, d.field, t.cells, Sb, nrec, ddrec, g->nt, g->nt - 1, st));
  return FWIME_OK;
}

int grad_backward_batch(fwime_ctx_t *ctx, const Common &c, const ExtGeom &eg, const GradPlan &pl,
                        const fwime_grid_t *g, int Sb, const DevTables &t, const float *wav_b, const float *coef,
                        float *uck, float *dck, const GradWork &wk, const float *r, double *acc, float *gacc,
                        hipStream_t st) {
  const Dims &d = c.d;
  const int K = pl.K, R = pl.R;
  HIPCHK(launch_zero(wk.lam, pl.ring_stride * Sb, st));
  HIPCHK(launch_zero(wk.er, pl.ring_stride * Sb, st));
  HIPCHK(launch_zero(wk.rho, pl.ring_stride * Sb, st));
  const bool two = ctx->two_step;
  int rc;
  for (int j = pl.nseg - 1; j >= 0; --j) {
    const int n0 = j * K, n1 = std::min(n0 + K, g->nt - 1), nk = n1 - n0;
    if (two) {
      // u from its checkpoint, two steps per launch, keeping T2 u_n
      Ring4 wu(wk.pairs, d.field * Sb);
      HIPCHK(launch_copy_fields(wu.prev(), d.field, uck + (2L * j) * d.field, pl.ck_stride, Sb, d.field, st));
      HIPCHK(launch_copy_fields(wu.cur(), d.field, uck + (2L * j + 1) * d.field, pl.ck_stride, Sb, d.field, st));
      rc = march2(ctx, c, wu, Sb, n0, n1, kModeT2, [&](Step2Args &p, int n, int k) {
        p.a.t2 = wk.t2u + (long)(n - n0) * d.field;
        p.t2b = k == 2 ? wk.t2u + (long)(n - n0 + 1) * d.field : nullptr;
        p.a.t2_sstride = pl.seg_stride;
        with_src2(p, t, wav_b, g, n);
      }, st);
      if (rc) return rc;
    } else {
      float *uc = uck + (2L * j + 1) * d.field, *up = uck + (2L * j) * d.field;
      for (int n = n0; n < n1; ++n) {
        StepArgs a = batch_args(c, Sb, pl.ck_stride);
        a.cur = uc;
        a.prev = up;
        a.out = up;
        a.t2 = wk.t2u + (long)(n - n0) * d.field;
        a.t2_sstride = pl.seg_stride;
        with_src_w(a, t, wav_b, g, n);
        HIPCHK(launch_step(a, d.TX, kModeT2, st));
        std::swap(uc, up);
      }
    }
    // t2d holds T2 du~ of the later segment outside the scatter's range: clear it
    HIPCHK(launch_zero(wk.t2d, pl.seg_stride * Sb, st));
    HIPCHK(launch_ext_scatter(coef, eg, +1, wk.t2u, d.field, wk.t2d, d.field, pl.seg_stride, Sb, nk, st));
    float *wc = dck + (2L * j + 1) * d.field, *wp = dck + (2L * j) * d.field;
    for (int n = n0; n < n1; ++n) {
      StepArgs a = batch_args(c, Sb, pl.ck_stride);
      a.cur = wc;
      a.prev = wp;
      a.out = wp;
      a.dsrc = wk.t2d + (long)(n - n0) * d.field;   // read the source, then
      a.dsrc_sstride = pl.seg_stride;
      a.t2 = wk.t2d + (long)(n - n0) * d.field;     // overwrite it with T2 du~_n
      a.t2_sstride = pl.seg_stride;
      HIPCHK(launch_step(a, d.TX, kModeT2 | kModeDsrc, st));
      std::swap(wc, wp);
    }
    if (two) {
      if ((rc = march2_back_lambda(ctx, c, wk.lam, pl.ring_stride, R, Sb, n0, n1, t, r, g->nt, st))) return rc;
    } else {
      for (int k = n1; k >= n0 + 1; --k) {
        StepArgs a = batch_args(c, Sb, pl.ring_stride);
        a.cur = wk.lam + (long)(k % R) * d.field;
        a.prev = wk.lam + (long)((k + 1) % R) * d.field;
        a.out = wk.lam + (long)((k - 1) % R) * d.field;
        with_rec_inject(a, t, r, g->nt, k);
        HIPCHK(launch_step(a, d.TX, kModePlain, st));
      }
    }
    HIPCHK(launch_ext_scatter(coef, eg, -1, wk.lam, d.field, wk.er, d.field, pl.ring_stride, Sb, nk, st, R, n0, R,
                              n0));
    auto er_slot = [&](int k) { return wk.er + (long)(k % R) * d.field; };
    if (two) {
      rc = march2_back_ring(ctx, c, wk.rho, pl.ring_stride, R, Sb, n0, n1, kModeNu, [&](Step2Args &p, int k, int kk) {
        p.a.nu = NuSource{er_slot(k - 1), er_slot(k), er_slot(k + 1), pl.ring_stride};
        if (kk == 2) p.nu2 = NuSource{er_slot(k - 2), er_slot(k - 1), er_slot(k), pl.ring_stride};
      }, st);
      if (rc) return rc;
    } else {
      for (int k = n1; k >= n0 + 1; --k) {
        StepArgs a = batch_args(c, Sb, pl.ring_stride);
        a.cur = wk.rho + (long)(k % R) * d.field;
        a.prev = wk.rho + (long)((k + 1) % R) * d.field;
        a.out = wk.rho + (long)((k - 1) % R) * d.field;
        a.nu = NuSource{er_slot(k - 1), er_slot(k), er_slot(k + 1), pl.ring_stride};
        HIPCHK(launch_step(a, d.TX, kModeNu, st));
      }
    }
    HIPCHK(launch_ext_image(wk.t2u, d.field, pl.seg_stride, wk.lam, d.field, pl.ring_stride, R, n0, Sb, nk, eg, acc,
                            wk.parts, st));
    HIPCHK(launch_grad_accum(wk.t2u, wk.t2d, d.field, pl.seg_stride, wk.lam, wk.rho, d.field, pl.ring_stride, R, n0,
                             Sb, nk, d.NZ, d.NX, d.LZ, gacc, st));
  }
  return FWIME_OK;
}

// the two-step path keeps four field buffers per wavefield (u and du~)
long grad_work_per_shot(const Dims &d, const GradPlan &pl, bool two) {
  return ((two ? 8L : 4L) + 2L * pl.K + 3L * pl.R) * d.field * 4;
}

void carve_work(Carve &cv, GradWork &wk, const Dims &d, const GradPlan &pl, int S, bool two) {
  cv.add(&wk.pairs, (two ? 8 : 4) * d.field * S);
  cv.add(&wk.t2u, (long)pl.K * d.field * S);
  cv.add(&wk.t2d, (long)pl.K * d.field * S);
  cv.add(&wk.lam, (long)pl.R * d.field * S);
  cv.add(&wk.er, (long)pl.R * d.field * S);
  cv.add(&wk.rho, (long)pl.R * d.field * S);
}

}  // namespace

// ---------------------------------------------------------------------------
// Tape: device-resident state between a forward and a backward call.
// ---------------------------------------------------------------------------
struct fwime_tape {
  fwime_ctx_t *ctx = nullptr;
  fwime_grid_t g{};
  int nh = 0, nshots = 0, nrec = 0;
  Dims d{};
  GradPlan pl{};
  std::vector<std::pair<int, int>> batches;
  TableSet ts;
  void *mem = nullptr;
  size_t bytes = 0;
  float *V = nullptr, *gz = nullptr, *gx = nullptr, *vel = nullptr, *pt = nullptr, *coef = nullptr, *wav = nullptr;
  float *uck = nullptr, *dck = nullptr;   // [nshots] x ck_stride each
  int *tables = nullptr;
  bool used = false;
};

extern "C" {

// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Variable-projection step (eqs. vp.obj, pert.opt, vp.pseudo.inv): linear
// conjugate gradient on (B~* B~ + eps^2 D* D) p~ = B~* (d_obs - f(m)) from
// p~ = 0.  Each iteration applies B~ and B~* once (four propagations per
// shot); the objective is tracked without further propagations as
// Phi_k = 1/2 ||d_obs - f(m)||^2 - 1/2 (b + r_k) . p~_k, which holds for any
// p~ with r = b - H p~ (b = B~* (d_obs - f(m)), H the normal matrix).
// The solver for either extension: subsurface offsets (tau false, nh
// offsets) or time lags (tau true, nh lags of `lag` steps).
static int vp_solve_run(fwime_ctx_t *ctx, const fwime_grid_t *g, const float *vel, const fwime_geom_t *geo,
                        int32_t nh, bool tau, int32_t lag, const float *dobs, double eps, const double *dso,
                        int32_t niter, float *ptilde_out, double *phi_out, void *stream) {
  if (!ctx) return FWIME_EINVAL;
  ctx->err.clear();
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if ((rc = check_grid(ctx, g)) || (rc = check_geom(ctx, g, geo)) ||
      (rc = tau ? check_tau(ctx, g, nh, lag) : check_nh(ctx, g, nh)))
    return rc;
  if (!dobs || !dso || !ptilde_out || !phi_out) return set_err(ctx, FWIME_EINVAL, "null pointer argument");
  if (niter < 0) return set_err(ctx, FWIME_EINVAL, "niter must be >= 0");
  if (!std::isfinite(eps)) return set_err(ctx, FWIME_EINVAL, "eps must be finite");
  for (int h = 0; h < nh; ++h)
    if (!std::isfinite(dso[h])) return set_err(ctx, FWIME_EINVAL, "dso must be finite");
  HIPCHK(hipSetDevice(ctx->device));
  const long ndata = (long)geo->nshots * geo->nrec * g->nt;
  const long plane = (long)g->nx * g->nz;
  const long img = (long)nh * plane;
  if ((rc = check_inputs(ctx, g, vel, geo, {{dobs, ndata}}, st))) return rc;

  // the background does not change during the step: the extended-precision
  // adjoint's checkpoints (2 nseg fields and their low parts per shot) are
  // kept for all shots when they fit, so every B~* after the first skips its
  // forward pass (FWIME_VP_NOCACHE=1 turns this off)
  const Dims dd = make_dims(g, ctx->tile_x);
  const int K = seg_len(g->nt);
  const long nseg = (g->nt - 1 + K - 1) / K;
  const long ck_elems = 2L * nseg * dd.field * geo->nshots;
  bool use_cache = ctx->two_step && !tau;          // the time-lag adjoint keeps no checkpoints
  if (const char *e = std::getenv("FWIME_VP_NOCACHE")) use_cache = use_cache && std::atoi(e) == 0;
  if (use_cache) {
    size_t avail = 0, total = 0;
    if (hipMemGetInfo(&avail, &total) != hipSuccess) avail = 0;
    // the solver's own buffer (possibly already holding a cache) counts as free here
    const size_t need = (size_t)ck_elems * 6;
    use_cache = need < (size_t)((avail + ctx->vp_bytes) * 0.5) && (!ctx->budget || need < ctx->budget / 2);
  }
  // solver vectors, kept in the context between calls
  float *r = nullptr, *sdir = nullptr, *q = nullptr, *b = nullptr, *dres = nullptr, *dtmp = nullptr,
        *e2d2 = nullptr;
  double *part = nullptr, *res = nullptr;
  AdjCache cache;
  Carve cv;
  if (use_cache) {
    cv.add(&cache.ckpt, ck_elems);
    cv.add(&cache.ckpt_lo, ck_elems);
  }
  cv.add(&r, img);
  cv.add(&sdir, img);
  cv.add(&q, img);
  cv.add(&b, img);
  cv.add(&dres, ndata);
  cv.add(&dtmp, ndata);
  cv.add(&e2d2, nh);
  cv.add(&part, dot_partials());
  cv.add(&res, 1);
  if (cv.total > ctx->vp_bytes) {
    HIPCHK(hipStreamSynchronize(st));
    if (ctx->vp) HIPCHK(hipFree(ctx->vp));
    ctx->vp = nullptr;
    ctx->vp_bytes = 0;
    if (hipMalloc(&ctx->vp, cv.total) != hipSuccess) {
      ctx->vp = nullptr;
      (void)hipGetLastError();
      return set_err(ctx, FWIME_ENOMEM, "cannot allocate the solver vectors");
    }
    ctx->vp_bytes = cv.total;
  }
  cv.assign(ctx->vp);
  // the operators below size their shot batches from what is left of the budget
  struct BudgetGuard {
    fwime_ctx_t *c;
    size_t saved;
    ~BudgetGuard() { c->budget = saved; }
  } guard{ctx, ctx->budget};
  if (ctx->budget) ctx->budget = ctx->budget > ctx->vp_bytes ? ctx->budget - ctx->vp_bytes : 1;

  auto dot = [&](const float *x, const float *y, long n, double &out) -> int {
    HIPCHK(launch_dot(x, y, n, part, res, st));
    HIPCHK(hipMemcpyAsync(ctx->host_red, res, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    out = ctx->host_red[0];
    return FWIME_OK;
  };
  std::vector<float> e2(nh);
  for (int h = 0; h < nh; ++h) e2[h] = (float)(eps * eps * dso[h] * dso[h]);
  HIPCHK(hipMemcpyAsync(e2d2, e2.data(), nh * sizeof(float), hipMemcpyHostToDevice, st));

  // residual of the background model and the right-hand side
  if ((rc = fwime_model(ctx, g, vel, geo, dtmp, stream))) return rc;
  HIPCHK(launch_sub(dobs, dtmp, dres, ndata, st));
  double c0 = 0.0, rr = 0.0;
  if ((rc = dot(dres, dres, ndata, c0))) return rc;
  c0 *= 0.5;
  AdjCache *cp = use_cache ? &cache : nullptr;
  auto fwd = [&](const float *x, float *d) {
    return tau ? fwime_born_ext_tau_fwd(ctx, g, vel, geo, nh, lag, x, d, stream)
               : fwime_born_ext_fwd(ctx, g, vel, geo, nh, x, d, stream);
  };
  auto adj = [&](const float *d, float *x) {
    return tau ? fwime_born_ext_tau_adj(ctx, g, vel, geo, nh, lag, d, x, stream)
               : born_ext_adj_run(ctx, g, vel, geo, nh, d, x, stream, cp);
  };
  if ((rc = adj(dres, b))) return rc;
  HIPCHK(launch_zero(ptilde_out, img, st));
  HIPCHK(hipMemcpyAsync(r, b, img * sizeof(float), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(sdir, b, img * sizeof(float), hipMemcpyDeviceToDevice, st));
  if ((rc = dot(r, r, img, rr))) return rc;
  phi_out[0] = c0;
  int k = 0;
  for (; k < niter; ++k) {
    // q = (B~* B~ + eps^2 D* D) s
    if ((rc = fwd(sdir, dtmp))) return rc;
    if ((rc = adj(dtmp, q))) return rc;
    HIPCHK(launch_add_diag(q, sdir, e2d2, plane, nh, st));
    double curv = 0.0;
    if ((rc = dot(sdir, q, img, curv))) return rc;
    if (!(curv > 0.0) || !std::isfinite(curv)) break;    // no curvature left along s: p~ is final
    const double alpha = rr / curv;
    HIPCHK(launch_cg_step(ptilde_out, r, sdir, q, (float)alpha, img, st));
    double rr_new = 0.0, bp = 0.0, rp = 0.0;
    if ((rc = dot(r, r, img, rr_new)) || (rc = dot(b, ptilde_out, img, bp)) || (rc = dot(r, ptilde_out, img, rp)))
      return rc;
    phi_out[k + 1] = c0 - 0.5 * (bp + rp);
    HIPCHK(launch_cg_dir(sdir, r, (float)(rr_new / rr), img, st));
    rr = rr_new;
  }
  for (int j = k + 1; j <= niter; ++j) phi_out[j] = phi_out[k];
  return FWIME_OK;
}

int fwime_vp_solve(fwime_ctx_t *ctx, const fwime_grid_t *g, const float *vel, const fwime_geom_t *geo,
                   int32_t nh, const float *dobs, double eps, const double *dso, int32_t niter,
                   float *ptilde_out, double *phi_out, void *stream) {
  return vp_solve_run(ctx, g, vel, geo, nh, false, 0, dobs, eps, dso, niter, ptilde_out, phi_out, stream);
}

int fwime_vp_solve_tau(fwime_ctx_t *ctx, const fwime_grid_t *g, const float *vel, const fwime_geom_t *geo,
                       int32_t ntau, int32_t lag, const float *dobs, double eps, const double *dso, int32_t niter,
                       float *ptau_out, double *phi_out, void *stream) {
  return vp_solve_run(ctx, g, vel, geo, ntau, true, lag, dobs, eps, dso, niter, ptau_out, phi_out, stream);
}

int fwime_gradient(fwime_ctx_t *ctx, const fwime_grid_t *g, const float *vel, const fwime_geom_t *geo, int32_t nh,
                   const float *ptilde, const float *dobs, double eps, const double *dso, double *obj,
                   float *grad_vel, float *grad_ptilde, void *stream) {
  if (!ctx) return FWIME_EINVAL;
  ctx->err.clear();
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if ((rc = check_grid(ctx, g)) || (rc = check_geom(ctx, g, geo)) || (rc = check_nh(ctx, g, nh))) return rc;
  if (!ptilde || !dobs || !dso || !obj || !grad_vel || !grad_ptilde)
    return set_err(ctx, FWIME_EINVAL, "null pointer argument");
  if (!std::isfinite(eps)) return set_err(ctx, FWIME_EINVAL, "eps must be finite");
  for (int h = 0; h < nh; ++h)
    if (!std::isfinite(dso[h])) return set_err(ctx, FWIME_EINVAL, "dso must be finite");
  HIPCHK(hipSetDevice(ctx->device));
  const long ndata = (long)geo->nshots * geo->nrec * g->nt;
  if ((rc = check_inputs(ctx, g, vel, geo, {{ptilde, (long)nh * g->nx * g->nz}, {dobs, ndata}}, st))) return rc;

  Common c;
  c.d = make_dims(g, ctx->tile_x);
  const Dims &d = c.d;
  ExtGeom eg{d.nz, d.nx, d.nb, d.NZ, d.NX, d.LZ, nh, (nh - 1) / 2};
  const GradPlan pl = grad_plan(d, g->nt);
  const long img = (long)nh * d.nx * d.nz;
  const long nrt = (long)geo->nrec * g->nt;
  const long per_shot =
      grad_work_per_shot(d, pl, ctx->two_step) + 2 * pl.ck_stride * 4 + 2 * nrt * 4 + (long)geo->nrec * 64;
  const size_t fixed = (size_t)d.field * 12 + (size_t)img * 4 * (5 + kImageGroups);
  const int S = choose_batch(ctx, per_shot, fixed, geo->nshots);
  auto batches = split_batches(geo->nshots, S);
  TableSet ts = build_table_set(d, geo, batches, ctx->two_step);

  double *acc = nullptr;
  float *coef = nullptr, *imgs = nullptr, *gacc = nullptr, *uck = nullptr, *dck = nullptr,
        *drec = nullptr, *ddrec = nullptr, *e2d2 = nullptr;
  double *sumsq = nullptr, *rpart = nullptr;
  GradWork wk;
  Carve cv;
  cv.add(&c.V, d.field);
  cv.add(&c.gz, d.LZ);
  cv.add(&c.gx, d.NX + kGxPad);
  cv.add(&c.tables, table_set_ints(ts) + 64 * batches.size() * 8);
  cv.add(&sumsq, 2);
  cv.add(&rpart, red_partials());
  cv.add(&e2d2, nh);
  cv.add(&coef, img);
  cv.add(&acc, img);
  cv.add(&imgs, img);
  cv.add(&gacc, d.field);
  cv.add(&uck, pl.ck_stride * S);
  cv.add(&dck, pl.ck_stride * S);
  carve_work(cv, wk, d, pl, S, ctx->two_step);
  cv.add(&wk.parts, kImageGroups * img);
  cv.add(&drec, nrt * S);
  cv.add(&ddrec, nrt * S);
  if ((rc = arena_get(ctx, cv))) return rc;
  if ((rc = upload_tables(ctx, ts, c.tables, st))) return rc;
  if ((rc = setup_common(ctx, c, g, vel, st))) return rc;
  std::vector<float> e2(nh);
  for (int h = 0; h < nh; ++h) e2[h] = (float)(eps * eps * dso[h] * dso[h]);
  HIPCHK(hipMemcpyAsync(e2d2, e2.data(), nh * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(launch_ext_coef(ptilde, vel, eg, (float)g->dt, coef, st));
  HIPCHK(launch_zero_d(acc, img, st));
  HIPCHK(launch_zero(gacc, d.field, st));
  HIPCHK(launch_zero_d(sumsq, 2, st));

  for (size_t bi = 0; bi < batches.size(); ++bi) {
    const int s0 = batches[bi].first, Sb = batches[bi].second;
    const DevTables &t = ts.dev[bi];
    const float *wav_b = geo->wavelet + (long)s0 * g->nt;
    if ((rc = grad_forward_batch(ctx, c, eg, pl, g, Sb, t, wav_b, coef, uck, dck, wk, drec, ddrec, geo->nrec, st)))
      return rc;
    HIPCHK(launch_residual(drec, ddrec, dobs + (long)s0 * nrt, nrt * Sb, rpart, sumsq, st));
    if ((rc = grad_backward_batch(ctx, c, eg, pl, g, Sb, t, wav_b, coef, uck, dck, wk, drec, acc, gacc, st)))
      return rc;
  }
  HIPCHK(launch_ext_finalize(acc, vel, eg, (float)g->dt, nullptr, nullptr, imgs, st));
  HIPCHK(launch_grad_finalize(gacc, c.V, vel, eg, (float)g->dt, ptilde, imgs, grad_vel, st));
  HIPCHK(launch_ext_finalize(acc, vel, eg, (float)g->dt, ptilde, e2d2, grad_ptilde, st));
  HIPCHK(launch_objective(sumsq, ptilde, e2d2, eg, rpart, obj, st));
  return FWIME_OK;
}

// ---------------------------------------------------------------------------
// FWIME objective and gradients with the time-lag extension.  Every history
// of a shot batch is kept whole (slot n of shot s at base + s hs + n field,
// hs = (nt + 1) fields): T2u and T2du~ of every step, the adjoint field of
// every time, and the scattering source, whose buffer then holds the spread
// e; rho runs in a ring of chunks of kTauChunk steps, each followed by its
// share of the gradient sums.
// ---------------------------------------------------------------------------
int fwime_gradient_tau(fwime_ctx_t *ctx, const fwime_grid_t *g, const float *vel, const fwime_geom_t *geo,
                       int32_t ntau, int32_t lag, const float *ptau, const float *dobs, double eps,
                       const double *dso, double *obj, float *grad_vel, float *grad_ptau, void *stream) {
  if (!ctx) return FWIME_EINVAL;
  ctx->err.clear();
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if ((rc = check_grid(ctx, g)) || (rc = check_geom(ctx, g, geo)) || (rc = check_tau(ctx, g, ntau, lag))) return rc;
  if (!ptau || !dobs || !dso || !obj || !grad_vel || !grad_ptau)
    return set_err(ctx, FWIME_EINVAL, "null pointer argument");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return set_err(ctx, FWIME_EINVAL, "eps must be finite and >= 0");
  for (int h = 0; h < ntau; ++h)
    if (!std::isfinite(dso[h])) return set_err(ctx, FWIME_EINVAL, "dso weights must be finite");
  HIPCHK(hipSetDevice(ctx->device));
  const long plane = (long)g->nx * g->nz, img = (long)ntau * plane;
  const long nrt = (long)geo->nrec * g->nt;
  if ((rc = check_inputs(ctx, g, vel, geo, {{ptau, img}, {dobs, nrt * geo->nshots}}, st))) return rc;

  constexpr int kTauChunk = 64;
  Common c;
  c.d = make_dims(g, ctx->tile_x);
  const Dims &d = c.d;
  ExtGeom eg{d.nz, d.nx, d.nb, d.NZ, d.NX, d.LZ, ntau, (ntau - 1) / 2};
  const int ns = g->nt - 1, R = g->nt + 1, RR = kTauChunk + 2;
  const long hs = (long)R * d.field, rs = (long)RR * d.field;
  // per shot: four histories of R fields, the rho ring, the wavefield rings
  // (8 fields) and the background's BF16 low parts (2), receiver data of u
  // and du~, tables
  const long per_shot = (4L * R + RR + 10) * d.field * 4 + 2 * nrt * 4 + (long)geo->nrec * 64;
  const size_t fixed = (size_t)d.field * 8 + (size_t)img * 4 * 3;
  const int S = choose_batch(ctx, per_shot, fixed, geo->nshots);
  auto batches = split_batches(geo->nshots, S);
  TableSet ts = build_table_set(d, geo, batches, true);

  float *coef = nullptr, *coefr = nullptr, *acc = nullptr, *gacc = nullptr, *e2d2 = nullptr, *pairs = nullptr,
        *hu = nullptr, *hdu = nullptr, *lam = nullptr, *sc = nullptr, *rho = nullptr, *drec = nullptr,
        *ddrec = nullptr;
  unsigned short *lows = nullptr;
  double *sumsq = nullptr, *rpart = nullptr;
  Carve cv;
  cv.add(&c.V, d.field);
  cv.add(&c.gz, d.LZ);
  cv.add(&c.gx, d.NX + kGxPad);
  cv.add(&c.tables, table_set_ints(ts) + 64 * batches.size() * 8);
  cv.add(&sumsq, 2);
  cv.add(&rpart, red_partials());
  cv.add(&e2d2, ntau);
  cv.add(&coef, img);
  cv.add(&coefr, img);
  cv.add(&acc, img);
  cv.add(&gacc, d.field);
  cv.add(&pairs, 8 * d.field * S);
  cv.add(&lows, 4 * d.field * S);
  cv.add(&hu, hs * S);
  cv.add(&hdu, hs * S);
  cv.add(&lam, hs * S);
  cv.add(&sc, hs * S);
  cv.add(&rho, rs * S);
  cv.add(&drec, nrt * S);
  cv.add(&ddrec, nrt * S);
  if ((rc = arena_get(ctx, cv))) return rc;
  if ((rc = upload_tables(ctx, ts, c.tables, st))) return rc;
  if ((rc = setup_common(ctx, c, g, vel, st))) return rc;
  std::vector<float> e2(ntau);
  for (int h = 0; h < ntau; ++h) e2[h] = (float)(eps * eps * dso[h] * dso[h]);
  HIPCHK(hipMemcpyAsync(e2d2, e2.data(), ntau * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(launch_ext_coef(ptau, vel, eg, (float)g->dt, coef, st));
  // the spread e_m = sum_k c_k lam_{m + 2kL} is the lag scatter with the
  // coefficient planes in reverse order: c'_k = c_{-k}
  for (int k = 0; k < ntau; ++k)
    HIPCHK(hipMemcpyAsync(coefr + (long)k * plane, coef + (long)(ntau - 1 - k) * plane, plane * sizeof(float),
                          hipMemcpyDeviceToDevice, st));
  HIPCHK(launch_zero(acc, img, st));
  HIPCHK(launch_zero(gacc, d.field, st));
  HIPCHK(launch_zero_d(sumsq, 2, st));

  for (size_t bi = 0; bi < batches.size(); ++bi) {
    const int s0 = batches[bi].first, Sb = batches[bi].second;
    const DevTables &t = ts.dev[bi];
    // background: T2u of every step, and its receiver data
    if ((rc = tau_background(ctx, c, g, geo, s0, Sb, t, pairs, lows, hu, hs, st, drec))) return rc;
    // scattering source history, then du~ with its T2 history and receivers
    HIPCHK(launch_zero(sc, hs * Sb, st));
    HIPCHK(launch_tau_scatter(coef, eg, lag, hu, sc, d.field, hs, ns, Sb, st));
    float *wp = pairs + 4 * d.field * Sb;
    HIPCHK(launch_zero(wp, 4 * d.field * Sb, st));
    Ring4 fw(wp, d.field * Sb);
    rc = march2(ctx, c, fw, Sb, 0, ns, kModeT2 | kModeDsrc, [&](Step2Args &p, int n, int k) {
      with_dsrc2(p, sc + (long)n * d.field, d.field, k, hs);
      p.a.t2 = hdu + (long)n * d.field;
      p.t2b = k == 2 ? hdu + (long)(n + 1) * d.field : nullptr;
      p.a.t2_sstride = hs;
      with_rec_extract(p.a, t, ddrec, g->nt, n);
    }, st);
    if (rc) return rc;
    HIPCHK(launch_gather(fw.cur(), d.field, t.cells, Sb, geo->nrec, ddrec, g->nt, g->nt - 1, st));
    // residual r = R(u + du~) - d_obs (into drec) and its sum of squares
    HIPCHK(launch_residual(drec, ddrec, dobs + (long)s0 * nrt, nrt * Sb, rpart, sumsq, st));
    // adjoint field of every time
    HIPCHK(launch_zero(lam, hs * Sb, st));
    if ((rc = march2_back_lambda(ctx, c, lam, hs, R, Sb, 0, g->nt - 1, t, drec, g->nt, st))) return rc;
    // spread e over the adjoint history (slots 0 .. ns-1; zero from ns on)
    HIPCHK(launch_zero(sc, hs * Sb, st));
    HIPCHK(launch_tau_scatter(coefr, eg, lag, lam, sc, d.field, hs, ns, Sb, st));
    // rho = M^-T nu, nu^k = e_{k-1}/g - 2 e_k + g e_{k+1}, chunk by chunk
    // backwards, each chunk followed by its gradient sums
    auto e_slot = [&](int k) { return sc + (long)k * d.field; };
    HIPCHK(launch_zero(rho, rs * Sb, st));
    const int nchunk = (ns + kTauChunk - 1) / kTauChunk;
    for (int j = nchunk - 1; j >= 0; --j) {
      const int n0 = j * kTauChunk, n1 = std::min(n0 + kTauChunk, ns);
      rc = march2_back_ring(ctx, c, rho, rs, RR, Sb, n0, n1, kModeNu, [&](Step2Args &p, int k, int kk) {
        p.a.nu = NuSource{e_slot(k - 1), e_slot(k), e_slot(k + 1), hs};
        if (kk == 2) p.nu2 = NuSource{e_slot(k - 2), e_slot(k - 1), e_slot(k), hs};
      }, st);
      if (rc) return rc;
      HIPCHK(launch_grad_accum2(hu + (long)n0 * d.field, hdu + (long)n0 * d.field, d.field, hs, lam, d.field, hs, R,
                                n0, rho, d.field, rs, RR, n0, Sb, n1 - n0, d.NZ, d.NX, d.LZ, gacc, st));
    }
    // B~_tau^T r (scaled by 2 / (v^3 dt^2) in the kernel)
    HIPCHK(launch_tau_image(hu, d.field, hs, lam, d.field, hs, ns, Sb, eg, lag, vel, (float)g->dt, acc, st));
  }
  HIPCHK(launch_grad_finalize(gacc, c.V, vel, eg, (float)g->dt, ptau, acc, grad_vel, st));
  HIPCHK(hipMemcpyAsync(grad_ptau, acc, img * sizeof(float), hipMemcpyDeviceToDevice, st));
  HIPCHK(launch_add_diag(grad_ptau, ptau, e2d2, plane, ntau, st));
  HIPCHK(launch_objective(sumsq, ptau, e2d2, eg, rpart, obj, st));
  return FWIME_OK;
}

// ---------------------------------------------------------------------------
void fwime_tape_free(fwime_tape_t *tape) {
  if (!tape) return;
  if (tape->mem) {
    (void)hipSetDevice(tape->ctx ? tape->ctx->device : 0);
    (void)hipDeviceSynchronize();
    (void)hipFree(tape->mem);
    if (tape->ctx) tape->ctx->tape_bytes -= tape->bytes;
  }
  delete tape;
}

int fwime_forward_tape(fwime_ctx_t *ctx, const fwime_grid_t *g, const float *vel, const fwime_geom_t *geo,
                       int32_t nh, const float *ptilde, float *data, fwime_tape_t **tape_out, void *stream) {
  if (!ctx) return FWIME_EINVAL;
  ctx->err.clear();
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if (!tape_out) return set_err(ctx, FWIME_EINVAL, "tape_out is null");
  *tape_out = nullptr;
  if ((rc = check_grid(ctx, g)) || (rc = check_geom(ctx, g, geo)) || (rc = check_nh(ctx, g, nh))) return rc;
  if (!ptilde || !data) return set_err(ctx, FWIME_EINVAL, "null pointer argument");
  HIPCHK(hipSetDevice(ctx->device));
  if ((rc = check_inputs(ctx, g, vel, geo, {{ptilde, (long)nh * g->nx * g->nz}}, st))) return rc;

  fwime_tape_t *tp = new fwime_tape_t();
  tp->ctx = ctx;
  tp->g = *g;
  tp->nh = nh;
  tp->nshots = geo->nshots;
  tp->nrec = geo->nrec;
  tp->d = make_dims(g, ctx->tile_x);
  const Dims &d = tp->d;
  tp->pl = grad_plan(d, g->nt);
  const GradPlan &pl = tp->pl;
  ExtGeom eg{d.nz, d.nx, d.nb, d.NZ, d.NX, d.LZ, nh, (nh - 1) / 2};
  const long img = (long)nh * d.nx * d.nz;
  const long nrt = (long)geo->nrec * g->nt;
  // checkpoints of every shot live in the tape; working fields in the arena
  const long per_shot = grad_work_per_shot(d, pl, ctx->two_step) + 2 * nrt * 4 + (long)geo->nrec * 64;
  const size_t tape_fixed = (size_t)(2 * pl.ck_stride * 4) * geo->nshots;
  const int S = choose_batch(ctx, per_shot, tape_fixed + (size_t)d.field * 8, geo->nshots);
  tp->batches = split_batches(geo->nshots, S);
  tp->ts = build_table_set(d, geo, tp->batches, ctx->two_step);

  Carve tc;   // tape memory
  tc.add(&tp->V, d.field);
  tc.add(&tp->gz, d.LZ);
  tc.add(&tp->gx, d.NX + kGxPad);
  tc.add(&tp->tables, table_set_ints(tp->ts) + 64 * tp->batches.size() * 8);
  tc.add(&tp->vel, (long)d.nx * d.nz);
  tc.add(&tp->pt, img);
  tc.add(&tp->coef, img);
  tc.add(&tp->wav, (long)geo->nshots * g->nt);
  tc.add(&tp->uck, pl.ck_stride * geo->nshots);
  tc.add(&tp->dck, pl.ck_stride * geo->nshots);
  if (ctx->budget && ctx->tape_bytes + tc.total + ctx->arena_bytes > ctx->budget) {
    delete tp;
    return set_err(ctx, FWIME_ENOMEM, "tape does not fit the HBM budget");
  }
  if (hipMalloc(&tp->mem, tc.total) != hipSuccess) {
    (void)hipGetLastError();
    delete tp;
    return set_err(ctx, FWIME_ENOMEM, "hipMalloc of the tape failed");
  }
  tp->bytes = tc.total;
  ctx->tape_bytes += tc.total;
  {
    char *p = (char *)tp->mem;
    for (auto &it : tc.items) {
      *it.first = p;
      p += it.second;
    }
  }
  auto fail = [&](int code) {
    fwime_tape_free(tp);
    return code;
  };
  if ((rc = upload_tables(ctx, tp->ts, tp->tables, st))) return fail(rc);
  Common c;
  c.d = d;
  c.V = tp->V;
  c.gz = tp->gz;
  c.gx = tp->gx;
  c.tables = tp->tables;
  if ((rc = setup_common(ctx, c, g, vel, st))) return fail(rc);
  if (hipMemcpyAsync(tp->vel, vel, sizeof(float) * d.nx * d.nz, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(tp->pt, ptilde, sizeof(float) * img, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(tp->wav, geo->wavelet, sizeof(float) * geo->nshots * g->nt, hipMemcpyDeviceToDevice, st) !=
          hipSuccess)
    return fail(set_err(ctx, FWIME_EHIP, "tape copy failed"));
  if (launch_ext_coef(tp->pt, tp->vel, eg, (float)g->dt, tp->coef, st) != hipSuccess)
    return fail(set_err(ctx, FWIME_EHIP, "coefficient launch failed"));

  float *drec = nullptr, *ddrec = nullptr;
  GradWork wk;
  Carve cv;
  carve_work(cv, wk, d, pl, S, ctx->two_step);
  cv.add(&drec, nrt * S);
  cv.add(&ddrec, nrt * S);
  if ((rc = arena_get(ctx, cv))) return fail(rc);
  for (size_t bi = 0; bi < tp->batches.size(); ++bi) {
    const int s0 = tp->batches[bi].first, Sb = tp->batches[bi].second;
    if ((rc = grad_forward_batch(ctx, c, eg, pl, g, Sb, tp->ts.dev[bi], tp->wav + (long)s0 * g->nt, tp->coef,
                                 tp->uck + s0 * pl.ck_stride, tp->dck + s0 * pl.ck_stride, wk, drec, ddrec,
                                 geo->nrec, st)))
      return fail(rc);
    // data = f(m) + B~ p~ for the batch
    if (launch_residual_sum(data + (long)s0 * nrt, drec, ddrec, nrt * Sb, st) != hipSuccess)
      return fail(set_err(ctx, FWIME_EHIP, "data sum failed"));
  }
  *tape_out = tp;
  return FWIME_OK;
}

int fwime_backward_tape(fwime_ctx_t *ctx, fwime_tape_t *tp, const float *adjsrc, float *grad_vel,
                        float *grad_ptilde, void *stream) {
  if (!ctx) return FWIME_EINVAL;
  ctx->err.clear();
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if (!tp || tp->ctx != ctx) return set_err(ctx, FWIME_EINVAL, "tape is null or belongs to another context");
  if (tp->used) return set_err(ctx, FWIME_EINVAL, "the tape's checkpoints were consumed by a previous backward");
  if (!adjsrc || !grad_vel || !grad_ptilde) return set_err(ctx, FWIME_EINVAL, "null pointer argument");
  HIPCHK(hipSetDevice(ctx->device));
  const fwime_grid_t *g = &tp->g;
  const Dims &d = tp->d;
  const GradPlan &pl = tp->pl;
  ExtGeom eg{d.nz, d.nx, d.nb, d.NZ, d.NX, d.LZ, tp->nh, (tp->nh - 1) / 2};
  const long img = (long)tp->nh * d.nx * d.nz;
  const long nrt = (long)tp->nrec * g->nt;
  {
    // finiteness of the adjoint source, checked before anything is written
    std::vector<double> r3;
    if ((rc = device_ranges(ctx, {{adjsrc, nrt * tp->nshots}}, st, r3))) return rc;
    if (r3[2] > 0) return set_err(ctx, FWIME_ENONFINITE, "adjoint source has non-finite values");
  }
  int S = 0;
  for (auto &b : tp->batches) S = std::max(S, b.second);
  double *acc = nullptr;
  float *imgs = nullptr, *gacc = nullptr;
  GradWork wk;
  Carve cv;
  cv.add(&acc, img);
  cv.add(&imgs, img);
  cv.add(&gacc, d.field);
  carve_work(cv, wk, d, pl, S, ctx->two_step);
  cv.add(&wk.parts, kImageGroups * img);
  if ((rc = arena_get(ctx, cv))) return rc;
  Common c;
  c.d = d;
  c.V = tp->V;
  c.gz = tp->gz;
  c.gx = tp->gx;
  c.tables = tp->tables;
  if ((rc = setup_common(ctx, c, g, tp->vel, st))) return rc;
  HIPCHK(launch_zero_d(acc, img, st));
  HIPCHK(launch_zero(gacc, d.field, st));
  tp->used = true;   // backward recomputes the segments in place over the checkpoints
  for (size_t bi = 0; bi < tp->batches.size(); ++bi) {
    const int s0 = tp->batches[bi].first, Sb = tp->batches[bi].second;
    if ((rc = grad_backward_batch(ctx, c, eg, pl, g, Sb, tp->ts.dev[bi], tp->wav + (long)s0 * g->nt, tp->coef,
                                  tp->uck + s0 * pl.ck_stride, tp->dck + s0 * pl.ck_stride, wk,
                                  adjsrc + (long)s0 * nrt, acc, gacc, st)))
      return rc;
  }
  HIPCHK(launch_ext_finalize(acc, tp->vel, eg, (float)g->dt, nullptr, nullptr, imgs, st));
  HIPCHK(launch_grad_finalize(gacc, c.V, tp->vel, eg, (float)g->dt, tp->pt, imgs, grad_vel, st));
  HIPCHK(hipMemcpyAsync(grad_ptilde, imgs, sizeof(float) * img, hipMemcpyDeviceToDevice, st));
  return FWIME_OK;
}

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Many modeling jobs of different grids in one launch per time step (two
// time steps per launch by default).
//
// Every job keeps its own padded velocity, taper, receiver tables and four
// (two with one step per launch) field buffers per shot; a device array of
// job descriptors lets one k_step2_multi (k_step_multi) launch advance all of
// them.  The time loop is recorded once as a graph of G (stencil, step-counter
// bump) node pairs on a private capture stream and replayed on the caller's
// stream until the longest job is done.
// The tile width comes from an autotuner: for a batch signature not seen
// before, each candidate width is timed on scratch fields (zero initial
// state, real velocity and sources) and the fastest is cached in the context.
// ---------------------------------------------------------------------------
struct BatchPlan {
  bool two = false;              // two time steps per launch (k_step2_multi)
  std::vector<int> order;        // position k in the launch -> caller's job index
  std::vector<Common> com;       // per position
  std::vector<TableSet> ts;
  std::vector<BatchJob> jobs;    // one-step descriptors
  std::vector<BatchJob2> jobs2;  // two-step descriptors
  std::vector<int> prefix;       // tiles before position k
  int total = 0;
  int nt_max = 0;
  bool fs = false;               // some job has a free surface
  int *dtile_job = nullptr;      // device: position k of every tile (two-step plans)
  int stride() const { return two ? 2 : 1; }
  // launches until the longest job has sampled its last time
  long launches() const { return two ? (nt_max - 1) / 2 + 1 : nt_max; }
  int nt_at(int k) const { return two ? jobs2[k].nt : jobs[k].nt; }
};

// Jobs are laid out in order of decreasing time-axis length, so the jobs still
// running at step n are a prefix of the list and a launch can stop at that
// prefix's last tile.
int batch_plan(fwime_ctx_t *ctx, int njobs, const fwime_job_t *jobs, int tx, BatchPlan &bp,
               std::vector<std::pair<void **, size_t>> *) {
  bp.two = ctx->two_step;
  bp.order.resize(njobs);
  for (int j = 0; j < njobs; ++j) bp.order[j] = j;
  std::stable_sort(bp.order.begin(), bp.order.end(),
                   [&](int a, int b) { return jobs[a].grid.nt > jobs[b].grid.nt; });
  bp.com.assign(njobs, Common());
  bp.ts.clear();
  bp.jobs.assign(bp.two ? 0 : njobs, BatchJob());
  bp.jobs2.assign(bp.two ? njobs : 0, BatchJob2());
  bp.prefix.assign(njobs + 1, 0);
  bp.total = 0;
  bp.nt_max = 0;
  bp.fs = false;
  for (int k = 0; k < njobs; ++k) {
    const int j = bp.order[k];
    bp.fs = bp.fs || jobs[j].grid.free_surface != 0;
    bp.com[k].d = make_dims(&jobs[j].grid, tx);
    const Dims &d = bp.com[k].d;
    bp.ts.push_back(build_table_set(d, &jobs[j].geom, {{0, jobs[j].geom.nshots}}, bp.two));
    if (bp.two) {
      bp.jobs2[k].tile_begin = bp.total;
      bp.jobs2[k].t0 = 0;
      bp.jobs2[k].nt = jobs[j].grid.nt;
      bp.total += d.ntz2 * d.ntx * jobs[j].geom.nshots;
    } else {
      bp.jobs[k].tile_begin = bp.total;
      bp.jobs[k].t0 = 0;
      bp.jobs[k].nt = jobs[j].grid.nt;
      bp.total += d.ntz * d.ntx * jobs[j].geom.nshots;
    }
    bp.prefix[k + 1] = bp.total;
    bp.nt_max = std::max(bp.nt_max, jobs[j].grid.nt);
  }
  return FWIME_OK;
}

// tiles of the jobs whose time index n is still within [0, nt - 1]
int batch_active_tiles(const BatchPlan &bp, long n) {
  int k = 0;
  const int nj = (int)bp.order.size();
  while (k < nj && n <= bp.nt_at(k) - 1) ++k;
  return bp.prefix[k];
}

// one multi-job launch (one or two time steps).  With a device step counter
// (graph replay) the launch is followed by the counter's bump; without one
// the global step is passed by value and nothing else is launched.
hipError_t batch_launch(const BatchPlan &bp, const void *djobs, int tiles, int *dstep, int step_val, int tx,
                        hipStream_t st) {
  const int nj = (int)bp.order.size();
  hipError_t e = bp.two ? launch_step2_multi((const BatchJob2 *)djobs, bp.dtile_job, nj, tiles, dstep, step_val, tx,
                                             bp.fs, st)
                        : launch_step_multi((const BatchJob *)djobs, nj, tiles, dstep, step_val, tx, bp.fs, st);
  if (e != hipSuccess || !dstep) return e;
  return launch_bump(dstep, bp.stride(), st);
}

int batch_carve_and_setup(fwime_ctx_t *ctx, int njobs, const fwime_job_t *jobs, BatchPlan &bp, void **djobs,
                          int **dstep, hipStream_t st) {
  Carve cv;
  std::vector<float *> fields(njobs);
  const int nf = bp.two ? 4 : 2;
  for (int k = 0; k < njobs; ++k) {
    const int j = bp.order[k];
    const Dims &d = bp.com[k].d;
    cv.add(&bp.com[k].V, d.field);
    cv.add(&bp.com[k].gz, d.LZ);
    cv.add(&bp.com[k].gx, d.NX + kGxPad);
    cv.add(&bp.com[k].tables, table_set_ints(bp.ts[k]) + 64 * 8);
    cv.add(&fields[k], nf * d.field * jobs[j].geom.nshots);
  }
  const size_t jb_bytes = bp.two ? sizeof(BatchJob2) : sizeof(BatchJob);
  char *dj = nullptr;
  cv.add(&dj, jb_bytes * njobs);
  cv.add(dstep, 1);
  if (bp.two) cv.add(&bp.dtile_job, bp.total);
  int rc = arena_get(ctx, cv);
  if (rc) return rc;
  for (int k = 0; k < njobs; ++k) {
    const int j = bp.order[k];
    const Dims &d = bp.com[k].d;
    const int S = jobs[j].geom.nshots;
    if ((rc = upload_tables(ctx, bp.ts[k], bp.com[k].tables, st, false))) return rc;
    if ((rc = setup_common(ctx, bp.com[k], &jobs[j].grid, jobs[j].vel, st))) return rc;
    HIPCHK(launch_zero(fields[k], nf * d.field * S, st));
    const DevTables &t = bp.ts[k].dev[0];
    if (bp.two) {
      BatchJob2 &bj = bp.jobs2[k];
      bj.p.a = batch_args(bp.com[k], S, d.field);
      bj.p.a.ntz = d.ntz2;
      with_src2(bj.p, t, jobs[j].geom.wavelet, &jobs[j].grid, 0);
      with_rec_extract(bj.p.a, t, jobs[j].data, jobs[j].grid.nt, 0);
      for (int q = 0; q < 4; ++q) bj.buf[q] = fields[k] + q * d.field * S;
    } else {
      BatchJob &bj = bp.jobs[k];
      bj.a = batch_args(bp.com[k], S, d.field);
      with_src(bj.a, t, &jobs[j].geom, &jobs[j].grid, 0, 0);
      with_rec_extract(bj.a, t, jobs[j].data, jobs[j].grid.nt, 0);
      bj.bufA = fields[k];
      bj.bufB = fields[k] + d.field * S;
    }
  }
  const void *host = bp.two ? (const void *)bp.jobs2.data() : (const void *)bp.jobs.data();
  HIPCHK(hipMemcpyAsync(dj, host, jb_bytes * njobs, hipMemcpyHostToDevice, st));
  // the job of every tile, so that a workgroup finds its job with one load
  std::vector<int> tile_job;
  if (bp.two) {
    tile_job.resize(bp.total);
    for (int k = 0; k < njobs; ++k)
      std::fill(tile_job.begin() + bp.prefix[k], tile_job.begin() + bp.prefix[k + 1], k);
    HIPCHK(hipMemcpyAsync(bp.dtile_job, tile_job.data(), sizeof(int) * bp.total, hipMemcpyHostToDevice, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  *djobs = dj;
  return FWIME_OK;
}

std::string batch_signature(int njobs, const fwime_job_t *jobs) {
  std::string sig;
  char buf[96];
  for (int j = 0; j < njobs; ++j) {
    std::snprintf(buf, sizeof buf, "%d,%d,%d,%d;", jobs[j].grid.nz + 2 * jobs[j].grid.nb,
                  jobs[j].grid.nx + 2 * jobs[j].grid.nb, jobs[j].geom.nshots, jobs[j].grid.nt > 1);
    sig += buf;
  }
  return sig;
}

// Times every tile width on the batch's first steps (receivers off) and
// keeps the context's width unless another is at least 2 % faster: the
// widths next to the best one are within a few per cent of it, and a choice
// made on noise would move the launch time from call to call.  Each width
// gets three timed windows of 8 launches; its time is the fastest window.
int batch_autotune(fwime_ctx_t *ctx, int njobs, const fwime_job_t *jobs, hipStream_t st, int *best_tx) {
  const int cand[5] = {16, 24, 32, 48, 64};
  float t_cand[5];
  *best_tx = ctx->tile_x;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  int rc = FWIME_OK;
  for (int ci = 0; ci < 5; ++ci) {
    const int tx = cand[ci];
    t_cand[ci] = 1e30f;
    BatchPlan bp;
    void *dj = nullptr;
    int *dstep = nullptr;
    if ((rc = batch_plan(ctx, njobs, jobs, tx, bp, nullptr))) break;
    if ((rc = batch_carve_and_setup(ctx, njobs, jobs, bp, &dj, &dstep, st))) break;
    // scratch run: receivers off, time kept below every job's last step
    for (auto &jb : bp.jobs) jb.a.ext.ptr = nullptr;
    for (auto &jb : bp.jobs2) jb.p.a.ext.ptr = nullptr;
    const void *host = bp.two ? (const void *)bp.jobs2.data() : (const void *)bp.jobs.data();
    const size_t jb_bytes = bp.two ? sizeof(BatchJob2) : sizeof(BatchJob);
    if (hipMemcpyAsync(dj, host, jb_bytes * njobs, hipMemcpyHostToDevice, st) != hipSuccess ||
        launch_zero(reinterpret_cast<float *>(dstep), 1, st) != hipSuccess) {   // all-zero bits: int 0
      rc = set_err(ctx, FWIME_EHIP, "autotune setup failed");
      break;
    }
    const int warm = 2, timed = 8, windows = 3;
    for (int i = 0; i < warm && rc == FWIME_OK; ++i)
      if (batch_launch(bp, dj, bp.total, dstep, 0, tx, st) != hipSuccess)
        rc = set_err(ctx, FWIME_EHIP, "autotune launch failed");
    for (int wdw = 0; wdw < windows && rc == FWIME_OK; ++wdw) {
      (void)hipEventRecord(e0, st);
      for (int i = 0; i < timed && rc == FWIME_OK; ++i)
        if (batch_launch(bp, dj, bp.total, dstep, 0, tx, st) != hipSuccess)
          rc = set_err(ctx, FWIME_EHIP, "autotune launch failed");
      if (rc) break;
      (void)hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess) {
        rc = set_err(ctx, FWIME_EHIP, "autotune sync failed");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      t_cand[ci] = std::min(t_cand[ci], ms);
    }
    if (rc) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  float t_def = 1e30f, t_best = 1e30f;
  int tx_best = ctx->tile_x;
  for (int ci = 0; ci < 5; ++ci) {
    if (cand[ci] == ctx->tile_x) t_def = t_cand[ci];
    if (t_cand[ci] < t_best) {
      t_best = t_cand[ci];
      tx_best = cand[ci];
    }
  }
  *best_tx = t_best < 0.98f * t_def ? tx_best : ctx->tile_x;
  return FWIME_OK;
}

}  // namespace

extern "C" {

int fwime_model_batch(fwime_ctx_t *ctx, int32_t njobs, const fwime_job_t *jobs, void *stream) {
  if (!ctx) return FWIME_EINVAL;
  ctx->err.clear();
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if (njobs < 1 || !jobs) return set_err(ctx, FWIME_EINVAL, "need njobs >= 1 and a job array");
  long nt_steps = 0;
  for (int j = 0; j < njobs; ++j) {
    if ((rc = check_grid(ctx, &jobs[j].grid)) || (rc = check_geom(ctx, &jobs[j].grid, &jobs[j].geom))) return rc;
    if (!jobs[j].data) return set_err(ctx, FWIME_EINVAL, "job data is null");
    nt_steps = std::max<long>(nt_steps, jobs[j].grid.nt);
  }
  HIPCHK(hipSetDevice(ctx->device));
  {
    // every job's velocity and wavelets in one device pass and one synchronization
    std::vector<std::pair<const float *, long>> arrays;
    for (int j = 0; j < njobs; ++j) {
      if (!jobs[j].vel) return set_err(ctx, FWIME_EINVAL, "job velocity is null");
      arrays.push_back({jobs[j].vel, (long)jobs[j].grid.nx * jobs[j].grid.nz});
      arrays.push_back({jobs[j].geom.wavelet, (long)jobs[j].geom.nshots * jobs[j].grid.nt});
    }
    std::vector<double> r;
    if ((rc = device_ranges(ctx, arrays, st, r))) return rc;
    for (int j = 0; j < njobs; ++j) {
      if ((rc = check_velocity_range(ctx, &jobs[j].grid, &r[6 * j]))) return rc;
      if (r[6 * j + 5] > 0) return set_err(ctx, FWIME_ENONFINITE, "input array has non-finite values");
    }
  }
  release_graph(ctx);   // the input checks synchronized the stream: earlier replays are done

  const std::string sig = batch_signature(njobs, jobs);
  int tx = ctx->tile_x;
  if (!std::getenv("FWIME_TILE_X")) {
    auto it = ctx->tuned.find(sig);
    if (it != ctx->tuned.end()) {
      tx = it->second;
    } else {
      if ((rc = batch_autotune(ctx, njobs, jobs, st, &tx))) return rc;
      ctx->tuned[sig] = tx;
    }
  }
  ctx->last_batch_tile = tx;

  BatchPlan bp;
  void *dj = nullptr;
  int *dstep = nullptr;
  if ((rc = batch_plan(ctx, njobs, jobs, tx, bp, nullptr))) return rc;
  if ((rc = batch_carve_and_setup(ctx, njobs, jobs, bp, &dj, &dstep, st))) return rc;
  HIPCHK(launch_zero(reinterpret_cast<float *>(dstep), 1, st));   // all-zero bits: int 0

  const int G = ctx->graph_steps;
  // Large batches: one direct launch per step over the still-running jobs
  // only (launch latency is negligible next to the step).  Small batches:
  // replay a captured graph of G full-width steps (idle jobs exit at once).
  const bool use_graph = !std::getenv("FWIME_NO_GRAPH") && bp.total <= kGraphMaxTiles;
  const long L = bp.launches();
  if (!use_graph) {
    HIPCHK(timing_begin(ctx, st));
    for (long i = 0; i < L; ++i)
      HIPCHK(batch_launch(bp, dj, batch_active_tiles(bp, i * bp.stride()), nullptr, (int)(i * bp.stride()), tx, st));
    HIPCHK(timing_end(ctx, st, L));
    return FWIME_OK;
  }
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // the capture stream is made on first use: contexts that never capture
  // (one per serving slot, say) do not take a hardware queue for it
  if (!ctx->capture) HIPCHK(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
  HIPCHK(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeRelaxed));
  hipError_t cap = hipSuccess;
  for (int i = 0; i < G && cap == hipSuccess; ++i) cap = batch_launch(bp, dj, bp.total, dstep, 0, tx, ctx->capture);
  hipError_t endc = hipStreamEndCapture(ctx->capture, &graph);
  if (cap != hipSuccess || endc != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return set_err(ctx, FWIME_EHIP, "graph capture failed");
  }
  if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return set_err(ctx, FWIME_EHIP, "graph instantiation failed");
  }
  const long replays = (L + G - 1) / G;
  HIPCHK(timing_begin(ctx, st));
  hipError_t le = hipSuccess;
  for (long r = 0; r < replays && le == hipSuccess; ++r) le = hipGraphLaunch(exec, st);
  if (le == hipSuccess) HIPCHK(timing_end(ctx, st, replays * G));
  ctx->graph = graph;          // kept until the replays have certainly finished
  ctx->graph_exec = exec;
  if (le != hipSuccess) return set_err(ctx, FWIME_EHIP, "graph launch failed");
  return FWIME_OK;
}

int fwime_footprint(const fwime_grid_t *g, int32_t nshots, int32_t nrec, int32_t nh, int32_t op, size_t *bytes) {
  if (!g || !bytes || nshots < 1 || nrec < 1 || nh < 1 || g->nt < 2) return FWIME_EINVAL;
  const Dims d = make_dims(g, 32);
  const long fb = d.field * 4;
  const long img = (long)nh * d.nx * d.nz * 4;
  const long nrt = (long)nrec * g->nt * 4;
  const GradPlan pl = grad_plan(d, g->nt);
  long per_shot = 0, fixed = fb + (long)(d.NX + d.LZ) * 4;
  // field buffers of the two-step path (the larger of the two paths)
  switch (op) {
    case FWIME_OP_MODEL: per_shot = 4 * fb; break;
    case FWIME_OP_BORN_FWD: per_shot = (8 + 2 * 16 + 4) * fb; fixed += img; break;
    case FWIME_OP_BORN_ADJ:
      per_shot = (4 + 2L * pl.nseg + pl.K + pl.R + 2 + (pl.R + 1) / 2 + pl.nseg) * fb;
      fixed += (2 + kImageGroups) * img;          // FP64 accumulator and partial images
      break;
    case FWIME_OP_GRADIENT:
      per_shot = grad_work_per_shot(d, pl, true) + 2 * pl.ck_stride * 4 + 2 * nrt;
      fixed += (5 + kImageGroups) * img;
      break;
    default: return FWIME_EINVAL;
  }
  *bytes = (size_t)(fixed + per_shot * nshots + (long)nrec * nshots * 64);
  return FWIME_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Continuous batching of modeling jobs (the request loop's engine).
//
// Jobs join a running multi-job time loop at the next round boundary and
// leave it when their last sample is recorded.  A round advances every
// active job by the same number of time steps in shared two-step launches
// (k_step2_multi, one launch per two steps over the tiles of all active
// jobs); a job's time index is the global step minus the step at which it
// joined, so jobs of different lengths and arrival times share launches.
// Per-job device memory (padded velocity, tapers, geometry tables, four
// wavefield buffers per shot) is allocated stream-ordered on the engine's
// stream when the job is submitted and freed the same way once its last
// round has completed; the job descriptors of a round go to one slot of a
// small device ring, reused only after that round's event has completed.
// ---------------------------------------------------------------------------
namespace {

struct EngineJob {
  int64_t ticket = 0;
  fwime_grid_t grid{};
  fwime_geom_t geom{};
  std::vector<int32_t> src_iz, src_ix, rec_iz, rec_ix;   // host copies of the geometry
  Common com;
  TableSet ts;
  void *mem = nullptr;
  BatchJob2 desc;
  int tiles = 0;
  long t0 = -1;            // global step at which the job's time index is 0
};

constexpr int kEngineRing = 4;

}  // namespace

struct fwime_engine {
  fwime_ctx_t *ctx = nullptr;
  hipStream_t st = nullptr;              // the engine's stream (all of its work)
  int steps = 64;                        // time steps per round (even)
  int max_jobs = 0;
  long step = 0;                         // global step counter
  int64_t next_ticket = 1;
  std::vector<EngineJob *> pending, active;
  std::vector<std::pair<EngineJob *, hipEvent_t>> finishing;
  std::vector<hipEvent_t> free_events;
  BatchJob2 *host_desc[kEngineRing] = {};
  BatchJob2 *dev_desc[kEngineRing] = {};
  hipEvent_t ring_ev[kEngineRing] = {};
  bool ring_used[kEngineRing] = {};
  int ring_i = 0;
  long rounds = 0;
  long launches = 0;
};

namespace {

void engine_release_job(fwime_engine_t *e, EngineJob *j) {
  if (j->mem) (void)hipFreeAsync(j->mem, e->st);
  delete j;
}

hipError_t engine_event(fwime_engine_t *e, hipEvent_t *ev) {
  if (!e->free_events.empty()) {
    *ev = e->free_events.back();
    e->free_events.pop_back();
    return hipSuccess;
  }
  return hipEventCreateWithFlags(ev, hipEventDisableTiming);
}

}  // namespace

extern "C" {

int fwime_engine_create(fwime_ctx_t *ctx, int32_t steps_per_round, int32_t max_jobs, void *stream,
                        fwime_engine_t **out) {
  if (!ctx || !out) return FWIME_EINVAL;
  *out = nullptr;
  if (steps_per_round < 2 || steps_per_round % 2 || max_jobs < 1)
    return set_err(ctx, FWIME_EINVAL, "steps_per_round must be even and >= 2, max_jobs >= 1");
  HIPCHK(hipSetDevice(ctx->device));
  fwime_engine_t *e = new fwime_engine_t();
  e->ctx = ctx;
  e->st = (hipStream_t)stream;
  e->steps = steps_per_round;
  e->max_jobs = max_jobs;
  const size_t bytes = sizeof(BatchJob2) * (size_t)max_jobs;
  for (int i = 0; i < kEngineRing; ++i) {
    if (hipHostMalloc((void **)&e->host_desc[i], bytes, hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void **)&e->dev_desc[i], bytes) != hipSuccess ||
        hipEventCreateWithFlags(&e->ring_ev[i], hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      fwime_engine_destroy(e);
      return set_err(ctx, FWIME_ENOMEM, "engine descriptor ring allocation failed");
    }
  }
  *out = e;
  return FWIME_OK;
}

int fwime_engine_submit(fwime_engine_t *e, const fwime_job_t *job, void *check_stream, int64_t *ticket) {
  if (!e || !job || !ticket) return FWIME_EINVAL;
  fwime_ctx_t *ctx = e->ctx;
  ctx->err.clear();
  int rc;
  if ((rc = check_grid(ctx, &job->grid)) || (rc = check_geom(ctx, &job->grid, &job->geom))) return rc;
  if (!job->data || !job->vel) return set_err(ctx, FWIME_EINVAL, "job data or velocity is null");
  if ((long)e->pending.size() + (long)e->active.size() >= e->max_jobs)
    return set_err(ctx, FWIME_ENOMEM, "the engine holds max_jobs jobs already");
  HIPCHK(hipSetDevice(ctx->device));
  {
    // velocity range and finite wavelets, on the stream that produced them
    std::vector<double> r;
    hipStream_t cs = (hipStream_t)check_stream;
    if ((rc = device_ranges(ctx, {{job->vel, (long)job->grid.nx * job->grid.nz},
                                  {job->geom.wavelet, (long)job->geom.nshots * job->grid.nt}}, cs, r)))
      return rc;
    if ((rc = check_velocity_range(ctx, &job->grid, r.data()))) return rc;
    if (r[5] > 0) return set_err(ctx, FWIME_ENONFINITE, "input array has non-finite values");
  }
  EngineJob *j = new EngineJob();
  j->grid = job->grid;
  j->geom = job->geom;
  const long ns = job->geom.nshots, nr = (long)job->geom.nshots * job->geom.nrec;
  j->src_iz.assign(job->geom.src_iz, job->geom.src_iz + ns);
  j->src_ix.assign(job->geom.src_ix, job->geom.src_ix + ns);
  j->rec_iz.assign(job->geom.rec_iz, job->geom.rec_iz + nr);
  j->rec_ix.assign(job->geom.rec_ix, job->geom.rec_ix + nr);
  j->geom.src_iz = j->src_iz.data();
  j->geom.src_ix = j->src_ix.data();
  j->geom.rec_iz = j->rec_iz.data();
  j->geom.rec_ix = j->rec_ix.data();
  Common &c = j->com;
  c.d = make_dims(&j->grid, ctx->tile_x);
  const Dims &d = c.d;
  const int S = (int)ns;
  j->ts = build_table_set(d, &j->geom, {{0, S}}, true);
  float *fields = nullptr;
  Carve cv;
  cv.add(&c.V, d.field);
  cv.add(&c.gz, d.LZ);
  cv.add(&c.gx, d.NX + kGxPad);
  cv.add(&c.tables, table_set_ints(j->ts) + 64 * 8);
  cv.add(&fields, 4 * d.field * S);
  if (ctx->budget && cv.total > ctx->budget) {
    delete j;
    return set_err(ctx, FWIME_ENOMEM, "the job exceeds the HBM budget");
  }
  if (hipMallocAsync(&j->mem, cv.total, e->st) != hipSuccess) {
    (void)hipGetLastError();
    delete j;
    return set_err(ctx, FWIME_ENOMEM, "hipMallocAsync of " + std::to_string(cv.total) + " bytes failed");
  }
  cv.assign(j->mem);
  // the blob stays alive in the job until it is released, after the copy
  if ((rc = upload_tables(ctx, j->ts, c.tables, e->st, false)) || (rc = setup_common(ctx, c, &j->grid, job->vel, e->st)) ||
      (launch_zero(fields, 4 * d.field * S, e->st) != hipSuccess ? (rc = FWIME_EHIP) : 0)) {
    engine_release_job(e, j);
    return rc ? rc : set_err(ctx, FWIME_EHIP, "engine job setup failed");
  }
  const DevTables &t = j->ts.dev[0];
  BatchJob2 &bj = j->desc;
  bj.p.a = batch_args(c, S, d.field);
  bj.p.a.ntz = d.ntz2;
  with_src2(bj.p, t, job->geom.wavelet, &j->grid, 0);
  with_rec_extract(bj.p.a, t, job->data, j->grid.nt, 0);
  for (int q = 0; q < 4; ++q) bj.buf[q] = fields + q * d.field * S;
  bj.nt = j->grid.nt;
  j->tiles = d.ntz2 * d.ntx * S;
  j->ticket = e->next_ticket++;
  e->pending.push_back(j);
  *ticket = j->ticket;
  return FWIME_OK;
}

int fwime_engine_run(fwime_engine_t *e) {
  if (!e) return FWIME_EINVAL;
  fwime_ctx_t *ctx = e->ctx;
  ctx->err.clear();
  HIPCHK(hipSetDevice(ctx->device));
  // jobs join at this round's boundary
  for (EngineJob *j : e->pending) {
    j->t0 = e->step;
    j->desc.t0 = (int)e->step;
    e->active.push_back(j);
  }
  e->pending.clear();
  if (e->active.empty()) return FWIME_OK;
  // descriptor slot of this round: free once the round that used it last is done
  const int i = e->ring_i;
  if (e->ring_used[i]) HIPCHK(hipEventSynchronize(e->ring_ev[i]));
  int total = 0;
  bool fs = false;
  const int nj = (int)e->active.size();
  for (int k = 0; k < nj; ++k) {
    EngineJob *j = e->active[k];
    j->desc.tile_begin = total;
    total += j->tiles;
    fs = fs || j->grid.free_surface != 0;
    e->host_desc[i][k] = j->desc;
  }
  HIPCHK(hipMemcpyAsync(e->dev_desc[i], e->host_desc[i], sizeof(BatchJob2) * nj, hipMemcpyHostToDevice, e->st));
  const int L = e->steps / 2;
  for (int l = 0; l < L; ++l)
    HIPCHK(launch_step2_multi(e->dev_desc[i], nullptr, nj, total, nullptr, (int)(e->step + 2L * l), ctx->tile_x, fs,
                              e->st));
  HIPCHK(hipEventRecord(e->ring_ev[i], e->st));
  e->ring_used[i] = true;
  e->ring_i = (i + 1) % kEngineRing;
  e->step += e->steps;
  e->rounds += 1;
  e->launches += L;
  // jobs whose last sample (time index nt - 1) was recorded in this round leave
  std::vector<EngineJob *> keep;
  for (EngineJob *j : e->active) {
    // the last launch of the round ran time index e->step - 2 - t0; the job
    // recorded its last sample once that index reached nt - 2 (two-step
    // launch) or nt - 1 (sample only): e->step - t0 >= nt, both being even
    if (e->step - j->t0 >= (long)j->grid.nt) {
      hipEvent_t ev;
      HIPCHK(engine_event(e, &ev));
      HIPCHK(hipEventRecord(ev, e->st));
      e->finishing.push_back({j, ev});
    } else {
      keep.push_back(j);
    }
  }
  e->active.swap(keep);
  return FWIME_OK;
}

int fwime_engine_poll(fwime_engine_t *e, int64_t *tickets, int32_t cap, int32_t *ndone) {
  if (!e || !ndone || (cap > 0 && !tickets)) return FWIME_EINVAL;
  fwime_ctx_t *ctx = e->ctx;
  HIPCHK(hipSetDevice(ctx->device));
  int n = 0;
  std::vector<std::pair<EngineJob *, hipEvent_t>> keep;
  for (auto &f : e->finishing) {
    if (n < cap && hipEventQuery(f.second) == hipSuccess) {
      tickets[n++] = f.first->ticket;
      e->free_events.push_back(f.second);
      engine_release_job(e, f.first);
    } else {
      (void)hipGetLastError();
      keep.push_back(f);
    }
  }
  e->finishing.swap(keep);
  *ndone = n;
  return FWIME_OK;
}

int fwime_engine_info(const fwime_engine_t *e, fwime_engine_info_t *out) {
  if (!e || !out) return FWIME_EINVAL;
  out->pending = (int32_t)e->pending.size();
  out->active = (int32_t)e->active.size();
  out->finishing = (int32_t)e->finishing.size();
  out->step = e->step;
  out->rounds = e->rounds;
  out->launches = e->launches;
  return FWIME_OK;
}

void fwime_engine_destroy(fwime_engine_t *e) {
  if (!e) return;
  (void)hipSetDevice(e->ctx->device);
  if (e->st) (void)hipStreamSynchronize(e->st);
  for (EngineJob *j : e->pending) engine_release_job(e, j);
  for (EngineJob *j : e->active) engine_release_job(e, j);
  for (auto &f : e->finishing) {
    engine_release_job(e, f.first);
    (void)hipEventDestroy(f.second);
  }
  if (e->st) (void)hipStreamSynchronize(e->st);
  for (hipEvent_t ev : e->free_events) (void)hipEventDestroy(ev);
  for (int i = 0; i < kEngineRing; ++i) {
    if (e->host_desc[i]) (void)hipHostFree(e->host_desc[i]);
    if (e->dev_desc[i]) (void)hipFree(e->dev_desc[i]);
    if (e->ring_ev[i]) (void)hipEventDestroy(e->ring_ev[i]);
  }
  delete e;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Linear spline operator S and its adjoint (Section 2's spline grid)
// ---------------------------------------------------------------------------
namespace fw {
hipError_t launch_spline_tables(const double *nodes, int nn, const double *pts, int nf, double h, int *cell,
                                float *wt, int *start, hipStream_t st);
hipError_t launch_spline_apply(const float *mc, int nzn, const int *cz, const float *tz, const int *cx,
                               const float *tx, int nz, int nx, float *out, hipStream_t st);
hipError_t launch_spline_adjoint(const float *f, int nz, int nx, const float *tz, const int *sz, int nzn,
                                 const float *tx, const int *sx, int nxn, float *tmp, float *out, hipStream_t st);
}  // namespace fw

namespace {

struct SplineAxes {
  double *zn = nullptr, *xn = nullptr;
  int *cz = nullptr, *cx = nullptr, *sz = nullptr, *sx = nullptr;
  float *tz = nullptr, *tx = nullptr;
};

int check_spline_axis(fwime_ctx_t *ctx, const double *n, int32_t nn, int32_t nf, double h, const char *name) {
  const std::string nm(name);
  if (nn < 2) return set_err(ctx, FWIME_EINVAL, nm + ": at least two spline nodes are needed");
  if (nn > kSplineMaxNodes) return set_err(ctx, FWIME_EINVAL, nm + ": more than 2^24 spline nodes");
  if (nf < 1 || nf > (1 << 30)) return set_err(ctx, FWIME_EINVAL, nm + ": the grid needs 1 to 2^30 points");
  if (!(h > 0.0) || !std::isfinite(h)) return set_err(ctx, FWIME_EINVAL, nm + ": grid spacing must be positive");
  if (!n) return set_err(ctx, FWIME_EINVAL, nm + " node coordinates are null");
  for (int j = 0; j < nn; ++j)
    if (!std::isfinite(n[j])) return set_err(ctx, FWIME_EINVAL, nm + " node coordinates must be finite");
  for (int j = 1; j < nn; ++j)
    if (!(n[j] > n[j - 1])) return set_err(ctx, FWIME_EINVAL, nm + " node coordinates must be strictly increasing");
  const double tol = 1e-9 * std::max(1.0, std::fabs(n[nn - 1] - n[0]));
  if (n[0] > tol || (nf - 1) * h > n[nn - 1] + tol)
    return set_err(ctx, FWIME_EINVAL, nm + " nodes must cover every grid point");
  return FWIME_OK;
}

// validates, carves the tables (plus `extra` floats) from the arena, uploads
// the node coordinates and builds the per-axis tables on `st`
int spline_setup(fwime_ctx_t *ctx, int32_t nz, int32_t nx, double dz, double dx, int32_t nzn, const double *zn,
                 int32_t nxn, const double *xn, const void *in, void *out, long extra, float **extra_ptr,
                 SplineAxes &a, hipStream_t st) {
  int rc;
  if ((rc = check_spline_axis(ctx, zn, nzn, nz, dz, "z")) || (rc = check_spline_axis(ctx, xn, nxn, nx, dx, "x")))
    return rc;
  if (!in || !out) return set_err(ctx, FWIME_EINVAL, "input or output is null");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(hipStreamSynchronize(st));      // earlier work on the stream may still use the arena
  Carve cv;
  cv.add(&a.zn, nzn);
  cv.add(&a.xn, nxn);
  cv.add(&a.cz, nz);
  cv.add(&a.cx, nx);
  cv.add(&a.tz, nz);
  cv.add(&a.tx, nx);
  cv.add(&a.sz, (long)nzn + 1);
  cv.add(&a.sx, (long)nxn + 1);
  if (extra > 0) cv.add(extra_ptr, extra);
  if ((rc = arena_get(ctx, cv))) return rc;
  // pageable sources are copied synchronously: nothing of the caller's is read later
  HIPCHK(hipMemcpyAsync(a.zn, zn, nzn * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(a.xn, xn, nxn * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(launch_spline_tables(a.zn, nzn, nullptr, nz, dz, a.cz, a.tz, a.sz, st));
  HIPCHK(launch_spline_tables(a.xn, nxn, nullptr, nx, dx, a.cx, a.tx, a.sx, st));
  return FWIME_OK;
}

}  // namespace

extern "C" {

int fwime_spline_apply(fwime_ctx_t *ctx, int32_t nz, int32_t nx, double dz, double dx, int32_t nzn, const double *zn,
                       int32_t nxn, const double *xn, const float *mc, float *out, void *stream) {
  if (!ctx) return FWIME_EINVAL;
  ctx->err.clear();
  hipStream_t st = (hipStream_t)stream;
  SplineAxes a;
  int rc = spline_setup(ctx, nz, nx, dz, dx, nzn, zn, nxn, xn, mc, out, 0, nullptr, a, st);
  if (rc) return rc;
  HIPCHK(launch_spline_apply(mc, nzn, a.cz, a.tz, a.cx, a.tx, nz, nx, out, st));
  return FWIME_OK;
}

int fwime_spline_adjoint(fwime_ctx_t *ctx, int32_t nz, int32_t nx, double dz, double dx, int32_t nzn,
                         const double *zn, int32_t nxn, const double *xn, const float *f, float *mc_out,
                         void *stream) {
  if (!ctx) return FWIME_EINVAL;
  ctx->err.clear();
  hipStream_t st = (hipStream_t)stream;
  SplineAxes a;
  float *tmp = nullptr;
  int rc = spline_setup(ctx, nz, nx, dz, dx, nzn, zn, nxn, xn, f, mc_out, (long)nx * nzn, &tmp, a, st);
  if (rc) return rc;
  HIPCHK(launch_spline_adjoint(f, nz, nx, a.tz, a.sz, nzn, a.tx, a.sx, nxn, tmp, mc_out, st));
  return FWIME_OK;
}

int fwime_spline_refine(fwime_ctx_t *ctx, int32_t nzn, const double *zn, int32_t nxn, const double *xn,
                        const float *mc, int32_t nzf, const double *zf, int32_t nxf, const double *xf,
                        float *mf_out, void *stream) {
  if (!ctx) return FWIME_EINVAL;
  ctx->err.clear();
  hipStream_t st = (hipStream_t)stream;
  // the new nodes: strictly increasing, inside the old nodes' span
  auto targets = [&](const double *t, int32_t nt_, const double *n, int32_t nn, const char *name) -> int {
    const std::string nm(name);
    if (nt_ < 1 || nt_ > kSplineMaxNodes) return set_err(ctx, FWIME_EINVAL, nm + ": 1 to 2^24 new nodes");
    if (!t) return set_err(ctx, FWIME_EINVAL, nm + " new node coordinates are null");
    for (int j = 0; j < nt_; ++j)
      if (!std::isfinite(t[j]) || (j > 0 && !(t[j] > t[j - 1])))
        return set_err(ctx, FWIME_EINVAL, nm + " new node coordinates must be finite and strictly increasing");
    if (nn >= 2 && n) {
      const double tol = 1e-9 * std::max(1.0, std::fabs(n[nn - 1] - n[0]));
      if (t[0] < n[0] - tol || t[nt_ - 1] > n[nn - 1] + tol)
        return set_err(ctx, FWIME_EINVAL, nm + " new nodes must lie within the old nodes");
    }
    return FWIME_OK;
  };
  int rc;
  if ((rc = check_spline_axis(ctx, zn, nzn, 1, 1.0, "z")) || (rc = check_spline_axis(ctx, xn, nxn, 1, 1.0, "x")) ||
      (rc = targets(zf, nzf, zn, nzn, "z")) || (rc = targets(xf, nxf, xn, nxn, "x")))
    return rc;
  if (!mc || !mf_out) return set_err(ctx, FWIME_EINVAL, "input or output is null");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(hipStreamSynchronize(st));      // earlier work on the stream may still use the arena
  SplineAxes a;
  double *zt = nullptr, *xt = nullptr;
  Carve cv;
  cv.add(&a.zn, nzn);
  cv.add(&a.xn, nxn);
  cv.add(&zt, nzf);
  cv.add(&xt, nxf);
  cv.add(&a.cz, nzf);
  cv.add(&a.cx, nxf);
  cv.add(&a.tz, nzf);
  cv.add(&a.tx, nxf);
  cv.add(&a.sz, (long)nzn + 1);
  cv.add(&a.sx, (long)nxn + 1);
  if ((rc = arena_get(ctx, cv))) return rc;
  HIPCHK(hipMemcpyAsync(a.zn, zn, nzn * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(a.xn, xn, nxn * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(zt, zf, nzf * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(xt, xf, nxf * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(launch_spline_tables(a.zn, nzn, zt, nzf, 0.0, a.cz, a.tz, a.sz, st));
  HIPCHK(launch_spline_tables(a.xn, nxn, xt, nxf, 0.0, a.cx, a.tx, a.sx, st));
  HIPCHK(launch_spline_apply(mc, nzn, a.cz, a.tz, a.cx, a.tx, nzf, nxf, mf_out, st));
  return FWIME_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// L-BFGS search direction (Section 3: the outer minimization uses L-BFGS)
// ---------------------------------------------------------------------------
namespace fw {
hipError_t launch_axpby(const float *x, float a, float *y, float b, long n, hipStream_t st);
}  // namespace fw

namespace {

constexpr int kLbfgsMaxEvals = 100;      // trial steps per line search
constexpr long kLbfgsWorkHead = 4096;    // floats of the workspace before the vectors (dot partials)

// d = H g by the two-loop recursion over the pairs S[i], Y[i] (oldest first),
// H_0 = (s.y / y.y of the newest pair) I; FP64 inner products, FP32 updates.
// Every pair's curvature is checked before d is written.
int two_loop(fwime_ctx_t *ctx, long n, const std::vector<const float *> &S, const std::vector<const float *> &Y,
             const float *g, float *d, double *part, double *res, hipStream_t st) {
  const int k = (int)S.size();
  int rc;
  auto dot = [&](const float *a, const float *b, double &out) -> int {
    HIPCHK(launch_dot(a, b, n, part, res, st));
    HIPCHK(hipMemcpyAsync(ctx->host_red, res, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    out = ctx->host_red[0];
    return FWIME_OK;
  };
  std::vector<double> rho(k), alpha(k);
  double sy = 0.0, yy = 1.0;
  for (int i = 0; i < k; ++i) {
    if ((rc = dot(S[i], Y[i], sy))) return rc;
    if (!(sy > 0.0) || !std::isfinite(sy))
      return set_err(ctx, FWIME_EINVAL, "pair " + std::to_string(i) + " has s.y <= 0 or non-finite");
    rho[i] = 1.0 / sy;
  }
  double gamma = 1.0;
  if (k > 0) {
    if ((rc = dot(Y[k - 1], Y[k - 1], yy))) return rc;
    gamma = (1.0 / rho[k - 1]) / yy;
  }
  if (d != g) HIPCHK(hipMemcpyAsync(d, g, (size_t)n * sizeof(float), hipMemcpyDeviceToDevice, st));
  for (int i = k - 1; i >= 0; --i) {
    double sq;
    if ((rc = dot(S[i], d, sq))) return rc;
    alpha[i] = rho[i] * sq;
    HIPCHK(launch_axpby(Y[i], (float)-alpha[i], d, 1.0f, n, st));
  }
  HIPCHK(launch_axpby(d, 0.0f, d, (float)gamma, n, st));
  for (int i = 0; i < k; ++i) {
    double yr;
    if ((rc = dot(Y[i], d, yr))) return rc;
    HIPCHK(launch_axpby(S[i], (float)(alpha[i] - rho[i] * yr), d, 1.0f, n, st));
  }
  return FWIME_OK;
}

}  // namespace

extern "C" {

int fwime_lbfgs_direction(fwime_ctx_t *ctx, int64_t n, int32_t npairs, const float *s, const float *y,
                          const float *g, float *d_out, void *stream) {
  if (!ctx) return FWIME_EINVAL;
  ctx->err.clear();
  hipStream_t st = (hipStream_t)stream;
  if (n < 1) return set_err(ctx, FWIME_EINVAL, "n must be >= 1");
  if (npairs < 0 || npairs > kLbfgsMaxPairs)
    return set_err(ctx, FWIME_EINVAL, "npairs must be in [0, " + std::to_string(kLbfgsMaxPairs) + "]");
  if (!g || !d_out || (npairs > 0 && (!s || !y))) return set_err(ctx, FWIME_EINVAL, "null vector");
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(hipStreamSynchronize(st));      // earlier work on the stream may still use the arena
  double *part = nullptr, *res = nullptr;
  Carve cv;
  cv.add(&part, dot_partials());
  cv.add(&res, 1);
  int rc;
  if ((rc = arena_get(ctx, cv))) return rc;
  std::vector<const float *> S(npairs), Y(npairs);
  for (int i = 0; i < npairs; ++i) {
    S[i] = s + (long)i * n;
    Y[i] = y + (long)i * n;
  }
  if ((rc = two_loop(ctx, (long)n, S, Y, g, d_out, part, res, st))) return rc;
  HIPCHK(launch_axpby(d_out, 0.0f, d_out, -1.0f, (long)n, st));
  return FWIME_OK;
}

int fwime_lbfgs_minimize(fwime_ctx_t *ctx, int64_t n, int32_t memory, int32_t maxiter, double gtol,
                         fwime_objective_fn fg, void *user, float *x, float *work, int64_t work_floats,
                         double *f_hist, int32_t *iters, void *stream) {
  if (!ctx) return FWIME_EINVAL;
  ctx->err.clear();
  hipStream_t st = (hipStream_t)stream;
  if (n < 1) return set_err(ctx, FWIME_EINVAL, "n must be >= 1");
  if (memory < 1 || memory > kLbfgsMaxPairs)
    return set_err(ctx, FWIME_EINVAL, "memory must be in [1, " + std::to_string(kLbfgsMaxPairs) + "]");
  if (maxiter < 0) return set_err(ctx, FWIME_EINVAL, "maxiter must be >= 0");
  if (!(gtol >= 0.0) || !std::isfinite(gtol)) return set_err(ctx, FWIME_EINVAL, "gtol must be finite and >= 0");
  if (!fg || !x || !work || !f_hist || !iters) return set_err(ctx, FWIME_EINVAL, "null argument");
  if ((reinterpret_cast<uintptr_t>(work) & 7) != 0) return set_err(ctx, FWIME_EINVAL, "work must be 8-byte aligned");
  if (n > (int64_t(1) << 40) || work_floats < kLbfgsWorkHead + (2 * (int64_t)memory + 6) * n)
    return set_err(ctx, FWIME_EINVAL, "work needs 4096 + (2 memory + 6) n floats");
  HIPCHK(hipSetDevice(ctx->device));
  // work: dot partials, then g, d, trial x, trial g and memory + 1 slots each of s and y
  double *part = (double *)work, *res = part + dot_partials();
  float *vec = work + kLbfgsWorkHead;
  auto V = [&](long j) { return vec + j * (long)n; };
  float *g = V(0), *d = V(1), *xt = V(2), *gt = V(3);
  std::vector<float *> sslot(memory + 1), yslot(memory + 1);
  for (int j = 0; j <= memory; ++j) {
    sslot[j] = V(4 + j);
    yslot[j] = V(5 + memory + j);
  }
  int rc;
  auto dot = [&](const float *a, const float *b, double &out) -> int {
    HIPCHK(launch_dot(a, b, (long)n, part, res, st));
    HIPCHK(hipMemcpyAsync(ctx->host_red, res, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    out = ctx->host_red[0];
    return FWIME_OK;
  };
  auto eval = [&](const float *at, float *grad, double &f) -> int {
    const int cb = fg(user, at, grad, &f);
    if (cb != 0) return set_err(ctx, FWIME_EINVAL, "objective callback returned " + std::to_string(cb));
    if (!std::isfinite(f)) return set_err(ctx, FWIME_ENONFINITE, "objective is not finite");
    return FWIME_OK;
  };
  double f = 0.0, gg = 0.0;
  if ((rc = eval(x, g, f)) || (rc = dot(g, g, gg))) return rc;
  const double g0 = std::sqrt(gg);
  f_hist[0] = f;
  // pairs kept oldest first, as slot indices; one slot is always free
  std::vector<int> pairs, free_slots;
  for (int j = memory; j >= 0; --j) free_slots.push_back(j);
  int it = 0;
  for (; it < maxiter; ++it) {
    if (std::sqrt(gg) <= gtol * g0) break;
    std::vector<const float *> S, Y;
    for (int j : pairs) {
      S.push_back(sslot[j]);
      Y.push_back(yslot[j]);
    }
    if ((rc = two_loop(ctx, (long)n, S, Y, g, d, part, res, st))) return rc;
    HIPCHK(launch_axpby(d, 0.0f, d, -1.0f, (long)n, st));   // descent direction -H g
    double dphi0;
    if ((rc = dot(g, d, dphi0))) return rc;
    if (!(dphi0 < 0.0)) break;
    MoreThuente ls;
    ls.stpmin = 0.0;
    ls.stpmax = 1e10;
    auto status = ls.start(1.0, f, dphi0);
    double ft = 0.0;
    for (int nfev = 0; status == MoreThuente::kEvaluate && nfev < kLbfgsMaxEvals; ++nfev) {
      HIPCHK(hipMemcpyAsync(xt, x, (size_t)n * sizeof(float), hipMemcpyDeviceToDevice, st));
      HIPCHK(launch_axpby(d, (float)ls.stp, xt, 1.0f, (long)n, st));
      double dphi;
      if ((rc = eval(xt, gt, ft)) || (rc = dot(gt, d, dphi))) return rc;
      status = ls.next(ft, dphi);
    }
    if (status != MoreThuente::kConverged) break;
    // new pair: s = x_t - x, y = g_t - g, kept if its curvature is positive
    const int slot = free_slots.back();
    float *sn = sslot[slot], *yn = yslot[slot];
    HIPCHK(hipMemcpyAsync(sn, xt, (size_t)n * sizeof(float), hipMemcpyDeviceToDevice, st));
    HIPCHK(launch_axpby(x, -1.0f, sn, 1.0f, (long)n, st));
    HIPCHK(hipMemcpyAsync(yn, gt, (size_t)n * sizeof(float), hipMemcpyDeviceToDevice, st));
    HIPCHK(launch_axpby(g, -1.0f, yn, 1.0f, (long)n, st));
    double sy, ss, yy;
    if ((rc = dot(sn, yn, sy)) || (rc = dot(sn, sn, ss)) || (rc = dot(yn, yn, yy))) return rc;
    if (sy > 1e-12 * std::sqrt(ss) * std::sqrt(yy)) {
      free_slots.pop_back();
      pairs.push_back(slot);
      if ((int)pairs.size() > memory) {
        free_slots.push_back(pairs.front());
        pairs.erase(pairs.begin());
      }
    }
    HIPCHK(hipMemcpyAsync(x, xt, (size_t)n * sizeof(float), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(g, gt, (size_t)n * sizeof(float), hipMemcpyDeviceToDevice, st));
    f = ft;
    if ((rc = dot(g, g, gg))) return rc;
    f_hist[it + 1] = f;
  }
  for (int j = it + 1; j <= maxiter; ++j) f_hist[j] = f;
  *iters = it;
  HIPCHK(hipStreamSynchronize(st));
  return FWIME_OK;
}

}  // extern "C"

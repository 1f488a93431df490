// Host runtime and C ABI of libbgk (declared in include/bgk.h).
//
// The runtime validates arguments, carves the caller's workspace, builds the
// per-instance descriptor tables the kernels read (written into the
// workspace by a tiny kernel that takes them as kernel arguments, so no host
// buffer has to outlive the call), and enqueues the kernel sequence of each
// operation on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "bgk_internal.h"

namespace bgk {
// Tuned tile shape of one grid class: velocity grid, x cells and batch
// rounded up to powers of two, steps per pass.
using TileKey = std::tuple<int, int, int, int, int, int>;
struct Tuned {
  Tiles t;
  double ms;         // time of the autotuner's timed sequence
  std::string arch;  // device architecture it was measured on
};
}  // namespace bgk

// What the library keeps between calls (include/bgk.h, plans): captured
// graphs, tuned tiles, and the workspaces each stream's calls used since its
// last bgk_check.  Separate locks: a capture (graph lock held) chooses tiles.
struct bgk_plan {
  std::mutex graph_mu;
  std::map<std::string, hipGraphExec_t> graphs;
  hipStream_t cap_stream = nullptr;  // private stream the graphs are captured on
  std::mutex tile_mu;
  std::map<bgk::TileKey, bgk::Tuned> tiles;
  std::mutex used_mu;
  std::map<void*, std::set<void*>> used;  // stream -> workspaces
};

namespace bgk {

static bgk_plan g_default_plan;
static thread_local bgk_plan* t_plan = nullptr;
static bgk_plan* cur_plan() { return t_plan ? t_plan : &g_default_plan; }

// Calls made by the allocation-free entry point: no timing events, no
// workspace registry entries (both would allocate host memory).
static thread_local bool t_noalloc = false;

// ---------------------------------------------------------------- errors --
static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return BGK_E_HIP;
}

static int invalid(const char* why) {
  set_error(why);
  return BGK_E_INVALID;
}

// --------------------------------------------------------- host helpers --
size_t align_up(size_t n, size_t a) { return (n + a - 1) / a * a; }

double dx_of(const bgk_problem& p) { return (p.x_hi - p.x_lo) / p.nx; }
double dv_of(const bgk_problem& p, int a) { return (p.v_hi[a] - p.v_lo[a]) / p.nv[a]; }

int check_problem(const bgk_problem* p) {
  if (p == nullptr) return invalid("problem is NULL");
  if (p->nx < 2) return invalid("nx must be >= 2");
  for (int a = 0; a < 3; ++a) {
    if (p->nv[a] < 1 || p->nv[a] > kMaxNv) return invalid("nv out of range [1, 256]");
    if (!(p->v_hi[a] > p->v_lo[a]) || !std::isfinite(p->v_hi[a] - p->v_lo[a]))
      return invalid("empty velocity box");
  }
  if (!(p->x_hi > p->x_lo) || !std::isfinite(p->x_hi - p->x_lo))
    return invalid("empty x domain");
  if (p->bc != 0 && p->bc != 1) return invalid("bc must be 0 (Neumann) or 1 (periodic)");
  if (!(p->eps > 0.0)) return invalid("eps must be > 0");
  if (!(p->cfl > 0.0 && p->cfl <= 1.0)) return invalid("cfl must be in (0, 1]");
  if (!(p->sound_gamma > 0.0) || !std::isfinite(p->sound_gamma))
    return invalid("sound_gamma must be > 0");
  const long long nv3 = (long long)p->nv[0] * p->nv[1] * p->nv[2];
  if (nv3 * p->nx > (1LL << 40)) return invalid("grid too large");
  return BGK_OK;
}

// Section 2.2 local step rule at velocity cell centres; with an exterior
// force (emax > 0) the x and v_x fluxes share the explicit step:
// dt (max|v_x| / dx + emax / dv_x) <= cfl.
int n_steps_for(const bgk_problem& p, double t_span, int32_t* n, double* dt, double emax) {
  if (!(t_span > 0.0) || !std::isfinite(t_span)) return invalid("t_span must be > 0");
  if (!(emax >= 0.0) || !std::isfinite(emax)) return invalid("e_max must be finite and >= 0");
  double vmax = 0.0;
  const double dv = dv_of(p, 0);
  for (int j = 0; j < p.nv[0]; ++j)
    vmax = std::max(vmax, std::fabs(p.v_lo[0] + (j + 0.5) * dv));
  const double dt_stab = emax > 0.0 ? p.cfl / (vmax / dx_of(p) + emax / dv)
                                    : p.cfl * dx_of(p) / vmax;
  const double r = t_span / dt_stab;
  if (!(r < 2.0e9)) return invalid("too many fine steps for t_span");
  int32_t k = (int32_t)std::ceil(r - 1e-9);
  if (k < 1) k = 1;
  *n = k;
  *dt = t_span / k;
  return BGK_OK;
}

// ----------------------------------------------------------------- tiles --
static std::mutex g_mu;
static Tiles g_override = {0, 0, -1};

static int pow2_ceil(long long n) {
  int v = 1;
  while (v < n && v < (1 << 30)) v <<= 1;
  return v;
}
static TileKey tile_key(const bgk_problem& p, int batch, int fuse) {
  return TileKey{p.nv[0], p.nv[1], p.nv[2], pow2_ceil(p.nx), pow2_ceil(batch), fuse};
}

static long long nv3_of(const bgk_problem& p) {
  return (long long)p.nv[0] * p.nv[1] * p.nv[2];
}

// Wave tiles per x cell: runs of 64 * elems flat velocities, or with the
// v_x-column mapping blocks of 64 (v_y, v_z) points by elems v_x points.
static long long ntiles_of(const bgk_problem& p, Tiles t) {
  if (t.vcol) {
    const long long nyz = (long long)p.nv[1] * p.nv[2];
    const long long span = (long long)kWave * (t.pair ? 2 : 1);
    return ((nyz + span - 1) / span) * ((p.nv[0] + t.elems - 1) / t.elems);
  }
  return (nv3_of(p) + kWave * t.elems - 1) / (kWave * t.elems);
}

static int part_tiles_of(const bgk_problem& p);

static long long blocks_for_tiles(const bgk_problem& p, int batch, Tiles t) {
  const long long ntiles = ntiles_of(p, t);
  const long long ntg = (ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
  return (long long)batch * ntg * ((p.nx + t.chunk - 1) / t.chunk);
}

static int g_fuse = 3;  // IMEX steps per pass (1, 2 or 3) where possible

// LDS and chunk limits of the three-step kernel.  With 4 velocities per lane
// (233 VGPRs) a CU holds one 8-wave block, which may then take all 160 KB of
// gfx950's LDS; with 2 (123 VGPRs) two blocks share it.
static size_t lds3_cap(int elems) { return elems == 4 ? (size_t)kLdsBytes : 65536; }
static int lds3_max_chunk(int elems) { return elems == 4 ? 64 : 24; }

// Longest factor row a three-step block stages: Ex of the v_x planes its
// eight tiles of 64 * elems velocities span, then Ey and Ez.
static int lds3_row(int nvx, int nvy, int nvz, int elems) {
  const long long nyz = (long long)nvy * nvz, nv3 = nyz * nvx;
  const long long span = (long long)kWavesPerBlock * kWave * elems;
  long long nj = 1;
  for (long long v0 = 0; v0 < nv3; v0 += span)
    nj = std::max(nj, (std::min(v0 + span, nv3) - 1) / nyz - v0 / nyz + 1);
  return (int)nj + nvy + nvz;
}

// The v_x-column mapping fits a grid whose tiles fit the partial-sum capacity.
static bool vcol_fits(const bgk_problem& p, Tiles t) {
  return ntiles_of(p, t) <= part_tiles_of(p);
}

Tiles choose_tiles(const bgk_problem& p, int batch, bool generic, bool force, bool limited) {
  std::lock_guard<std::mutex> lk(g_mu);
  const int pair = (p.nv[2] % 2 == 0 && !generic) ? 1 : 0;
  // measured best on the 512 x 32^3 x 64-slice batch with 8-wave blocks:
  // fused passes 8 velocities per lane over 8-cell chunks, single steps 8
  // over short chunks; fused passes on unpaired lanes (odd nv_z) take 4
  // (8 spill in their two-step march)
  Tiles t = g_fuse >= 2 ? (pair ? Tiles{8, 8, 1} : Tiles{4, 8, 0}) : Tiles{8, 4, pair};
  bool tuned = false;
  if (!generic && !force && !limited) {
    bgk_plan* pl = cur_plan();
    std::lock_guard<std::mutex> lt(pl->tile_mu);
    auto it = pl->tiles.find(tile_key(p, batch, g_fuse));
    if (it != pl->tiles.end() && (it->second.t.pair == 0 || pair)) {
      t = it->second.t;
      tuned = true;
    }
  }
  const long long cells = (long long)batch * p.nx * nv3_of(p);
  // The exterior-force step runs on v_x columns (the v_x neighbours of a
  // lane's elements in its own registers) when a v_x plane fills a wave, or
  // when asked to (pair = 2: one (v_y, v_z) point per lane, 3: two), else on
  // the flat mapping below.  Built-in: two points per lane (16-byte
  // accesses) when nvy nvz is even.
  const long long nyz = (long long)p.nv[1] * p.nv[2];
  const int ov = g_override.pair;
  if (force && (ov >= 2 || (ov != 0 && nyz >= kWave))) {
    // measured on the 100 x 256x16x16 two-beam grid: 4 v_x points by 2
    // (v_y, v_z) points per lane over 8-cell chunks for 1 and 20 slices;
    // 16-cell chunks with the second-order x flux where the grid keeps
    // enough blocks
    Tiles c = {4, limited ? 16 : 8, (nyz % 2 == 0 && ov != 2) ? 1 : 0, 1};
    while (c.chunk > 1 && blocks_for_tiles(p, batch, c) < (limited ? 192 : 128)) c.chunk /= 2;
    if (g_override.elems) c.elems = g_override.elems;
    if (g_override.chunk) c.chunk = g_override.chunk;
    if (c.elems == 8) c.pair = 0;  // paired columns take 2 or 4 v_x points
    if (vcol_fits(p, c)) return c;
  }
  if (generic) {
    // the exterior-force step on the flat mapping: 2 velocities per lane
    // keep the extra registers unspilled.  The second-order step without
    // force is VALU-bound: 4 velocities per lane (170 VGPRs, no spills)
    // halve the per-update share of the wave's moment reduction, and
    // 64-cell chunks amortise its 5-row window (measured on the 512 x 32^3
    // x 64-slice batch: 3.38 ms per step against 3.80 with 2 per lane over
    // 16 cells; 2 per lane where a tile of 256 velocities would be short)
    t = (limited && !force && nv3_of(p) >= 4 * kWave * 4) ? Tiles{4, 64, 0}
                                                          : Tiles{2, limited ? 16 : 8, 0};
    while (t.chunk > 1 && blocks_for_tiles(p, batch, t) < 512) t.chunk /= 2;
  } else if (tuned) {
    // a shape bgk_autotune measured for this grid class
  } else if (pair && g_fuse >= 2 && cells < (1LL << 24)) {
    // latency-bound sizes (f fits the last-level cache): short velocity
    // tiles, x chunks as long as the grid keeps about two blocks per CU
    t = Tiles{2, 16, 1};
    while (t.chunk > 1 && blocks_for_tiles(p, batch, t) < 512) t.chunk /= 2;
  } else {
    // enough work items to fill 256 CUs several times over.  Three-step
    // passes (grids whose v_x planes are whole tiles) hold three levels of
    // rows: 4 velocities per lane (non-temporal row loads) where a v_x plane
    // is whole tiles of 256 velocities, else 2; long chunks amortise the
    // deeper halo (measured with 4 per lane: on the 512 x 32^3 x 64-slice
    // batch 3.51, 3.37, 3.30, 3.24, 3.21 ms per pass over 12, 16, 24, 32, 48
    // cells; on 4 slices of 2048 x 48^3 3.17, 3.01, 2.97 ms over 14, 24, 32;
    // 2 per lane 3.47 ms over 24)
    if (pair && g_fuse == 4 && p.nx >= 4 && nyz % (kWave * 2) == 0) {
      // four levels of rows: one velocity pair per lane (two spill), the
      // longest chunk whose four levels of factor rows fit the LDS
      const long long rl = lds3_row(p.nv[0], p.nv[1], p.nv[2], 2);
      int ch = kMaxChunk;
      while (ch > 1 && (4LL * ch + 20) * rl * (long long)sizeof(double) > kLdsBytes) --ch;
      t = Tiles{2, ch, 1};
    } else if (pair && g_fuse >= 3 && p.nx >= 3 && nyz % (kWave * 2) == 0) {
      // the longest chunk whose three levels of factor rows fit the LDS
      const int e = nyz % (kWave * 4) == 0 ? 4 : 2;
      const long long rl = lds3_row(p.nv[0], p.nv[1], p.nv[2], e);
      int ch = lds3_max_chunk(e);
      while (ch > 1 && (size_t)(3LL * ch + 12) * rl * sizeof(double) > lds3_cap(e)) --ch;
      t = Tiles{e, ch, 1};
    }
    while (t.chunk > 1 && blocks_for_tiles(p, batch, t) < 4096) t.chunk /= 2;
    // fewer velocities per lane (more tiles) where blocks are still short
    if (blocks_for_tiles(p, batch, t) < 2048 && t.elems > 4) t.elems = 4;
    if (blocks_for_tiles(p, batch, t) < 1024 && t.elems > 2) t.elems = 2;
  }
  if (g_override.elems) t.elems = g_override.elems;
  if (g_override.chunk) t.chunk = g_override.chunk;
  if ((g_override.pair == 0 || g_override.pair == 1) && p.nv[2] % 2 == 0 && !generic)
    t.pair = g_override.pair;
  if (limited && t.elems > 4) t.elems = 4;  // second-order flat kernels take 2 or 4
  // keep the factor rows a step kernel stages within gfx950's 160 KB of LDS
  // (x-flat mappings: chunk + 2 rows per level, + 4 with the limiter, two
  // levels of 2 chunk + 6 rows in the fused two-step pass)
  if (!t.vcol) {
    const long long nvs = (long long)p.nv[0] + p.nv[1] + p.nv[2];
    auto rows = [&](int c) -> long long {
      if (limited) return c + 4;
      return g_fuse >= 2 ? 2LL * c + 6 : c + 2;
    };
    while (t.chunk > 1 && rows(t.chunk) * nvs * (long long)sizeof(double) > kLdsBytes)
      t.chunk /= 2;
  }
  return t;
}

// The paired kernel needs 16-byte aligned rows of f.
// Columns without pairs have more tiles: back to the flat mapping where they
// exceed the partial-sum capacity.
static Tiles aligned_tiles(Tiles t, const bgk_problem& p,
                           std::initializer_list<const void*> ptrs) {
  for (const void* q : ptrs)
    if (q && reinterpret_cast<uintptr_t>(q) % 16 != 0) t.pair = 0;
  if (t.vcol && !vcol_fits(p, t)) t = Tiles{2, t.chunk, 0, 0};
  return t;
}

// ------------------------------------------------------------- workspace --
// Every workspace starts with WsHeader, then a descriptor table, then the
// regions of the operation.
struct Carve {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  }
};

constexpr int kMaxInst = 4096;

struct FineRegions {  // fine solve of B members of one grid
  size_t buf0, buf1, part, fac, vg, vout, fac2, aux, fac3, aux2, fac4, aux3;
};
constexpr size_t kNone = ~(size_t)0;  // region not allocated

// Capacity per x cell, in 5-double units: one record (5 or 15 doubles) per
// wave tile of at least 64 * kMinElems velocities.
static int part_tiles_of(const bgk_problem& p) {
  return 3 * (int)((nv3_of(p) + kWave * kMinElems - 1) / (kWave * kMinElems));
}

// nbufs: phase-space buffers of B members to carve (0, 1 or 2).
static FineRegions carve_fine(Carve& c, const bgk_problem& p, int B, int nbufs) {
  FineRegions r;
  const size_t f = (size_t)B * p.nx * nv3_of(p) * sizeof(double);
  r.buf0 = nbufs >= 1 ? c.take(f) : kNone;
  r.buf1 = nbufs >= 2 ? c.take(f) : kNone;
  r.part = c.take((size_t)B * p.nx * part_tiles_of(p) * 5 * sizeof(double));
  r.fac = c.take((size_t)B * p.nx * (p.nv[0] + p.nv[1] + p.nv[2]) * sizeof(double));
  r.vg = c.take((size_t)B * p.nx * 5 * sizeof(double));
  r.vout = c.take((size_t)B * p.nx * 5 * sizeof(double));
  r.fac2 = c.take((size_t)B * p.nx * (p.nv[0] + p.nv[1] + p.nv[2]) * sizeof(double));
  r.aux = c.take((size_t)B * p.nx * kAux * sizeof(double));
  r.fac3 = c.take((size_t)B * p.nx * (p.nv[0] + p.nv[1] + p.nv[2]) * sizeof(double));
  r.aux2 = c.take((size_t)B * p.nx * kAux2 * sizeof(double));
  r.fac4 = c.take((size_t)B * p.nx * (p.nv[0] + p.nv[1] + p.nv[2]) * sizeof(double));
  r.aux3 = c.take((size_t)B * p.nx * kAux3 * sizeof(double));
  return r;
}

struct Layout {
  size_t header = 0, insts = 0;
  FineRegions fine{};
  size_t coarse = 0;                 // Euler scratch
  size_t U0 = 0, U1 = 0, Gc = 0, VF = 0, errs = 0;
  size_t states = 0, fbA = 0, fbB = 0, part6 = 0, coef = 0, dle = 0;
  size_t total = 0;
};

static Layout layout_of(const bgk_problem& p, int op, int batch) {
  Carve c;
  Layout L;
  L.header = c.take(sizeof(WsHeader));
  // descriptor table: 4 entries; the adjoint keeps one per step of a
  // checkpoint segment for the recomputation and one for the backward step
  L.insts = c.take(sizeof(Inst) * (op == BGK_OP_ADJOINT ? std::max(4, 2 * batch) : 4));
  const size_t f1 = (size_t)p.nx * nv3_of(p) * sizeof(double);
  const size_t sl = (size_t)p.nx * 5 * sizeof(double);
  switch (op) {
    case BGK_OP_FINE_STEP:
      L.fine = carve_fine(c, p, 1, 1);
      break;
    case BGK_OP_MOMENTS:
    case BGK_OP_LIFT:
      L.fine = carve_fine(c, p, 1, 0);
      break;
    case BGK_OP_COARSE:
      L.coarse = c.take((size_t)batch * kCoarseScratch * p.nx * sizeof(double));
      break;
    case BGK_OP_PROPAGATE:
      L.fine = carve_fine(c, p, batch, 2);
      break;
    case BGK_OP_PARAREAL:
      L.fine = carve_fine(c, p, batch, 2);
      L.coarse = c.take((size_t)kCoarseScratch * p.nx * sizeof(double));
      L.errs = c.take((size_t)(batch + 1) * sizeof(double));
      L.U0 = c.take(sl * (batch + 1));
      L.U1 = c.take(sl * (batch + 1));
      L.Gc = c.take(sl * (batch + 1));
      L.VF = c.take(sl * (batch + 1));
      break;
    case BGK_OP_ADJOINT: {
      L.fine = carve_fine(c, p, 1, 1);
      L.states = c.take(f1 * batch);
      L.fbA = c.take(f1);
      L.fbB = c.take(f1);
      const size_t nt = (nv3_of(p) + kWave * kAdjElems - 1) / (kWave * kAdjElems);
      L.part6 = c.take((size_t)p.nx * nt * 6 * sizeof(double));
      L.coef = c.take(sl);
      L.dle = c.take((size_t)p.nx * sizeof(double));
      break;
    }
    default:
      break;
  }
  L.total = c.off;
  return L;
}

template <class T>
static T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

static int check_ws(void* ws, size_t ws_bytes, size_t need) {
  if (ws == nullptr) {
    set_error("workspace is NULL");
    return BGK_E_WORKSPACE;
  }
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) {
    set_error("workspace must be 256-byte aligned");
    return BGK_E_WORKSPACE;
  }
  if (ws_bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return BGK_E_WORKSPACE;
  }
  return BGK_OK;
}

// Records that a call enqueued on `stream` uses workspace `ws`, whose sticky
// status bgk_check(stream) reads.
static void note_ws(void* ws, void* stream) {
  if (t_noalloc) return;
  bgk_plan* pl = cur_plan();
  std::lock_guard<std::mutex> lk(pl->used_mu);
  pl->used[stream].insert(ws);
}

// -------------------------------------------------- descriptor uploads --
constexpr int kPack = 12;  // descriptors per upload launch (kernel-argument bytes)
struct InstPack {
  Inst v[kPack];
  int n;
};

__global__ void k_put_insts(Inst* dst, InstPack p) {
  constexpr int W = sizeof(Inst) / sizeof(unsigned long long);
  static_assert(sizeof(Inst) % sizeof(unsigned long long) == 0, "Inst padding");
  const unsigned long long* s = reinterpret_cast<const unsigned long long*>(p.v);
  unsigned long long* d = reinterpret_cast<unsigned long long*>(dst);
  for (int k = threadIdx.x; k < p.n * W; k += blockDim.x) d[k] = s[k];
}

static int put_insts(Inst* d_dst, const Inst* h, int n, hipStream_t s) {
  for (int b = 0; b < n; b += kPack) {
    InstPack pk;
    std::memset(&pk, 0, sizeof(pk));
    pk.n = std::min(kPack, n - b);
    for (int k = 0; k < pk.n; ++k) pk.v[k] = h[b + k];
    hipLaunchKernelGGL(k_put_insts, dim3(1), dim3(256), 0, s, d_dst + b, pk);
    BGK_HIP(hipGetLastError());
  }
  return BGK_OK;
}

__global__ void k_fill_int(int* p, int v) {
  if (threadIdx.x == 0) *p = v;
}

__global__ void k_prim_to_cons(const double* __restrict__ W, double* V, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* w = W + 5 * (long long)i;
  double* v = V + 5 * (long long)i;
  const double rho = w[0];
  const double usq = w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
  v[0] = rho;
  v[1] = rho * w[1];
  v[2] = rho * w[2];
  v[3] = rho * w[3];
  v[4] = 0.5 * rho * usq + 1.5 * rho * w[4];
}

int launch_prim_to_cons(const double* W, double* V, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_prim_to_cons, dim3((n + 255) / 256), dim3(256), 0, s, W, V, n);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

// Two (or three) IMEX steps per pass over f, paired or unpaired lanes;
// switchable.
static bool fused_for(const Tiles& t, int n_steps) {
  (void)t;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_fuse >= 2 && n_steps >= 2;
}

// Descriptor of B members of one grid advanced with step dt.  ns: sums per
// moment partial (15 when the steps run fused two per pass).
static Inst make_inst(const bgk_problem& p, int B, double dt, Tiles t, int ns = 5) {
  Inst I;
  std::memset(&I, 0, sizeof(I));
  I.nx = p.nx;
  I.nvx = p.nv[0];
  I.nvy = p.nv[1];
  I.nvz = p.nv[2];
  I.nv3 = (int)nv3_of(p);
  I.nvs = p.nv[0] + p.nv[1] + p.nv[2];
  I.bc = p.bc;
  I.nbatch = B;
  I.ntiles = (int)ntiles_of(p, t);
  I.ntg = (I.ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
  I.nsum = ns;
  // fused passes on grids whose tiles each lie in one v_x plane write
  // compact 4-value partial records
  if (ns == 15 && t.pair && ((long long)p.nv[1] * p.nv[2]) % (kWave * t.elems) == 0)
    I.crec = kWave * t.elems;
  I.order = 1;
  I.nvz_live = p.nv[2];
  I.nparts = I.ntiles;  // one partial record per wave tile
  I.nchunks = (p.nx + t.chunk - 1) / t.chunk;
  I.items = (long long)B * I.ntg * I.nchunks;
  I.part_tiles = part_tiles_of(p);
  for (int a = 0; a < 3; ++a) {
    I.dv[a] = dv_of(p, a);
    I.vlo[a] = p.v_lo[a];
  }
  I.dv3 = I.dv[0] * I.dv[1] * I.dv[2];
  I.r = dt / dx_of(p);
  const double lam = dt / p.eps;
  if (std::isinf(lam)) {
    I.a = 0.0;
    I.al = 1.0;
  } else {
    I.a = 1.0 / (1.0 + lam);
    I.al = lam / (1.0 + lam);
  }
  return I;
}

static void attach_fine(Inst& I, void* ws, const FineRegions& r, double* buf1) {
  I.buf[0] = r.buf0 == kNone ? nullptr : at<double>(ws, r.buf0);
  I.buf[1] = buf1 ? buf1 : (r.buf1 == kNone ? nullptr : at<double>(ws, r.buf1));
  I.part = at<double>(ws, r.part);
  I.fac = at<double>(ws, r.fac);
  I.vg = at<double>(ws, r.vg);
  I.vout = at<double>(ws, r.vout);
  I.fac2 = at<double>(ws, r.fac2);
  I.aux = at<double>(ws, r.aux);
  I.fac3 = at<double>(ws, r.fac3);
  I.aux2 = at<double>(ws, r.aux2);
  I.fac4 = at<double>(ws, r.fac4);
  I.aux3 = at<double>(ws, r.aux3);
}

static int lds_doubles(const Inst& I, Tiles t) {
  return (t.chunk + (I.order == 2 ? 4 : 2)) * I.nvs;
}
static int lds_doubles2(const Inst& I, Tiles t) { return (2 * t.chunk + 6) * I.nvs; }
static int lds_doubles3(const Inst& I, Tiles t) {
  return (3 * t.chunk + 12) * lds3_row(I.nvx, I.nvy, I.nvz, t.elems);
}
static int lds_doubles4(const Inst& I, Tiles t) {
  return (4 * t.chunk + 20) * lds3_row(I.nvx, I.nvy, I.nvz, t.elems);
}

static int fuse_mode() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_fuse;
}

// Three IMEX steps per pass: on when asked for, on grids with compact records
// (every tile in one v_x plane), nx >= 3 (ghost rows three deep), 2 or 4
// velocities per lane (three levels of rows in registers) and factor rows of
// the three levels within the LDS cap (lds3_cap).
static bool triple_for(const Inst& h, Tiles t) {
  int fuse;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    fuse = g_fuse;
  }
  return fuse >= 3 && h.crec != 0 && h.nsum == 15 && h.nx >= 3 && t.pair && t.elems <= 4 &&
         (size_t)lds_doubles3(h, t) * sizeof(double) <= lds3_cap(t.elems);
}

// Four IMEX steps per pass: on when asked for, on grids with compact records,
// nx >= 4 (ghost rows four deep), one velocity pair per lane (four levels of
// rows in registers) and factor rows of the four levels within the LDS.
static bool quad_for(const Inst& h, Tiles t) {
  int fuse;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    fuse = g_fuse;
  }
  return fuse == 4 && h.crec != 0 && h.nsum == 15 && h.nx >= 4 && t.pair && t.elems == 2 &&
         (long long)lds_doubles4(h, t) * (long long)sizeof(double) <= kLdsBytes;
}

// Runs `n` relax-then-transport steps on the (uploaded) descriptor d_I.
// first_mode: kCopy (read fin) or kLift (factors of the lifted Maxwellian
// already in fac, and in aux when h.nsum == 15).  With h.nsum == 15 the steps
// run two per pass where possible.  The last reduction writes the relaxation
// factors of g^n, or with project_last the projected relaxed moments into
// vout.  *last_sel receives the buffer index holding g^n.
static int run_steps(const Inst* d_I, const Inst& h, int n, int first_mode,
                     bool project_last, Tiles t, int* d_status, hipStream_t s,
                     int* last_sel) {
  const long long cells = (long long)h.nbatch * h.nx;
  const double upd = (double)cells * h.nv3;
  int phase = 1;  // a pass reads buf[phase] and writes buf[phase ^ 1]
  int rc;
  auto single = [&](int mode) -> int {
    prof_before(s);
    int r = launch_step(d_I, 1, h.items, mode, phase, t, lds_doubles(h, t), d_status, s,
                        h.nsum, h.efield != nullptr, h.order == 2 ? 2 : 1,
                        h.order == 2 && h.crec != 0);
    prof_after(s, upd, mode == kLift ? 8.0 : 16.0, BGK_PROF_ONE_STEP);
    phase ^= 1;
    return r;
  };
  auto reduce = [&](int mode) { return launch_reduce(d_I, 1, cells, mode, 0, d_status, s); };
  if (h.nsum != 15) {
    for (int k = 1; k <= n; ++k) {
      if ((rc = single(k == 1 ? first_mode : kRelax))) return rc;
      if ((rc = reduce((project_last && k == n) ? kRedProject : kRedRelaxFactors))) return rc;
    }
    *last_sel = phase;
    return BGK_OK;
  }
  int done = 0;
  auto pair_pass = [&](int mode) -> int {
    prof_before(s);
    const bool uni = (h.nvy * h.nvz) % (kWave * t.elems) == 0;
    int r = launch_step2x2(d_I, 1, h.items, mode, phase, t, lds_doubles2(h, t), uni, s);
    prof_after(s, 2.0 * upd, mode == kLift ? 4.0 : 8.0,
               mode == kLift ? BGK_PROF_TWO_STEP_LIFT : BGK_PROF_TWO_STEP);
    phase ^= 1;
    done += 2;
    return r;
  };
  if (quad_for(h, t)) {
    auto quad_pass = [&](int mode) -> int {
      prof_before(s);
      int r = launch_step4x(d_I, 1, h.items, mode, phase, t, lds_doubles4(h, t), s);
      prof_after(s, 4.0 * upd, mode == kLift ? 2.0 : 4.0,
                 mode == kLift ? BGK_PROF_FOUR_STEP_LIFT : BGK_PROF_FOUR_STEP);
      phase ^= 1;
      done += 4;
      return r;
    };
    auto quad_reductions = [&]() -> int {
      int r;
      if ((r = reduce(kRedW1x4))) return r;
      if ((r = reduce(kRedW2x4))) return r;
      if ((r = reduce(kRedW3x4))) return r;
      return reduce(kRedW4x4);
    };
    // the first pass: four steps from the lift (its weighted sums to the
    // third power come with the lift factors), or one step from the copy
    if (first_mode == kLift && n >= 4) {
      if ((rc = reduce(kRedW2x4))) return rc;
      if ((rc = reduce(kRedW3x4))) return rc;
      if ((rc = reduce(kRedW4x4))) return rc;
      if ((rc = quad_pass(kLift))) return rc;
    } else {
      if ((rc = single(first_mode))) return rc;
      done = 1;
    }
    // When only the projected moments leave the call, the n - done mod 4 steps
    // left after the last four-step pass close on the moments (weighted sums
    // of the last stored field).
    const int virt = (project_last && first_mode == kLift && n >= 4) ? (n - done) % 4 : 0;
    while (n - done - virt >= 4) {
      if ((rc = quad_reductions())) return rc;
      if ((rc = quad_pass(kRelax))) return rc;
    }
    if (virt == 1) {
      if ((rc = reduce(kRedW1))) return rc;
      if ((rc = reduce(kRedW2Project))) return rc;
      *last_sel = phase;
      return BGK_OK;
    }
    if (virt == 2) {
      if ((rc = reduce(kRedW1x3))) return rc;
      if ((rc = reduce(kRedW2x3))) return rc;
      if ((rc = reduce(kRedW3x3Project))) return rc;
      *last_sel = phase;
      return BGK_OK;
    }
    if (virt == 3) {
      if ((rc = reduce(kRedW1x4))) return rc;
      if ((rc = reduce(kRedW2x4))) return rc;
      if ((rc = reduce(kRedW3x4))) return rc;
      if ((rc = reduce(kRedW4x4Project))) return rc;
      *last_sel = phase;
      return BGK_OK;
    }
    // fewer than four steps left: two-step passes, then one step
    while (n - done >= 2) {
      if ((rc = reduce(kRedW1))) return rc;
      if ((rc = reduce(kRedW2))) return rc;
      if ((rc = pair_pass(kRelax))) return rc;
    }
    if (n - done == 1) {
      if ((rc = reduce(kRedRelaxFactors))) return rc;
      if ((rc = single(kRelax))) return rc;
      done += 1;
    }
    if ((rc = reduce(project_last ? kRedProject : kRedRelaxFactors))) return rc;
    *last_sel = phase;
    return BGK_OK;
  }
  if (triple_for(h, t)) {
    auto triple_pass = [&](int mode) -> int {
      prof_before(s);
      int r = launch_step3x(d_I, 1, h.items, mode, phase, t, lds_doubles3(h, t), s);
      prof_after(s, 3.0 * upd, mode == kLift ? 8.0 / 3.0 : 16.0 / 3.0,
                 mode == kLift ? BGK_PROF_THREE_STEP_LIFT : BGK_PROF_THREE_STEP);
      phase ^= 1;
      done += 3;
      return r;
    };
    // When only the projected moments leave the call, the last one or two
    // steps are not written out: their moments follow from the weighted sums
    // of the last stored field (linearity of the transport; the reductions
    // before a three-step pass give the moments of the next two fields).
    // Then the first pass takes two steps from the lift (cheaper than three),
    // three-step passes follow, and virt = (n - 2) mod 3 steps close on the
    // moments.
    // For n = 2 mod 3 (n >= 5) the first pass takes three steps from the lift
    // and two steps close on the moments: one relax pass fewer than a
    // two-step first pass followed by triples.
    const bool proj_lift = project_last && first_mode == kLift && n >= 4;
    const bool lift3 = proj_lift && n >= 5 && n % 3 == 2;
    const int virt = lift3 ? 2 : (proj_lift ? (n - 2) % 3 : 0);
    // the first pass starts from the lift (write-only) or the copy: n mod 3
    // decides whether it takes three, two or one step
    if (lift3) {
      if ((rc = reduce(kRedW2x3))) return rc;
      if ((rc = reduce(kRedW3x3))) return rc;
      if ((rc = triple_pass(kLift))) return rc;
    } else if (virt) {
      if ((rc = reduce(kRedW2))) return rc;
      if ((rc = pair_pass(kLift))) return rc;
    } else if (first_mode == kLift && n >= 3 && n % 3 == 0) {
      if ((rc = reduce(kRedW2x3))) return rc;
      if ((rc = reduce(kRedW3x3))) return rc;
      if ((rc = triple_pass(kLift))) return rc;
    } else if (first_mode == kLift && n >= 2 && n % 3 == 2) {
      if ((rc = reduce(kRedW2))) return rc;
      if ((rc = pair_pass(kLift))) return rc;
    } else {
      if ((rc = single(first_mode))) return rc;
      done = 1;
    }
    if (!virt && (n - done) % 3 == 2) {
      if ((rc = reduce(kRedW1))) return rc;
      if ((rc = reduce(kRedW2))) return rc;
      if ((rc = pair_pass(kRelax))) return rc;
    }
    while (n - done - virt >= 3) {
      if ((rc = reduce(kRedW1x3))) return rc;
      if ((rc = reduce(kRedW2x3))) return rc;
      if ((rc = reduce(kRedW3x3))) return rc;
      if ((rc = triple_pass(kRelax))) return rc;
    }
    if (virt == 1) {
      if ((rc = reduce(kRedW1))) return rc;
      if ((rc = reduce(kRedW2Project))) return rc;
      *last_sel = phase;  // the last field written (the call returns moments only)
      return BGK_OK;
    }
    if (virt == 2) {
      if ((rc = reduce(kRedW1x3))) return rc;
      if ((rc = reduce(kRedW2x3))) return rc;
      if ((rc = reduce(kRedW3x3Project))) return rc;
      *last_sel = phase;
      return BGK_OK;
    }
    if (n - done == 1) {
      if ((rc = reduce(kRedRelaxFactors))) return rc;
      if ((rc = single(kRelax))) return rc;
      done += 1;
    }
    if ((rc = reduce(project_last ? kRedProject : kRedRelaxFactors))) return rc;
    *last_sel = phase;
    return BGK_OK;
  }
  // An odd step count takes its single step first, from the lift: that pass
  // only writes f (8 bytes per update instead of the 16 of a later single).
  // When only the projected moments leave the call, the odd step is the last
  // one instead, not written out (its moments from the weighted sums).
  const bool last_on_moments = project_last && first_mode == kLift && n >= 3 && n % 2 == 1;
  if (first_mode == kLift && n >= 2 && (n % 2 == 0 || last_on_moments)) {
    if ((rc = reduce(kRedW2))) return rc;
    if ((rc = pair_pass(kLift))) return rc;
  } else {
    if ((rc = single(first_mode))) return rc;
    done = 1;
  }
  while (n - done >= 2) {
    if ((rc = reduce(kRedW1))) return rc;
    if ((rc = reduce(kRedW2))) return rc;
    if ((rc = pair_pass(kRelax))) return rc;
  }
  if (n - done == 1 && last_on_moments) {
    if ((rc = reduce(kRedW1))) return rc;
    if ((rc = reduce(kRedW2Project))) return rc;
    *last_sel = phase;  // the last field written (the call returns moments only)
    return BGK_OK;
  }
  if (n - done == 1) {
    if ((rc = reduce(kRedRelaxFactors))) return rc;
    if ((rc = single(kRelax))) return rc;
    done += 1;
  }
  if ((rc = reduce(project_last ? kRedProject : kRedRelaxFactors))) return rc;
  *last_sel = phase;
  return BGK_OK;
}

// Lift (factors from the conserved vin of every member) then n steps.
static int lift_and_run(const Inst* d_I, const Inst& h, int n, bool project_last, Tiles t,
                        int* d_status, hipStream_t s, int* last_sel) {
  // a three-step first pass needs the nu+^2, nu-^2 weighted sums of the lift
  int rc = launch_lift_factors(d_I, 1, (long long)h.nbatch * h.nx, nullptr, d_status, s,
                               h.nsum == 15 ? (quad_for(h, t) ? 3 : (triple_for(h, t) ? 2 : 1))
                                            : 0);
  if (rc) return rc;
  return run_steps(d_I, h, n, kLift, project_last, t, d_status, s, last_sel);
}

// Lifting of order lift_order (0: Maxwellian, fused into the first pass;
// 1: first Chapman-Enskog correction, written into buf[1], which the first
// step then reads in copy mode; prepare_lift must have set h.fin before the
// descriptor was uploaded) followed by n steps and the projection.
static void prepare_lift(Inst& h, int lift_order) {
  if (lift_order == 1) h.fin = h.buf[1];
}

static int run_lifted(const Inst* d_I, const Inst& h, int n, int lift_order,
                      const bgk_problem& p, Tiles t, int* d_status, hipStream_t s,
                      int* last_sel) {
  if (lift_order == 0) return lift_and_run(d_I, h, n, true, t, d_status, s, last_sel);
  int rc = launch_lift_ce(d_I, h, dx_of(p), p.eps, d_status, s);
  if (rc) return rc;
  return run_steps(d_I, h, n, kCopy, true, t, d_status, s, last_sel);
}

static int check_lift_order(const bgk_problem& p, int lift_order) {
  if (lift_order != 0 && lift_order != 1) return invalid("lift_order must be 0 or 1");
  if (lift_order == 1 && !std::isfinite(p.eps))
    return invalid("the order-one lifting needs a finite eps");
  return BGK_OK;
}

static long long relax_out_blocks(const Inst& h) {
  const long long slabs = (h.nv3 + 4 * kBlock - 1) / (4 * kBlock);
  return (long long)h.nbatch * h.nx * slabs;
}

// ------------------------------------------------------------- profiling --
struct ProfRec {
  hipEvent_t a, b;
  double cells, bytes;
  int kind;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<ProfRec> g_prof;
static std::vector<hipEvent_t> g_prof_pool;
static hipEvent_t g_prof_pending = nullptr;

static hipEvent_t prof_event() {
  if (!g_prof_pool.empty()) {
    hipEvent_t e = g_prof_pool.back();
    g_prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void noalloc_mode(bool on) { t_noalloc = on; }

void prof_before(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof_on || t_noalloc) return;
  g_prof_pending = prof_event();
  if (g_prof_pending) (void)hipEventRecord(g_prof_pending, s);
}

void prof_after(hipStream_t s, double cells, double bytes_per_cell, int kind) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof_on || t_noalloc || !g_prof_pending) return;
  hipEvent_t e = prof_event();
  if (!e) return;
  (void)hipEventRecord(e, s);
  g_prof.push_back({g_prof_pending, e, cells, cells * bytes_per_cell, kind});
  g_prof_pending = nullptr;
}

// ----------------------------------------------------------- hipGraphs --
// Launch-bound sequences (one parareal iteration, the serial chain of slice
// solves) are captured once per (workspace, shape, iteration) on a private
// capture stream and replayed on the caller's stream.  Everything a captured
// sequence touches lives in the workspace, so the key names the workspace.
static std::mutex g_graph_mu;  // guards g_graphs_on
static bool g_graphs_on = true;
constexpr size_t kMaxGraphs = 512;  // per plan; a full plan is emptied

// The fields of a problem as key bytes (not the struct's own bytes: the
// padding after bc is whatever the caller left there).
static void add_problem_key(std::string& k, const bgk_problem& p) {
  const double d[13] = {p.x_lo, p.x_hi, p.v_lo[0], p.v_lo[1], p.v_lo[2], p.v_hi[0],
                        p.v_hi[1], p.v_hi[2], p.eps, p.cfl, p.sound_gamma,
                        (double)p.nx, (double)p.bc};
  const int32_t v[3] = {p.nv[0], p.nv[1], p.nv[2]};
  k.append(reinterpret_cast<const char*>(d), sizeof(d));
  k.append(reinterpret_cast<const char*>(v), sizeof(v));
}

// Key of a captured sequence: its tag, the workspace, the problem, the
// launch parameters xs and the raw bytes of the device pointers it reads
// or writes outside the workspace.
static std::string graph_key(const char* tag, const void* ws, size_t ws_bytes,
                             const bgk_problem& p, std::initializer_list<double> xs,
                             std::initializer_list<const void*> ptrs = {}) {
  std::string k(tag);
  auto add = [&](const void* q, size_t n) { k.append(static_cast<const char*>(q), n); };
  add(&ws, sizeof(ws));
  add(&ws_bytes, sizeof(ws_bytes));
  add_problem_key(k, p);
  for (double x : xs) add(&x, sizeof(x));
  for (const void* q : ptrs) add(&q, sizeof(q));
  return k;
}

template <class F>
static int run_graph(const std::string& key, hipStream_t user, F&& enqueue) {
  bool use;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    use = g_graphs_on && !g_prof_on;
  }
  if (!use) return enqueue(user);
  bgk_plan* pl = cur_plan();
  std::lock_guard<std::mutex> lk(pl->graph_mu);
  auto it = pl->graphs.find(key);
  if (it == pl->graphs.end()) {
    if (pl->graphs.size() >= kMaxGraphs) {
      BGK_HIP(hipDeviceSynchronize());
      for (auto& kv : pl->graphs) (void)hipGraphExecDestroy(kv.second);
      pl->graphs.clear();
    }
    if (!pl->cap_stream)
      BGK_HIP(hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking));
    BGK_HIP(hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue(pl->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(pl->cap_stream, &g);
    if (rc || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return rc ? rc : hip_fail(e, "hipStreamEndCapture");
    }
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    it = pl->graphs.emplace(key, ex).first;
  }
  BGK_HIP(hipGraphLaunch(it->second, user));
  return BGK_OK;
}

// ------------------------------------------------------ fine-step method --
// E: device [nx] exterior force at the x centres (null: none); emax: the
// Rusanov coefficient of the v_x flux, which must bound max |E_i|; order: x
// transport, 1 upwind (Section 3.1), 2 with the van Leer limited correction.
struct Force {
  const double* E = nullptr;
  double emax = 0.0;
  int order = 1;
  bool on() const { return E != nullptr; }
};

constexpr int kStatusBadForce = 2;  // sticky status: |E_i| > emax or not finite

__global__ void k_check_force(const double* __restrict__ E, int n, double emax, int* status) {
  for (int i = threadIdx.x + blockIdx.x * blockDim.x; i < n; i += blockDim.x * gridDim.x)
    if (!(fabs(E[i]) <= emax)) *status = kStatusBadForce;
}

static int check_force(const bgk_problem& p, const Force& F, int* d_status, hipStream_t s) {
  if (!F.on()) return BGK_OK;
  if (!(F.emax >= 0.0) || !std::isfinite(F.emax)) return invalid("e_max must be finite and >= 0");
  hipLaunchKernelGGL(k_check_force, dim3((p.nx + 255) / 256), dim3(256), 0, s, F.E, p.nx,
                     F.emax, d_status);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

// Method fields of a descriptor (the v_x flux needs dt / dv_x).
static void attach_force(Inst& I, const bgk_problem& p, const Force& F, double dt, Tiles t) {
  I.efield = F.E;
  I.emax = F.emax;
  I.rv = dt / dv_of(p, 0);
  I.order = F.order;
  // the limited step without force on tiles that each lie in one v_x plane
  // writes compact records
  if (F.order == 2 && !F.on() && !t.vcol && !t.pair &&
      ((long long)p.nv[1] * p.nv[2]) % (kWave * t.elems) == 0)
    I.crec = kWave * t.elems;
}

// Tiles and sums per partial for a fine solve of `n` steps: the force step
// and the second-order step run one step per pass on the generic lane mapping.
static Tiles fine_tiles(const bgk_problem& p, int batch, const Force& F) {
  return choose_tiles(p, batch, F.on() || F.order == 2, F.on(), F.order == 2);
}
static int fine_nsum(const Tiles& t, int n, const Force& F) {
  return (!F.on() && F.order != 2 && fused_for(t, n)) ? 15 : 5;
}

static int status_code(int st) {
  if (st == 0) return BGK_OK;
  if (st == kStatusBadForce) {
    set_error("exterior force exceeds e_max or is not finite");
    return BGK_E_INVALID;
  }
  return BGK_E_NONPHYSICAL;
}

}  // namespace bgk

using namespace bgk;

// ======================================================================
//                                C ABI
// ======================================================================
extern "C" {

const char* bgk_last_error(void) { return g_last_error.c_str(); }

const char* bgk_status_string(int st) {
  switch (st) {
    case BGK_OK: return "ok";
    case BGK_E_INVALID: return "invalid argument";
    case BGK_E_NONPHYSICAL: return "non-physical state (rho <= 0, theta <= 0 or NaN)";
    case BGK_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case BGK_E_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

size_t bgk_workspace_bytes(const bgk_problem* prob, int32_t op, int32_t batch) {
  if (check_problem(prob) || batch < 1 || op < 0 || op > BGK_OP_ADJOINT) return 0;
  return layout_of(*prob, op, batch).total;
}

int bgk_n_steps(const bgk_problem* prob, double t_span, int32_t* n, double* dt) {
  int rc = check_problem(prob);
  if (rc) return rc;
  int32_t nn;
  double d;
  rc = n_steps_for(*prob, t_span, &nn, &d);
  if (rc) return rc;
  if (n) *n = nn;
  if (dt) *dt = d;
  return BGK_OK;
}

}  // extern "C"

namespace bgk {
// Reads and clears the sticky status word of ws (stream already idle).
static int take_status(void* ws, hipStream_t s) {
  int st = 0;
  BGK_HIP(hipMemcpy(&st, at<WsHeader>(ws, 0), sizeof(int), hipMemcpyDeviceToHost));
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, &at<WsHeader>(ws, 0)->status, 0);
  BGK_HIP(hipGetLastError());
  BGK_HIP(hipStreamSynchronize(s));
  return status_code(st);
}
}  // namespace bgk

extern "C" {

int bgk_status(void* ws, void* stream) {
  if (ws == nullptr) return BGK_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  BGK_HIP(hipStreamSynchronize(s));
  return take_status(ws, s);
}

int bgk_check(void* stream) {
  hipStream_t s = (hipStream_t)stream;
  BGK_HIP(hipStreamSynchronize(s));
  std::set<void*> list;
  {
    bgk_plan* pl = cur_plan();
    std::lock_guard<std::mutex> lk(pl->used_mu);
    auto it = pl->used.find(stream);
    if (it == pl->used.end()) return BGK_OK;
    list.swap(it->second);
    pl->used.erase(it);
  }
  int worst = BGK_OK;
  std::string msg;
  for (void* ws : list) {
    const int rc = take_status(ws, s);
    if (rc != BGK_OK && worst == BGK_OK) {
      worst = rc;
      msg = g_last_error;
    }
  }
  if (worst != BGK_OK && worst != BGK_E_HIP) set_error(msg);
  return worst;
}

// ------------------------------------------------------------------ plans --
int bgk_plan_create(bgk_plan** plan) {
  if (!plan) return invalid("plan is NULL");
  *plan = new (std::nothrow) bgk_plan();
  if (!*plan) {
    set_error("out of host memory for a plan");
    return BGK_E_INVALID;
  }
  return BGK_OK;
}

int bgk_plan_use(bgk_plan* plan) {
  t_plan = plan;
  return BGK_OK;
}

int bgk_plan_destroy(bgk_plan* plan) {
  if (!plan) return BGK_OK;
  if (plan == &g_default_plan) return invalid("the default plan cannot be destroyed");
  if (t_plan == plan) t_plan = nullptr;
  {
    std::lock_guard<std::mutex> lk(plan->graph_mu);
    if (!plan->graphs.empty() || plan->cap_stream) {
      BGK_HIP(hipDeviceSynchronize());
      for (auto& kv : plan->graphs) (void)hipGraphExecDestroy(kv.second);
      plan->graphs.clear();
      if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
      plan->cap_stream = nullptr;
    }
  }
  delete plan;
  return BGK_OK;
}

int bgk_plan_info(const bgk_plan* plan, int32_t* n_graphs, int32_t* n_tiles) {
  bgk_plan* pl = plan ? const_cast<bgk_plan*>(plan) : cur_plan();
  {
    std::lock_guard<std::mutex> lk(pl->graph_mu);
    if (n_graphs) *n_graphs = (int32_t)pl->graphs.size();
  }
  std::lock_guard<std::mutex> lk(pl->tile_mu);
  if (n_tiles) *n_tiles = (int32_t)pl->tiles.size();
  return BGK_OK;
}

int bgk_lift(const bgk_problem* prob, const double* W, double* f, void* ws,
             size_t ws_bytes, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if (!W || !f) return invalid("NULL array");
  const Layout L = layout_of(*prob, BGK_OP_LIFT, 1);
  if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
  note_ws(ws, stream);
  hipStream_t s = (hipStream_t)stream;
  const Tiles t = choose_tiles(*prob, 1);
  Inst I = make_inst(*prob, 1, 1.0, t);
  attach_fine(I, ws, L.fine, nullptr);
  I.fout = f;
  Inst* dI = at<Inst>(ws, L.insts);
  int* st = &at<WsHeader>(ws, 0)->status;
  if ((rc = put_insts(dI, &I, 1, s))) return rc;
  if ((rc = launch_lift_factors(dI, 1, prob->nx, W, st, s))) return rc;
  return launch_relax_out_blocks(dI, 1, relax_out_blocks(I), I.nvs, -1, s);
}

int bgk_moments(const bgk_problem* prob, const double* f, double* V, double* W,
                void* ws, size_t ws_bytes, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if (!f) return invalid("NULL array");
  const Layout L = layout_of(*prob, BGK_OP_MOMENTS, 1);
  if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
  note_ws(ws, stream);
  hipStream_t s = (hipStream_t)stream;
  Tiles t = choose_tiles(*prob, 1);
  t.pair = 0;  // the moment-partials kernel uses the generic lane mapping
  Inst I = make_inst(*prob, 1, 1.0, t);
  attach_fine(I, ws, L.fine, nullptr);
  I.fin = f;
  if (V) I.vg = V;
  I.vout = W;  // primitive output (nullable)
  Inst* dI = at<Inst>(ws, L.insts);
  int* st = &at<WsHeader>(ws, 0)->status;
  if ((rc = put_insts(dI, &I, 1, s))) return rc;
  if ((rc = launch_partials(dI, 1, I.items, t.elems, t.chunk, s))) return rc;
  return launch_reduce(dI, 1, prob->nx, kRedMomentsOnly, 0, st, s);
}

static int fine_steps_impl(const bgk_problem* prob, const Force& F, const double* f_in,
                           double* f_out, double dt, int32_t n_steps, void* ws,
                           size_t ws_bytes, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if (!f_in || !f_out) return invalid("NULL array");
  if (!(dt > 0.0) || !std::isfinite(dt)) return invalid("dt must be > 0");
  if (n_steps < 0) return invalid("n_steps must be >= 0");
  const size_t fbytes = (size_t)prob->nx * nv3_of(*prob) * sizeof(double);
  const char* a0 = (const char*)f_in;
  const char* b0 = (const char*)f_out;
  if (a0 < b0 + fbytes && b0 < a0 + fbytes) return invalid("f_in and f_out overlap");
  const Layout L = layout_of(*prob, BGK_OP_FINE_STEP, 1);
  if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
  note_ws(ws, stream);
  hipStream_t s = (hipStream_t)stream;
  if (n_steps == 0) {
    BGK_HIP(hipMemcpyAsync(f_out, f_in, fbytes, hipMemcpyDeviceToDevice, s));
    return BGK_OK;
  }
  const Tiles t = aligned_tiles(fine_tiles(*prob, 1, F), *prob, {f_in, f_out});
  Inst I = make_inst(*prob, 1, dt, t, fine_nsum(t, n_steps, F));
  attach_fine(I, ws, L.fine, f_out);  // ping-pong between ws and f_out
  attach_force(I, *prob, F, dt, t);
  I.fin = f_in;
  I.fout = f_out;
  Inst* dI = at<Inst>(ws, L.insts);
  int* st = &at<WsHeader>(ws, 0)->status;
  if ((rc = check_force(*prob, F, st, s))) return rc;
  if ((rc = put_insts(dI, &I, 1, s))) return rc;
  int last = 0;
  if ((rc = run_steps(dI, I, n_steps, kCopy, false, t, st, s, &last))) return rc;
  return launch_relax_out_blocks(dI, 1, relax_out_blocks(I), I.nvs, last, s);
}

int bgk_fine_steps(const bgk_problem* prob, const double* f_in, double* f_out,
                   double dt, int32_t n_steps, void* ws, size_t ws_bytes,
                   void* stream) {
  return fine_steps_impl(prob, Force{}, f_in, f_out, dt, n_steps, ws, ws_bytes, stream);
}

int bgk_fine_steps_force(const bgk_problem* prob, const double* E, double e_max,
                         const double* f_in, double* f_out, double dt, int32_t n_steps,
                         void* ws, size_t ws_bytes, void* stream) {
  if (!E) return invalid("E is NULL");
  return fine_steps_impl(prob, Force{E, e_max}, f_in, f_out, dt, n_steps, ws, ws_bytes,
                         stream);
}

static int fine_step_impl(const bgk_problem* prob, const Force& F, const double* f_in,
                          double* f_out, double t_span, int32_t* n_steps_out, void* ws,
                          size_t ws_bytes, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  int32_t n;
  double dt;
  if ((rc = n_steps_for(*prob, t_span, &n, &dt, F.emax))) return rc;
  if (n_steps_out) *n_steps_out = n;
  return fine_steps_impl(prob, F, f_in, f_out, dt, n, ws, ws_bytes, stream);
}

int bgk_fine_step(const bgk_problem* prob, const double* f_in, double* f_out,
                  double t_span, int32_t* n_steps_out, void* ws, size_t ws_bytes,
                  void* stream) {
  return fine_step_impl(prob, Force{}, f_in, f_out, t_span, n_steps_out, ws, ws_bytes,
                        stream);
}

int bgk_fine_step_force(const bgk_problem* prob, const double* E, double e_max,
                        const double* f_in, double* f_out, double t_span,
                        int32_t* n_steps_out, void* ws, size_t ws_bytes, void* stream) {
  if (!E) return invalid("E is NULL");
  return fine_step_impl(prob, Force{E, e_max}, f_in, f_out, t_span, n_steps_out, ws,
                        ws_bytes, stream);
}

static int propagate_impl(const bgk_problem* prob, const Force& F, int lift_order,
                          int32_t batch, const double* V_in, double* V_out, double t_span,
                          void* ws, size_t ws_bytes, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if ((rc = check_lift_order(*prob, lift_order))) return rc;
  if (batch < 1) return invalid("batch must be >= 1");
  if (!V_in || !V_out) return invalid("NULL array");
  const size_t vb = (size_t)batch * prob->nx * 5 * sizeof(double);
  const char* a0 = (const char*)V_in;
  const char* b0 = (const char*)V_out;
  if (a0 < b0 + vb && b0 < a0 + vb) return invalid("V_in and V_out overlap");
  int32_t n;
  double dt;
  if ((rc = n_steps_for(*prob, t_span, &n, &dt, F.emax))) return rc;
  const Layout L = layout_of(*prob, BGK_OP_PROPAGATE, batch);
  if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
  note_ws(ws, stream);
  hipStream_t s = (hipStream_t)stream;
  const Tiles t = fine_tiles(*prob, batch, F);
  Inst I = make_inst(*prob, batch, dt, t, fine_nsum(t, n, F));
  attach_fine(I, ws, L.fine, nullptr);
  attach_force(I, *prob, F, dt, t);
  prepare_lift(I, lift_order);
  I.vin = V_in;
  I.vout = V_out;
  Inst* dI = at<Inst>(ws, L.insts);
  int* st = &at<WsHeader>(ws, 0)->status;
  if ((rc = check_force(*prob, F, st, s))) return rc;
  if ((rc = put_insts(dI, &I, 1, s))) return rc;
  int last = 0;
  return run_lifted(dI, I, n, lift_order, *prob, t, st, s, &last);
}

}  // extern "C"

namespace bgk {
size_t propagate_ws_bytes(const bgk_problem& p, int batch) {
  return layout_of(p, BGK_OP_PROPAGATE, batch).total;
}
int propagate_plain(const bgk_problem* prob, int32_t batch, const double* V_in,
                    double* V_out, double t_span, void* ws, size_t ws_bytes,
                    void* stream) {
  return propagate_impl(prob, Force{}, 0, batch, V_in, V_out, t_span, ws, ws_bytes, stream);
}
}  // namespace bgk

extern "C" {

int bgk_fine_propagate_moments(const bgk_problem* prob, int32_t batch,
                               const double* V_in, double* V_out, double t_span,
                               void* ws, size_t ws_bytes, void* stream) {
  return propagate_impl(prob, Force{}, 0, batch, V_in, V_out, t_span, ws, ws_bytes, stream);
}

int bgk_fine_propagate_moments_force(const bgk_problem* prob, const double* E,
                                     double e_max, int32_t batch, const double* V_in,
                                     double* V_out, double t_span, void* ws,
                                     size_t ws_bytes, void* stream) {
  if (!E) return invalid("E is NULL");
  return propagate_impl(prob, Force{E, e_max}, 0, batch, V_in, V_out, t_span, ws, ws_bytes,
                        stream);
}

static int euler_impl(const bgk_problem* prob, const double* E, bool viscous, int32_t batch,
                      const double* V_in, double* V_out, double t_span, int32_t* n_sub_out,
                      void* ws, size_t ws_bytes, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if (viscous && !std::isfinite(prob->eps)) return invalid("the Navier-Stokes model needs a finite eps");
  if (batch < 1) return invalid("batch must be >= 1");
  if (!V_in || !V_out) return invalid("NULL array");
  if (!(t_span > 0.0) || !std::isfinite(t_span)) return invalid("t_span must be > 0");
  const Layout L = layout_of(*prob, BGK_OP_COARSE, batch);
  if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
  note_ws(ws, stream);
  return launch_euler(*prob, batch, V_in, V_out, t_span, n_sub_out,
                      at<double>(ws, L.coarse), &at<WsHeader>(ws, 0)->status,
                      (hipStream_t)stream, E, viscous);
}

int euler_coarse_step(const bgk_problem* prob, int32_t batch, const double* V_in,
                      double* V_out, double t_span, int32_t* n_sub_out, void* ws,
                      size_t ws_bytes, void* stream) {
  return euler_impl(prob, nullptr, false, batch, V_in, V_out, t_span, n_sub_out, ws,
                    ws_bytes, stream);
}

int euler_coarse_step_force(const bgk_problem* prob, const double* E, int32_t batch,
                            const double* V_in, double* V_out, double t_span,
                            int32_t* n_sub_out, void* ws, size_t ws_bytes, void* stream) {
  if (!E) return invalid("E is NULL");
  return euler_impl(prob, E, false, batch, V_in, V_out, t_span, n_sub_out, ws, ws_bytes,
                    stream);
}

int euler_coarse_step_cns(const bgk_problem* prob, const double* E, int32_t batch,
                          const double* V_in, double* V_out, double t_span,
                          int32_t* n_sub_out, void* ws, size_t ws_bytes, void* stream) {
  return euler_impl(prob, E, true, batch, V_in, V_out, t_span, n_sub_out, ws, ws_bytes,
                    stream);
}

static int parareal_impl(const bgk_problem* prob, const Force& F, bool viscous,
                         int lift_order, const double* W0,
                         int32_t n_slices, double T, int32_t k_max, double tol,
                         double* V_out, double* err_hist, int32_t* k_done, void* ws,
                         size_t ws_bytes, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if (!W0 || !V_out) return invalid("NULL array");
  if (n_slices < 1 || k_max < 0) return invalid("n_slices >= 1 and k_max >= 0 required");
  if (k_max > 0 && !err_hist) return invalid("err_hist is NULL");
  if (!(T > 0.0) || !std::isfinite(T) || std::isnan(tol)) return invalid("bad T or tol");
  if (viscous && !std::isfinite(prob->eps)) return invalid("the Navier-Stokes model needs a finite eps");
  if ((rc = check_lift_order(*prob, lift_order))) return rc;
  const double span = T / n_slices;
  int32_t n;
  double dt;
  if ((rc = n_steps_for(*prob, span, &n, &dt, F.emax))) return rc;
  const Layout L = layout_of(*prob, BGK_OP_PARAREAL, n_slices);
  if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
  note_ws(ws, stream);
  hipStream_t s = (hipStream_t)stream;
  WsHeader* hd = at<WsHeader>(ws, 0);
  int* st = &hd->status;
  const size_t sl = (size_t)prob->nx * 5;
  double* U[2] = {at<double>(ws, L.U0), at<double>(ws, L.U1)};
  double* Gc = at<double>(ws, L.Gc);
  double* VF = at<double>(ws, L.VF);
  double* scratch = at<double>(ws, L.coarse);
  double* errs = at<double>(ws, L.errs);  // per-iteration errors (fixed K)
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, st, 0);
  BGK_HIP(hipGetLastError());
  if ((rc = check_force(*prob, F, st, s))) return rc;
  if ((rc = launch_pararealsweep_init(*prob, n_slices, W0, U[0], Gc, span, scratch, st, s,
                                      F.E, viscous)))
    return rc;
  int cur = 0;
  int32_t kd = 0;
  Inst* dI = at<Inst>(ws, L.insts);
  for (int k = 0; k < k_max; ++k) {
    const int B = n_slices - k;
    const Tiles t = fine_tiles(*prob, B, F);
    Inst I = make_inst(*prob, B, dt, t, fine_nsum(t, n, F));
    attach_fine(I, ws, L.fine, nullptr);
    attach_force(I, *prob, F, dt, t);
    prepare_lift(I, lift_order);
    I.vin = U[cur] + (size_t)k * sl;        // U^{n-1,k}, n = k+1..N
    I.vout = VF + (size_t)(k + 1) * sl;     // P F L(U^{n-1,k})
    // one iteration: batched lift + fine steps + projection of the active
    // slices, then the sequential correction sweep (replayed as one graph)
    auto iteration = [&](hipStream_t q) -> int {
      int r;
      if ((r = put_insts(dI, &I, 1, q))) return r;
      int last = 0;
      if ((r = run_lifted(dI, I, n, lift_order, *prob, t, st, q, &last))) return r;
      return launch_parareal_sweep(*prob, n_slices, k, U[cur], U[cur ^ 1], VF, Gc, span,
                                   scratch, tol > 0.0 ? &hd->err : errs + k, st, q, F.E,
                                   viscous);
    };
    if ((rc = run_graph(graph_key("pit", ws, ws_bytes, *prob,
                                  {(double)n_slices, span, (double)k, (double)t.elems,
                                   (double)t.chunk, (double)(t.pair + 2 * t.vcol),
                                   (double)I.nsum, (double)fuse_mode(),
                                   tol > 0.0 ? 1.0 : 0.0, F.emax,
                                   viscous ? 1.0 : 0.0, (double)lift_order},
                                  {F.E}),
                        s, iteration)))
      return rc;
    cur ^= 1;
    kd = k + 1;
    if (!(tol > 0.0)) continue;  // fixed K: nothing to decide on the host yet
    struct {
      int status;
      int pad;
      double err;
    } h;
    BGK_HIP(hipMemcpyAsync(&h, hd, sizeof(h), hipMemcpyDeviceToHost, s));
    BGK_HIP(hipStreamSynchronize(s));
    err_hist[k] = h.err;
    if (h.status) {
      // reported here: cleared, so that a later check does not report it again
      hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, st, 0);
      BGK_HIP(hipGetLastError());
      if (k_done) *k_done = kd;
      set_error("non-physical state during parareal iteration");
      return status_code(h.status);
    }
    if (h.err < tol) break;
  }
  if (!(tol > 0.0) && kd > 0) {
    // one readback for all iterations
    int st_h = 0;
    BGK_HIP(hipMemcpyAsync(err_hist, errs, sizeof(double) * kd, hipMemcpyDeviceToHost, s));
    BGK_HIP(hipMemcpyAsync(&st_h, st, sizeof(int), hipMemcpyDeviceToHost, s));
    BGK_HIP(hipStreamSynchronize(s));
    if (st_h) {
      hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, st, 0);
      BGK_HIP(hipGetLastError());
      if (k_done) *k_done = kd;
      set_error("non-physical state during parareal iteration");
      return status_code(st_h);
    }
  }
  if (k_done) *k_done = kd;
  BGK_HIP(hipMemcpyAsync(V_out, U[cur], sl * (n_slices + 1) * sizeof(double),
                         hipMemcpyDeviceToDevice, s));
  return BGK_OK;
}

int parareal_iterate(const bgk_problem* prob, const double* W0, int32_t n_slices,
                     double T, int32_t k_max, double tol, double* V_out,
                     double* err_hist, int32_t* k_done, void* ws, size_t ws_bytes,
                     void* stream) {
  return parareal_impl(prob, Force{}, false, 0, W0, n_slices, T, k_max, tol, V_out, err_hist,
                       k_done, ws, ws_bytes, stream);
}

int parareal_iterate_force(const bgk_problem* prob, const double* E, double e_max,
                           const double* W0, int32_t n_slices, double T, int32_t k_max,
                           double tol, double* V_out, double* err_hist, int32_t* k_done,
                           void* ws, size_t ws_bytes, void* stream) {
  if (!E) return invalid("E is NULL");
  return parareal_impl(prob, Force{E, e_max}, false, 0, W0, n_slices, T, k_max, tol, V_out,
                       err_hist, k_done, ws, ws_bytes, stream);
}

int parareal_iterate_cns(const bgk_problem* prob, const double* E, double e_max,
                         const double* W0, int32_t n_slices, double T, int32_t k_max,
                         double tol, double* V_out, double* err_hist, int32_t* k_done,
                         void* ws, size_t ws_bytes, void* stream) {
  const Force F = E ? Force{E, e_max} : Force{};
  return parareal_impl(prob, F, true, 0, W0, n_slices, T, k_max, tol, V_out, err_hist, k_done,
                       ws, ws_bytes, stream);
}

static int serial_impl(const bgk_problem* prob, const Force& F, int lift_order,
                       const double* W0, int32_t n_slices, double T, double* V_out,
                       void* ws, size_t ws_bytes, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if ((rc = check_lift_order(*prob, lift_order))) return rc;
  if (!W0 || !V_out) return invalid("NULL array");
  if (n_slices < 1 || !(T > 0.0) || !std::isfinite(T)) return invalid("bad n_slices or T");
  const double span = T / n_slices;
  int32_t n;
  double dt;
  if ((rc = n_steps_for(*prob, span, &n, &dt, F.emax))) return rc;
  const Layout L = layout_of(*prob, BGK_OP_PARAREAL, n_slices);
  if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
  note_ws(ws, stream);
  hipStream_t s = (hipStream_t)stream;
  int* st = &at<WsHeader>(ws, 0)->status;
  const size_t sl = (size_t)prob->nx * 5;
  double* U = at<double>(ws, L.U0);  // chain computed in the workspace
  if ((rc = check_force(*prob, F, st, s))) return rc;
  if ((rc = launch_prim_to_cons(W0, U, prob->nx, s))) return rc;
  const Tiles t = fine_tiles(*prob, 1, F);
  Inst* dI = at<Inst>(ws, L.insts);
  const int ns = fine_nsum(t, n, F);
  auto chain = [&](hipStream_t q) -> int {
    int r;
    Inst I = make_inst(*prob, 1, dt, t, ns);
    attach_fine(I, ws, L.fine, nullptr);
    attach_force(I, *prob, F, dt, t);
    prepare_lift(I, lift_order);
    for (int m = 1; m <= n_slices; ++m) {
      I.vin = U + (size_t)(m - 1) * sl;
      I.vout = U + (size_t)m * sl;
      if ((r = put_insts(dI, &I, 1, q))) return r;
      int last = 0;
      if ((r = run_lifted(dI, I, n, lift_order, *prob, t, st, q, &last))) return r;
    }
    return BGK_OK;
  };
  if ((rc = run_graph(graph_key("ser", ws, ws_bytes, *prob,
                                {(double)n_slices, span, (double)t.elems, (double)t.chunk,
                                 (double)(t.pair + 2 * t.vcol), (double)ns,
                                 (double)fuse_mode(), F.emax,
                                 (double)lift_order},
                                {F.E}),
                      s, chain)))
    return rc;
  BGK_HIP(hipMemcpyAsync(V_out, U, sl * (n_slices + 1) * sizeof(double),
                         hipMemcpyDeviceToDevice, s));
  return BGK_OK;
}

int bgk_serial_fine(const bgk_problem* prob, const double* W0, int32_t n_slices,
                    double T, double* V_out, void* ws, size_t ws_bytes,
                    void* stream) {
  return serial_impl(prob, Force{}, 0, W0, n_slices, T, V_out, ws, ws_bytes, stream);
}

int bgk_serial_fine_force(const bgk_problem* prob, const double* E, double e_max,
                          const double* W0, int32_t n_slices, double T, double* V_out,
                          void* ws, size_t ws_bytes, void* stream) {
  if (!E) return invalid("E is NULL");
  return serial_impl(prob, Force{E, e_max}, 0, W0, n_slices, T, V_out, ws, ws_bytes, stream);
}

static Force force_of(const bgk_options* o) {
  Force F = (o && o->E) ? Force{o->E, o->e_max} : Force{};
  F.order = (o && o->fine_order == 2) ? 2 : 1;
  return F;
}

static int check_options(const bgk_options* o) {
  if (o && o->coarse != BGK_COARSE_EULER && o->coarse != BGK_COARSE_NAVIER_STOKES)
    return invalid("coarse must be BGK_COARSE_EULER or BGK_COARSE_NAVIER_STOKES");
  if (o && o->fine_order != 0 && o->fine_order != 1 && o->fine_order != 2)
    return invalid("fine_order must be 1 or 2 (0 means 1)");
  return BGK_OK;
}

int bgk_fine_steps_opts(const bgk_problem* prob, const bgk_options* opts, const double* f_in,
                        double* f_out, double dt, int32_t n_steps, void* ws, size_t ws_bytes,
                        void* stream) {
  int rc = check_options(opts);
  if (rc) return rc;
  return fine_steps_impl(prob, force_of(opts), f_in, f_out, dt, n_steps, ws, ws_bytes, stream);
}

int bgk_fine_propagate_moments_opts(const bgk_problem* prob, const bgk_options* opts,
                                    int32_t batch, const double* V_in, double* V_out,
                                    double t_span, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_options(opts);
  if (rc) return rc;
  return propagate_impl(prob, force_of(opts), opts ? opts->lift_order : 0, batch, V_in,
                        V_out, t_span, ws, ws_bytes, stream);
}

int parareal_iterate_opts(const bgk_problem* prob, const bgk_options* opts,
                          const double* W0, int32_t n_slices, double T, int32_t k_max,
                          double tol, double* V_out, double* err_hist, int32_t* k_done,
                          void* ws, size_t ws_bytes, void* stream) {
  int rc = check_options(opts);
  if (rc) return rc;
  return parareal_impl(prob, force_of(opts),
                       opts && opts->coarse == BGK_COARSE_NAVIER_STOKES,
                       opts ? opts->lift_order : 0, W0, n_slices, T, k_max, tol, V_out,
                       err_hist, k_done, ws, ws_bytes, stream);
}

int bgk_serial_fine_opts(const bgk_problem* prob, const bgk_options* opts, const double* W0,
                         int32_t n_slices, double T, double* V_out, void* ws,
                         size_t ws_bytes, void* stream) {
  int rc = check_options(opts);
  if (rc) return rc;
  return serial_impl(prob, force_of(opts), opts ? opts->lift_order : 0, W0, n_slices, T,
                     V_out, ws, ws_bytes, stream);
}

int bgk_lift_ce(const bgk_problem* prob, const double* W, double* f, void* ws,
                size_t ws_bytes, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if ((rc = check_lift_order(*prob, 1))) return rc;
  if (!W || !f) return invalid("NULL array");
  const Layout L = layout_of(*prob, BGK_OP_LIFT, 1);
  if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
  note_ws(ws, stream);
  hipStream_t s = (hipStream_t)stream;
  const Tiles t = choose_tiles(*prob, 1);
  Inst I = make_inst(*prob, 1, 1.0, t);
  attach_fine(I, ws, L.fine, f);  // the lift writes buf[1] = f
  double* V = at<double>(ws, L.fine.vg);  // conserved moments of W
  if ((rc = launch_prim_to_cons(W, V, prob->nx, s))) return rc;
  I.vin = V;
  Inst* dI = at<Inst>(ws, L.insts);
  int* st = &at<WsHeader>(ws, 0)->status;
  if ((rc = put_insts(dI, &I, 1, s))) return rc;
  return launch_lift_ce(dI, I, dx_of(*prob), prob->eps, st, s);
}

int bgk_n_steps_force(const bgk_problem* prob, double e_max, double t_span, int32_t* n,
                      double* dt) {
  int rc = check_problem(prob);
  if (rc) return rc;
  int32_t nn;
  double d;
  if ((rc = n_steps_for(*prob, t_span, &nn, &d, e_max))) return rc;
  if (n) *n = nn;
  if (dt) *dt = d;
  return BGK_OK;
}

int bgk_set_step_fusion(int32_t steps_per_pass) {
  if (steps_per_pass < 1 || steps_per_pass > 4)
    return invalid("steps_per_pass must be 1, 2, 3 or 4");
  std::lock_guard<std::mutex> lk(g_mu);
  g_fuse = steps_per_pass;
  return BGK_OK;
}

int bgk_set_graphs(int32_t on) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  g_graphs_on = on != 0;
  return BGK_OK;
}

int bgk_release_graphs(void) {
  bgk_plan* pl = cur_plan();
  std::lock_guard<std::mutex> lk(pl->graph_mu);
  if (pl->graphs.empty()) return BGK_OK;
  BGK_HIP(hipDeviceSynchronize());
  for (auto& kv : pl->graphs) (void)hipGraphExecDestroy(kv.second);
  pl->graphs.clear();
  return BGK_OK;
}

int bgk_fine_adjoint(const bgk_problem* prob, const double* f_ckpt,
                     int32_t ckpt_every, int32_t n_steps, double dt,
                     const double* fbar_T, double* fbar_0, double* dlog_eps,
                     void* ws, size_t ws_bytes, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if (!f_ckpt || !fbar_T || !fbar_0 || !dlog_eps) return invalid("NULL array");
  if (ckpt_every < 1 || n_steps < 0) return invalid("ckpt_every >= 1, n_steps >= 0");
  if (!(dt > 0.0) || !std::isfinite(dt)) return invalid("dt must be > 0");
  const size_t nf = (size_t)prob->nx * nv3_of(*prob);
  const size_t fbytes = nf * sizeof(double);
  {
    const char* a0 = (const char*)fbar_T;
    const char* b0 = (const char*)fbar_0;
    if (a0 < b0 + fbytes && b0 < a0 + fbytes) return invalid("fbar_T and fbar_0 overlap");
  }
  const Layout L = layout_of(*prob, BGK_OP_ADJOINT, ckpt_every);
  if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
  note_ws(ws, stream);
  hipStream_t s = (hipStream_t)stream;
  int* st = &at<WsHeader>(ws, 0)->status;
  const Tiles t = choose_tiles(*prob, 1);
  Inst base = make_inst(*prob, 1, dt, t);
  attach_fine(base, ws, L.fine, nullptr);
  double* states = at<double>(ws, L.states);
  double* fb[2] = {at<double>(ws, L.fbA), at<double>(ws, L.fbB)};
  double* part6 = at<double>(ws, L.part6);
  double* coef = at<double>(ws, L.coef);
  double* dle = at<double>(ws, L.dle);
  Inst* dI = at<Inst>(ws, L.insts);
  const int n_seg = (n_steps + ckpt_every - 1) / ckpt_every;
  // descriptors by position j in a segment: the recomputation of state j
  // from state j - 1 (entry j), the backward step from state j (entry
  // ckpt_every + j); the same for every segment, uploaded once
  std::vector<Inst> tab(2 * (size_t)ckpt_every, base);
  for (int j = 0; j < ckpt_every; ++j) {
    if (j > 0) {
      tab[j].fin = states + (size_t)(j - 1) * nf;
      tab[j].fout = states + (size_t)j * nf;
    }
    tab[ckpt_every + j].fin = states + (size_t)j * nf;
  }
  // cells whose velocities fit one block take the whole-cell kernels (one
  // launch per recomputed state, two per backward step); larger cells the
  // tiled kernels with separate per-cell reductions
  const bool whole_cell = adj_cell_ept(base) > 0;
  auto sequence = [&](hipStream_t q) -> int {
    int r;
    if ((r = put_insts(dI, tab.data(), 2 * ckpt_every, q))) return r;
    BGK_HIP(hipMemcpyAsync(fb[0], fbar_T, fbytes, hipMemcpyDeviceToDevice, q));
    int cur = 0;
    for (int c = n_seg - 1; c >= 0; --c) {
      const int s0 = c * ckpt_every;
      const int s1 = std::min(s0 + ckpt_every, (int)n_steps);
      BGK_HIP(hipMemcpyAsync(states, f_ckpt + (size_t)c * nf, fbytes,
                             hipMemcpyDeviceToDevice, q));
      // forward states s0+1 .. s1-1 of the segment (transport, moments, relax)
      for (int k = s0 + 1; k < s1; ++k) {
        const Inst* d = dI + (k - s0);
        if (whole_cell) {
          if ((r = launch_adj_cell(dI, base, false, states + (size_t)(k - 1 - s0) * nf,
                                   states + (size_t)(k - s0) * nf, nullptr, nullptr, nullptr,
                                   false, st, q)))
            return r;
          continue;
        }
        if ((r = launch_step(d, 1, base.items, kCopy, 1, t, lds_doubles(base, t), st, q)))
          return r;
        if ((r = launch_reduce(d, 1, prob->nx, kRedRelaxFactors, 0, st, q))) return r;
        if ((r = launch_relax_out_blocks(d, 1, relax_out_blocks(base), base.nvs, 0, q)))
          return r;
      }
      for (int k = s1 - 1; k >= s0; --k) {
        const Inst* d = dI + ckpt_every + (k - s0);
        // per-cell log-eps terms summed over the steps, then over the cells
        const bool acc = k != (int)n_steps - 1;
        if (whole_cell) {
          // g = T f^k, its moments and Maxwellian, the sums and coefficients
          if ((r = launch_adj_cell(dI, base, true, states + (size_t)(k - s0) * nf, nullptr,
                                   fb[cur], coef, dle, acc, st, q)))
            return r;
        } else {
          // g = T f^k into buf[0], moments and the unscaled Maxwellian of U(g)
          if ((r = launch_step(d, 1, base.items, kCopy, 1, t, lds_doubles(base, t), st, q)))
            return r;
          if ((r = launch_reduce(d, 1, prob->nx, kRedMaxwellFactors, 0, st, q))) return r;
          if ((r = launch_adjoint_sums(d, base, 0, fb[cur], part6, q))) return r;
          if ((r = launch_adjoint_reduce(d, base, part6, coef, dle, acc, q))) return r;
        }
        if ((r = launch_adjoint_transpose(d, base, t.chunk, fb[cur], coef, fb[cur ^ 1], q)))
          return r;
        cur ^= 1;
      }
    }
    if (n_steps > 0 && (r = launch_sum_into(dle, prob->nx, dlog_eps, q))) return r;
    BGK_HIP(hipMemcpyAsync(fbar_0, fb[cur], fbytes, hipMemcpyDeviceToDevice, q));
    return BGK_OK;
  };
  // the whole sequence is captured once per (workspace, problem, buffers,
  // steps) and replayed
  return run_graph(graph_key("adj", ws, ws_bytes, *prob,
                             {(double)ckpt_every, (double)n_steps, dt, (double)t.elems,
                              (double)t.chunk, (double)(t.pair + 2 * t.vcol)},
                             {f_ckpt, fbar_T, fbar_0, dlog_eps}),
                   s, sequence);
}

int bgk_lift_adjoint_rho(const bgk_problem* prob, const double* W,
                         const double* fbar, double* rhobar, void* ws,
                         size_t ws_bytes, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if (!W || !fbar || !rhobar) return invalid("NULL array");
  const Layout L = layout_of(*prob, BGK_OP_LIFT, 1);
  if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
  note_ws(ws, stream);
  hipStream_t s = (hipStream_t)stream;
  const Tiles t = choose_tiles(*prob, 1);
  Inst I = make_inst(*prob, 1, 1.0, t);
  attach_fine(I, ws, L.fine, nullptr);
  Inst* dI = at<Inst>(ws, L.insts);
  int* st = &at<WsHeader>(ws, 0)->status;
  if ((rc = put_insts(dI, &I, 1, s))) return rc;
  if ((rc = launch_lift_factors(dI, 1, prob->nx, W, st, s))) return rc;
  return launch_lift_adjoint_rho(dI, I, W, fbar, rhobar, s);
}

__global__ void k_density_adjoint(const double* __restrict__ rhobar, double* fbar,
                                  long long nv3, long long n, double dv3) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) fbar[k] = rhobar[k / nv3] * dv3;
}

int bgk_density_adjoint(const bgk_problem* prob, const double* rhobar, double* fbar,
                        void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if (!rhobar || !fbar) return invalid("NULL array");
  const long long nv3 = nv3_of(*prob);
  const long long n = nv3 * prob->nx;
  const double dv3 = dv_of(*prob, 0) * dv_of(*prob, 1) * dv_of(*prob, 2);
  hipLaunchKernelGGL(k_density_adjoint, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, rhobar, fbar, nv3, n, dv3);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

// -------------------------------------------------- uneven batches (C ABI) --
// A grid with odd nv_z has no 16-byte pairs of z neighbours, and its x rows
// alternate in alignment.  The fused passes run it on a padded copy instead:
// each z row gains one point above the box (same spacing) whose Maxwellian
// factor is zero, so f stays exactly zero there and every sum is unchanged;
// its fields live in two workspace buffers, filled from f_in with the pad
// points cleared and written back to f_out without them by the final
// relaxation.
static bool batched_padded(const bgk_problem& p) { return p.nv[2] % 2 != 0; }

static bgk_problem padded_problem(const bgk_problem& p) {
  bgk_problem q = p;
  q.nv[2] += 1;
  q.v_hi[2] = p.v_hi[2] + dv_of(p, 2);
  return q;
}

struct BatchedLayout {
  size_t header, insts;
  std::vector<FineRegions> regions;
  size_t total;
};

static BatchedLayout batched_layout(const bgk_problem* probs, int n) {
  Carve c;
  BatchedLayout L;
  L.header = c.take(sizeof(WsHeader));
  L.insts = c.take(sizeof(Inst) * (size_t)n);
  for (int q = 0; q < n; ++q)
    L.regions.push_back(batched_padded(probs[q]) ? carve_fine(c, padded_problem(probs[q]), 1, 2)
                                                 : carve_fine(c, probs[q], 1, 1));
  L.total = c.off;
  return L;
}

size_t bgk_workspace_bytes_batched(const bgk_problem* probs, int32_t n) {
  if (!probs || n < 1 || n > kMaxInst) return 0;
  for (int q = 0; q < n; ++q)
    if (check_problem(&probs[q])) return 0;
  return batched_layout(probs, n).total;
}

int bgk_fine_step_batched(const bgk_problem* probs, int32_t n,
                          const double* const* f_in, double* const* f_out,
                          const double* t_span, int32_t* n_steps_out, void* ws,
                          size_t ws_bytes, void* stream) {
  if (!probs || !f_in || !f_out || !t_span) return invalid("NULL argument");
  if (n < 1 || n > kMaxInst) return invalid("n must be in [1, 4096]");
  int rc;
  std::vector<int32_t> steps(n);
  std::vector<double> dts(n);
  for (int q = 0; q < n; ++q) {
    if ((rc = check_problem(&probs[q]))) return rc;
    if (!f_in[q] || !f_out[q]) return invalid("NULL array");
    if ((rc = n_steps_for(probs[q], t_span[q], &steps[q], &dts[q]))) return rc;
    const size_t fb = (size_t)probs[q].nx * nv3_of(probs[q]) * sizeof(double);
    const char* a0 = (const char*)f_in[q];
    const char* b0 = (const char*)f_out[q];
    if (a0 < b0 + fb && b0 < a0 + fb) return invalid("f_in and f_out overlap");
  }
  const BatchedLayout L = batched_layout(probs, n);
  if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
  note_ws(ws, stream);
  if (n_steps_out)
    for (int q = 0; q < n; ++q) n_steps_out[q] = steps[q];
  hipStream_t s = (hipStream_t)stream;
  // Tile shape: 4 velocities per lane over 8-cell chunks (or the override).
  // With two or more steps per pass set, every instance runs fused two-step
  // passes: first the instances whose rows can be read in 16-byte pairs
  // (nvz even with aligned f_in and f_out, or nvz odd on the padded copy),
  // then the others (even nvz, unaligned f) on unpaired lanes, each group
  // with its own tile mapping.  Without fusion all instances take one step
  // per launch (paired lanes only if every instance allows them).
  // Within a group the instances are sorted by step count (descending), so
  // that its active instances at any step form a prefix.
  // Built-in shapes, measured on the 29-instance seeded batch: paired lanes
  // four pairs per lane over 8-cell chunks (5.3 TB/s), unpaired lanes four
  // velocities per lane over 24-cell chunks (4.0 TB/s; 8-cell chunks 3.3,
  // eight per lane spill); an override applies to both groups.
  Tiles t = {8, 8, 1}, tflat = {4, 24, 0};
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (Tiles* x : {&t, &tflat}) {
      if (g_override.elems) x->elems = g_override.elems;
      if (g_override.chunk) x->chunk = g_override.chunk;
    }
    if (g_override.pair == 0) t.pair = 0;
  }
  const bool fused = fuse_mode() >= 2;
  std::vector<char> pairable(n), padded(n);
  for (int q = 0; q < n; ++q) {
    padded[q] = fused && t.pair == 1 && batched_padded(probs[q]);
    pairable[q] = t.pair == 1 && (padded[q] || (probs[q].nv[2] % 2 == 0 &&
                                  aligned_tiles(t, probs[q], {f_in[q], f_out[q]}).pair == 1));
  }
  // the grid each instance's kernels run on
  std::vector<bgk_problem> grid(n);
  for (int q = 0; q < n; ++q) grid[q] = padded[q] ? padded_problem(probs[q]) : probs[q];
  auto first_group = [&](int q) { return fused && pairable[q]; };
  std::vector<int> order(n);
  for (int q = 0; q < n; ++q) order[q] = q;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    if (first_group(x) != first_group(y)) return first_group(x);
    return steps[x] > steps[y];
  });
  int nA = 0;
  while (nA < n && first_group(order[nA])) ++nA;
  Tiles tA = t, tB = t;
  for (int k = nA; k < n; ++k)
    if (!pairable[order[k]]) tB = tflat;
  // factor rows of the group's largest velocity grid within the LDS (two
  // levels of 2 chunk + 6 rows in a two-step pass, chunk + 2 in one step)
  for (int grp = 0; grp < 2; ++grp) {
    Tiles& tt = grp ? tB : tA;
    long long nvs_m = 0;
    for (int k = grp ? nA : 0; k < (grp ? n : nA); ++k) {
      const bgk_problem& pq = grid[order[k]];
      nvs_m = std::max(nvs_m, (long long)pq.nv[0] + pq.nv[1] + pq.nv[2]);
    }
    while (tt.chunk > 1 && (fused ? 2LL * tt.chunk + 6 : tt.chunk + 2LL) * nvs_m * 8 > kLdsBytes)
      tt.chunk /= 2;
  }
  std::vector<Inst> h(n);
  long long items = 0;
  int nvs_a = 0, nvs_b = 0;
  std::vector<long long> items_prefix(n + 1, 0), cells_prefix(n + 1, 0);
  for (int k = 0; k < n; ++k) {
    const int q = order[k];
    // fused passes need the nu-weighted partial sums (15 per record)
    Inst I = make_inst(grid[q], 1, dts[q], k < nA ? tA : tB, fused ? 15 : 5);
    if (padded[q]) {
      // the real grid's spacing and live z points; f_in is copied into buf[1]
      I.dv[2] = dv_of(probs[q], 2);
      I.dv3 = I.dv[0] * I.dv[1] * I.dv[2];
      I.nvz_live = probs[q].nv[2];
      attach_fine(I, ws, L.regions[q], nullptr);
      I.fin = I.buf[1];
    } else {
      attach_fine(I, ws, L.regions[q], f_out[q]);
      I.fin = f_in[q];
    }
    I.fout = f_out[q];
    I.steps = steps[q];
    I.item_begin = items;
    I.cell_begin = cells_prefix[k];
    items += I.items;
    items_prefix[k + 1] = items;
    cells_prefix[k + 1] = cells_prefix[k] + I.nx;
    (k < nA ? nvs_a : nvs_b) = std::max(k < nA ? nvs_a : nvs_b, I.nvs);
    h[k] = I;
  }
  Inst* dI = at<Inst>(ws, L.insts);
  int* st = &at<WsHeader>(ws, 0)->status;
  // phase-space cells of entries [a, b) on their own grids (pad points not
  // counted)
  auto cells_of = [&](int a, int b) {
    double c = 0.0;
    for (int k = a; k < b; ++k) c += (double)h[k].nx * nv3_of(probs[order[k]]);
    return c;
  };
  // Entries [a0, a1) one step per launch over the instances still stepping
  // (a launch over entries [a, b) takes the table from entry a).
  auto single_steps = [&](int a0, int a1, Tiles tt, int nvs_m, hipStream_t q) -> int {
    int r;
    if (a0 == a1) return BGK_OK;
    const int smax = h[a0].steps;
    int w_prev = 1;
    for (int k = 1; k <= smax; ++k) {
      int e = a0;
      while (e < a1 && h[e].steps >= k) ++e;
      const int mode = (k == 1) ? kCopy : kRelax;
      const int phase = w_prev;
      prof_before(q);
      r = launch_step(dI + a0, e - a0, items_prefix[e] - items_prefix[a0], mode, phase, tt,
                      (tt.chunk + 2) * nvs_m, st, q);
      prof_after(q, cells_of(a0, e), 16.0, BGK_PROF_ONE_STEP);
      if (r) return r;
      if ((r = launch_reduce(dI + a0, e - a0, cells_prefix[e] - cells_prefix[a0],
                             kRedRelaxFactors, 0, st, q)))
        return r;
      w_prev = phase ^ 1;
    }
    // final relaxation, each instance from the buffer its last step wrote:
    // step k writes buf[(k - 1) & 1]
    for (int k = a0; k < a1; ++k) {
      const int sel = (h[k].steps - 1) & 1;
      if ((r = launch_relax_out_blocks(dI + k, 1, relax_out_blocks(h[k]), h[k].nvs, sel, q)))
        return r;
    }
    return BGK_OK;
  };
  // Entries [a0, a1) fused: every instance's first step alone (from f_in),
  // then in each round the instances with two or more steps left (a prefix)
  // take one two-step pass and those with one left (the next entries) one
  // step, so all active instances stay in the same buffer phase.
  auto fused_steps = [&](int a0, int a1, Tiles tt, int nvs_m, hipStream_t q) -> int {
    int r;
    if (a0 == a1) return BGK_OK;
    std::vector<int> rem(a1 - a0), sel(a1 - a0, 0);
    for (int k = a0; k < a1; ++k) rem[k - a0] = h[k].steps;
    auto prefix_end = [&](int m) {
      int c = a0;
      while (c < a1 && rem[c - a0] >= m) ++c;
      return c;
    };
    int phase = 1;  // a pass reads buf[phase] (f_in in copy mode), writes buf[phase ^ 1]
    auto advance = [&](int a, int b, int by) {
      for (int k = a; k < b; ++k) {
        rem[k - a0] -= by;
        if (rem[k - a0] == 0) sel[k - a0] = phase ^ 1;
      }
    };
    auto span_items = [&](int a, int b) { return items_prefix[b] - items_prefix[a]; };
    auto span_cells = [&](int a, int b) { return cells_prefix[b] - cells_prefix[a]; };
    prof_before(q);
    r = launch_step(dI + a0, a1 - a0, span_items(a0, a1), kCopy, phase, tt,
                    (tt.chunk + 2) * nvs_m, st, q, 15);
    prof_after(q, cells_of(a0, a1), 16.0, BGK_PROF_ONE_STEP);
    if (r) return r;
    advance(a0, a1, 1);
    phase ^= 1;
    for (;;) {
      const int e1 = prefix_end(1), e2 = prefix_end(2);
      if (e1 == a0) break;
      if (e2 > a0) {
        if ((r = launch_reduce(dI + a0, e2 - a0, span_cells(a0, e2), kRedW1, 0, st, q)))
          return r;
        if ((r = launch_reduce(dI + a0, e2 - a0, span_cells(a0, e2), kRedW2, 0, st, q)))
          return r;
      }
      if (e1 > e2 && (r = launch_reduce(dI + e2, e1 - e2, span_cells(e2, e1),
                                        kRedRelaxFactors, 0, st, q)))
        return r;
      if (e2 > a0) {
        prof_before(q);
        r = launch_step2x2(dI + a0, e2 - a0, span_items(a0, e2), kRelax, phase, tt,
                           (2 * tt.chunk + 6) * nvs_m, false, q);
        prof_after(q, 2.0 * cells_of(a0, e2), 8.0, BGK_PROF_TWO_STEP);
        if (r) return r;
      }
      if (e1 > e2) {
        prof_before(q);
        r = launch_step(dI + e2, e1 - e2, span_items(e2, e1), kRelax, phase, tt,
                        (tt.chunk + 2) * nvs_m, st, q, 15);
        prof_after(q, cells_of(e2, e1), 16.0, BGK_PROF_ONE_STEP);
        if (r) return r;
      }
      advance(a0, e2, 2);
      advance(e2, e1, 1);
      phase ^= 1;
    }
    // factors of every instance's last field, then its relaxed output
    if ((r = launch_reduce(dI + a0, a1 - a0, span_cells(a0, a1), kRedRelaxFactors, 0, st, q)))
      return r;
    for (int k = a0; k < a1; ++k)
      if ((r = launch_relax_out_blocks(dI + k, 1, relax_out_blocks(h[k]), h[k].nvs,
                                       sel[k - a0], q)))
        return r;
    return BGK_OK;
  };
  auto sequence = [&](hipStream_t q) -> int {
    int r;
    if ((r = put_insts(dI, h.data(), n, q))) return r;
    for (int k = 0; k < n; ++k)
      if (padded[order[k]] &&
          (r = launch_pad_rows(f_in[order[k]], h[k].buf[1],
                               (long long)h[k].nx * h[k].nvx * h[k].nvy, h[k].nvz_live, q)))
        return r;
    if (!fused) return single_steps(0, n, tB, nvs_b, q);
    if ((r = fused_steps(0, nA, tA, nvs_a, q))) return r;
    return fused_steps(nA, n, tB, nvs_b, q);
  };
  // the whole sequence is captured once per (workspace, problems, buffers,
  // spans, tiles, fusion) and replayed
  std::string key("bat");
  auto add = [&](const void* q, size_t nb) { key.append(static_cast<const char*>(q), nb); };
  add(&ws, sizeof(ws));
  add(&ws_bytes, sizeof(ws_bytes));
  add(&n, sizeof(n));
  for (int q = 0; q < n; ++q) add_problem_key(key, probs[q]);
  add(f_in, sizeof(const double*) * (size_t)n);
  add(f_out, sizeof(double*) * (size_t)n);
  add(t_span, sizeof(double) * (size_t)n);
  add(&tA, sizeof(tA));
  add(&tB, sizeof(tB));
  add(&fused, sizeof(fused));
  return run_graph(key, s, sequence);
}

// ------------------------------------------------------- tiles / autotune --
int bgk_set_tiles(int32_t elems, int32_t chunk, int32_t pair) {
  if (!(elems == 0 || elems == 2 || elems == 4 || elems == 8))
    return invalid("elems_per_lane must be 0, 2, 4 or 8");
  if (chunk < 0 || chunk > kMaxChunk) return invalid("x_chunk must be in [0, 64]");
  if (pair < -1 || pair > 3) return invalid("pair must be -1, 0, 1, 2 or 3");
  std::lock_guard<std::mutex> lk(g_mu);
  g_override = {elems, chunk, pair};
  return BGK_OK;
}

}  // extern "C"

namespace bgk {
// Architecture name of the current device ("gfx950"), looked up once per
// device.
static std::string device_arch() {
  static std::mutex mu;
  static std::map<int, std::string> names;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "unknown";
  std::lock_guard<std::mutex> lk(mu);
  auto it = names.find(dev);
  if (it != names.end()) return it->second;
  hipDeviceProp_t prop;
  std::string name = "unknown";
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    name = prop.gcnArchName;
    const size_t c = name.find(':');
    if (c != std::string::npos) name = name.substr(0, c);
  }
  names[dev] = name;
  return name;
}

// LDS bytes of the passes a fused sequence of `steps` steps runs with tiles t.
static long long seq_lds_bytes(const Inst& h, Tiles t, int steps) {
  if (fused_for(t, steps) && triple_for(h, t)) return (long long)lds_doubles3(h, t) * 8;
  if (fused_for(t, steps)) return (long long)lds_doubles2(h, t) * 8;
  return (long long)lds_doubles(h, t) * 8;
}
}  // namespace bgk

extern "C" {

int bgk_autotune(const bgk_problem* prob, int32_t batch, void* ws, size_t ws_bytes,
                 void* stream, int32_t* best_elems, int32_t* best_chunk,
                 int32_t* best_pair) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if (batch < 1) return invalid("batch must be >= 1");
  const Layout L = layout_of(*prob, BGK_OP_PROPAGATE, batch);
  if ((rc = check_ws(ws, ws_bytes, L.total))) return rc;
  note_ws(ws, stream);
  hipStream_t s = (hipStream_t)stream;
  // moments of a smooth state to lift from
  std::vector<double> hV((size_t)batch * prob->nx * 5);
  for (int b = 0; b < batch; ++b)
    for (int i = 0; i < prob->nx; ++i) {
      double* v = &hV[((size_t)b * prob->nx + i) * 5];
      v[0] = 1.0 + 0.1 * std::sin(6.283185307179586 * (i + 0.5) / prob->nx);
      v[1] = v[2] = v[3] = 0.0;
      v[4] = 1.5 * v[0];
    }
  double* Vin = at<double>(ws, L.fine.vg);   // borrow: lifted from before steps
  double* Vout = at<double>(ws, L.fine.vout);
  // nine steps: whole passes with three steps per pass (one from the lift,
  // two reading and writing f) and with two
  const int steps = 9;
  const double dt = 0.5 * dx_of(*prob) / std::max(std::fabs(prob->v_lo[0]), std::fabs(prob->v_hi[0]));
  const int fuse = fuse_mode();
  // candidates: the built-in choice (without a tuned entry), a grid of
  // shapes, and for three-step grids the longest chunks whose factor rows fit
  // the LDS; shapes whose passes would need more than 160 KB of LDS are left
  // out
  std::vector<Tiles> cands;
  {
    bgk_plan* pl = cur_plan();
    std::map<TileKey, Tuned> saved;
    {
      std::lock_guard<std::mutex> lk(pl->tile_mu);
      saved.swap(pl->tiles);
    }
    cands.push_back(choose_tiles(*prob, batch));
    std::lock_guard<std::mutex> lk(pl->tile_mu);
    for (auto& kv : saved) pl->tiles.emplace(kv.first, kv.second);
  }
  const int Es[3] = {2, 4, 8};
  const int Cs[8] = {1, 2, 4, 8, 16, 24, 32, 48};
  for (int pr = 0; pr < 2; ++pr)
    for (int ei = 0; ei < 3; ++ei) {
      for (int ci = 0; ci < 8; ++ci) cands.push_back(Tiles{Es[ei], Cs[ci], pr});
      if (pr && Es[ei] <= 4) {
        const long long rl = lds3_row(prob->nv[0], prob->nv[1], prob->nv[2], Es[ei]);
        int ch = lds3_max_chunk(Es[ei]);
        while (ch > 1 && (3LL * ch + 12) * rl * 8 > (long long)lds3_cap(Es[ei])) --ch;
        cands.push_back(Tiles{Es[ei], ch, 1});
      }
    }
  hipEvent_t e0, e1;
  BGK_HIP(hipEventCreate(&e0));
  BGK_HIP(hipEventCreate(&e1));
  Tiles best = cands[0];
  float best_ms = 1e30f;
  std::set<std::tuple<int, int, int>> seen;
  for (const Tiles& t : cands) {
    if (t.chunk < 1 || t.chunk > prob->nx || (t.pair && prob->nv[2] % 2 != 0)) continue;
    if (!seen.insert({t.elems, t.chunk, t.pair}).second) continue;
    Inst I = make_inst(*prob, batch, dt, t, fused_for(t, steps) ? 15 : 5);
    if (seq_lds_bytes(I, t, steps) > kLdsBytes) continue;
    attach_fine(I, ws, L.fine, nullptr);
    I.vin = Vin;
    I.vout = Vout;
    Inst* dI = at<Inst>(ws, L.insts);
    int* st = &at<WsHeader>(ws, 0)->status;
    float ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {
      BGK_HIP(hipMemcpyAsync(Vin, hV.data(), hV.size() * sizeof(double),
                             hipMemcpyHostToDevice, s));
      if ((rc = put_insts(dI, &I, 1, s))) break;
      BGK_HIP(hipEventRecord(e0, s));
      int last = 0;
      if ((rc = lift_and_run(dI, I, steps, false, t, st, s, &last))) break;
      BGK_HIP(hipEventRecord(e1, s));
      BGK_HIP(hipEventSynchronize(e1));
      BGK_HIP(hipEventElapsedTime(&ms, e0, e1));
    }
    if (rc) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return rc;
    }
    if (ms < best_ms) {
      best_ms = ms;
      best = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  {
    bgk_plan* pl = cur_plan();
    std::lock_guard<std::mutex> lk(pl->tile_mu);
    pl->tiles[tile_key(*prob, batch, fuse)] = Tuned{best, (double)best_ms, device_arch()};
  }
  if (best_elems) *best_elems = best.elems;
  if (best_chunk) *best_chunk = best.chunk;
  if (best_pair) *best_pair = best.pair;
  return BGK_OK;
}

// Tuned tiles as JSON: {"bgk_tiles": 1, "entries": [{"arch": "gfx950",
// "nv": [a, b, c], "nx_bucket": n, "batch_bucket": m, "steps_per_pass": k,
// "elems": e, "chunk": c, "pair": p, "ms": t}, ...]}
int bgk_plan_save_tiles(const bgk_plan* plan, const char* path) {
  if (!path) return invalid("path is NULL");
  bgk_plan* pl = plan ? const_cast<bgk_plan*>(plan) : cur_plan();
  std::string out = "{\"bgk_tiles\": 1, \"entries\": [";
  {
    std::lock_guard<std::mutex> lk(pl->tile_mu);
    bool first = true;
    for (auto& kv : pl->tiles) {
      const TileKey& k = kv.first;
      const Tuned& v = kv.second;
      char buf[512];
      std::snprintf(buf, sizeof(buf),
                    "%s\n  {\"arch\": \"%s\", \"nv\": [%d, %d, %d], \"nx_bucket\": %d, "
                    "\"batch_bucket\": %d, \"steps_per_pass\": %d, \"elems\": %d, "
                    "\"chunk\": %d, \"pair\": %d, \"ms\": %.6g}",
                    first ? "" : ",", v.arch.c_str(), std::get<0>(k), std::get<1>(k),
                    std::get<2>(k), std::get<3>(k), std::get<4>(k), std::get<5>(k),
                    v.t.elems, v.t.chunk, v.t.pair, v.ms);
      out += buf;
      first = false;
    }
  }
  out += "\n]}\n";
  FILE* fh = std::fopen(path, "w");
  if (!fh) return invalid("cannot open the tile file for writing");
  const size_t wr = std::fwrite(out.data(), 1, out.size(), fh);
  const int cl = std::fclose(fh);
  if (wr != out.size() || cl != 0) return invalid("cannot write the tile file");
  return BGK_OK;
}

}  // extern "C"

namespace bgk {
// Value text after "name": in one entry object (nullptr if absent).
static const char* json_field(const std::string& obj, const char* name, size_t* pos) {
  const std::string k = std::string("\"") + name + "\"";
  const size_t a = obj.find(k);
  if (a == std::string::npos) return nullptr;
  const size_t c = obj.find(':', a + k.size());
  if (c == std::string::npos) return nullptr;
  *pos = c + 1;
  return obj.c_str() + c + 1;
}
static bool json_int(const std::string& obj, const char* name, int* v) {
  size_t pos;
  const char* t = json_field(obj, name, &pos);
  return t && std::sscanf(t, " %d", v) == 1;
}
}  // namespace bgk

extern "C" {

int bgk_plan_load_tiles(bgk_plan* plan, const char* path) {
  if (!path) return invalid("path is NULL");
  FILE* fh = std::fopen(path, "r");
  if (!fh) return invalid("cannot open the tile file");
  std::string txt;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), fh)) > 0) txt.append(buf, n);
  std::fclose(fh);
  if (txt.find("\"bgk_tiles\"") == std::string::npos) return invalid("not a tile file");
  bgk_plan* pl = plan ? plan : cur_plan();
  std::vector<std::pair<std::string, std::pair<TileKey, Tuned>>> entries;
  size_t at_ = txt.find('[');
  if (at_ == std::string::npos) return invalid("tile file has no entries");
  for (;;) {
    const size_t a = txt.find('{', at_);
    if (a == std::string::npos) break;
    const size_t b = txt.find('}', a);
    if (b == std::string::npos) return invalid("truncated tile file");
    const std::string obj = txt.substr(a, b - a + 1);
    at_ = b + 1;
    size_t pos;
    const char* t = json_field(obj, "arch", &pos);
    char a_name[64] = {0};
    if (!t || std::sscanf(t, " \"%63[^\"]\"", a_name) != 1) return invalid("tile entry without arch");
    int nv[3], nxb, bb, fu, e, c, pr;
    const char* tv = json_field(obj, "nv", &pos);
    if (!tv || std::sscanf(tv, " [ %d , %d , %d ]", &nv[0], &nv[1], &nv[2]) != 3 ||
        !json_int(obj, "nx_bucket", &nxb) || !json_int(obj, "batch_bucket", &bb) ||
        !json_int(obj, "steps_per_pass", &fu) || !json_int(obj, "elems", &e) ||
        !json_int(obj, "chunk", &c) || !json_int(obj, "pair", &pr))
      return invalid("malformed tile entry");
    if (!(e == 2 || e == 4 || e == 8) || c < 1 || c > kMaxChunk || pr < 0 || pr > 1)
      return invalid("tile entry out of range");
    double ms = 0.0;
    const char* tm = json_field(obj, "ms", &pos);
    if (tm) std::sscanf(tm, " %lf", &ms);
    entries.push_back({a_name, {TileKey{nv[0], nv[1], nv[2], nxb, bb, fu},
                                Tuned{Tiles{e, c, pr, 0}, ms, a_name}}});
  }
  if (entries.empty()) return BGK_OK;
  const std::string arch = device_arch();
  std::lock_guard<std::mutex> lk(pl->tile_mu);
  for (auto& en : entries)
    if (en.first == arch) pl->tiles[en.second.first] = en.second.second;  // else another arch
  return BGK_OK;
}

// max |E_i| of an exterior force (the Rusanov coefficient of the v_x flux).
int bgk_force_bound(const bgk_problem* prob, const double* E, int32_t E_on_device,
                    double* e_max, void* stream) {
  int rc = check_problem(prob);
  if (rc) return rc;
  if (!E || !e_max) return invalid("NULL array");
  std::vector<double> h;
  const double* src = E;
  if (E_on_device) {
    // nx values: read back on the stream rather than reduced on the device
    h.resize(prob->nx);
    hipStream_t s = (hipStream_t)stream;
    BGK_HIP(hipMemcpyAsync(h.data(), E, sizeof(double) * prob->nx, hipMemcpyDeviceToHost, s));
    BGK_HIP(hipStreamSynchronize(s));
    src = h.data();
  }
  double m = 0.0;
  for (int i = 0; i < prob->nx; ++i) {
    const double a = std::fabs(src[i]);
    if (std::isnan(a)) {
      m = a;
      break;
    }
    m = std::max(m, a);
  }
  *e_max = m;
  return BGK_OK;
}

// -------------------------------------------------------------- profiling --
int bgk_prof_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& r : g_prof) {
    g_prof_pool.push_back(r.a);
    g_prof_pool.push_back(r.b);
  }
  g_prof.clear();
  g_prof_on = on != 0;
  return BGK_OK;
}

int bgk_prof_read(int32_t kind, double* total_ms, int64_t* launches, double* cells,
                  double* bytes) {
  if (kind < BGK_PROF_ALL || kind > BGK_PROF_FOUR_STEP_LIFT) return invalid("unknown timing kind");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  double ms = 0.0, c = 0.0, by = 0.0;
  int64_t n = 0;
  for (auto& r : g_prof) {
    if (kind != BGK_PROF_ALL && r.kind != kind) continue;
    BGK_HIP(hipEventSynchronize(r.b));
    float x = 0.f;
    BGK_HIP(hipEventElapsedTime(&x, r.a, r.b));
    ms += x;
    c += r.cells;
    by += r.bytes;
    ++n;
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = n;
  if (cells) *cells = c;
  if (bytes) *bytes = by;
  return BGK_OK;
}

}  // extern "C"

// Fine kinetic propagator kernels for gfx950 (CDNA4), FP64.
//
// One IMEX step (Section 3.1) is upwind transport in x, moments of the
// transported field, the Maxwellian of those moments and the implicit BGK
// relaxation f = (f* + lambda M[P f*]) / (1 + lambda).  The relaxation only
// needs each x cell's moments, so the kernels store g = f* (the transported,
// not yet relaxed field) and relax it on the fly when it is read by the next
// step ("relax-then-transport"): every step then reads g once and writes it
// once (16 bytes per phase-space update), and the moments are carried between
// steps as deterministic per-wave partial sums.
//
// Layout: g[member][x][v] with the flat velocity index fastest.  A wave owns a
// tile of 64*E velocities (element e of lane l at tile*64E + e*64 + l, so every
// load and store instruction of a wave covers 512 contiguous bytes) and
// marches along a chunk of x cells, keeping rows i-1, i, i+1 in registers;
// only the two halo rows of a chunk are read twice.  The Maxwellian is
// separable, M = C Ex(v_x) Ey(v_y) Ez(v_z), so a step needs 3 Nv exponentials
// per x cell (computed once per cell by the reduce kernel) and a workgroup
// stages the factor rows of its chunk in LDS.
#include "bgk_internal.h"

#include <type_traits>

namespace bgk {

// ------------------------------------------------------------- helpers --


__device__ __forceinline__ int ghost_row(int i, int nx, int bc) {
  if (i < 0) return bc == 1 ? i + nx : 0;
  if (i >= nx) return bc == 1 ? i - nx : nx - 1;
  return i;
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_mov(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xf, true);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xf, true);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave; the total is valid in lane 63.  Fixed
// combination order, so results are bitwise reproducible.
__device__ __forceinline__ double wave_sum_to_last(double v) {
  v += dpp_mov<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov<0x114, 0xf>(v);  // row_shr:4
  v += dpp_mov<0x118, 0xf>(v);  // row_shr:8   -> lane 15 of each row
  v += dpp_mov<0x142, 0xa>(v);  // row_bcast:15 into rows 1, 3
  v += dpp_mov<0x143, 0xc>(v);  // row_bcast:31 into rows 2, 3
  return v;
}

// A wave-uniform double moved to scalar registers.
__device__ __forceinline__ double uniform_d(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum_all(double v) {
  return readlane_d(wave_sum_to_last(v), kWave - 1);
}

// Instance of a work item: the last entry whose item_begin is <= item
// (binary search; entries are in item order).  A launch may take a table
// that starts inside a batch (its first entry's item_begin > 0): the kernels
// add that offset to their block's item before the search.
__device__ __forceinline__ int find_inst(const Inst* insts, int n_inst,
                                         long long item) {
  int lo = 0, hi = n_inst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (insts[mid].item_begin <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Work item -> (member b, tile group tg, x chunk c), tile groups fastest, so
// the blocks that run together on one XCD cover whole rows of a few x chunks
// (a compact address window; shared halo rows stay in that XCD's L2).
__device__ __forceinline__ void decode_item(const Inst& I, long long local, int& b, int& tg,
                                            int& c) {
  tg = (int)(local % I.ntg);
  const long long t = local / I.ntg;
  c = (int)(t % I.nchunks);
  b = (int)(t / I.nchunks);
}

__device__ __forceinline__ double vgrid(const Inst& I, int a, int j) {
  return I.vlo[a] + (j + 0.5) * I.dv[a];
}

// Per-lane velocity elements of one tile.
template <int E>
struct Elems {
  unsigned off[E];  // LDS factor offsets: ox | oy << 10 | oz << 20
  double vx[E], vy[E], vz[E];
  bool ok[E];
};

template <int E>
__device__ __forceinline__ void setup_elems(const Inst& I, int tile, int lane,
                                            Elems<E>& el) {
  const int nyz = I.nvy * I.nvz;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    int j = tile * (kWave * E) + e * kWave + lane;
    el.ok[e] = j < I.nv3;
    int jj = el.ok[e] ? j : 0;
    int jx = jj / nyz;
    int rem = jj - jx * nyz;
    int jy = rem / I.nvz;
    int jz = rem - jy * I.nvz;
    el.off[e] = (unsigned)jx | ((unsigned)(I.nvx + jy) << 10) |
                ((unsigned)(I.nvx + I.nvy + jz) << 20);
    el.vx[e] = vgrid(I, 0, jx);
    el.vy[e] = vgrid(I, 1, jy);
    el.vz[e] = vgrid(I, 2, jz);
  }
}

__device__ __forceinline__ double fac3(const double* row, unsigned off) {
  return row[off & 1023u] * row[(off >> 10) & 1023u] * row[off >> 20];
}

// ------------------------------------------------ lane reductions --
// Lane exchanges without the LDS pipe (no LDS-counter waits on the row loop's
// critical path).  Partner lane ^ (1 << STAGE) for bits 0-3 by DPP: quad
// permutations for bits 0-1; for bit 2 a row shift by 4 (right in lanes with
// bit 2 set, left in the others); for bit 3 a rotation by 8 inside the row of
// 16.  Bits 4 and 5 only ever enter sums, v + partner(v): the gfx950 permlane
// swaps with both operands v leave a lane's own value in one result and its
// partner's in the other, so the sum of the two results is that sum.
template <int STAGE>
__device__ __forceinline__ double xor_lane(double v, int lane) {
  static_assert(STAGE >= 0 && STAGE <= 3, "bits 4 and 5: sum_across");
  if (STAGE == 0) return dpp_mov<0xb1, 0xf>(v);  // quad_perm [1,0,3,2]
  if (STAGE == 1) return dpp_mov<0x4e, 0xf>(v);  // quad_perm [2,3,0,1]
  if (STAGE == 2) {
    const double from_below = dpp_mov<0x114, 0xf>(v);  // row_shr:4: lane - 4
    const double from_above = dpp_mov<0x104, 0xf>(v);  // row_shl:4: lane + 4
    return (lane & 4) ? from_below : from_above;
  }
  return dpp_mov<0x128, 0xf>(v);  // row_ror:8: lane ^ 8 inside the row
}

// v plus the value of partner lane ^ (1 << STAGE), every lane.
template <int STAGE>
__device__ __forceinline__ double sum_across(double v, int lane) {
  if constexpr (STAGE <= 3) {
    return v + xor_lane<STAGE>(v, lane);
  } else {
    const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
    if constexpr (STAGE == 4) {
      const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
      const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
      return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
    } else {
      const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
      const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
      return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
    }
  }
}

// One reduce-scatter stage: the lanes split by bit STAGE; each keeps one half
// of its H*2 running sums (the half its partner does not keep), adds the
// partner's copy of that half, and drops the other.
template <int STAGE, int H, int N>
__device__ __forceinline__ void scatter_stage(double (&s)[N], int lane) {
  const bool upper = (lane >> STAGE) & 1;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const double send = upper ? s[i] : s[i + H];
    const double keep = upper ? s[i + H] : s[i];
    s[i] = keep + xor_lane<STAGE>(send, lane);
  }
}

// Sums of 16 values over the 64 lanes of a wave by reduce-scatter: 17 lane
// exchanges instead of 16 x 6.  Returns this lane's total of value
// index 8 b0 + 4 b1 + 2 b2 + b3 (b = bits of the lane id); lanes 0..15 hold
// all 16 totals.  Fixed combination order: bitwise reproducible.
__device__ __forceinline__ double wave_reduce_scatter16(double (&s)[16], int lane) {
  scatter_stage<0, 8>(s, lane);
  scatter_stage<1, 4>(s, lane);
  scatter_stage<2, 2>(s, lane);
  scatter_stage<3, 1>(s, lane);
  s[0] = sum_across<4>(s[0], lane);
  s[0] = sum_across<5>(s[0], lane);
  return s[0];
}

__device__ __forceinline__ int scatter16_index(int lane) {
  return 8 * (lane & 1) + 4 * ((lane >> 1) & 1) + 2 * ((lane >> 2) & 1) + ((lane >> 3) & 1);
}

// Lane holding total c after wave_reduce_scatter16 (the 4-bit reversal).
__device__ __forceinline__ constexpr int lane_of_slot16(int c) {
  return ((c & 1) << 3) | ((c & 2) << 1) | ((c & 4) >> 1) | ((c & 8) >> 3);
}

// Sums of N values over the 64 lanes, every total returned to every lane:
// reduce-scatter in groups of 16 (17 lane exchanges per group instead of 96),
// then each total read from the lane that holds it.  Fixed order: bitwise
// reproducible.
template <int N>
__device__ __forceinline__ void wave_sum_all_n(double (&v)[N], int lane) {
#pragma unroll
  for (int g = 0; g < N; g += 16) {
    double t[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) t[c] = g + c < N ? v[g + c] : 0.0;
    const double tot = wave_reduce_scatter16(t, lane);
#pragma unroll
    for (int c = 0; c < 16; ++c)
      if (g + c < N) v[g + c] = readlane_d(tot, lane_of_slot16(c));
  }
}

// Per-pair velocity data of one lane: |v|^2 of both velocities of the pair
// and nu = v_x dt/dx held in registers.
template <int P>
struct PairEls {
  int jofs[P];
  unsigned off[P];
  double vx[P], vy[P], vz[P];
  double q0_[P], q1_[P], nu_[P];
  double r, dvz;
  bool ok[P];
  __device__ __forceinline__ double q0(int p) const { return q0_[p]; }
  __device__ __forceinline__ double q1(int p) const { return q1_[p]; }
  __device__ __forceinline__ double nu(int p) const { return nu_[p]; }
};

// Velocity data of a lane's pairs and their offsets into a factor row laid
// out as [Ex | Ey | Ez]; jx_base and row_nx describe a row holding only the
// Ex values of v_x planes jx_base .. jx_base + row_nx - 1 (defaults: all).
template <int P, bool FULL>
__device__ __forceinline__ void setup_pairs(const Inst& I, int tile, int lane,
                                            PairEls<P>& e, int jx_base = 0,
                                            int row_nx = -1) {
  const int nyz = I.nvy * I.nvz;
  if (row_nx < 0) row_nx = I.nvx;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int j = tile * (128 * P) + p * 128 + 2 * lane;
    e.ok[p] = FULL || j < I.nv3;
    const int jj = e.ok[p] ? j : 0;
    e.jofs[p] = jj;
    const int jx = jj / nyz;
    const int rem = jj - jx * nyz;
    const int jy = rem / I.nvz;
    const int jz = rem - jy * I.nvz;
    e.off[p] = (unsigned)(jx - jx_base) | ((unsigned)(row_nx + jy) << 10) |
               ((unsigned)(row_nx + I.nvy + jz) << 20);
    e.vx[p] = vgrid(I, 0, jx);
    e.vy[p] = vgrid(I, 1, jy);
    e.vz[p] = vgrid(I, 2, jz);
    const double vxy = e.vx[p] * e.vx[p] + e.vy[p] * e.vy[p];
    e.q0_[p] = vxy + e.vz[p] * e.vz[p];
    const double vz1 = vgrid(I, 2, jz + 1);
    e.q1_[p] = vxy + vz1 * vz1;
    e.nu_[p] = e.vx[p] * I.r;
  }
  e.r = I.r;
  e.dvz = I.dv[2];
}

// Readlane of a double from a uniform lane.
__device__ __forceinline__ double bcast_lane(double v, int lane) {
  return readlane_d(v, lane);
}

// Sums of NSLOT (4, 8 or 16) values over the 64 lanes by reduce-scatter;
// returns this lane's total, of value index slot_of_lane<NSLOT>(lane).
template <int NSLOT>
__device__ __forceinline__ double wave_reduce_scatter(double (&s)[NSLOT], int lane) {
  if (NSLOT >= 16) scatter_stage<0, 8>(s, lane);
  if (NSLOT >= 8) scatter_stage<(NSLOT >= 16 ? 1 : 0), 4>(s, lane);
  scatter_stage<(NSLOT >= 16 ? 2 : (NSLOT >= 8 ? 1 : 0)), 2>(s, lane);
  scatter_stage<(NSLOT >= 16 ? 3 : (NSLOT >= 8 ? 2 : 1)), 1>(s, lane);
  // remaining lane bits: plain sums of the one value each lane holds
  if (NSLOT <= 8) s[0] = sum_across<(NSLOT >= 8 ? 3 : 2)>(s[0], lane);
  if (NSLOT <= 4) s[0] = sum_across<3>(s[0], lane);
  s[0] = sum_across<4>(s[0], lane);
  s[0] = sum_across<5>(s[0], lane);
  return s[0];
}

template <int NSLOT>
__device__ __forceinline__ int slot_of_lane(int lane) {
  if (NSLOT == 16) return scatter16_index(lane);
  if (NSLOT == 8) return 4 * (lane & 1) + 2 * ((lane >> 1) & 1) + ((lane >> 2) & 1);
  return 2 * (lane & 1) + ((lane >> 1) & 1);
}

// Lane holding slot k after a 4-slot reduce-scatter.
__device__ __forceinline__ constexpr int lane_of_slot4(int k) {
  return (k >> 1) | ((k & 1) << 1);
}

// ---------------------------------------------------- fused step kernel --
// Work item = (instance, member b, tile group, x chunk); the waves of a block
// share the chunk (and its LDS factor rows) and take consecutive tiles.
// FORCE: the step also transports in v_x under the exterior force E_i of the
// x cell (Rusanov flux, coefficient emax, no flux through the ends of the v_x
// range).  A lane's v_x neighbours lie nvy*nvz elements away in the same x
// row; they are read directly (other waves of the block or nearby blocks
// read them as their own centre values, so they mostly hit L2) and relaxed
// with the factor of the neighbouring v_x point.
// LIMITED: second order in x, the upwind flux with the Lax-Wendroff
// correction limited by van Leer's limiter (five-point stencil, so the march
// keeps rows i-2 .. i+2 and the ghost cells are two deep).
// Harmonic-mean slope 2ab/(a+b) of van Leer's limiter, 0 where a b <= 0.
// The quotient takes the hardware reciprocal of s = a+b refined by one
// Newton-Raphson step r <- r + r(1 - s r), then one residual correction of
// the quotient q <- q + r(n - s q), at fewer instructions than the division
// (the second-order step is VALU-bound).  Measured on gfx950 against the
// rounded division on 4M random same-sign pairs spread over 60 binades:
// identical in every case (a second Newton step changes nothing; with none,
// 43 % differ by up to 19 ulp).  s != 0 where the value is used (a b > 0
// means a and b have one sign).
__device__ __forceinline__ double vl_limited(double a, double b) {
  const double p = a * b;
  const double s = a + b;
  double r = __builtin_amdgcn_rcp(s);
  r = fma(r, fma(-s, r, 1.0), r);
  const double n = 2.0 * p;
  double q = n * r;
  q = fma(r, fma(-s, q, n), q);
  return p > 0.0 ? q : 0.0;
}

// Limited flux through the face between f0 (cell i) and fp (cell i+1): the
// upwind value plus the limited correction taken on the upwind side, one
// limiter per face (pos: v_x > 0; anu = |nu|).  For v_x < 0 the factor
// -(1 - |nu|)/2 equals -(1 + nu)/2 exactly.
__device__ __forceinline__ double flux2(double vx, double anu, double fm, double f0,
                                        double fp, double fp2) {
  const bool pos = vx > 0.0;
  const double up = pos ? f0 : fp;
  const double d1 = pos ? f0 - fm : fp2 - fp;
  const double h = 0.5 * (1.0 - anu);
  const double c = pos ? h : -h;
  return vx * (up + c * vl_limited(d1, fp - f0));
}

// flux2 with the sign of v_x known (SGN = +1: v_x > 0, -1: v_x <= 0) for a
// whole tile, so the upwind side needs no selects; SGN = 0 decides per
// velocity.
template <int SGN>
__device__ __forceinline__ double flux2s(double vx, double anu, double fm, double f0,
                                         double fp, double fp2) {
  if (SGN == 0) return flux2(vx, anu, fm, f0, fp, fp2);
  const double up = SGN > 0 ? f0 : fp;
  const double d1 = SGN > 0 ? f0 - fm : fp2 - fp;
  const double h = 0.5 * (1.0 - anu);
  return vx * (up + (SGN > 0 ? h : -h) * vl_limited(d1, fp - f0));
}

// NS = 15: the records also carry the nu+ and nu- weighted sums (fused
// passes on grids without paired rows; plain step only).  UNI (the limited
// step without force): every tile lies in one v_x plane, so v_x and nu are
// the wave's, the upwind side is uniform, and the record is compact (sum g,
// sum v_y g, sum v_z g, sum |v|^2 g; the reduction rebuilds sum v_x g).
template <int E, int MODE, bool FORCE = false, bool LIMITED = false, int NS = 5,
          bool UNI = false>
__global__ __launch_bounds__(kBlock) void k_step(const Inst* __restrict__ insts,
                                                 int n_inst, int chunk,
                                                 int phase) {
  constexpr int H = LIMITED ? 2 : 1;  // stencil half-width in x
  extern __shared__ double lds[];
  const long long item = xcd_item(blockIdx.x, gridDim.x) + insts[0].item_begin;
  const int q = find_inst(insts, n_inst, item);
  const Inst& I = insts[q];
  const long long local = item - I.item_begin;
  int b, tg, c;
  decode_item(I, local, b, tg, c);
  const int nx = I.nx, nv3 = I.nv3, nvs = I.nvs;
  const int i0 = c * chunk;
  const int i1 = min(i0 + chunk, nx);
  const int rbase = i0 - H;  // first staged factor row

  if (MODE != kCopy) {
    // factor rows of cells i0-H .. i1+H-1 (ghosts mapped by the BC)
    const int rows = i1 - i0 + 2 * H;
    gptr<const double> fac = gmem(I.fac) + (long long)b * nx * nvs;
    for (int idx = threadIdx.x; idx < rows * nvs; idx += kBlock) {
      int rr = idx / nvs;
      int k = idx - rr * nvs;
      lds[idx] = fac[(long long)ghost_row(rbase + rr, nx, I.bc) * nvs + k];
    }
    __syncthreads();
  }

  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int tile = tg * kWavesPerBlock + wave;
  if (tile >= I.ntiles) return;

  Elems<E> el;
  setup_elems<E>(I, tile, lane, el);
  const long long mbase = (long long)b * nx * nv3;
  gptr<const double> src = gmem((MODE == kCopy) ? I.fin : I.buf[phase]);
  gptr<double> dst = gmem(I.buf[phase ^ 1]);
  src += mbase + tile * (kWave * E) + lane;
  dst += mbase + tile * (kWave * E) + lane;
  const double a = I.a;
  static_assert(!UNI || (LIMITED && !FORCE && NS == 5), "uniform tiles: limited step only");
  double nu[E], vsq[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    nu[e] = el.vx[e] * I.r;
    vsq[e] = el.vx[e] * el.vx[e] + el.vy[e] * el.vy[e] + el.vz[e] * el.vz[e];
  }
  // the tile's v_x and nu (UNI)
  const double vxu = UNI ? uniform_d(vgrid(I, 0, (tile * kWave * E) / (I.nvy * I.nvz))) : 0.0;
  const double nuu = vxu * I.r;

  // relaxed value of row r (global row index, ghost-mapped) from raw g
  // (UNI tiles are whole, a v_x plane holding whole tiles, and share one Ex
  // factor per row)
  auto relax_row = [&](int r, const double* raw, double* out) {
    const double* frow = lds + (r - rbase) * nvs;
    const double mxu = (UNI && MODE != kCopy) ? frow[el.off[0] & 1023u] : 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const double m = UNI ? mxu * frow[(el.off[e] >> 10) & 1023u] * frow[el.off[e] >> 20]
                           : fac3(frow, el.off[e]);
      double v;
      if (MODE == kCopy) v = raw[e];
      else if (MODE == kRelax) v = fma(a, raw[e], m);
      else v = m;
      out[e] = (UNI || el.ok[e]) ? v : 0.0;
    }
  };
  auto load_row = [&](int r, double* raw) {
    if (MODE == kLift) return;
    const long long ro = (long long)ghost_row(r, nx, I.bc) * nv3;
#pragma unroll
    for (int e = 0; e < E; ++e) raw[e] = (UNI || el.ok[e]) ? src[ro + e * kWave] : 0.0;
  };

  // relaxed rows i-H .. i+H of the march; raw row i+H (rawp) and i+H+1 (rawn)
  double w[2 * H + 1][E], rawp[E], rawn[E];
#pragma unroll
  for (int e = 0; e < E; ++e) rawn[e] = 0.0;
#pragma unroll
  for (int k = 0; k < 2 * H; ++k) {
    double raw[E];
    load_row(i0 - H + k, raw);
    relax_row(i0 - H + k, raw, w[k]);
  }
  load_row(i0 + H, rawp);
  // FORCE: raw values at the v_x neighbours (dn: -nyz, up: +nyz) of each
  // element, loaded one row ahead of their use; relaxed with the factor of
  // the neighbouring v_x point (the Ex index is the low field of off)
  const int nyz = I.nvy * I.nvz;
  double dn_cur[FORCE ? E : 1], up_cur[FORCE ? E : 1];
  double dn_nxt[FORCE ? E : 1], up_nxt[FORCE ? E : 1];
  auto load_vnb = [&](int r, double* dn, double* up) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int jx = (int)(el.off[e] & 1023u);
      const long long o = (long long)r * nv3 + e * kWave;
      dn[e] = (MODE != kLift && el.ok[e] && jx > 0) ? src[o - nyz] : 0.0;
      up[e] = (MODE != kLift && el.ok[e] && jx + 1 < I.nvx) ? src[o + nyz] : 0.0;
    }
  };
  auto relax_vnb = [&](int r, int e, int dir, double raw) -> double {
    const double* frow = lds + (r - rbase) * nvs;
    const unsigned off = el.off[e] + (unsigned)dir;
    if (MODE == kCopy) return raw;
    if (MODE == kRelax) return fma(a, raw, fac3(frow, off));
    return fac3(frow, off);
  };
  if (FORCE) load_vnb(i0, dn_cur, up_cur);
  // LIMITED: flux through the left face of the current row, carried over
  // from the right face of the previous one (computed once per face)
  double fcar[LIMITED ? E : 1];
  if (LIMITED) {
#pragma unroll
    for (int e = 0; e < E; ++e)
      fcar[e] = flux2(UNI ? vxu : el.vx[e], fabs(UNI ? nuu : nu[e]), w[0][e], w[1][e], w[2][e],
                      w[3 < 2 * H ? 3 : 0][e]);
  }
  static_assert(NS == 5 || (NS == 15 && !FORCE && !LIMITED), "weighted sums: plain step");
  gptr<double> part = gmem(I.part) + ((long long)b * nx) * I.part_tiles * 5 + (long long)tile * NS;
  // one output row; SG: the tile's sign of v_x (UNI), else 0 (per velocity)
  auto row = [&](int i, auto sg) {
    constexpr int SG = decltype(sg)::value;
    if (i + 2 <= i1) load_row(i + H + 1, rawn);  // prefetch the next row
    if (FORCE && i + 1 < i1) load_vnb(i + 1, dn_nxt, up_nxt);
    relax_row(i + H, rawp, w[2 * H]);
    double Ei = 0.0;
    if (FORCE) Ei = gmem(I.efield)[i];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
    double sw[NS == 15 ? 10 : 1];
#pragma unroll
    for (int c = 0; c < (NS == 15 ? 10 : 1); ++c) sw[c] = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      double gs;
      if (LIMITED) {
        const double fr = flux2s<SG>(UNI ? vxu : el.vx[e], fabs(UNI ? nuu : nu[e]), w[H - 1][e],
                                     w[H][e], w[H + 1][e], w[H + 2 < 2 * H + 1 ? H + 2 : 2 * H][e]);
        gs = w[H][e] - I.r * (fr - fcar[e]);
        fcar[e] = fr;
      } else {
        const double nb = nu[e] > 0.0 ? w[H - 1][e] : w[H + 1][e];
        gs = fma(fabs(nu[e]), nb - w[H][e], w[H][e]);
      }
      if (FORCE && el.ok[e]) {
        const int jx = (int)(el.off[e] & 1023u);
        const double c = w[H][e];
        double g_up = 0.0, g_down = 0.0;
        if (jx + 1 < I.nvx) {
          const double u = relax_vnb(i, e, 1, up_cur[e]);
          g_up = 0.5 * Ei * (c + u) - 0.5 * I.emax * (u - c);
        }
        if (jx > 0) {
          const double d = relax_vnb(i, e, -1, dn_cur[e]);
          g_down = 0.5 * Ei * (d + c) - 0.5 * I.emax * (c - d);
        }
        gs -= I.rv * (g_up - g_down);
      }
      if (UNI || el.ok[e]) dst[(long long)i * nv3 + e * kWave] = gs;
      if (UNI && e == 0) {
        // the sums start from the first velocity's terms (no additions of 0)
        s0 = gs;
        s2 = el.vy[e] * gs;
        s3 = el.vz[e] * gs;
        s4 = vsq[e] * gs;
      } else {
        s0 += gs;
        if (!UNI) s1 = fma(el.vx[e], gs, s1);
        s2 = fma(el.vy[e], gs, s2);
        s3 = fma(el.vz[e], gs, s3);
        s4 = fma(vsq[e], gs, s4);
      }
      if (NS == 15) {
        const double cp = nu[e] > 0.0 ? nu[e] : 0.0, cm = nu[e] < 0.0 ? -nu[e] : 0.0;
        const double m[5] = {gs, el.vx[e] * gs, el.vy[e] * gs, el.vz[e] * gs, vsq[e] * gs};
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          sw[c] = fma(cp, m[c], sw[c]);
          sw[5 + c] = fma(cm, m[c], sw[5 + c]);
        }
      }
    }
    if (NS == 15) {
      // the fifteen sums by reduce-scatter: lanes 0..15 hold the totals
      double t16[16] = {s0, s1, s2, s3, s4};
#pragma unroll
      for (int c = 0; c < 10; ++c) t16[5 + c] = sw[c];
      t16[15] = 0.0;
      const double tot = wave_reduce_scatter<16>(t16, lane);
      const int slot = slot_of_lane<16>(lane);
      if (lane < 16 && slot < 15) part[(long long)i * I.part_tiles * 5 + slot] = tot;
    } else if (UNI) {
      // compact record: the four totals by reduce-scatter (lanes 0..3)
      double t4[4] = {s0, s2, s3, s4};
      const double tot = wave_reduce_scatter<4>(t4, lane);
      gptr<double> crec = gmem(I.part) + ((long long)b * nx + i) * I.part_tiles * 5 + tile * 4;
      if (lane < 4) crec[slot_of_lane<4>(lane)] = tot;
    } else {
      // the wave's five sums by reduce-scatter: lanes 0..7 hold the totals
      double t8[8] = {s0, s1, s2, s3, s4, 0.0, 0.0, 0.0};
      const double tot = wave_reduce_scatter<8>(t8, lane);
      const int slot = slot_of_lane<8>(lane);
      if (lane < 8 && slot < 5) part[(long long)i * I.part_tiles * 5 + slot] = tot;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
#pragma unroll
      for (int k = 0; k < 2 * H; ++k) w[k][e] = w[k + 1][e];
      rawp[e] = rawn[e];
      if (FORCE) {
        dn_cur[e] = dn_nxt[e];
        up_cur[e] = up_nxt[e];
      }
    }
  };
  // the tile's sign of v_x is uniform (UNI): one loop per sign, no
  // per-velocity selects of the upwind side
  if (UNI && vxu > 0.0) {
    for (int i = i0; i < i1; ++i) row(i, std::integral_constant<int, 1>{});
  } else if (UNI) {
    for (int i = i0; i < i1; ++i) row(i, std::integral_constant<int, -1>{});
  } else {
    for (int i = i0; i < i1; ++i) row(i, std::integral_constant<int, 0>{});
  }
}

// ------------------------------------------- paired-velocity step kernel --
// Same step, lanes own pairs of adjacent velocities (v_z and v_z + dv_z, same
// v_x and v_y): 16-byte loads and stores, one transport select, one Ex*Ey
// product and one ds_read2 per pair.  Pair p of lane l covers the flat
// velocities tile*128P + p*128 + 2l + {0,1} (requires even nv_z, so a pair
// never straddles a v_z row, and 16-byte aligned rows).
//
// Moment partials, one record per wave and x cell: the five moment sums
// (NS = 5), joined with NS = 15 by the same sums weighted by nu+ = max(nu,0)
// and nu- = max(-nu,0) (needed to predict the next step's moments, see the
// two-step kernel), reduced over the wave by reduce-scatter.

// Running moment sums of one wave over its tile, for one x cell, and their
// reduction into the partial-sum record of the wave: NS values, the five
// moment sums (1, v_x, v_y, v_z, |v|^2) and, with NS = 15, the same sums
// weighted by nu+ = max(nu,0) and nu- = max(-nu,0), nu = v_x dt/dx.
// UNI: the tile lies in one v_x plane, so v_x and nu are the same for all
// its velocities: the v_x and nu-weighted sums are multiples of the plain
// sum and only four sums need a cross-lane reduction.
template <int NS, bool UNI>
struct Acc {
  static constexpr int N = UNI ? 4 : NS;
  double s[N];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int c = 0; c < N; ++c) s[c] = 0.0;
  }
  __device__ __forceinline__ void add(double2 g, double vx, double vy, double vz,
                                      double dvz, double q0, double q1, double nu) {
    const double gs = g.x + g.y;
    if (UNI) {
      s[0] += gs;
      s[1] = fma(vy, gs, s[1]);
      s[2] = fma(vz, gs, fma(dvz, g.y, s[2]));
      s[3] = fma(q0, g.x, fma(q1, g.y, s[3]));
      return;
    }
    const double m[5] = {gs, vx * gs, vy * gs, fma(vz, gs, dvz * g.y),
                         fma(q0, g.x, q1 * g.y)};
#pragma unroll
    for (int c = 0; c < 5; ++c) s[c] += m[c];
    if (NS == 15) {
      const double cp = nu > 0.0 ? nu : 0.0;
      const double cm = nu < 0.0 ? -nu : 0.0;
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        s[5 + c] = fma(cp, m[c], s[5 + c]);
        s[10 + c] = fma(cm, m[c], s[10 + c]);
      }
    }
  }
  // vxu, nuu: the tile's v_x and nu (used when UNI)
  __device__ __forceinline__ void store(const Inst& I, int b, int r, int tile, int lane,
                                        double vxu, double nuu) {
    gptr<double> rec = gmem(I.part) + ((long long)b * I.nx + r) * I.part_tiles * 5 + tile * NS;
    if (UNI) {
      double t4[4] = {s[0], s[1], s[2], s[3]};
      const double tot = wave_reduce_scatter<4>(t4, lane);
      if (I.crec) {
        // compact record: the four totals; the reduction rebuilds the v_x and
        // nu-weighted sums from the tile's v_x
        gptr<double> crec = gmem(I.part) + ((long long)b * I.nx + r) * I.part_tiles * 5 + tile * 4;
        if (lane < 4) crec[slot_of_lane<4>(lane)] = tot;
        return;
      }
      const double T0 = bcast_lane(tot, lane_of_slot4(0));
      const double T1 = bcast_lane(tot, lane_of_slot4(1));
      const double T2 = bcast_lane(tot, lane_of_slot4(2));
      const double T3 = bcast_lane(tot, lane_of_slot4(3));
      if (lane < NS) {
        const int c = lane % 5, w = lane / 5;
        const double S = c == 0 ? T0 : (c == 1 ? vxu * T0 : (c == 2 ? T1 : (c == 3 ? T2 : T3)));
        const double wt = w == 0 ? 1.0 : (w == 1 ? (nuu > 0.0 ? nuu : 0.0)
                                                  : (nuu < 0.0 ? -nuu : 0.0));
        rec[lane] = wt * S;
      }
      return;
    }
    constexpr int NSLOT = NS <= 8 ? 8 : 16;
    double t[NSLOT];
#pragma unroll
    for (int c = 0; c < NSLOT; ++c) t[c] = c < NS ? s[c] : 0.0;
    const double tot = wave_reduce_scatter<NSLOT>(t, lane);
    const int idx = slot_of_lane<NSLOT>(lane);
    if (lane < NSLOT && idx < NS) rec[idx] = tot;
  }
};

// ----------------------------------------- v_x-column exterior-force step --
// The exterior-force step with lanes owning (v_y, v_z) points and the E
// elements of a lane running along v_x.  The v_x neighbours of every element
// but the first and the last are then in registers, and the two v_x planes
// just outside the tile (its halo planes) are one coalesced load each; the
// factor of element e is (Mx[x0 + e] My[v_y]) Mz[v_z], the same product as
// in the other step kernels, with My and Mz read once per x row.  A lane owns
// PY adjacent (v_y, v_z) points (PY = 2: 16-byte loads and stores; needs an
// even nvy nvz and 16-byte aligned f).  Tile t of an x cell covers the
// (v_y, v_z) points 64 PY (t mod nyzb) + PY lane + {0 .. PY-1} and the v_x
// points x0 + e, x0 = E (t div nyzb), with nyzb = ceil(nvy nvz / (64 PY)).
// The v_x flux through the face between two neighbouring v_x points is
// computed once and used by both (Rusanov flux, no flux through the ends of
// the v_x range).
template <int PY>
struct Col {
  double v[PY];
};

template <int PY>
__device__ __forceinline__ Col<PY> ld_col(gptr<const double> p) {
  Col<PY> c;
  if constexpr (PY == 2) {
    const double2 t = ld2(p);
    c.v[0] = t.x;
    c.v[1] = t.y;
  } else {
    c.v[0] = *p;
  }
  return c;
}

template <int PY>
__device__ __forceinline__ void st_col(gptr<double> p, const Col<PY>& c) {
  if constexpr (PY == 2) {
    st2(p, c.v[0], c.v[1]);
  } else {
    *p = c.v[0];
  }
}

template <int E, int MODE, bool LIMITED, int PY>
__global__ __launch_bounds__(kBlock) void k_step_vcol(const Inst* __restrict__ insts,
                                                      int n_inst, int chunk, int phase) {
  constexpr int H = LIMITED ? 2 : 1;
  extern __shared__ double lds[];
  const long long item = xcd_item(blockIdx.x, gridDim.x) + insts[0].item_begin;
  const int q = find_inst(insts, n_inst, item);
  const Inst& I = insts[q];
  const long long local = item - I.item_begin;
  int b, tg, c;
  decode_item(I, local, b, tg, c);
  const int nx = I.nx, nv3 = I.nv3, nvs = I.nvs;
  const int i0 = c * chunk;
  const int i1 = min(i0 + chunk, nx);
  const int rbase = i0 - H;

  if (MODE != kCopy) {
    const int rows = i1 - i0 + 2 * H;
    gptr<const double> fac = gmem(I.fac) + (long long)b * nx * nvs;
    for (int idx = threadIdx.x; idx < rows * nvs; idx += kBlock) {
      int rr = idx / nvs;
      int k = idx - rr * nvs;
      lds[idx] = fac[(long long)ghost_row(rbase + rr, nx, I.bc) * nvs + k];
    }
    __syncthreads();
  }

  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int tile = __builtin_amdgcn_readfirstlane(tg * kWavesPerBlock + wave);
  if (tile >= I.ntiles) return;

  const int nvx = I.nvx;
  const int nyz = I.nvy * I.nvz;
  const int nyzb = (nyz + kWave * PY - 1) / (kWave * PY);
  const int yz = (tile % nyzb) * (kWave * PY) + PY * lane;
  const int x0 = (tile / nyzb) * E;       // first v_x point of the tile
  const int nel = min(E, nvx - x0);       // v_x points in the tile (wave-uniform)
  const bool ok = yz < nyz;               // PY = 2: nyz even, so yz + 1 < nyz too
  const bool has_dn = x0 > 0;             // v_x plane x0 - 1 exists
  const bool has_up = x0 + E < nvx;       // v_x plane x0 + E exists (nel == E)
  int oy[PY], oz[PY];                     // factor-row offsets
  double vy[PY], vz[PY], vyz2[PY];
#pragma unroll
  for (int p = 0; p < PY; ++p) {
    const int jj = ok ? yz + p : 0;
    const int jy = jj / I.nvz;
    const int jz = jj - jy * I.nvz;
    oy[p] = nvx + jy;
    oz[p] = nvx + I.nvy + jz;
    vy[p] = vgrid(I, 1, jy);
    vz[p] = vgrid(I, 2, jz);
    vyz2[p] = vy[p] * vy[p] + vz[p] * vz[p];
  }
  // v_x, nu of the tile's v_x points: wave-uniform, kept in scalar registers
  double vx[E], nu[E];
  int ox[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    ox[e] = min(x0 + e, nvx - 1);
    vx[e] = uniform_d(vgrid(I, 0, ox[e]));
    nu[e] = uniform_d(vx[e] * I.r);
  }
  const long long mbase = (long long)b * nx * nv3 + (long long)x0 * nyz + yz;
  gptr<const double> src = gmem((MODE == kCopy) ? I.fin : I.buf[phase]) + mbase;
  gptr<double> dst = gmem(I.buf[phase ^ 1]) + mbase;
  const double a = I.a;

  auto relax1 = [&](double raw, double fe) -> double {
    if (MODE == kCopy) return raw;
    if (MODE == kRelax) return fma(a, raw, fe);
    return fe;
  };
  // (values of dead elements, e >= nel or a lane past nvy nvz, are finite
  // and never used: their results are zeroed and their faces carry no flux)
  auto relax_row = [&](int r, const Col<PY>* raw, Col<PY>* out) {
    const double* frow = lds + (r - rbase) * nvs;
    double my[PY], mz[PY];
#pragma unroll
    for (int p = 0; p < PY; ++p) {
      my[p] = (MODE == kCopy) ? 0.0 : frow[oy[p]];
      mz[p] = (MODE == kCopy) ? 0.0 : frow[oz[p]];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const double mx = (MODE == kCopy) ? 0.0 : frow[ox[e]];
#pragma unroll
      for (int p = 0; p < PY; ++p) out[e].v[p] = relax1(raw[e].v[p], mx * my[p] * mz[p]);
    }
  };
  auto load_row = [&](int r, Col<PY>* raw) {
    if (MODE == kLift) return;
    const long long ro = (long long)ghost_row(r, nx, I.bc) * nv3;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (ok && e < nel) raw[e] = ld_col<PY>(src + ro + (long long)e * nyz);
      else
#pragma unroll
        for (int p = 0; p < PY; ++p) raw[e].v[p] = 0.0;
    }
  };
  // raw values of the halo planes of centre row r (loaded one row ahead)
  auto load_halo = [&](int r, Col<PY>& dn, Col<PY>& up) {
    const long long ro = (long long)r * nv3;
#pragma unroll
    for (int p = 0; p < PY; ++p) dn.v[p] = up.v[p] = 0.0;
    if (MODE == kLift || !ok) return;
    if (has_dn) dn = ld_col<PY>(src + ro - nyz);
    if (has_up) up = ld_col<PY>(src + ro + (long long)E * nyz);
  };

  // one raw row in flight: row i+H is relaxed at the top of step i, then the
  // same registers take the load of row i+H+1 (likewise the halo planes)
  Col<PY> w[2 * H + 1][E], rawp[E];
#pragma unroll
  for (int e = 0; e < E; ++e)
#pragma unroll
    for (int p = 0; p < PY; ++p) rawp[e].v[p] = 0.0;
#pragma unroll
  for (int k = 0; k < 2 * H; ++k) {
    Col<PY> raw[E];
    load_row(i0 - H + k, raw);
    relax_row(i0 - H + k, raw, w[k]);
  }
  load_row(i0 + H, rawp);
  Col<PY> dn_raw, up_raw;
  load_halo(i0, dn_raw, up_raw);
  const double hm = 0.5 * I.emax;
  // LIMITED: x flux through the left face of the current row, carried over
  // from the right face of the previous one (computed once per face)
  double fcar[LIMITED ? E : 1][PY];
  if (LIMITED) {
#pragma unroll
    for (int e = 0; e < E; ++e)
#pragma unroll
      for (int p = 0; p < PY; ++p)
        fcar[e][p] = flux2(vx[e], fabs(nu[e]), w[0][e].v[p], w[1][e].v[p], w[2][e].v[p],
                           w[3 < 2 * H ? 3 : 0][e].v[p]);
  }
  gptr<double> part = gmem(I.part) + ((long long)b * nx * I.part_tiles + tile) * 5;
  for (int i = i0; i < i1; ++i) {
    relax_row(i + H, rawp, w[2 * H]);
    if (i + 2 <= i1) load_row(i + H + 1, rawp);  // prefetch the next row
    const double* frow = lds + (i - rbase) * nvs;
    // relaxed halo values of row i (factors of row i), then the next halo loads
    double hd_[PY], hu_[PY];
#pragma unroll
    for (int p = 0; p < PY; ++p) {
      const double myz = (MODE == kCopy) ? 0.0 : frow[oy[p]];
      const double mzz = (MODE == kCopy) ? 0.0 : frow[oz[p]];
      hd_[p] = has_dn ? relax1(dn_raw.v[p], (MODE == kCopy) ? 0.0 : frow[x0 - 1] * myz * mzz)
                     : 0.0;
      hu_[p] = has_up ? relax1(up_raw.v[p], (MODE == kCopy) ? 0.0 : frow[x0 + E] * myz * mzz)
                     : 0.0;
    }
    if (i + 1 < i1) load_halo(i + 1, dn_raw, up_raw);
    const double he = 0.5 * gmem(I.efield)[i];
    // v_x face fluxes (face k lies below element k), carried along the
    // column: each face's flux is computed once
    auto face = [&](double lo, double hi) { return he * (lo + hi) - hm * (hi - lo); };
    double glo[PY];
#pragma unroll
    for (int p = 0; p < PY; ++p) glo[p] = has_dn ? face(hd_[p], w[H][0].v[p]) : 0.0;
    double u0[PY], t1 = 0.0, t4 = 0.0;
#pragma unroll
    for (int p = 0; p < PY; ++p) u0[p] = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const bool live = ok && e < nel;
      Col<PY> out;
#pragma unroll
      for (int p = 0; p < PY; ++p) {
        double gs;
        if (LIMITED) {
          const int hp2 = H + 2 < 2 * H + 1 ? H + 2 : 2 * H;
          const double fr = flux2(vx[e], fabs(nu[e]), w[H - 1][e].v[p], w[H][e].v[p],
                                  w[H + 1][e].v[p], w[hp2][e].v[p]);
          gs = w[H][e].v[p] - I.r * (fr - fcar[e][p]);
          fcar[e][p] = fr;
        } else {
          const double nb = nu[e] > 0.0 ? w[H - 1][e].v[p] : w[H + 1][e].v[p];
          gs = fma(fabs(nu[e]), nb - w[H][e].v[p], w[H][e].v[p]);
        }
        double ghi;
        if (e + 1 < E) ghi = (e + 1 < nel) ? face(w[H][e].v[p], w[H][e + 1].v[p]) : 0.0;
        else ghi = has_up ? face(w[H][E - 1].v[p], hu_[p]) : 0.0;
        gs -= I.rv * (ghi - glo[p]);
        glo[p] = ghi;
        gs = live ? gs : 0.0;
        out.v[p] = gs;
        u0[p] += gs;
        t1 = fma(vx[e], gs, t1);
        t4 = fma(vx[e] * vx[e], gs, t4);
      }
      if (live) st_col<PY>(dst + (long long)i * nv3 + (long long)e * nyz, out);
    }
    double t0 = 0.0, t2 = 0.0, t3 = 0.0;
#pragma unroll
    for (int p = 0; p < PY; ++p) {
      t0 += u0[p];
      t2 = fma(vy[p], u0[p], t2);
      t3 = fma(vz[p], u0[p], t3);
      t4 = fma(vyz2[p], u0[p], t4);
    }
    // the wave's five sums by reduce-scatter: lanes 0..7 hold the totals
    double t8[8] = {t0, t1, t2, t3, t4, 0.0, 0.0, 0.0};
    const double tot = wave_reduce_scatter<8>(t8, lane);
    const int slot = slot_of_lane<8>(lane);
    if (lane < 8 && slot < 5) part[(long long)i * I.part_tiles * 5 + slot] = tot;
#pragma unroll
    for (int e = 0; e < E; ++e)
#pragma unroll
      for (int k = 0; k < 2 * H; ++k) w[k][e] = w[k + 1][e];
  }
}

// Non-temporal store of a pair of g (streamed once, read back only by the
// next pass).
__device__ __forceinline__ void store_pair(gptr<double> drow, int jofs, double2 g) {
  __builtin_nontemporal_store(g.x, drow + jofs);
  __builtin_nontemporal_store(g.y, drow + jofs + 1);
}

// One upwind transport of a pair: centre c, its neighbours behind (march
// position k-1) and ahead (k+1).  The upwind cell is x-1 for v_x > 0.
// SGN != 0: the sign of nu is known (uniform over the wave), no select.
template <int DIR, int SGN>
__device__ __forceinline__ double2 transport_pair(double nu, double2 behind,
                                                  double2 c, double2 ahead) {
  const bool take_behind = SGN != 0 ? ((SGN > 0) == (DIR > 0)) : ((nu > 0.0) == (DIR > 0));
  const double cn = fabs(nu);
  const double2 nb = take_behind ? behind : ahead;
  double2 g;
  g.x = fma(cn, nb.x - c.x, c.x);
  g.y = fma(cn, nb.y - c.y, c.y);
  return g;
}

// Relaxed pair from raw g (or the Maxwellian alone in lift mode) with the
// factor row `fr` (al*C*Ex | Ey | Ez, or C*Ex | Ey | Ez for the lift).
template <int MODE>
__device__ __forceinline__ double2 relax_pair(const double* fr, unsigned o,
                                              double a, double2 raw) {
  if (MODE == kCopy) return raw;
  const double fxy = fr[o & 1023u] * fr[(o >> 10) & 1023u];
  const double* fz = fr + (o >> 20);
  const double m0 = fxy * fz[0], m1 = fxy * fz[1];
  double2 v;
  if (MODE == kRelax) {
    v.x = fma(a, raw.x, m0);
    v.y = fma(a, raw.y, m1);
  } else {
    v.x = m0;
    v.y = m1;
  }
  return v;
}

// Tile classes of the paired kernels: a full tile inside one v_x plane with
// nu > 0 or nu < 0 (uniform fast path), a full mixed tile, a ragged tile.
enum TileCase : int { kTilePos = 0, kTileNeg = 1, kTileMixed = 2, kTileRagged = 3 };

__device__ __forceinline__ int tile_case(const Inst& I, int tile, int P, double* vxu,
                                         double* nuu) {
  const int t0 = tile * 128 * P;
  const int t1 = t0 + 128 * P;  // exclusive
  const int nyz = I.nvy * I.nvz;
  const int jx = t0 / nyz;
  *vxu = vgrid(I, 0, jx);
  *nuu = *vxu * I.r;
  if (t1 > I.nv3) return kTileRagged;
  if ((t1 - 1) / nyz != jx) return kTileMixed;
  return *nuu > 0.0 ? kTilePos : kTileNeg;
}

// DIR = +1 marches the chunk's x cells upward, -1 downward.  Neighbouring
// chunks march in opposite directions, so the two halo rows they share are
// read by both blocks at nearly the same time (both at their start or both at
// their end) and the second read hits L2.
template <int P, int MODE, int CASE, int DIR, int NS>
__device__ __forceinline__ void step2_march(const Inst& I, const double* lds,
                                            int b, int tile, int lane, int i0,
                                            int i1, int phase, double vxu, double nuu) {
  constexpr bool FULL = CASE != kTileRagged;
  constexpr bool UNI = CASE == kTilePos || CASE == kTileNeg;
  constexpr int SGN = CASE == kTilePos ? 1 : (CASE == kTileNeg ? -1 : 0);
  const int nx = I.nx, nv3 = I.nv3, nvs = I.nvs;
  PairEls<P> e;
  setup_pairs<P, FULL>(I, tile, lane, e);
  const double dvz = I.dv[2];
  const long long mbase = (long long)b * nx * nv3;
  gptr<const double> src = gmem((MODE == kCopy) ? I.fin : I.buf[phase]) + mbase;
  gptr<double> dst = gmem(I.buf[phase ^ 1]) + mbase;
  const double a = I.a;
  const int len = i1 - i0;
  // global row of march position k (k = -1 and k = len are the halo rows)
  auto row_at = [&](int k) { return DIR > 0 ? i0 + k : i1 - 1 - k; };
  auto load_row = [&](int r, double2 (&raw)[P]) {
    if (MODE == kLift) return;
    gptr<const double> row = src + (long long)ghost_row(r, nx, I.bc) * nv3;
#pragma unroll
    for (int p = 0; p < P; ++p)
      raw[p] = e.ok[p] ? ld2(row + e.jofs[p])
                       : make_double2(0.0, 0.0);
  };
  auto relax_row = [&](int r, const double2 (&raw)[P], double2 (&out)[P]) {
    const double* fr = lds + (r - (i0 - 1)) * nvs;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      double2 v = relax_pair<MODE>(fr, e.off[p], a, raw[p]);
      if (!FULL && !e.ok[p]) v = make_double2(0.0, 0.0);
      out[p] = v;
    }
  };

  // fb: relaxed row behind (k-1), f0: current (k), fa: ahead (k+1);
  // r1: raw row k+1, r2: raw row k+2 (in flight)
  double2 fb[P], f0[P], fa[P], r1[P], r2[P];
#pragma unroll
  for (int p = 0; p < P; ++p) r2[p] = make_double2(0.0, 0.0);
  {
    double2 t0[P];
    load_row(row_at(-1), t0);
    load_row(row_at(0), r1);
    relax_row(row_at(-1), t0, fb);
    load_row(row_at(1), t0);
    relax_row(row_at(0), r1, f0);
#pragma unroll
    for (int p = 0; p < P; ++p) r1[p] = t0[p];
  }
  for (int k = 0; k < len; ++k) {
    if (k + 2 <= len) load_row(row_at(k + 2), r2);  // prefetch
    relax_row(row_at(k + 1), r1, fa);
    const int r = row_at(k);
    Acc<NS, UNI> acc;
    acc.zero();
    gptr<double> drow = dst + (long long)r * nv3;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const double nu = UNI ? nuu : e.nu(p);
      const double2 g = transport_pair<DIR, SGN>(nu, fb[p], f0[p], fa[p]);
      if (FULL || e.ok[p]) store_pair(drow, e.jofs[p], g);
      acc.add(g, e.vx[p], e.vy[p], e.vz[p], dvz, e.q0(p), e.q1(p), nu);
    }
    acc.store(I, b, r, tile, lane, vxu, nuu);
#pragma unroll
    for (int p = 0; p < P; ++p) {
      fb[p] = f0[p];
      f0[p] = fa[p];
      r1[p] = r2[p];
    }
  }
}

__device__ __forceinline__ void stage_rows(const Inst& I, const double* fac, int b,
                                           int first_row, int rows, double* lds) {
  const int nx = I.nx, nvs = I.nvs;
  gptr<const double> f = gmem(fac) + (long long)b * nx * nvs;
  for (int idx = threadIdx.x; idx < rows * nvs; idx += kBlock) {
    int rr = idx / nvs;
    int k = idx - rr * nvs;
    lds[idx] = f[(long long)ghost_row(first_row + rr, nx, I.bc) * nvs + k];
  }
}

// Dispatch of a march over the tile class and march direction.
#define BGK_MARCH_DISPATCH(CALL, ...)                                            \
  do {                                                                           \
    const int tc_ = tile_case(I, tile, P, &vxu, &nuu);                           \
    if (c & 1) {                                                                 \
      if (tc_ == kTilePos) CALL::template run<kTilePos, -1>(__VA_ARGS__);        \
      else if (tc_ == kTileNeg) CALL::template run<kTileNeg, -1>(__VA_ARGS__);   \
      else if (tc_ == kTileMixed) CALL::template run<kTileMixed, -1>(__VA_ARGS__); \
      else CALL::template run<kTileRagged, -1>(__VA_ARGS__);                     \
    } else {                                                                     \
      if (tc_ == kTilePos) CALL::template run<kTilePos, 1>(__VA_ARGS__);         \
      else if (tc_ == kTileNeg) CALL::template run<kTileNeg, 1>(__VA_ARGS__);    \
      else if (tc_ == kTileMixed) CALL::template run<kTileMixed, 1>(__VA_ARGS__); \
      else CALL::template run<kTileRagged, 1>(__VA_ARGS__);                      \
    }                                                                            \
  } while (0)

// Variant for grids whose v_x planes are whole multiples of a tile (then
// every tile is uniform in sign): only the two uniform cases are compiled
// into the kernel, whose register budget is then not set by the mixed case.
#define BGK_MARCH_DISPATCH_UNI(CALL, ...)                                        \
  do {                                                                           \
    const int tc_ = tile_case(I, tile, P, &vxu, &nuu);                           \
    if (c & 1) {                                                                 \
      if (tc_ == kTileNeg) CALL::template run<kTileNeg, -1>(__VA_ARGS__);        \
      else CALL::template run<kTilePos, -1>(__VA_ARGS__);                        \
    } else {                                                                     \
      if (tc_ == kTileNeg) CALL::template run<kTileNeg, 1>(__VA_ARGS__);         \
      else CALL::template run<kTilePos, 1>(__VA_ARGS__);                         \
    }                                                                            \
  } while (0)

template <int P, int MODE, int NS>
struct Step2Call {
  template <int CASE, int DIR>
  static __device__ __forceinline__ void run(const Inst& I, const double* lds, int b,
                                             int tile, int lane, int i0, int i1,
                                             int phase, double vxu, double nuu) {
    step2_march<P, MODE, CASE, DIR, NS>(I, lds, b, tile, lane, i0, i1, phase, vxu, nuu);
  }
};

template <int P, int MODE, int NS>
__global__ __launch_bounds__(kBlock) void k_step2(const Inst* __restrict__ insts,
                                                  int n_inst, int chunk,
                                                  int phase) {
  extern __shared__ double lds[];
  const long long item = xcd_item(blockIdx.x, gridDim.x) + insts[0].item_begin;
  const int q = find_inst(insts, n_inst, item);
  const Inst& I = insts[q];
  const long long local = item - I.item_begin;
  int b, tg, c;
  decode_item(I, local, b, tg, c);
  const int i0 = c * chunk;
  const int i1 = min(i0 + chunk, I.nx);
  if (MODE != kCopy) {
    stage_rows(I, I.fac, b, i0 - 1, i1 - i0 + 2, lds);
    __syncthreads();
  }
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int tile = tg * kWavesPerBlock + wave;
  if (tile >= I.ntiles) return;
  double vxu, nuu;
  using Call = Step2Call<P, MODE, NS>;
  BGK_MARCH_DISPATCH(Call, I, lds, b, tile, lane, i0, i1, phase, vxu, nuu);
}

// ------------------------------------------------ two steps in one pass --
// Reads g^m once, writes g^{m+2} once: 8 bytes per phase-space update.
//   f^m     = a g^m + al M[U(g^m)]            (lift: f^0 = M[U0])  -- factors fac
//   g^{m+1} = T f^m                           (in registers)
//   f^{m+1} = a g^{m+1} + al M[U(g^{m+1})]                          -- factors fac2
//   g^{m+2} = T f^{m+1}                       (stored, with 15 weighted sums)
// U(g^{m+1}) is known before the pass: transport is linear, so the moments of
// T f^m at cell i follow from the nu-weighted moment sums of g^m and of
// M[U(g^m)] at cells i-1, i, i+1 (the reduce kernel's kRedW2 mode).
// The march keeps level-1 rows k..k+2 and level-2 rows k-1..k+1.  Level-2
// values outside the domain are ghost copies of the boundary cell (Neumann)
// or the wrapped cell (periodic), exactly as a single step would see them.
// Raw rows in flight in the two-step marches: one on paired lanes (a second
// row spills the 4-pair march: measured 3.3 against 5.3 TB/s on the uneven
// batch's paired instances), three on unpaired lanes, loaded non-temporally
// (3.97 TB/s on the batch's odd-nv_z instances run unpaired, against 3.76
// with one row, 3.92 with two).
constexpr int kRowsInFlight2x = 1;
constexpr int kRowsInFlight2xFlat = 3;

template <int P, int MODE, int CASE, int DIR>
__device__ __forceinline__ void step2x2_march(const Inst& I, const double* lds1,
                                              const double* lds2, int b, int tile,
                                              int lane, int i0, int i1, int phase,
                                              double vxu, double nuu) {
  constexpr int R = kRowsInFlight2x;
  constexpr bool FULL = CASE != kTileRagged;
  constexpr bool UNI = CASE == kTilePos || CASE == kTileNeg;
  constexpr int SGN = CASE == kTilePos ? 1 : (CASE == kTileNeg ? -1 : 0);
  const int nx = I.nx, nv3 = I.nv3, nvs = I.nvs;
  PairEls<P> e;
  setup_pairs<P, FULL>(I, tile, lane, e);
  const double dvz = I.dv[2];
  const long long mbase = (long long)b * nx * nv3;
  gptr<const double> src = gmem(I.buf[phase]) + mbase;
  gptr<double> dst = gmem(I.buf[phase ^ 1]) + mbase;
  const double a = I.a;
  const bool neumann = I.bc == 0;
  const int len = i1 - i0;
  auto row_at = [&](int k) { return DIR > 0 ? i0 + k : i1 - 1 - k; };
  auto outside = [&](int r) { return r < 0 || r >= nx; };
  auto load_row = [&](int r, double2 (&raw)[P]) {
    if (MODE == kLift) return;
    gptr<const double> row = src + (long long)ghost_row(r, nx, I.bc) * nv3;
#pragma unroll
    for (int p = 0; p < P; ++p)
      raw[p] = e.ok[p] ? ld2(row + e.jofs[p])
                       : make_double2(0.0, 0.0);
  };
  // level 1: rows i0-2 .. i1+1 staged in lds1; level 2: rows i0-1 .. i1 in lds2
  auto relax1 = [&](int r, const double2 (&raw)[P], double2 (&out)[P]) {
    const double* fr = lds1 + (r - (i0 - 2)) * nvs;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      double2 v = relax_pair<MODE>(fr, e.off[p], a, raw[p]);
      if (!FULL && !e.ok[p]) v = make_double2(0.0, 0.0);
      out[p] = v;
    }
  };
  auto level2 = [&](int r, const double2 (&b1)[P], const double2 (&c1)[P],
                    const double2 (&a1)[P], double2 (&out)[P]) {
    const double* fr = lds2 + (r - (i0 - 1)) * nvs;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const double nu = UNI ? nuu : e.nu(p);
      const double2 g = transport_pair<DIR, SGN>(nu, b1[p], c1[p], a1[p]);
      double2 v = relax_pair<kRelax>(fr, e.off[p], a, g);
      if (!FULL && !e.ok[p]) v = make_double2(0.0, 0.0);
      out[p] = v;
    }
  };

  double2 f1b[P], f1c[P], f1a[P];  // level 1 at positions k, k+1, k+2
  double2 f2b[P], f2c[P], f2a[P];  // level 2 at positions k-1, k, k+1
  // raw rows in flight: rows k+2 .. k+1+R in R buffers used in turn
  double2 raw[R][P];
  {
    double2 ra[P], rb[P], l0[P], l1[P];
    load_row(row_at(-2), ra);
    load_row(row_at(-1), rb);
    relax1(row_at(-2), ra, l0);        // level 1 at -2
    load_row(row_at(0), ra);
    relax1(row_at(-1), rb, l1);        // level 1 at -1
    load_row(row_at(1), rb);
    relax1(row_at(0), ra, f1b);        // level 1 at 0
#pragma unroll
    for (int j = 0; j < R; ++j)
      if (2 + j <= len + 1) load_row(row_at(2 + j), raw[j]);
    relax1(row_at(1), rb, f1c);        // level 1 at 1
    level2(row_at(-1), l0, l1, f1b, f2b);   // level 2 at -1
    level2(row_at(0), l1, f1b, f1c, f2c);   // level 2 at 0
    if (neumann && outside(row_at(-1))) {
#pragma unroll
      for (int p = 0; p < P; ++p) f2b[p] = f2c[p];
    }
  }
  // output row k; rw holds raw row k+2 and takes the load of row k+2+R
  auto step = [&](int k, double2 (&rw)[P]) {
    relax1(row_at(k + 2), rw, f1a);
    if (k + 2 + R <= len + 1) load_row(row_at(k + 2 + R), rw);  // in flight meanwhile
    level2(row_at(k + 1), f1b, f1c, f1a, f2a);
    if (neumann && outside(row_at(k + 1))) {
#pragma unroll
      for (int p = 0; p < P; ++p) f2a[p] = f2c[p];
    }
    const int r = row_at(k);
    Acc<15, UNI> acc;
    acc.zero();
    gptr<double> drow = dst + (long long)r * nv3;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const double nu = UNI ? nuu : e.nu(p);
      const double2 g = transport_pair<DIR, SGN>(nu, f2b[p], f2c[p], f2a[p]);
      if (FULL || e.ok[p]) store_pair(drow, e.jofs[p], g);
      acc.add(g, e.vx[p], e.vy[p], e.vz[p], dvz, e.q0(p), e.q1(p), nu);
    }
    acc.store(I, b, r, tile, lane, vxu, nuu);
#pragma unroll
    for (int p = 0; p < P; ++p) {
      f1b[p] = f1c[p];
      f1c[p] = f1a[p];
      f2b[p] = f2c[p];
      f2c[p] = f2a[p];
    }
  };
  for (int k = 0; k < len; k += R) {
#pragma unroll
    for (int j = 0; j < R; ++j)
      if (k + j < len) step(k + j, raw[j]);
  }
}

template <int P, int MODE>
struct Step2x2Call {
  template <int CASE, int DIR>
  static __device__ __forceinline__ void run(const Inst& I, const double* lds1,
                                             const double* lds2, int b, int tile,
                                             int lane, int i0, int i1, int phase,
                                             double vxu, double nuu) {
    step2x2_march<P, MODE, CASE, DIR>(I, lds1, lds2, b, tile, lane, i0, i1, phase, vxu,
                                      nuu);
  }
};

template <int P, int MODE, bool UNI_ONLY>
__global__ __launch_bounds__(kBlock) void k_step2x2(const Inst* __restrict__ insts,
                                                    int n_inst, int chunk,
                                                    int phase) {
  extern __shared__ double lds[];
  const long long item = xcd_item(blockIdx.x, gridDim.x) + insts[0].item_begin;
  const int q = find_inst(insts, n_inst, item);
  const Inst& I = insts[q];
  const long long local = item - I.item_begin;
  int b, tg, c;
  decode_item(I, local, b, tg, c);
  const int i0 = c * chunk;
  const int i1 = min(i0 + chunk, I.nx);
  const int len = i1 - i0;
  double* lds1 = lds;
  double* lds2 = lds + (len + 4) * I.nvs;
  stage_rows(I, I.fac, b, i0 - 2, len + 4, lds1);
  stage_rows(I, I.fac2, b, i0 - 1, len + 2, lds2);
  __syncthreads();
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int tile = tg * kWavesPerBlock + wave;
  if (tile >= I.ntiles) return;
  double vxu, nuu;
  using Call = Step2x2Call<P, MODE>;
  if (UNI_ONLY)
    BGK_MARCH_DISPATCH_UNI(Call, I, lds1, lds2, b, tile, lane, i0, i1, phase, vxu, nuu);
  else
    BGK_MARCH_DISPATCH(Call, I, lds1, lds2, b, tile, lane, i0, i1, phase, vxu, nuu);
}

// ------------------------------- two steps per pass, unpaired lanes --
// The two-step pass for grids whose rows cannot be read in 16-byte pairs
// (odd nv_z, or f off 16-byte alignment): E velocities per lane at stride 64 (flat index tile * 64 E +
// e * 64 + lane, one 8-byte access each), as in the one-step kernel.  Same
// levels as the paired march: level 1 at rows k .. k+2 from the factors
// fac, level 2 at rows k-1 .. k+1 from fac2, output row k; every velocity
// has its own v_x, nu and factors.  Records: the fifteen sums per wave.
template <int E, int MODE, int DIR, int R>
__device__ __forceinline__ void step2x2_flat_march(const Inst& I, const double* lds1,
                                                   const double* lds2, int b, int tile,
                                                   int lane, int i0, int i1, int phase) {
  const int nx = I.nx, nv3 = I.nv3, nvs = I.nvs;
  Elems<E> el;
  setup_elems<E>(I, tile, lane, el);
  double nu[E], q[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    nu[e] = el.vx[e] * I.r;
    q[e] = el.vx[e] * el.vx[e] + el.vy[e] * el.vy[e] + el.vz[e] * el.vz[e];
  }
  const long long mbase = (long long)b * nx * nv3 + (long long)tile * (kWave * E) + lane;
  gptr<const double> src = gmem(I.buf[phase]) + mbase;
  gptr<double> dst = gmem(I.buf[phase ^ 1]) + mbase;
  const double a = I.a;
  const bool neumann = I.bc == 0;
  const int len = i1 - i0;
  auto row_at = [&](int k) { return DIR > 0 ? i0 + k : i1 - 1 - k; };
  auto outside = [&](int r) { return r < 0 || r >= nx; };
  auto load_row = [&](int r, double (&raw)[E]) {
    if (MODE == kLift) return;
    gptr<const double> row = src + (long long)ghost_row(r, nx, I.bc) * nv3;
#pragma unroll
    for (int e = 0; e < E; ++e)
      raw[e] = el.ok[e] ? __builtin_nontemporal_load(row + e * kWave) : 0.0;
  };
  // upwind transport of one velocity: centre c, neighbours behind (march
  // position k-1) and ahead (k+1); the upwind cell is x-1 for v_x > 0
  auto transport = [&](int e, double bh, double c, double ah) {
    const double nb = ((nu[e] > 0.0) == (DIR > 0)) ? bh : ah;
    return fma(fabs(nu[e]), nb - c, c);
  };
  // level 1: rows i0-2 .. i1+1 staged in lds1; level 2: rows i0-1 .. i1 in lds2
  auto relax1 = [&](int r, const double (&raw)[E], double (&out)[E]) {
    const double* fr = lds1 + (r - (i0 - 2)) * nvs;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const double m = fac3(fr, el.off[e]);
      const double v = MODE == kRelax ? fma(a, raw[e], m) : m;
      out[e] = el.ok[e] ? v : 0.0;
    }
  };
  auto level2 = [&](int r, const double (&b1)[E], const double (&c1)[E],
                    const double (&a1)[E], double (&out)[E]) {
    const double* fr = lds2 + (r - (i0 - 1)) * nvs;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const double v = fma(a, transport(e, b1[e], c1[e], a1[e]), fac3(fr, el.off[e]));
      out[e] = el.ok[e] ? v : 0.0;
    }
  };
  auto copy = [&](double (&d)[E], const double (&s)[E]) {
#pragma unroll
    for (int e = 0; e < E; ++e) d[e] = s[e];
  };

  double f1b[E], f1c[E], f1a[E];  // level 1 at positions k, k+1, k+2
  double f2b[E], f2c[E], f2a[E];  // level 2 at positions k-1, k, k+1
  // raw rows in flight: rows k+2 .. k+1+R in R buffers used in turn (the
  // loop is unrolled by R, so no buffer is copied while its load is
  // outstanding)
  double raw[R][E];
  {
    double ra[E], rb[E], l0[E], l1[E];
    load_row(row_at(-2), ra);
    load_row(row_at(-1), rb);
    relax1(row_at(-2), ra, l0);       // level 1 at -2
    load_row(row_at(0), ra);
    relax1(row_at(-1), rb, l1);       // level 1 at -1
    load_row(row_at(1), rb);
    relax1(row_at(0), ra, f1b);       // level 1 at 0
#pragma unroll
    for (int j = 0; j < R; ++j)
      if (2 + j <= len + 1) load_row(row_at(2 + j), raw[j]);
    relax1(row_at(1), rb, f1c);       // level 1 at 1
    level2(row_at(-1), l0, l1, f1b, f2b);  // level 2 at -1
    level2(row_at(0), l1, f1b, f1c, f2c);  // level 2 at 0
    if (neumann && outside(row_at(-1))) copy(f2b, f2c);
  }
  // output row k; rw holds raw row k+2 and takes the load of row k+2+R
  auto step = [&](int k, double (&rw)[E]) {
    relax1(row_at(k + 2), rw, f1a);
    if (k + 2 + R <= len + 1) load_row(row_at(k + 2 + R), rw);  // in flight meanwhile
    level2(row_at(k + 1), f1b, f1c, f1a, f2a);
    if (neumann && outside(row_at(k + 1))) copy(f2a, f2c);
    const int r = row_at(k);
    Acc<15, false> acc;
    acc.zero();
    gptr<double> drow = dst + (long long)r * nv3;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const double g = transport(e, f2b[e], f2c[e], f2a[e]);
      if (el.ok[e]) __builtin_nontemporal_store(g, drow + e * kWave);
      // one velocity: the pair accumulation with a zero second member
      acc.add(make_double2(g, 0.0), el.vx[e], el.vy[e], el.vz[e], 0.0, q[e], 0.0, nu[e]);
    }
    acc.store(I, b, r, tile, lane, 0.0, 0.0);
    copy(f1b, f1c);
    copy(f1c, f1a);
    copy(f2b, f2c);
    copy(f2c, f2a);
  };
  for (int k = 0; k < len; k += R) {
#pragma unroll
    for (int j = 0; j < R; ++j)
      if (k + j < len) step(k + j, raw[j]);
  }
}

template <int E, int MODE>
__global__ __launch_bounds__(kBlock) void k_step2x2_flat(const Inst* __restrict__ insts,
                                                         int n_inst, int chunk, int phase) {
  extern __shared__ double lds[];
  const long long item = xcd_item(blockIdx.x, gridDim.x) + insts[0].item_begin;
  const int q = find_inst(insts, n_inst, item);
  const Inst& I = insts[q];
  const long long local = item - I.item_begin;
  int b, tg, c;
  decode_item(I, local, b, tg, c);
  const int i0 = c * chunk;
  const int i1 = min(i0 + chunk, I.nx);
  const int len = i1 - i0;
  double* lds1 = lds;
  double* lds2 = lds + (len + 4) * I.nvs;
  stage_rows(I, I.fac, b, i0 - 2, len + 4, lds1);
  stage_rows(I, I.fac2, b, i0 - 1, len + 2, lds2);
  __syncthreads();
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int tile = tg * kWavesPerBlock + wave;
  if (tile >= I.ntiles) return;
  // neighbouring chunks march in opposite directions (shared halo rows)
  if (c & 1)
    step2x2_flat_march<E, MODE, -1, kRowsInFlight2xFlat>(I, lds1, lds2, b, tile, lane, i0,
                                                         i1, phase);
  else
    step2x2_flat_march<E, MODE, 1, kRowsInFlight2xFlat>(I, lds1, lds2, b, tile, lane, i0,
                                                        i1, phase);
}

// ---------------------------------------------- three steps in one pass --
// Reads g^m once, writes g^{m+3} once: 16/3 bytes per phase-space update.
//   f^m     = a g^m + al M[U(g^m)]           (lift: f^0 = M[U0])  -- factors fac
//   g^{m+1} = T f^m,  f^{m+1} = a g^{m+1} + al M[U(g^{m+1})]         -- fac2
//   g^{m+2} = T f^{m+1},  f^{m+2} = a g^{m+2} + al M[U(g^{m+2})]     -- fac3
//   g^{m+3} = T f^{m+2}                      (stored, with compact records)
// U(g^{m+1}) and U(g^{m+2}) are known before the pass.  Upwind transport is
// T h_i = (1 - nu+ - nu-) h_i + nu+ h_{i-1} + nu- h_{i+1} per velocity, so the
// moments of T h and their nu+ and nu- weighted sums (nu+ nu- = 0) follow
// from the sums of h weighted by 1, nu+, nu-, nu+^2, nu-^2 at cells i-1, i,
// i+1; for h = a g + al M those come from the records of g and from 1-D sums
// of the separable M (reductions kRedW1x3, kRedW2x3, kRedW3x3).  Tiles lie in
// one v_x plane (uniform nu).  The march keeps level-1 rows k+1 .. k+3,
// level-2 rows k .. k+2 and level-3 rows k-1 .. k+1 around output row k;
// level-2 and level-3 values outside the domain are, for Neumann ends, copies
// of the boundary row of the same level (the single step's ghost cells).
// Raw rows in flight in the three-step march.
constexpr int kRowsInFlight3x = 2;

template <int P, int MODE, int CASE, int DIR>
__device__ __forceinline__ void step3x_march(const Inst& I, const double* lds1,
                                             const double* lds2, const double* lds3,
                                             int b, int tile, int lane, int i0, int i1,
                                             int phase, double vxu, double nuu,
                                             int jx_base, int row_nx) {
  constexpr int SGN = CASE == kTilePos ? 1 : -1;
  const int nx = I.nx, nv3 = I.nv3;
  const int nvs = row_nx + I.nvy + I.nvz;  // compact factor rows in LDS
  PairEls<P> e;
  setup_pairs<P, true>(I, tile, lane, e, jx_base, row_nx);
  const double dvz = I.dv[2];
  const long long mbase = (long long)b * nx * nv3;
  gptr<const double> src = gmem(I.buf[phase]) + mbase;
  gptr<double> dst = gmem(I.buf[phase ^ 1]) + mbase;
  const double a = I.a;
  const bool neumann = I.bc == 0;
  const int len = i1 - i0;
  auto row_at = [&](int k) { return DIR > 0 ? i0 + k : i1 - 1 - k; };
  auto outside = [&](int k) {
    const int r = row_at(k);
    return r < 0 || r >= nx;
  };
  // raw rows: non-temporal loads with two pairs per lane (measured on the
  // 64-slice 512 x 32^3 batch: 3.26 against 3.47 ms per pass; with one pair
  // per lane, and in the one- and two-step passes, they are slower)
  auto load_row = [&](int k, double2 (&raw)[P]) {
    if (MODE == kLift) return;
    gptr<const double> row = src + (long long)ghost_row(row_at(k), nx, I.bc) * nv3;
#pragma unroll
    for (int p = 0; p < P; ++p)
      raw[p] = P == 2 ? ld2_nt(row + e.jofs[p]) : ld2(row + e.jofs[p]);
  };
  // level 1 at position k: rows i0-3 .. i1+2 staged in lds1
  auto level1 = [&](int k, const double2 (&raw)[P], double2 (&out)[P]) {
    const double* fr = lds1 + (row_at(k) - (i0 - 3)) * nvs;
#pragma unroll
    for (int p = 0; p < P; ++p) out[p] = relax_pair<MODE>(fr, e.off[p], a, raw[p]);
  };
  // level L+1 at position k from level L at k-1, k, k+1 (lds: the factor
  // rows of level L+1, first row `first`)
  auto next = [&](const double* lds, int first, int k, const double2 (&bh)[P],
                  const double2 (&c)[P], const double2 (&ah)[P], double2 (&out)[P]) {
    const double* fr = lds + (row_at(k) - first) * nvs;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const double2 g = transport_pair<DIR, SGN>(nuu, bh[p], c[p], ah[p]);
      out[p] = relax_pair<kRelax>(fr, e.off[p], a, g);
    }
  };
  auto copy = [&](double2 (&d)[P], const double2 (&s)[P]) {
#pragma unroll
    for (int p = 0; p < P; ++p) d[p] = s[p];
  };

  double2 l1b[P], l1c[P];  // level 1 at positions k+1, k+2
  double2 l2b[P], l2c[P];  // level 2 at k, k+1
  double2 l3b[P], l3c[P];  // level 3 at k-1, k
  // raw rows in flight: rows k+3 .. k+2+R in R buffers used in turn (the loop
  // is unrolled by R, so no buffer is copied while its load is outstanding)
  constexpr int R = kRowsInFlight3x;
  double2 raw[R][P];
  {
    double2 x0[P], x1[P], x2[P], r0[P], r1[P], y0[P], y1[P];
    load_row(-3, r0);
    load_row(-2, r1);
    level1(-3, r0, x0);
    load_row(-1, r0);
    level1(-2, r1, x1);
    load_row(0, r1);
    level1(-1, r0, x2);
    next(lds2, i0 - 2, -2, x0, x1, x2, y0);  // level 2 at -2
    load_row(1, r0);
    level1(0, r1, x0);
    next(lds2, i0 - 2, -1, x1, x2, x0, y1);  // level 2 at -1
    load_row(2, r1);
    level1(1, r0, x1);
    next(lds2, i0 - 2, 0, x2, x0, x1, l2b);  // level 2 at 0
#pragma unroll
    for (int j = 0; j < R; ++j)
      if (3 + j <= len + 2) load_row(3 + j, raw[j]);
    level1(2, r1, x2);
    next(lds2, i0 - 2, 1, x0, x1, x2, l2c);  // level 2 at 1
    if (neumann) {
      // position 0 is inside; outside positions copy their inner neighbour
      if (outside(1)) copy(l2c, l2b);
      if (outside(-1)) copy(y1, l2b);
      if (outside(-2)) copy(y0, y1);
    }
    next(lds3, i0 - 1, -1, y0, y1, l2b, l3b);  // level 3 at -1
    next(lds3, i0 - 1, 0, y1, l2b, l2c, l3c);  // level 3 at 0
    if (neumann && outside(-1)) copy(l3b, l3c);
    copy(l1b, x1);
    copy(l1c, x2);
  }
  // output row k; rw holds row k+3 and takes the load of row k+3+R
  auto step = [&](int k, double2 (&rw)[P]) {
    double2 l1a[P], l2a[P], l3a[P];
    level1(k + 3, rw, l1a);
    if (k + 3 + R <= len + 2) load_row(k + 3 + R, rw);  // in flight meanwhile
    next(lds2, i0 - 2, k + 2, l1b, l1c, l1a, l2a);
    if (neumann && outside(k + 2)) copy(l2a, l2c);
    next(lds3, i0 - 1, k + 1, l2b, l2c, l2a, l3a);
    if (neumann && outside(k + 1)) copy(l3a, l3c);
    const int r = row_at(k);
    Acc<15, true> acc;
    acc.zero();
    gptr<double> drow = dst + (long long)r * nv3;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const double2 g = transport_pair<DIR, SGN>(nuu, l3b[p], l3c[p], l3a[p]);
      store_pair(drow, e.jofs[p], g);
      acc.add(g, e.vx[p], e.vy[p], e.vz[p], dvz, e.q0(p), e.q1(p), nuu);
    }
    acc.store(I, b, r, tile, lane, vxu, nuu);
    copy(l1b, l1c);
    copy(l1c, l1a);
    copy(l2b, l2c);
    copy(l2c, l2a);
    copy(l3b, l3c);
    copy(l3c, l3a);
  };
  for (int k = 0; k < len; k += R) {
#pragma unroll
    for (int j = 0; j < R; ++j)
      if (k + j < len) step(k + j, raw[j]);
  }
}

template <int P, int MODE>
struct Step3xCall {
  template <int CASE, int DIR>
  static __device__ __forceinline__ void run(const Inst& I, const double* lds1,
                                             const double* lds2, const double* lds3, int b,
                                             int tile, int lane, int i0, int i1, int phase,
                                             double vxu, double nuu, int jx_base,
                                             int row_nx) {
    step3x_march<P, MODE, CASE, DIR>(I, lds1, lds2, lds3, b, tile, lane, i0, i1, phase,
                                     vxu, nuu, jx_base, row_nx);
  }
};

// Factor rows of `rows` x cells from first_row on, keeping of Ex only the
// v_x planes jx_base .. jx_base + row_nx - 1 (the planes the block's tiles
// lie in): [Ex(jx_base ..) | Ey | Ez], row_nx + nvy + nvz values per row.
__device__ __forceinline__ void stage_rows_compact(const Inst& I, const double* fac, int b,
                                                   int first_row, int rows, int jx_base,
                                                   int row_nx, double* lds) {
  const int nx = I.nx, nvs = I.nvs;
  const int rl = row_nx + I.nvy + I.nvz;
  gptr<const double> f = gmem(fac) + (long long)b * nx * nvs;
  for (int idx = threadIdx.x; idx < rows * rl; idx += kBlock) {
    const int rr = idx / rl;
    const int k = idx - rr * rl;
    const int src = k < row_nx ? jx_base + k : I.nvx + (k - row_nx);
    lds[idx] = f[(long long)ghost_row(first_row + rr, nx, I.bc) * nvs + src];
  }
}

template <int P, int MODE>
__global__ __launch_bounds__(kBlock) void k_step3x(const Inst* __restrict__ insts,
                                                   int n_inst, int chunk, int phase) {
  extern __shared__ double lds[];
  const long long item = xcd_item(blockIdx.x, gridDim.x) + insts[0].item_begin;
  const int q = find_inst(insts, n_inst, item);
  const Inst& I = insts[q];
  const long long local = item - I.item_begin;
  int b, tg, c;
  decode_item(I, local, b, tg, c);
  const int i0 = c * chunk;
  const int i1 = min(i0 + chunk, I.nx);
  const int len = i1 - i0;
  // the v_x planes of the block's tiles (every tile lies in one plane)
  constexpr int kTileV = 128 * P;
  const int nyz = I.nvy * I.nvz;
  const int v_first = tg * kWavesPerBlock * kTileV;
  const int v_last = min((tg + 1) * kWavesPerBlock * kTileV, I.nv3) - 1;
  const int jx_base = v_first / nyz;
  const int row_nx = v_last / nyz - jx_base + 1;
  const int rl = row_nx + I.nvy + I.nvz;
  double* lds1 = lds;
  double* lds2 = lds1 + (len + 6) * rl;
  double* lds3 = lds2 + (len + 4) * rl;
  stage_rows_compact(I, I.fac, b, i0 - 3, len + 6, jx_base, row_nx, lds1);
  stage_rows_compact(I, I.fac2, b, i0 - 2, len + 4, jx_base, row_nx, lds2);
  stage_rows_compact(I, I.fac3, b, i0 - 1, len + 2, jx_base, row_nx, lds3);
  __syncthreads();
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int tile = tg * kWavesPerBlock + wave;
  if (tile >= I.ntiles) return;
  double vxu, nuu;
  using Call = Step3xCall<P, MODE>;
  BGK_MARCH_DISPATCH_UNI(Call, I, lds1, lds2, lds3, b, tile, lane, i0, i1, phase, vxu, nuu,
                         jx_base, row_nx);
}

// ----------------------------------------------- four steps in one pass --
// The three-step pass extended by one level: reads g^m once and writes
// g^{m+4} once (4 bytes per phase-space update).  The moments of g^{m+1},
// g^{m+2} and g^{m+3} are known before the pass (reductions kRedW1x4,
// kRedW2x4, kRedW3x4, kRedW4x4 from sums of g^m and M^m weighted by nu+ and
// nu- up to the third power).  Output row k takes level 4 at k-1 .. k+1,
// level 4 at k+1 takes level 3 at k .. k+2, level 3 at k+2 level 2 at
// k+1 .. k+3, level 2 at k+3 level 1 at k+2 .. k+4.  Four levels of rows fit
// the registers with one velocity pair per lane (147 VGPRs with two rows in
// flight; two pairs per lane spill).  With four rows in flight the pass takes
// 30.9 ms on the 32-slice 2048 x 48^3 batch (47-cell chunks), 7.7 ms per IMEX
// step against 7.1 for the three-step pass (two pairs per lane): one pair
// per lane and one block per CU leave too few loads in flight.
constexpr int kRowsInFlight4x = 4;

template <int P, int MODE, int CASE, int DIR>
__device__ __forceinline__ void step4x_march(const Inst& I, const double* lds1,
                                             const double* lds2, const double* lds3,
                                             const double* lds4, int b, int tile, int lane,
                                             int i0, int i1, int phase, double vxu,
                                             double nuu, int jx_base, int row_nx) {
  constexpr int SGN = CASE == kTilePos ? 1 : -1;
  const int nx = I.nx, nv3 = I.nv3;
  const int nvs = row_nx + I.nvy + I.nvz;  // compact factor rows in LDS
  PairEls<P> e;
  setup_pairs<P, true>(I, tile, lane, e, jx_base, row_nx);
  const double dvz = I.dv[2];
  const long long mbase = (long long)b * nx * nv3;
  gptr<const double> src = gmem(I.buf[phase]) + mbase;
  gptr<double> dst = gmem(I.buf[phase ^ 1]) + mbase;
  const double a = I.a;
  const bool neumann = I.bc == 0;
  const int len = i1 - i0;
  auto row_at = [&](int k) { return DIR > 0 ? i0 + k : i1 - 1 - k; };
  auto outside = [&](int k) {
    const int r = row_at(k);
    return r < 0 || r >= nx;
  };
  auto load_row = [&](int k, double2 (&raw)[P]) {
    if (MODE == kLift) return;
    gptr<const double> row = src + (long long)ghost_row(row_at(k), nx, I.bc) * nv3;
#pragma unroll
    for (int p = 0; p < P; ++p)
      raw[p] = P == 2 ? ld2_nt(row + e.jofs[p]) : ld2(row + e.jofs[p]);
  };
  // level 1 at position k: rows i0-4 .. i1+3 staged in lds1
  auto level1 = [&](int k, const double2 (&raw)[P], double2 (&out)[P]) {
    const double* fr = lds1 + (row_at(k) - (i0 - 4)) * nvs;
#pragma unroll
    for (int p = 0; p < P; ++p) out[p] = relax_pair<MODE>(fr, e.off[p], a, raw[p]);
  };
  // level L+1 at position k from level L at k-1, k, k+1 (lds: the factor
  // rows of level L+1, first row `first`)
  auto next = [&](const double* lds, int first, int k, const double2 (&bh)[P],
                  const double2 (&c)[P], const double2 (&ah)[P], double2 (&out)[P]) {
    const double* fr = lds + (row_at(k) - first) * nvs;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const double2 g = transport_pair<DIR, SGN>(nuu, bh[p], c[p], ah[p]);
      out[p] = relax_pair<kRelax>(fr, e.off[p], a, g);
    }
  };
  auto copy = [&](double2 (&d)[P], const double2 (&s)[P]) {
#pragma unroll
    for (int p = 0; p < P; ++p) d[p] = s[p];
  };

  double2 l1b[P], l1c[P];  // level 1 at positions k+2, k+3
  double2 l2b[P], l2c[P];  // level 2 at k+1, k+2
  double2 l3b[P], l3c[P];  // level 3 at k, k+1
  double2 l4b[P], l4c[P];  // level 4 at k-1, k
  constexpr int R = kRowsInFlight4x;
  double2 raw[R][P];
  {
    // level 1 at -4 .. 3 (streamed), level 2 at -3 .. 2, then the Neumann
    // copies outside the domain, level 3 at -2 .. 1, level 4 at -1 .. 0
    double2 r0[P], r1[P], x0[P], x1[P], x2[P];
    double2 m3[P], m2[P], m1[P], z0[P];  // level 2 at -3, -2, -1, 0
    load_row(-4, r0);
    load_row(-3, r1);
    level1(-4, r0, x0);
    load_row(-2, r0);
    level1(-3, r1, x1);
    load_row(-1, r1);
    level1(-2, r0, x2);
    next(lds2, i0 - 3, -3, x0, x1, x2, m3);  // level 2 at -3
    load_row(0, r0);
    level1(-1, r1, x0);
    next(lds2, i0 - 3, -2, x1, x2, x0, m2);  // level 2 at -2
    load_row(1, r1);
    level1(0, r0, x1);
    next(lds2, i0 - 3, -1, x2, x0, x1, m1);  // level 2 at -1
    load_row(2, r0);
    level1(1, r1, x2);
    next(lds2, i0 - 3, 0, x0, x1, x2, z0);   // level 2 at 0
    load_row(3, r1);
#pragma unroll
    for (int j = 0; j < R; ++j)
      if (4 + j <= len + 3) load_row(4 + j, raw[j]);
    level1(2, r0, x0);
    next(lds2, i0 - 3, 1, x1, x2, x0, l2b);  // level 2 at 1
    level1(3, r1, x1);
    next(lds2, i0 - 3, 2, x2, x0, x1, l2c);  // level 2 at 2
    copy(l1b, x0);
    copy(l1c, x1);
    if (neumann) {
      if (outside(1)) copy(l2b, z0);
      if (outside(2)) copy(l2c, l2b);
      if (outside(-1)) copy(m1, z0);
      if (outside(-2)) copy(m2, m1);
      if (outside(-3)) copy(m3, m2);
    }
    double2 y2[P], y1[P];                       // level 3 at -2, -1
    next(lds3, i0 - 2, -2, m3, m2, m1, y2);
    next(lds3, i0 - 2, -1, m2, m1, z0, y1);
    next(lds3, i0 - 2, 0, m1, z0, l2b, l3b);    // level 3 at 0
    next(lds3, i0 - 2, 1, z0, l2b, l2c, l3c);   // level 3 at 1
    if (neumann) {
      if (outside(1)) copy(l3c, l3b);
      if (outside(-1)) copy(y1, l3b);
      if (outside(-2)) copy(y2, y1);
    }
    next(lds4, i0 - 1, -1, y2, y1, l3b, l4b);   // level 4 at -1
    next(lds4, i0 - 1, 0, y1, l3b, l3c, l4c);   // level 4 at 0
    if (neumann && outside(-1)) copy(l4b, l4c);
  }
  // output row k; rw holds raw row k+4 and takes the load of row k+4+R
  auto step = [&](int k, double2 (&rw)[P]) {
    double2 l1a[P], l2a[P], l3a[P], l4a[P];
    level1(k + 4, rw, l1a);
    if (k + 4 + R <= len + 3) load_row(k + 4 + R, rw);  // in flight meanwhile
    next(lds2, i0 - 3, k + 3, l1b, l1c, l1a, l2a);
    if (neumann && outside(k + 3)) copy(l2a, l2c);
    next(lds3, i0 - 2, k + 2, l2b, l2c, l2a, l3a);
    if (neumann && outside(k + 2)) copy(l3a, l3c);
    next(lds4, i0 - 1, k + 1, l3b, l3c, l3a, l4a);
    if (neumann && outside(k + 1)) copy(l4a, l4c);
    const int r = row_at(k);
    Acc<15, true> acc;
    acc.zero();
    gptr<double> drow = dst + (long long)r * nv3;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const double2 g = transport_pair<DIR, SGN>(nuu, l4b[p], l4c[p], l4a[p]);
      store_pair(drow, e.jofs[p], g);
      acc.add(g, e.vx[p], e.vy[p], e.vz[p], dvz, e.q0(p), e.q1(p), nuu);
    }
    acc.store(I, b, r, tile, lane, vxu, nuu);
    copy(l1b, l1c);
    copy(l1c, l1a);
    copy(l2b, l2c);
    copy(l2c, l2a);
    copy(l3b, l3c);
    copy(l3c, l3a);
    copy(l4b, l4c);
    copy(l4c, l4a);
  };
  for (int k = 0; k < len; k += R) {
#pragma unroll
    for (int j = 0; j < R; ++j)
      if (k + j < len) step(k + j, raw[j]);
  }
}

template <int P, int MODE>
struct Step4xCall {
  template <int CASE, int DIR>
  static __device__ __forceinline__ void run(const Inst& I, const double* lds1,
                                             const double* lds2, const double* lds3,
                                             const double* lds4, int b, int tile, int lane,
                                             int i0, int i1, int phase, double vxu,
                                             double nuu, int jx_base, int row_nx) {
    step4x_march<P, MODE, CASE, DIR>(I, lds1, lds2, lds3, lds4, b, tile, lane, i0, i1,
                                     phase, vxu, nuu, jx_base, row_nx);
  }
};

template <int P, int MODE>
__global__ __launch_bounds__(kBlock) void k_step4x(const Inst* __restrict__ insts,
                                                   int n_inst, int chunk, int phase) {
  extern __shared__ double lds[];
  const long long item = xcd_item(blockIdx.x, gridDim.x) + insts[0].item_begin;
  const int q = find_inst(insts, n_inst, item);
  const Inst& I = insts[q];
  const long long local = item - I.item_begin;
  int b, tg, c;
  decode_item(I, local, b, tg, c);
  const int i0 = c * chunk;
  const int i1 = min(i0 + chunk, I.nx);
  const int len = i1 - i0;
  constexpr int kTileV = 128 * P;
  const int nyz = I.nvy * I.nvz;
  const int v_first = tg * kWavesPerBlock * kTileV;
  const int v_last = min((tg + 1) * kWavesPerBlock * kTileV, I.nv3) - 1;
  const int jx_base = v_first / nyz;
  const int row_nx = v_last / nyz - jx_base + 1;
  const int rl = row_nx + I.nvy + I.nvz;
  double* lds1 = lds;
  double* lds2 = lds1 + (len + 8) * rl;
  double* lds3 = lds2 + (len + 6) * rl;
  double* lds4 = lds3 + (len + 4) * rl;
  stage_rows_compact(I, I.fac, b, i0 - 4, len + 8, jx_base, row_nx, lds1);
  stage_rows_compact(I, I.fac2, b, i0 - 3, len + 6, jx_base, row_nx, lds2);
  stage_rows_compact(I, I.fac3, b, i0 - 2, len + 4, jx_base, row_nx, lds3);
  stage_rows_compact(I, I.fac4, b, i0 - 1, len + 2, jx_base, row_nx, lds4);
  __syncthreads();
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int tile = tg * kWavesPerBlock + wave;
  if (tile >= I.ntiles) return;
  double vxu, nuu;
  using Call = Step4xCall<P, MODE>;
  BGK_MARCH_DISPATCH_UNI(Call, I, lds1, lds2, lds3, lds4, b, tile, lane, i0, i1, phase, vxu,
                         nuu, jx_base, row_nx);
}

// -------------------------------------------- partial sums of a field --
// Moments of an arbitrary f (source fin), same tiling, no transport.
template <int E>
__global__ __launch_bounds__(kBlock) void k_partials(
    const Inst* __restrict__ insts, int n_inst, int chunk) {
  const long long item = xcd_item(blockIdx.x, gridDim.x) + insts[0].item_begin;
  const int q = find_inst(insts, n_inst, item);
  const Inst& I = insts[q];
  const long long local = item - I.item_begin;
  int b, tg, c;
  decode_item(I, local, b, tg, c);
  const int wave = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int tile = tg * kWavesPerBlock + wave;
  if (tile >= I.ntiles) return;
  const int nx = I.nx, nv3 = I.nv3;
  const int i0 = c * chunk, i1 = min(i0 + chunk, nx);
  Elems<E> el;
  setup_elems<E>(I, tile, lane, el);
  gptr<const double> src = gmem(I.fin) + (long long)b * nx * nv3 + tile * (kWave * E) + lane;
  gptr<double> part = gmem(I.part) + (((long long)b * nx) * I.part_tiles + tile) * 5;
  for (int i = i0; i < i1; ++i) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const double g = el.ok[e] ? src[(long long)i * nv3 + e * kWave] : 0.0;
      const double vsq = el.vx[e] * el.vx[e] + el.vy[e] * el.vy[e] +
                         el.vz[e] * el.vz[e];
      s0 += g;
      s1 = fma(el.vx[e], g, s1);
      s2 = fma(el.vy[e], g, s2);
      s3 = fma(el.vz[e], g, s3);
      s4 = fma(vsq, g, s4);
    }
    s0 = wave_sum_to_last(s0);
    s1 = wave_sum_to_last(s1);
    s2 = wave_sum_to_last(s2);
    s3 = wave_sum_to_last(s3);
    s4 = wave_sum_to_last(s4);
    if (lane == kWave - 1) {
      gptr<double> pp = part + (long long)i * I.part_tiles * 5;
      pp[0] = s0;
      pp[1] = s1;
      pp[2] = s2;
      pp[3] = s3;
      pp[4] = s4;
    }
  }
}

// ------------------------------------------------------- cell reduction --
// Instance of an x cell counted from the table's first entry, and the cell
// within that instance (binary search over cell_begin, as find_inst).
__device__ __forceinline__ int find_inst_cell(const Inst* insts, int n_inst,
                                              long long cell,
                                              long long* cell_local) {
  cell += insts[0].cell_begin;
  int lo = 0, hi = n_inst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (insts[mid].cell_begin <= cell) lo = mid;
    else hi = mid - 1;
  }
  *cell_local = cell - insts[lo].cell_begin;
  return lo;
}

__device__ __forceinline__ bool physical(double rho, double th) {
  return rho > 0.0 && th > 0.0 && isfinite(rho) && isfinite(th);
}

// Writes factor row k in [0, nvs): Ex scaled by C, Ey, Ez.
__device__ __forceinline__ void write_factors(const Inst& I, double* row,
                                              int lane, double C,
                                              const double u[3], double th) {
  const double inv2t = 1.0 / (2.0 * th);
  for (int k = lane; k < I.nvs; k += kWave) {
    int ax = (k < I.nvx) ? 0 : (k < I.nvx + I.nvy ? 1 : 2);
    int j = k - (ax == 0 ? 0 : (ax == 1 ? I.nvx : I.nvx + I.nvy));
    double d = vgrid(I, ax, j) - u[ax];
    double e = exp(-d * d * inv2t);
    if (ax == 2 && j >= I.nvz_live) e = 0.0;  // pad points of the z rows
    row[k] = ax == 0 ? C * e : e;
  }
}

// Separable moment sums of the Maxwellian with factors exp(-(v-u)^2/(2 theta))
// per axis (C0 * dv3 applied by the caller): for weights w of v_x in {1, nu+,
// nu-} (NW = 3), also nu+^2, nu-^2 (NW = 5) and nu+^3, nu-^3 (NW = 7),
// nu = v_x dt/dx, A^w = (rho,
// m_x, m_y, m_z, E) moments of w M, scaled by K = C0 dv3: 5 NW values in that
// weight order.  All lanes return the same values.
// row (nullable): also writes the factor row of the same exponentials (Ex
// scaled by Cx, Ey, Ez), as write_factors does.
template <int NW>
__device__ __forceinline__ void maxwell_weighted_sums(const Inst& I, int lane,
                                                      const double u[3], double th,
                                                      double K, double (&A)[5 * NW],
                                                      double* row = nullptr,
                                                      double Cx = 0.0) {
  // x: X^w_k = sum w(vx) vx^k Ex, k = 0..2 (3 NW values); y, z: k = 0..2
  constexpr int NT = 3 * NW + 6;
  double t[NT];
#pragma unroll
  for (int c = 0; c < NT; ++c) t[c] = 0.0;
  const double inv2t = 1.0 / (2.0 * th);
  for (int kk = lane; kk < I.nvs; kk += kWave) {
    int ax = (kk < I.nvx) ? 0 : (kk < I.nvx + I.nvy ? 1 : 2);
    int j = kk - (ax == 0 ? 0 : (ax == 1 ? I.nvx : I.nvx + I.nvy));
    const double v = vgrid(I, ax, j);
    const double d = v - u[ax];
    const double ex = (ax == 2 && j >= I.nvz_live) ? 0.0 : exp(-d * d * inv2t);
    if (row != nullptr) row[kk] = ax == 0 ? Cx * ex : ex;
    const double e1 = v * ex, e2 = v * v * ex;
    if (ax == 0) {
      const double nu = v * I.r;
      const double wp = nu > 0.0 ? nu : 0.0, wm = nu < 0.0 ? -nu : 0.0;
      t[0] += ex; t[1] += e1; t[2] += e2;
      t[3] += wp * ex; t[4] += wp * e1; t[5] += wp * e2;
      t[6] += wm * ex; t[7] += wm * e1; t[8] += wm * e2;
      if (NW >= 5) {
        const double wpp = wp * wp, wmm = wm * wm;
        t[9] += wpp * ex; t[10] += wpp * e1; t[11] += wpp * e2;
        t[12] += wmm * ex; t[13] += wmm * e1; t[14] += wmm * e2;
        if (NW == 7) {
          const double w3p = wpp * wp, w3m = wmm * wm;
          t[15] += w3p * ex; t[16] += w3p * e1; t[17] += w3p * e2;
          t[18] += w3m * ex; t[19] += w3m * e1; t[20] += w3m * e2;
        }
      }
    } else if (ax == 1) {
      t[3 * NW] += ex; t[3 * NW + 1] += e1; t[3 * NW + 2] += e2;
    } else {
      t[3 * NW + 3] += ex; t[3 * NW + 4] += e1; t[3 * NW + 5] += e2;
    }
  }
  wave_sum_all_n<NT>(t, lane);
  const double Y0 = t[3 * NW], Y1 = t[3 * NW + 1], Y2 = t[3 * NW + 2];
  const double Z0 = t[3 * NW + 3], Z1 = t[3 * NW + 4], Z2 = t[3 * NW + 5];
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const double X0 = t[3 * w], X1 = t[3 * w + 1], X2 = t[3 * w + 2];
    A[5 * w + 0] = K * X0 * Y0 * Z0;
    A[5 * w + 1] = K * X1 * Y0 * Z0;
    A[5 * w + 2] = K * X0 * Y1 * Z0;
    A[5 * w + 3] = K * X0 * Y0 * Z1;
    A[5 * w + 4] = 0.5 * K * (X2 * Y0 * Z0 + X0 * Y2 * Z0 + X0 * Y0 * Z2);
  }
}

// Primitive (rho, u, theta) from conserved (rho, m, E): one division, the
// other quotients by its reciprocal.
__device__ __forceinline__ void cons_to_prim(const double* V, double& rho, double u[3],
                                             double& th) {
  rho = V[0];
  const double irho = 1.0 / rho;
  u[0] = V[1] * irho;
  u[1] = V[2] * irho;
  u[2] = V[3] * irho;
  const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  th = (2.0 * V[4] * irho - usq) * (1.0 / 3.0);
}

// Offset of weight class w (0: 1; 2q - 1: nu+^q; 2q: nu-^q) in an aux-style
// layout, for the sums of g (maxw false) or of its Maxwellian (true).
__device__ __forceinline__ constexpr int aux_off(int w, bool maxw) {
  return w == 0 ? (maxw ? 15 : 0)
                : (w <= 2 ? 5 * w + (maxw ? 15 : 0)
                          : 30 + 20 * ((w + 1) / 2 - 2) + (w % 2 == 0 ? 5 : 0) +
                                (maxw ? 10 : 0));
}
static_assert(aux_off(0, false) == 0 && aux_off(1, false) == 5 && aux_off(2, false) == 10 &&
                  aux_off(0, true) == 15 && aux_off(1, true) == 20 && aux_off(2, true) == 25 &&
                  aux_off(3, false) == 30 && aux_off(4, false) == 35 && aux_off(3, true) == 40 &&
                  aux_off(4, true) == 45 && aux_off(5, false) == 50 && aux_off(6, false) == 55 &&
                  aux_off(5, true) == 60 && aux_off(6, true) == 65,
              "aux layout");

// Moments of the next transported field T(a g + al M[U(g)]) at a cell and its
// sums weighted by nu+^q, nu-^q up to q = PIN - 1, from the sums of g and M
// at cells i-1, i, i+1 (input layout of highest power PIN: upwind transport
// T h_i = (1 - nu+ - nu-) h_i + nu+ h_{i-1} + nu- h_{i+1} with nu+ nu- = 0
// gives S^0[T h]_i = S^0_i - S^{1+}_i - S^{1-}_i + S^{1+}_{i-1} + S^{1-}_{i+1},
// S^{q+}[T h]_i = S^{q+}_i - S^{(q+1)+}_i + S^{(q+1)+}_{i-1} and the mirror
// for q-).  Writes the factor row of the new field's Maxwellian into fac_out
// and, for PIN >= 2, its sums and the Maxwellian's into out (layout of
// highest power PIN - 1); with PROJECT instead the projected relaxed moments
// a V + al V(M) into vout.  One wave per cell; every lane returns.
template <int PIN, bool PROJECT>
__device__ __forceinline__ void advance_reduce(const Inst& I, long long cl, int lane,
                                               const double* in, int in_stride,
                                               double* fac_out, double* out, int out_stride,
                                               int* status) {
  constexpr int NWO = 2 * PIN - 1;  // weight classes of the output
  const int nx = I.nx;
  const long long b = cl / nx;
  const int i = (int)(cl - b * nx);
  gptr<const double> ac = gmem(in) + cl * in_stride;
  gptr<const double> am = gmem(in) + (b * nx + ghost_row(i - 1, nx, I.bc)) * in_stride;
  gptr<const double> ap = gmem(in) + (b * nx + ghost_row(i + 1, nx, I.bc)) * in_stride;
  double val = 0.0;
  if (lane < 5 * NWO) {
    const int w = lane / 5, c = lane - 5 * (lane / 5);
    double tg, tm;
    if (w == 0) {
      tg = ac[c] - ac[5 + c] - ac[10 + c] + am[5 + c] + ap[10 + c];
      tm = ac[15 + c] - ac[20 + c] - ac[25 + c] + am[20 + c] + ap[25 + c];
    } else {
      // class w = (q, sign); the next power of the same sign is class w + 2
      const bool plus = (w % 2) == 1;
      const int og = aux_off(w, false), og1 = aux_off(w + 2, false);
      const int om = aux_off(w, true), om1 = aux_off(w + 2, true);
      gptr<const double> nb = plus ? am : ap;
      tg = ac[og + c] - ac[og1 + c] + nb[og1 + c];
      tm = ac[om + c] - ac[om1 + c] + nb[om1 + c];
    }
    val = I.a * tg + I.al * tm;
  }
  double V[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) V[c] = readlane_d(val, c);
  double rho, u[3], th;
  cons_to_prim(V, rho, u, th);
  if (lane == 0 && !physical(rho, th)) *status = 1;
  const double C0 = maxwell_norm(rho, th);
  if (PROJECT) {
    double A[15];
    maxwell_weighted_sums<3>(I, lane, u, th, C0 * I.dv3, A);
    if (lane == 0) {
      double* vo = I.vout + cl * 5;
#pragma unroll
      for (int c = 0; c < 5; ++c) vo[c] = I.a * V[c] + I.al * A[c];
    }
    return;
  }
  double* frow = fac_out + cl * I.nvs;
  if (NWO == 1) {
    write_factors(I, frow, lane, I.al * C0, u, th);
    return;
  }
  double A[5 * NWO];
  maxwell_weighted_sums<NWO>(I, lane, u, th, C0 * I.dv3, A, frow, I.al * C0);
  double* ax = out + cl * out_stride;
  if (lane < 5 * NWO) ax[aux_off(lane / 5, false) + lane % 5] = val;
  if (lane == 0) {
#pragma unroll
    for (int w = 0; w < NWO; ++w)
#pragma unroll
      for (int c = 0; c < 5; ++c) ax[aux_off(w, true) + c] = A[5 * w + c];
  }
}

// One wave per (instance, member, x cell).  The mode is a template argument
// so that the independent wave reductions are unrolled and interleaved.
template <int mode>
__global__ __launch_bounds__(kBlock) void k_reduce(const Inst* __restrict__ insts,
                                                   int n_inst,
                                                   long long total_cells,
                                                   int* status) {
  const long long cell = (long long)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  if (cell >= total_cells) return;
  const int lane = threadIdx.x % kWave;
  long long cl;
  const int q = find_inst_cell(insts, n_inst, cell, &cl);
  const Inst& I = insts[q];
  if (mode == kRedW2x4) {
    advance_reduce<3, false>(I, cl, lane, I.aux, kAux, I.fac2, I.aux2, kAux2, status);
    return;
  }
  if (mode == kRedW3x4) {
    advance_reduce<2, false>(I, cl, lane, I.aux2, kAux2, I.fac3, I.aux3, kAux3, status);
    return;
  }
  if (mode == kRedW4x4) {
    advance_reduce<1, false>(I, cl, lane, I.aux3, kAux3, I.fac4, nullptr, 0, status);
    return;
  }
  if (mode == kRedW4x4Project) {
    advance_reduce<1, true>(I, cl, lane, I.aux3, kAux3, nullptr, nullptr, 0, status);
    return;
  }
  if (mode == kRedW2 || mode == kRedW2x3 || mode == kRedW3x3 || mode == kRedW2Project ||
      mode == kRedW3x3Project) {
    // moments of the next transported field T(a g + al M[U(g)]) at this cell
    // from the weighted sums of g and M at cells i-1, i, i+1 (upwind
    // transport: T h_i = (1 - nu+ - nu-) h_i + nu+ h_{i-1} + nu- h_{i+1})
    const int nx = I.nx;
    const long long b = cl / nx;
    const int i = (int)(cl - b * nx);
    const bool second = mode == kRedW3x3 || mode == kRedW3x3Project;  // from aux2
    gptr<const double> base = gmem(second ? I.aux2 : I.aux);
    const int stride = second ? kAux2 : kAux;
    gptr<const double> ac = base + cl * stride;
    gptr<const double> am = base + (b * nx + ghost_row(i - 1, nx, I.bc)) * stride;
    gptr<const double> ap = base + (b * nx + ghost_row(i + 1, nx, I.bc)) * stride;
    // lane 5 w + c forms component c of the plain (w = 0) moments of T h and,
    // for kRedW2x3, of its nu+ (w = 1) and nu- (w = 2) weighted sums (nu+ nu-
    // = 0: the sums of h weighted by nu+ and nu+^2 at i and i-1, by nu- and
    // nu-^2 at i and i+1)
    double val = 0.0;
    if (lane < (mode == kRedW2x3 ? 15 : 5)) {
      const int w = lane / 5, c = lane - 5 * (lane / 5);
      double tg, tm;
      if (w == 0) {
        tg = ac[c] - ac[5 + c] - ac[10 + c] + am[5 + c] + ap[10 + c];
        tm = ac[15 + c] - ac[20 + c] - ac[25 + c] + am[20 + c] + ap[25 + c];
      } else if (w == 1) {
        tg = ac[5 + c] - ac[30 + c] + am[30 + c];
        tm = ac[20 + c] - ac[40 + c] + am[40 + c];
      } else {
        tg = ac[10 + c] - ac[35 + c] + ap[35 + c];
        tm = ac[25 + c] - ac[45 + c] + ap[45 + c];
      }
      val = I.a * tg + I.al * tm;
    }
    double V[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) V[c] = readlane_d(val, c);
    double rho, u[3], th;
    cons_to_prim(V, rho, u, th);
    if (lane == 0 && !physical(rho, th)) *status = 1;
    const double C0 = maxwell_norm(rho, th);
    if (mode == kRedW2Project || mode == kRedW3x3Project) {
      // the next field's relaxation, projected (as kRedProject does from
      // records): P f = a V(g) + al V(M[U(g)])
      double A[15];
      maxwell_weighted_sums<3>(I, lane, u, th, C0 * I.dv3, A);
      if (lane == 0) {
        double* vo = I.vout + cl * 5;
#pragma unroll
        for (int c = 0; c < 5; ++c) vo[c] = I.a * V[c] + I.al * A[c];
      }
      return;
    }
    double* fout = (mode == kRedW3x3 ? I.fac3 : I.fac2) + cl * I.nvs;
    if (mode != kRedW2x3) write_factors(I, fout, lane, I.al * C0, u, th);
    if (mode == kRedW2x3) {
      double A[15];
      maxwell_weighted_sums<3>(I, lane, u, th, C0 * I.dv3, A, fout, I.al * C0);
      double* ax = I.aux2 + cl * kAux2;
      if (lane < 15) ax[lane] = val;
      if (lane == 0) {
#pragma unroll
        for (int c = 0; c < 15; ++c) ax[15 + c] = A[c];
      }
    }
    return;
  }
  const int ns = I.nsum;
  gptr<const double> pp = gmem(I.part) + cl * I.part_tiles * 5;
  // weight classes of the sums: 1 (and nu+, nu- for W1; and nu+^2, nu-^2
  // for W1x3, which needs compact records)
  constexpr int NW = mode == kRedW1x4 ? 7 : (mode == kRedW1x3 ? 5 : (mode == kRedW1 ? 3 : 1));
  double s[35];
#pragma unroll
  for (int c = 0; c < 35; ++c) s[c] = 0.0;
  if (I.crec) {
    // compact records (tiles inside one v_x plane): (sum g, sum v_y g,
    // sum v_z g, sum |v|^2 g); v_x and nu are the tile's
    // a record's tile lies in v_x plane t / (tiles per plane); crec divides
    // nvy nvz, and the 32-bit quotient avoids a 64-bit division per record
    const unsigned tiles_per_plane = (unsigned)(I.nvy * I.nvz / I.crec);
    // the records of up to RU tiles per lane are loaded before any is summed
    // (loads in flight together); summed in tile order as in one pass
    constexpr int RU = 4;
    for (int t0 = lane; t0 < I.nparts; t0 += RU * kWave) {
      double q[RU][4];
#pragma unroll
      for (int r = 0; r < RU; ++r) {
        const int t = t0 + r * kWave;
        // (records are 8-byte aligned only: part_tiles * 5 may be odd)
        if (t < I.nparts) {
#pragma unroll
          for (int c = 0; c < 4; ++c) q[r][c] = pp[t * 4 + c];
        }
      }
#pragma unroll
      for (int r = 0; r < RU; ++r) {
        const int t = t0 + r * kWave;
        if (t >= I.nparts) break;
        const double vx = vgrid(I, 0, (int)((unsigned)t / tiles_per_plane));
        const double m[5] = {q[r][0], vx * q[r][0], q[r][1], q[r][2], q[r][3]};
#pragma unroll
        for (int c = 0; c < 5; ++c) s[c] += m[c];
        if (NW >= 3) {
          const double nu = vx * I.r;
          const double wp = nu > 0.0 ? nu : 0.0, wm = nu < 0.0 ? -nu : 0.0;
#pragma unroll
          for (int c = 0; c < 5; ++c) {
            s[5 + c] += wp * m[c];
            s[10 + c] += wm * m[c];
          }
          if (NW >= 5) {
            const double wpp = wp * wp, wmm = wm * wm;
#pragma unroll
            for (int c = 0; c < 5; ++c) {
              s[15 + c] += wpp * m[c];
              s[20 + c] += wmm * m[c];
            }
            if (NW == 7) {
              const double w3p = wpp * wp, w3m = wmm * wm;
#pragma unroll
              for (int c = 0; c < 5; ++c) {
                s[25 + c] += w3p * m[c];
                s[30 + c] += w3m * m[c];
              }
            }
          }
        }
      }
    }
  } else {
    for (int t = lane; t < I.nparts; t += kWave) {
#pragma unroll
      for (int c = 0; c < 5; ++c) s[c] += pp[t * ns + c];
      if (mode == kRedW1) {
#pragma unroll
        for (int c = 5; c < 15; ++c) s[c] += pp[t * ns + c];
      }
    }
  }
  {
    double t[5 * NW];
#pragma unroll
    for (int c = 0; c < 5 * NW; ++c) t[c] = s[c];
    wave_sum_all_n<5 * NW>(t, lane);
#pragma unroll
    for (int c = 0; c < 5 * NW; ++c) s[c] = t[c];
  }
  // conserved units: rho, m from sums times dv3; E = sum |v|^2 g dv3 / 2
#pragma unroll
  for (int w = 0; w < NW; ++w) {
#pragma unroll
    for (int c = 0; c < 4; ++c) s[5 * w + c] *= I.dv3;
    s[5 * w + 4] *= 0.5 * I.dv3;
  }
  const double rho = s[0];
  const double m[3] = {s[1], s[2], s[3]};
  const double E = s[4];
  const double irho = 1.0 / rho;
  const double u[3] = {m[0] * irho, m[1] * irho, m[2] * irho};
  const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const double th = (2.0 * E * irho - usq) * (1.0 / 3.0);
  if (lane == 0) {
    double* vg = I.vg + cl * 5;
    vg[0] = rho;
    vg[1] = m[0];
    vg[2] = m[1];
    vg[3] = m[2];
    vg[4] = E;
    if (!physical(rho, th)) *status = 1;
  }
  if (mode == kRedMomentsOnly) {
    if (I.vout != nullptr && lane == 0) {
      double* w = I.vout + cl * 5;
      w[0] = rho;
      w[1] = u[0];
      w[2] = u[1];
      w[3] = u[2];
      w[4] = th;
    }
    return;
  }
  const double C0 = maxwell_norm(rho, th);
  if (mode == kRedRelaxFactors || mode == kRedMaxwellFactors || mode == kRedW1 ||
      mode == kRedW1x3 || mode == kRedW1x4) {
    // (W1, W1x3: the factor row is written with the weighted sums' exponentials)
    if (mode == kRedRelaxFactors || mode == kRedMaxwellFactors)
      write_factors(I, I.fac + cl * I.nvs, lane,
                    mode == kRedMaxwellFactors ? C0 : I.al * C0, u, th);
    if (mode == kRedW1x4) {
      double A[35];
      maxwell_weighted_sums<7>(I, lane, u, th, C0 * I.dv3, A, I.fac + cl * I.nvs, I.al * C0);
      if (lane == 0) {
        double* ax = I.aux + cl * kAux;
#pragma unroll
        for (int w = 0; w < 7; ++w)
#pragma unroll
          for (int c = 0; c < 5; ++c) {
            ax[aux_off(w, false) + c] = s[5 * w + c];
            ax[aux_off(w, true) + c] = A[5 * w + c];
          }
      }
    }
    if (mode == kRedW1x3) {
      double A[25];
      maxwell_weighted_sums<5>(I, lane, u, th, C0 * I.dv3, A, I.fac + cl * I.nvs, I.al * C0);
      if (lane == 0) {
        double* ax = I.aux + cl * kAux;
#pragma unroll
        for (int c = 0; c < 15; ++c) {
          ax[c] = s[c];
          ax[15 + c] = A[c];
        }
#pragma unroll
        for (int c = 0; c < 10; ++c) {
          ax[30 + c] = s[15 + c];
          ax[40 + c] = A[15 + c];
        }
      }
    }
    if (mode == kRedW1) {
      double A[15];
      maxwell_weighted_sums<3>(I, lane, u, th, C0 * I.dv3, A, I.fac + cl * I.nvs, I.al * C0);
      if (lane == 0) {
        double* ax = I.aux + cl * kAux;
#pragma unroll
        for (int c = 0; c < 15; ++c) ax[c] = s[c];
#pragma unroll
        for (int c = 0; c < 15; ++c) ax[15 + c] = A[c];
      }
    }
    return;
  }
  // kRedProject: moments of the relaxed field a g + al M[U(g)], with the
  // moments of the separable Maxwellian as products of 1D sums.
  double A[15];
  maxwell_weighted_sums<3>(I, lane, u, th, C0 * I.dv3, A);
  const double vgv[5] = {rho, m[0], m[1], m[2], E};
  if (lane == 0) {
    double* vo = I.vout + cl * 5;
#pragma unroll
    for (int c = 0; c < 5; ++c) vo[c] = I.a * vgv[c] + I.al * A[c];
  }
}

// Lift factors: C = rho (2 pi theta)^{-3/2} from primitive W (if given) or
// from the conserved vin of each member.  with_aux: also the weighted
// Maxwellian sums into aux (both the "g" and the "M" slots: the lifted field
// is its own Maxwellian), for a two-step (1) or three-step (2) first pass.
__global__ __launch_bounds__(kBlock) void k_lift_factors(
    const Inst* __restrict__ insts, int n_inst, long long total_cells,
    const double* __restrict__ W, int* status, int with_aux) {
  const long long cell = (long long)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  if (cell >= total_cells) return;
  const int lane = threadIdx.x % kWave;
  long long cl;
  const int q = find_inst_cell(insts, n_inst, cell, &cl);
  const Inst& I = insts[q];
  double rho, u[3], th;
  if (W != nullptr) {
    const double* w = W + cl * 5;
    rho = w[0];
    u[0] = w[1];
    u[1] = w[2];
    u[2] = w[3];
    th = w[4];
  } else {
    cons_to_prim(I.vin + cl * 5, rho, u, th);
  }
  if (!physical(rho, th) || !isfinite(u[0]) || !isfinite(u[1]) || !isfinite(u[2])) {
    if (lane == 0) *status = 1;
  }
  const double C0 = maxwell_norm(rho, th);
  double* row = I.fac + cl * I.nvs;
  if (!with_aux) write_factors(I, row, lane, C0, u, th);
  if (with_aux == 1) {
    double A[15];
    maxwell_weighted_sums<3>(I, lane, u, th, C0 * I.dv3, A, row, C0);
    if (lane == 0) {
      double* ax = I.aux + cl * kAux;
#pragma unroll
      for (int c = 0; c < 15; ++c) {
        ax[c] = A[c];
        ax[15 + c] = A[c];
      }
    }
  } else if (with_aux == 3) {
    // to the third power, for a four-step first pass
    double A[35];
    maxwell_weighted_sums<7>(I, lane, u, th, C0 * I.dv3, A, row, C0);
    if (lane == 0) {
      double* ax = I.aux + cl * kAux;
#pragma unroll
      for (int w = 0; w < 7; ++w)
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          ax[aux_off(w, false) + c] = A[5 * w + c];
          ax[aux_off(w, true) + c] = A[5 * w + c];
        }
    }
  } else if (with_aux == 2) {
    // with the nu+^2, nu-^2 weighted sums, for a three-step first pass
    double A[25];
    maxwell_weighted_sums<5>(I, lane, u, th, C0 * I.dv3, A, row, C0);
    if (lane == 0) {
      double* ax = I.aux + cl * kAux;
#pragma unroll
      for (int c = 0; c < 15; ++c) {
        ax[c] = A[c];
        ax[15 + c] = A[c];
      }
#pragma unroll
      for (int c = 0; c < 10; ++c) {
        ax[30 + c] = A[15 + c];
        ax[40 + c] = A[15 + c];
      }
    }
  }
}

// f_out = a g + F (relaxation of the last transported field), or f_out = F
// when src_sel < 0 (pure lift).  One block per (cell, 1024-element slab).
__global__ __launch_bounds__(kBlock) void k_relax_out(
    const Inst* __restrict__ insts, int n_inst, long long total_cells,
    int src_sel) {
  extern __shared__ double lds[];
  const long long blk = blockIdx.x;
  // find the cell: each instance contributes nbatch*nx*slabs blocks
  long long begin = 0;
  int q = 0;
  long long slabs = 0;
  for (;;) {
    slabs = (insts[q].nv3 + 4 * kBlock - 1) / (4 * kBlock);
    long long n = (long long)insts[q].nbatch * insts[q].nx * slabs;
    if (blk < begin + n || q + 1 == n_inst) break;
    begin += n;
    ++q;
  }
  const Inst& I = insts[q];
  const long long local = blk - begin;
  const long long cl = local / slabs;
  const int slab = (int)(local % slabs);
  gptr<const double> frow = gmem(I.fac) + cl * I.nvs;
  for (int k = threadIdx.x; k < I.nvs; k += kBlock) lds[k] = frow[k];
  __syncthreads();
  const int nyz = I.nvy * I.nvz;
  // rows with pad points: the output holds only the live ones (nvz_live per
  // z row, nvx nvy nvz_live per x cell)
  const int nzl = I.nvz_live;
  const long long out_nv3 = (long long)I.nvx * I.nvy * nzl;
  gptr<const double> g = src_sel >= 0 ? gmem(I.buf[src_sel]) + cl * I.nv3 : nullptr;
  gptr<double> out = gmem(I.fout) + cl * out_nv3;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    int j = slab * 4 * kBlock + e * kBlock + threadIdx.x;
    if (j >= I.nv3) break;
    int jx = j / nyz;
    int rem = j - jx * nyz;
    int jy = rem / I.nvz;
    int jz = rem - jy * I.nvz;
    if (jz >= nzl) continue;
    double F = lds[jx] * lds[I.nvx + jy] * lds[I.nvx + I.nvy + jz];
    const int jo = nzl == I.nvz ? j : (jx * I.nvy + jy) * nzl + jz;
    out[jo] = g ? fma(I.a, g[j], F) : F;
  }
  (void)total_cells;
}

// Rows of f with nz_live values per z row copied into rows of nz_live + 1
// values, the pad point set to zero: cells x cells, nxy = nvx nvy z rows each.
__global__ __launch_bounds__(kBlock) void k_pad_rows(const double* __restrict__ src,
                                                     double* __restrict__ dst,
                                                     long long rows, int nz_live) {
  const int nz = nz_live + 1;
  const long long n = rows * nz;
  for (long long t = (long long)blockIdx.x * kBlock + threadIdx.x; t < n;
       t += (long long)gridDim.x * kBlock) {
    const long long row = t / nz;
    const int jz = (int)(t - row * nz);
    dst[t] = jz < nz_live ? src[row * nz_live + jz] : 0.0;
  }
}

// ------------------------------------------------------------- launchers --
static int blocks_for(long long n) { return (int)n; }

int launch_step(const Inst* d_insts, int n_inst, long long total_items, int mode,
                int phase, Tiles t, int lds_doubles, int* d_status, hipStream_t s,
                int ns, bool force, int order, bool uni) {
  (void)d_status;
  if (total_items <= 0) return BGK_OK;
  dim3 grid(blocks_for(total_items)), block(kBlock);
  size_t lds = (mode == kCopy) ? 0 : (size_t)lds_doubles * sizeof(double);
  const int chunk = t.chunk;
#define BGK_STEP_CASE(KER, EE, MM)                                          \
  if (t.elems == EE && mode == MM) {                                        \
    hipLaunchKernelGGL(KER, grid, block, lds, s, d_insts, n_inst, chunk,    \
                       phase);                                              \
    hipError_t e_ = hipGetLastError();                                      \
    return e_ == hipSuccess ? BGK_OK : hip_fail(e_, "k_step");              \
  }
  if (t.vcol) {
    if (!force || ns != 5) {
      set_error("the v_x-column lane mapping serves the exterior-force step only");
      return BGK_E_INVALID;
    }
#define BGK_VCOL_CASES(EE, LIM, PYY)                                \
  BGK_STEP_CASE((k_step_vcol<EE, kCopy, LIM, PYY>), EE, kCopy)      \
  BGK_STEP_CASE((k_step_vcol<EE, kRelax, LIM, PYY>), EE, kRelax)    \
  BGK_STEP_CASE((k_step_vcol<EE, kLift, LIM, PYY>), EE, kLift)
    if (t.pair) {
      if (order == 2) {
        BGK_VCOL_CASES(2, true, 2)
        BGK_VCOL_CASES(4, true, 2)
      } else {
        BGK_VCOL_CASES(2, false, 2)
        BGK_VCOL_CASES(4, false, 2)
      }
    } else if (order == 2) {
      BGK_VCOL_CASES(2, true, 1)
      BGK_VCOL_CASES(4, true, 1)
      BGK_VCOL_CASES(8, true, 1)
    } else {
      BGK_VCOL_CASES(2, false, 1)
      BGK_VCOL_CASES(4, false, 1)
      BGK_VCOL_CASES(8, false, 1)
    }
#undef BGK_VCOL_CASES
  } else if (order == 2) {
    if (t.pair || ns != 5) {
      set_error("the second-order step uses the generic lane mapping, one step per pass");
      return BGK_E_INVALID;
    }
    if (force) {
      BGK_STEP_CASE((k_step<2, kCopy, true, true>), 2, kCopy)
      BGK_STEP_CASE((k_step<2, kRelax, true, true>), 2, kRelax)
      BGK_STEP_CASE((k_step<2, kLift, true, true>), 2, kLift)
      BGK_STEP_CASE((k_step<4, kCopy, true, true>), 4, kCopy)
      BGK_STEP_CASE((k_step<4, kRelax, true, true>), 4, kRelax)
      BGK_STEP_CASE((k_step<4, kLift, true, true>), 4, kLift)
    } else if (uni) {
      BGK_STEP_CASE((k_step<2, kCopy, false, true, 5, true>), 2, kCopy)
      BGK_STEP_CASE((k_step<2, kRelax, false, true, 5, true>), 2, kRelax)
      BGK_STEP_CASE((k_step<2, kLift, false, true, 5, true>), 2, kLift)
      BGK_STEP_CASE((k_step<4, kCopy, false, true, 5, true>), 4, kCopy)
      BGK_STEP_CASE((k_step<4, kRelax, false, true, 5, true>), 4, kRelax)
      BGK_STEP_CASE((k_step<4, kLift, false, true, 5, true>), 4, kLift)
    } else {
      BGK_STEP_CASE((k_step<2, kCopy, false, true>), 2, kCopy)
      BGK_STEP_CASE((k_step<2, kRelax, false, true>), 2, kRelax)
      BGK_STEP_CASE((k_step<2, kLift, false, true>), 2, kLift)
      BGK_STEP_CASE((k_step<4, kCopy, false, true>), 4, kCopy)
      BGK_STEP_CASE((k_step<4, kRelax, false, true>), 4, kRelax)
      BGK_STEP_CASE((k_step<4, kLift, false, true>), 4, kLift)
    }
  } else if (force) {
    if (t.pair) {
      set_error("the force step uses the generic lane mapping");
      return BGK_E_INVALID;
    }
    BGK_STEP_CASE((k_step<2, kCopy, true>), 2, kCopy)
    BGK_STEP_CASE((k_step<2, kRelax, true>), 2, kRelax)
    BGK_STEP_CASE((k_step<2, kLift, true>), 2, kLift)
    BGK_STEP_CASE((k_step<4, kCopy, true>), 4, kCopy)
    BGK_STEP_CASE((k_step<4, kRelax, true>), 4, kRelax)
    BGK_STEP_CASE((k_step<4, kLift, true>), 4, kLift)
    BGK_STEP_CASE((k_step<8, kCopy, true>), 8, kCopy)
    BGK_STEP_CASE((k_step<8, kRelax, true>), 8, kRelax)
    BGK_STEP_CASE((k_step<8, kLift, true>), 8, kLift)
  } else if (t.pair && ns == 15) {
    BGK_STEP_CASE((k_step2<1, kCopy, 15>), 2, kCopy)
    BGK_STEP_CASE((k_step2<1, kRelax, 15>), 2, kRelax)
    BGK_STEP_CASE((k_step2<1, kLift, 15>), 2, kLift)
    BGK_STEP_CASE((k_step2<2, kCopy, 15>), 4, kCopy)
    BGK_STEP_CASE((k_step2<2, kRelax, 15>), 4, kRelax)
    BGK_STEP_CASE((k_step2<2, kLift, 15>), 4, kLift)
    BGK_STEP_CASE((k_step2<4, kCopy, 15>), 8, kCopy)
    BGK_STEP_CASE((k_step2<4, kRelax, 15>), 8, kRelax)
    BGK_STEP_CASE((k_step2<4, kLift, 15>), 8, kLift)
  } else if (t.pair) {
    BGK_STEP_CASE((k_step2<1, kCopy, 5>), 2, kCopy)
    BGK_STEP_CASE((k_step2<1, kRelax, 5>), 2, kRelax)
    BGK_STEP_CASE((k_step2<1, kLift, 5>), 2, kLift)
    BGK_STEP_CASE((k_step2<2, kCopy, 5>), 4, kCopy)
    BGK_STEP_CASE((k_step2<2, kRelax, 5>), 4, kRelax)
    BGK_STEP_CASE((k_step2<2, kLift, 5>), 4, kLift)
    BGK_STEP_CASE((k_step2<4, kCopy, 5>), 8, kCopy)
    BGK_STEP_CASE((k_step2<4, kRelax, 5>), 8, kRelax)
    BGK_STEP_CASE((k_step2<4, kLift, 5>), 8, kLift)
  } else if (ns == 15) {
    BGK_STEP_CASE((k_step<2, kCopy, false, false, 15>), 2, kCopy)
    BGK_STEP_CASE((k_step<2, kRelax, false, false, 15>), 2, kRelax)
    BGK_STEP_CASE((k_step<2, kLift, false, false, 15>), 2, kLift)
    BGK_STEP_CASE((k_step<4, kCopy, false, false, 15>), 4, kCopy)
    BGK_STEP_CASE((k_step<4, kRelax, false, false, 15>), 4, kRelax)
    BGK_STEP_CASE((k_step<4, kLift, false, false, 15>), 4, kLift)
    BGK_STEP_CASE((k_step<8, kCopy, false, false, 15>), 8, kCopy)
    BGK_STEP_CASE((k_step<8, kRelax, false, false, 15>), 8, kRelax)
    BGK_STEP_CASE((k_step<8, kLift, false, false, 15>), 8, kLift)
  } else {
    BGK_STEP_CASE((k_step<2, kCopy>), 2, kCopy)
    BGK_STEP_CASE((k_step<2, kRelax>), 2, kRelax)
    BGK_STEP_CASE((k_step<2, kLift>), 2, kLift)
    BGK_STEP_CASE((k_step<4, kCopy>), 4, kCopy)
    BGK_STEP_CASE((k_step<4, kRelax>), 4, kRelax)
    BGK_STEP_CASE((k_step<4, kLift>), 4, kLift)
    BGK_STEP_CASE((k_step<8, kCopy>), 8, kCopy)
    BGK_STEP_CASE((k_step<8, kRelax>), 8, kRelax)
    BGK_STEP_CASE((k_step<8, kLift>), 8, kLift)
  }
  set_error("unsupported tile shape");
  return BGK_E_INVALID;
}

int launch_step2x2(const Inst* d_insts, int n_inst, long long total_items, int mode,
                   int phase, Tiles t, int lds_doubles, bool uni_only, hipStream_t s) {
  if (total_items <= 0) return BGK_OK;
  dim3 grid(blocks_for(total_items)), block(kBlock);
  size_t lds = (size_t)lds_doubles * sizeof(double);
  const int chunk = t.chunk;
  if (!t.pair) {
    BGK_STEP_CASE((k_step2x2_flat<2, kRelax>), 2, kRelax)
    BGK_STEP_CASE((k_step2x2_flat<2, kLift>), 2, kLift)
    BGK_STEP_CASE((k_step2x2_flat<4, kRelax>), 4, kRelax)
    BGK_STEP_CASE((k_step2x2_flat<4, kLift>), 4, kLift)
    BGK_STEP_CASE((k_step2x2_flat<8, kRelax>), 8, kRelax)
    BGK_STEP_CASE((k_step2x2_flat<8, kLift>), 8, kLift)
    set_error("unsupported tile shape");
    return BGK_E_INVALID;
  }
  if (uni_only) {
    BGK_STEP_CASE((k_step2x2<1, kRelax, true>), 2, kRelax)
    BGK_STEP_CASE((k_step2x2<1, kLift, true>), 2, kLift)
    BGK_STEP_CASE((k_step2x2<2, kRelax, true>), 4, kRelax)
    BGK_STEP_CASE((k_step2x2<2, kLift, true>), 4, kLift)
    BGK_STEP_CASE((k_step2x2<4, kRelax, true>), 8, kRelax)
    BGK_STEP_CASE((k_step2x2<4, kLift, true>), 8, kLift)
  }
  BGK_STEP_CASE((k_step2x2<1, kRelax, false>), 2, kRelax)
  BGK_STEP_CASE((k_step2x2<1, kLift, false>), 2, kLift)
  BGK_STEP_CASE((k_step2x2<2, kRelax, false>), 4, kRelax)
  BGK_STEP_CASE((k_step2x2<2, kLift, false>), 4, kLift)
  BGK_STEP_CASE((k_step2x2<4, kRelax, false>), 8, kRelax)
  BGK_STEP_CASE((k_step2x2<4, kLift, false>), 8, kLift)
#undef BGK_STEP_CASE
  set_error("unsupported tile shape");
  return BGK_E_INVALID;
}

int launch_step3x(const Inst* d_insts, int n_inst, long long total_items, int mode,
                  int phase, Tiles t, int lds_doubles, hipStream_t s) {
  if (total_items <= 0) return BGK_OK;
  if (!t.pair) {
    set_error("three-step passes need the paired lane mapping");
    return BGK_E_INVALID;
  }
  dim3 grid(blocks_for(total_items)), block(kBlock);
  const size_t lds = (size_t)lds_doubles * sizeof(double);
#define BGK_STEP3_CASE(PP, MM)                                                    \
  if (t.elems == 2 * PP && mode == MM) {                                          \
    hipLaunchKernelGGL((k_step3x<PP, MM>), grid, block, lds, s, d_insts, n_inst,  \
                       t.chunk, phase);                                           \
    hipError_t e_ = hipGetLastError();                                            \
    return e_ == hipSuccess ? BGK_OK : hip_fail(e_, "k_step3x");                  \
  }
  BGK_STEP3_CASE(1, kRelax)
  BGK_STEP3_CASE(1, kLift)
  BGK_STEP3_CASE(2, kRelax)
  BGK_STEP3_CASE(2, kLift)
#undef BGK_STEP3_CASE
  set_error("unsupported tile shape for a three-step pass");
  return BGK_E_INVALID;
}

int launch_step4x(const Inst* d_insts, int n_inst, long long total_items, int mode,
                  int phase, Tiles t, int lds_doubles, hipStream_t s) {
  if (total_items <= 0) return BGK_OK;
  if (!t.pair || t.elems != 2) {
    set_error("four-step passes need the paired lane mapping with one pair per lane");
    return BGK_E_INVALID;
  }
  dim3 grid(blocks_for(total_items)), block(kBlock);
  const size_t lds = (size_t)lds_doubles * sizeof(double);
  if (mode == kRelax)
    hipLaunchKernelGGL((k_step4x<1, kRelax>), grid, block, lds, s, d_insts, n_inst, t.chunk,
                       phase);
  else if (mode == kLift)
    hipLaunchKernelGGL((k_step4x<1, kLift>), grid, block, lds, s, d_insts, n_inst, t.chunk,
                       phase);
  else {
    set_error("unsupported mode for a four-step pass");
    return BGK_E_INVALID;
  }
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

int launch_partials(const Inst* d_insts, int n_inst, long long total_items,
                    int elems, int chunk, hipStream_t s) {
  if (total_items <= 0) return BGK_OK;
  dim3 grid(blocks_for(total_items)), block(kBlock);
  if (elems == 2)
    hipLaunchKernelGGL(k_partials<2>, grid, block, 0, s, d_insts, n_inst, chunk);
  else if (elems == 4)
    hipLaunchKernelGGL(k_partials<4>, grid, block, 0, s, d_insts, n_inst, chunk);
  else if (elems == 8)
    hipLaunchKernelGGL(k_partials<8>, grid, block, 0, s, d_insts, n_inst, chunk);
  else {
    set_error("unsupported tile shape");
    return BGK_E_INVALID;
  }
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

int launch_reduce(const Inst* d_insts, int n_inst, long long total_cells,
                  int mode, int phase, int* d_status, hipStream_t s) {
  (void)phase;
  if (total_cells <= 0) return BGK_OK;
  dim3 grid((unsigned)((total_cells + kWavesPerBlock - 1) / kWavesPerBlock));
  switch (mode) {
#define BGK_REDUCE_CASE(M)                                                       \
  case M:                                                                       \
    hipLaunchKernelGGL(k_reduce<M>, grid, dim3(kBlock), 0, s, d_insts, n_inst, \
                       total_cells, d_status);                                  \
    break;
    BGK_REDUCE_CASE(kRedRelaxFactors)
    BGK_REDUCE_CASE(kRedProject)
    BGK_REDUCE_CASE(kRedMomentsOnly)
    BGK_REDUCE_CASE(kRedMaxwellFactors)
    BGK_REDUCE_CASE(kRedW1)
    BGK_REDUCE_CASE(kRedW2)
    BGK_REDUCE_CASE(kRedW1x3)
    BGK_REDUCE_CASE(kRedW2x3)
    BGK_REDUCE_CASE(kRedW3x3)
    BGK_REDUCE_CASE(kRedW2Project)
    BGK_REDUCE_CASE(kRedW3x3Project)
    BGK_REDUCE_CASE(kRedW1x4)
    BGK_REDUCE_CASE(kRedW2x4)
    BGK_REDUCE_CASE(kRedW3x4)
    BGK_REDUCE_CASE(kRedW4x4)
    BGK_REDUCE_CASE(kRedW4x4Project)
#undef BGK_REDUCE_CASE
    default:
      set_error("unknown reduction mode");
      return BGK_E_INVALID;
  }
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

int launch_lift_factors(const Inst* d_insts, int n_inst, long long total_cells,
                        const double* W, int* d_status, hipStream_t s, int with_aux) {
  if (total_cells <= 0) return BGK_OK;
  dim3 grid((unsigned)((total_cells + kWavesPerBlock - 1) / kWavesPerBlock));
  hipLaunchKernelGGL(k_lift_factors, grid, dim3(kBlock), 0, s, d_insts, n_inst,
                     total_cells, W, d_status, with_aux);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

int launch_relax_out_blocks(const Inst* d_insts, int n_inst, long long blocks,
                            int nvs_max, int src_sel, hipStream_t s) {
  if (blocks <= 0) return BGK_OK;
  hipLaunchKernelGGL(k_relax_out, dim3((unsigned)blocks), dim3(kBlock),
                     (size_t)nvs_max * sizeof(double), s, d_insts, n_inst,
                     (long long)0, src_sel);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

int launch_pad_rows(const double* src, double* dst, long long rows, int nz_live,
                    hipStream_t s) {
  if (rows <= 0) return BGK_OK;
  const long long n = rows * (nz_live + 1);
  const long long blocks = std::min<long long>((n + kBlock - 1) / kBlock, 8192);
  hipLaunchKernelGGL(k_pad_rows, dim3((unsigned)blocks), dim3(kBlock), 0, s, src, dst, rows,
                     nz_live);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

}  // namespace bgk

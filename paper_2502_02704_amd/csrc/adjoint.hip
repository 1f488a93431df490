// Adjoint of the fine IMEX step for gfx950, FP64.
//
// One step is f^{n+1} = R(g), g = T f^n with T the upwind transport and
// R(g) = (g + lambda M[U(g)]) / (1 + lambda).  Given fbar = dL/df^{n+1}:
//   with w = lambda/(1+lambda) fbar, per x cell
//     rhobar = sum w M / rho,  ubar = sum w M (v - u) / theta,
//     thetabar = sum w M (|v-u|^2 / (2 theta^2) - 3 / (2 theta)),
//   mapped through U(rho, m, E) (u = m/rho, theta = (2E/rho - |u|^2)/3) to
//     Etil = 2 thetabar / (3 rho),  mtil = ubar/rho - 2 thetabar u / (3 rho),
//     rhotil = rhobar - ubar.u/rho + thetabar (|u|^2 - 3 theta) / (3 rho),
//   gbar_j = fbar_j / (1+lambda) + dv^3 (rhotil + mtil.v_j + Etil |v_j|^2/2),
//   fbar^n = T^t gbar (transposed upwind stencil with transposed ghost cells),
//   dL/dlog eps += -lambda/(1+lambda)^2 sum fbar (M - g).
// The per-cell sums use deterministic wave partials, as in the forward step.
#include "bgk_internal.h"

namespace bgk {

namespace {

constexpr int E = kAdjElems;

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_mov_a(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xf, true);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xf, true);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wsum_last(double v) {
  v += dpp_mov_a<0xb1, 0xf>(v);
  v += dpp_mov_a<0x4e, 0xf>(v);
  v += dpp_mov_a<0x114, 0xf>(v);
  v += dpp_mov_a<0x118, 0xf>(v);
  v += dpp_mov_a<0x142, 0xa>(v);
  v += dpp_mov_a<0x143, 0xc>(v);
  return v;
}

__device__ __forceinline__ double wsum_all(double v) {
  v = wsum_last(v);
  int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double vg_at(const Inst& I, int a, int j) {
  return I.vlo[a] + (j + 0.5) * I.dv[a];
}

struct El {
  int jx, jy, jz;
  bool ok;
};

__device__ __forceinline__ El el_of(const Inst& I, int j) {
  El r;
  r.ok = j < I.nv3;
  int jj = r.ok ? j : 0;
  int nyz = I.nvy * I.nvz;
  r.jx = jj / nyz;
  int rem = jj - r.jx * nyz;
  r.jy = rem / I.nvz;
  r.jz = rem - r.jy * I.nvz;
  return r;
}

// x row read for row i (ghost rows: periodic wrap, or the boundary row)
__device__ __forceinline__ int ghost_row_a(int i, int nx, int bc) {
  if (i < 0) return bc == 1 ? i + nx : 0;
  if (i >= nx) return bc == 1 ? i - nx : nx - 1;
  return i;
}

// grid: nx * ceil(ntiles4 / 4) blocks; block = (cell, tile group)
__global__ __launch_bounds__(kBlock) void k_adj_sums(
    const Inst* __restrict__ inst, int g_sel, const double* __restrict__ fbar,
    double* part6, int ntiles, int ntg) {
  extern __shared__ double lds[];
  const Inst& I = *inst;
  const int cell = blockIdx.x / ntg;
  const int tg = blockIdx.x % ntg;
  for (int k = threadIdx.x; k < I.nvs; k += kBlock) lds[k] = I.fac[(long long)cell * I.nvs + k];
  __syncthreads();
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int tile = tg * kWavesPerBlock + wave;
  if (tile >= ntiles) return;
  const double* g = I.buf[g_sel] + (long long)cell * I.nv3;
  const double* fb = fbar + (long long)cell * I.nv3;
  double s[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int j = tile * (kWave * E) + e * kWave + lane;
    const El el = el_of(I, j);
    if (!el.ok) continue;
    const double M = lds[el.jx] * lds[I.nvx + el.jy] * lds[I.nvx + I.nvy + el.jz];
    const double vx = vg_at(I, 0, el.jx), vy = vg_at(I, 1, el.jy), vz = vg_at(I, 2, el.jz);
    const double fm = fb[j] * M;
    s[0] += fm;
    s[1] += fm * vx;
    s[2] += fm * vy;
    s[3] += fm * vz;
    s[4] += fm * (vx * vx + vy * vy + vz * vz);
    s[5] += fb[j] * (M - g[j]);
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) s[c] = wsum_last(s[c]);
  if (lane == kWave - 1) {
    double* p = part6 + ((long long)cell * ntiles + tile) * 6;
#pragma unroll
    for (int c = 0; c < 6; ++c) p[c] = s[c];
  }
}

// The cell's coefficients of gbar (rhotil, mtil, Etil/2, times dv^3) and its
// log-eps term from the sums s = (fbar M, fbar M v, fbar M |v|^2, fbar (M - g))
// and the moments of g; the log-eps term is stored, or added to the terms of
// the steps already taken (accumulate).
__device__ __forceinline__ void adj_coefficients(const Inst& I, double rho, const double u[3],
                                                 double usq, double th, const double* s,
                                                 double* cf, double* dle, int accumulate) {
  const double al = I.al;
  // sums of w M = al fbar M and its velocity moments
  const double S0 = s[0], S1[3] = {s[1], s[2], s[3]}, S2 = s[4];
  const double uS1 = u[0] * S1[0] + u[1] * S1[1] + u[2] * S1[2];
  const double rhobar = al * S0 / rho;
  double ubar[3];
  for (int a = 0; a < 3; ++a) ubar[a] = al * (S1[a] - u[a] * S0) / th;
  const double c2 = S2 - 2.0 * uS1 + usq * S0;  // sum fbar M |v-u|^2
  const double thbar = al * (c2 / (2.0 * th * th) - 1.5 * S0 / th);
  const double ubu = ubar[0] * u[0] + ubar[1] * u[1] + ubar[2] * u[2];
  const double Etil = 2.0 * thbar / (3.0 * rho);
  const double rtil = rhobar - ubu / rho + thbar * (usq - 3.0 * th) / (3.0 * rho);
  cf[0] = I.dv3 * rtil;
  for (int a = 0; a < 3; ++a)
    cf[1 + a] = I.dv3 * (ubar[a] / rho - 2.0 * thbar * u[a] / (3.0 * rho));
  cf[4] = I.dv3 * 0.5 * Etil;
  const double d = -al * I.a * s[5];
  *dle = accumulate ? *dle + d : d;
}

// one wave per x cell
__global__ __launch_bounds__(kBlock) void k_adj_reduce(
    const Inst* __restrict__ inst, const double* __restrict__ part6, int ntiles,
    double* coef, double* dle_cells, int accumulate) {
  const Inst& I = *inst;
  const int cell = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  if (cell >= I.nx) return;
  const int lane = threadIdx.x % kWave;
  double s[6] = {0, 0, 0, 0, 0, 0};
  for (int t = lane; t < ntiles; t += kWave) {
#pragma unroll
    for (int c = 0; c < 6; ++c) s[c] += part6[((long long)cell * ntiles + t) * 6 + c];
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) s[c] = wsum_all(s[c]);
  if (lane != 0) return;
  const double* vg = I.vg + (long long)cell * 5;
  const double rho = vg[0];
  const double u[3] = {vg[1] / rho, vg[2] / rho, vg[3] / rho};
  const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const double th = (2.0 * vg[4] / rho - usq) / 3.0;
  adj_coefficients(I, rho, u, usq, th, s, coef + (long long)cell * 5, dle_cells + cell,
                   accumulate);
}

// fbar_prev = T^t gbar; work item = (x chunk, tile group); rows of gbar are
// formed on the fly from fbar_next and the per-cell coefficients.
__global__ __launch_bounds__(kBlock) void k_adj_transpose(
    const Inst* __restrict__ inst, int chunk, int ntiles, int ntg,
    const double* __restrict__ fbar, const double* __restrict__ coef,
    double* out) {
  const Inst& I = *inst;
  const int c = blockIdx.x % I.nchunks;
  const int tg = blockIdx.x / I.nchunks;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int tile = tg * kWavesPerBlock + wave;
  if (tile >= ntiles) return;
  const int nx = I.nx;
  const int i0 = c * chunk, i1 = min(i0 + chunk, nx);
  const bool periodic = I.bc == 1;
  double vx[E], vy[E], vz[E], vsq[E], cL[E], cR[E], cS[E];
  int j[E];
  bool ok[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    j[e] = tile * (kWave * E) + e * kWave + lane;
    const El el = el_of(I, j[e]);
    ok[e] = el.ok;
    vx[e] = vg_at(I, 0, el.jx);
    vy[e] = vg_at(I, 1, el.jy);
    vz[e] = vg_at(I, 2, el.jz);
    vsq[e] = vx[e] * vx[e] + vy[e] * vy[e] + vz[e] * vz[e];
    const double nu = vx[e] * I.r;
    cL[e] = nu > 0.0 ? nu : 0.0;
    cR[e] = nu < 0.0 ? -nu : 0.0;
    cS[e] = 1.0 - fabs(nu);
  }
  // gbar of row r; rows outside [0, nx) are zero unless periodic
  auto grow = [&](int r, double* gb) {
    bool inside = r >= 0 && r < nx;
    int rr = r;
    if (!inside && periodic) {
      rr = r < 0 ? r + nx : r - nx;
      inside = true;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) gb[e] = 0.0;
    if (!inside) return;
    const double* cf = coef + (long long)rr * 5;
    const double* fb = fbar + (long long)rr * I.nv3;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (!ok[e]) continue;
      gb[e] = I.a * fb[j[e]] + cf[0] + cf[1] * vx[e] + cf[2] * vy[e] +
              cf[3] * vz[e] + cf[4] * vsq[e];
    }
  };
  double gm[E], g0[E], gp[E];
  grow(i0 - 1, gm);
  grow(i0, g0);
  for (int i = i0; i < i1; ++i) {
    grow(i + 1, gp);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      double v = cS[e] * g0[e] + cL[e] * gp[e] + cR[e] * gm[e];
      if (!periodic) {
        if (i == 0) v += cL[e] * g0[e];        // left ghost copies cell 0
        if (i == nx - 1) v += cR[e] * g0[e];   // right ghost copies cell nx-1
      }
      if (ok[e]) out[(long long)i * I.nv3 + j[e]] = v;
      gm[e] = g0[e];
      g0[e] = gp[e];
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_sum_into(const double* __restrict__ x,
                                                     int n, double* acc) {
  __shared__ double red[kBlock];
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += kBlock) s += x[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *acc += red[0];
}

// rhobar_i = sum_j fbar_ij M_ij / rho_i; factors of the lift (C included).
__global__ __launch_bounds__(kBlock) void k_lift_adj_rho(
    const Inst* __restrict__ inst, const double* __restrict__ W,
    const double* __restrict__ fbar, double* rhobar) {
  __shared__ double red[kBlock];
  extern __shared__ double lds[];
  const Inst& I = *inst;
  const int cell = blockIdx.x;
  for (int k = threadIdx.x; k < I.nvs; k += kBlock) lds[k] = I.fac[(long long)cell * I.nvs + k];
  __syncthreads();
  double s = 0.0;
  const double* fb = fbar + (long long)cell * I.nv3;
  for (int j = threadIdx.x; j < I.nv3; j += kBlock) {
    const El el = el_of(I, j);
    s += fb[j] * lds[el.jx] * lds[I.nvx + el.jy] * lds[I.nvx + I.nvy + el.jz];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) rhobar[cell] = red[0] / W[(long long)cell * 5];
}

// ------------------------------------------------ whole-cell adjoint step --
// One block per x cell holding all of the cell's velocities (EPT per thread),
// so the per-cell sums are block reductions inside the kernel.  The
// recomputation of a state (FWD) is then one launch: g = T f^k at the cell,
// its moments, the Maxwellian factors al M[U(g)] and f^{k+1} = a g + al M.
// The backward step (BWD) is one launch up to the transposed stencil: g and
// its moments, the unscaled factors of M[U(g)], the sums of fbar M {1, v,
// |v|^2} and of fbar (M - g), and from them the cell's coefficients of gbar
// and its log-eps term.
constexpr int kCellBlock = 512;
constexpr int kCellWaves = kCellBlock / kWave;

// Sum over the block of N values per thread (deterministic order: DPP within
// waves, then the waves in order); every thread receives the sums.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double* red) {
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
#pragma unroll
  for (int c = 0; c < N; ++c) v[c] = wsum_last(v[c]);
  if (lane == kWave - 1)
#pragma unroll
    for (int c = 0; c < N; ++c) red[wave * N + c] = v[c];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < N; ++c) {
    double t = 0.0;
    for (int w = 0; w < kCellWaves; ++w) t += red[w * N + c];
    v[c] = t;
  }
  __syncthreads();
}

template <int EPT, bool BWD>
__global__ __launch_bounds__(kCellBlock) void k_adj_cell(
    const Inst* __restrict__ inst, const double* __restrict__ f, double* __restrict__ fnext,
    const double* __restrict__ fbar, double* coef, double* dle_cells, int accumulate,
    int* status) {
  // factor row [nvs], the reduction scratch, and the cell's g [nv3]
  extern __shared__ double lds[];
  double* red = lds + inst->nvs;
  double* gl = red + kCellWaves * 6;
  const Inst& I = *inst;
  // neighbouring cells on one XCD: the rows i-1 and i+1 a block reads are
  // its neighbours' own rows, in the same L2
  const int nx = I.nx, nv3 = I.nv3;
  const int i = (int)xcd_item(blockIdx.x, (unsigned)nx);
  const double* fc = f + (long long)i * nv3;
  const double* fm = f + (long long)ghost_row_a(i - 1, nx, I.bc) * nv3;
  const double* fp = f + (long long)ghost_row_a(i + 1, nx, I.bc) * nv3;
  // element j = threadIdx.x + k kCellBlock: its (jx, jy, jz) advance by the
  // digits of kCellBlock in the (nvx, nvy, nvz) radix, with carries
  const El el0 = el_of(I, threadIdx.x);
  const int sz = kCellBlock % I.nvz, sy = (kCellBlock / I.nvz) % I.nvy,
            sx = kCellBlock / (I.nvz * I.nvy);
  auto advance = [&](El& el) {
    el.jz += sz;
    if (el.jz >= I.nvz) { el.jz -= I.nvz; ++el.jy; }
    el.jy += sy;
    if (el.jy >= I.nvy) { el.jy -= I.nvy; ++el.jx; }
    el.jx += sx;
  };
  // loads in batches of KB elements issued together (indices past the cell
  // clamped to its last element, their values unused)
  constexpr int KB = EPT < 8 ? EPT : 8;
  double s[5] = {0, 0, 0, 0, 0};
  // batches run as a loop (not unrolled), so no per-element value stays live
  // from one phase into the next
  El el = el0;
#pragma unroll 1
  for (int k0 = 0; k0 < EPT; k0 += KB) {
    double c[KB], up[KB];
    El e2 = el;
#pragma unroll
    for (int k = k0; k < k0 + KB; ++k) {
      if (k > k0) advance(e2);
      const int j = min((int)threadIdx.x + k * kCellBlock, nv3 - 1);
      c[k - k0] = fc[j];
      up[k - k0] = (vg_at(I, 0, e2.jx) > 0.0 ? fm : fp)[j];
    }
#pragma unroll
    for (int k = k0; k < k0 + KB; ++k) {
      if (k > k0) advance(el);
      const bool live = (int)threadIdx.x + k * kCellBlock < nv3;
      const double vx = vg_at(I, 0, el.jx), vy = vg_at(I, 1, el.jy), vz = vg_at(I, 2, el.jz);
      const double nu = vx * I.r;
      const double cc = c[k - k0];
      const double g = live ? fma(fabs(nu), up[k - k0] - cc, cc) : 0.0;
      if (live) gl[threadIdx.x + k * kCellBlock] = g;
      s[0] += g;
      s[1] += g * vx;
      s[2] += g * vy;
      s[3] += g * vz;
      s[4] += g * (vx * vx + vy * vy + vz * vz);
    }
    // el: element k0 + KB - 1; the next batch starts one element on
    if (k0 + KB < EPT) advance(el);
    __builtin_amdgcn_sched_barrier(0);  // batches stay apart (register pressure)
  }
  block_sum<5>(s, red);
  const double rho = s[0] * I.dv3;
  const double mom[3] = {s[1] * I.dv3, s[2] * I.dv3, s[3] * I.dv3};
  const double En = 0.5 * s[4] * I.dv3;
  const double u[3] = {mom[0] / rho, mom[1] / rho, mom[2] / rho};
  const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const double th = (2.0 * En / rho - usq) / 3.0;
  if (threadIdx.x == 0 && !(rho > 0.0 && th > 0.0 && isfinite(rho) && isfinite(th)))
    *status = 1;
  const double C0 = maxwell_norm(rho, th);
  const double inv2t = 1.0 / (2.0 * th);
  for (int k = threadIdx.x; k < I.nvs; k += kCellBlock) {
    const int ax = k < I.nvx ? 0 : (k < I.nvx + I.nvy ? 1 : 2);
    const int jj = k - (ax == 0 ? 0 : (ax == 1 ? I.nvx : I.nvx + I.nvy));
    const double d = vg_at(I, ax, jj) - u[ax];
    const double e = exp(-d * d * inv2t);
    lds[k] = ax == 0 ? (BWD ? C0 : I.al * C0) * e : e;
  }
  __syncthreads();
  if (!BWD) {
    double* out = fnext + (long long)i * nv3;
    el = el0;
#pragma unroll 4
    for (int k = 0; k < EPT; ++k) {
      const int j = threadIdx.x + k * kCellBlock;
      if (k > 0) advance(el);
      if (j >= nv3) continue;
      const double M = (lds[el.jx] * lds[I.nvx + el.jy]) * lds[I.nvx + I.nvy + el.jz];
      out[j] = fma(I.a, gl[j], M);
    }
    return;
  }
  const double* fb = fbar + (long long)i * nv3;
  double w[6] = {0, 0, 0, 0, 0, 0};
  el = el0;
#pragma unroll 1
  for (int k0 = 0; k0 < EPT; k0 += KB) {
    double fbv[KB];
#pragma unroll
    for (int k = k0; k < k0 + KB; ++k)
      fbv[k - k0] = fb[min((int)threadIdx.x + k * kCellBlock, nv3 - 1)];
#pragma unroll
    for (int k = k0; k < k0 + KB; ++k) {
      if (k > 0) advance(el);
      if ((int)threadIdx.x + k * kCellBlock >= nv3) continue;
      const double vx = vg_at(I, 0, el.jx), vy = vg_at(I, 1, el.jy), vz = vg_at(I, 2, el.jz);
      const double M = (lds[el.jx] * lds[I.nvx + el.jy]) * lds[I.nvx + I.nvy + el.jz];
      const double fmv = fbv[k - k0] * M;
      w[0] += fmv;
      w[1] += fmv * vx;
      w[2] += fmv * vy;
      w[3] += fmv * vz;
      w[4] += fmv * (vx * vx + vy * vy + vz * vz);
      w[5] += fbv[k - k0] * (M - gl[threadIdx.x + k * kCellBlock]);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  block_sum<6>(w, red);
  if (threadIdx.x != 0) return;
  adj_coefficients(I, rho, u, usq, th, w, coef + (long long)i * 5, dle_cells + i, accumulate);
}

int adj_ntiles(const Inst& I) { return (I.nv3 + kWave * E - 1) / (kWave * E); }

}  // namespace

int launch_adjoint_sums(const Inst* d_inst, const Inst& h, int g_sel,
                        const double* fbar_next, double* part6, hipStream_t s) {
  const int nt = adj_ntiles(h);
  const int ntg = (nt + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL(k_adj_sums, dim3((unsigned)(h.nx * ntg)), dim3(kBlock),
                     (size_t)h.nvs * sizeof(double), s, d_inst, g_sel, fbar_next,
                     part6, nt, ntg);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

int launch_adjoint_reduce(const Inst* d_inst, const Inst& h, const double* part6,
                          double* coef, double* dle_cells, bool accumulate, hipStream_t s) {
  const int nt = adj_ntiles(h);
  hipLaunchKernelGGL(k_adj_reduce,
                     dim3((unsigned)((h.nx + kWavesPerBlock - 1) / kWavesPerBlock)),
                     dim3(kBlock), 0, s, d_inst, part6, nt, coef, dle_cells,
                     accumulate ? 1 : 0);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

int launch_adjoint_transpose(const Inst* d_inst, const Inst& h, int chunk,
                             const double* fbar_next, const double* coef,
                             double* fbar_prev, hipStream_t s) {
  const int nt = adj_ntiles(h);
  const int ntg = (nt + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL(k_adj_transpose, dim3((unsigned)(h.nchunks * ntg)),
                     dim3(kBlock), 0, s, d_inst, chunk, nt, ntg, fbar_next, coef,
                     fbar_prev);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

int adj_cell_ept(const Inst& h) {
  // the cell's g is kept in LDS next to the factor row
  if (((long long)h.nv3 + h.nvs + kCellWaves * 6) * 8 > kLdsBytes) return 0;
  for (int e = 1; e <= 32; e *= 2)
    if ((long long)e * kCellBlock >= h.nv3) return e;
  return 0;
}

int launch_adj_cell(const Inst* d_inst, const Inst& h, bool backward, const double* f,
                    double* fnext, const double* fbar, double* coef, double* dle_cells,
                    bool accumulate, int* status, hipStream_t s) {
  const int ept = adj_cell_ept(h);
  const size_t lds = ((size_t)h.nvs + (size_t)kCellWaves * 6 + (size_t)h.nv3) * sizeof(double);
  const dim3 grid((unsigned)h.nx), block(kCellBlock);
  const int acc = accumulate ? 1 : 0;
#define BGK_ADJ_CELL(EE)                                                                  \
  if (ept == EE) {                                                                        \
    if (backward)                                                                         \
      hipLaunchKernelGGL((k_adj_cell<EE, true>), grid, block, lds, s, d_inst, f, fnext, fbar, \
                         coef, dle_cells, acc, status);                                   \
    else                                                                                  \
      hipLaunchKernelGGL((k_adj_cell<EE, false>), grid, block, lds, s, d_inst, f, fnext,  \
                         fbar, coef, dle_cells, acc, status);                             \
    BGK_HIP(hipGetLastError());                                                           \
    return BGK_OK;                                                                        \
  }
  BGK_ADJ_CELL(1)
  BGK_ADJ_CELL(2)
  BGK_ADJ_CELL(4)
  BGK_ADJ_CELL(8)
  BGK_ADJ_CELL(16)
  BGK_ADJ_CELL(32)
#undef BGK_ADJ_CELL
  return BGK_E_INVALID;
}

int launch_sum_into(const double* cells, int n, double* acc, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_into, dim3(1), dim3(kBlock), 0, s, cells, n, acc);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

int launch_lift_adjoint_rho(const Inst* d_inst, const Inst& h, const double* W,
                            const double* fbar, double* rhobar, hipStream_t s) {
  hipLaunchKernelGGL(k_lift_adj_rho, dim3((unsigned)h.nx), dim3(kBlock),
                     (size_t)h.nvs * sizeof(double), s, d_inst, W, fbar, rhobar);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

}  // namespace bgk

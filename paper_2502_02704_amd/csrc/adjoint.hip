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

// one wave per x cell; the cell's log-eps term is stored, or added to the
// terms of the steps already taken (accumulate), and summed over cells once
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
  double* cf = coef + (long long)cell * 5;
  cf[0] = I.dv3 * rtil;
  for (int a = 0; a < 3; ++a)
    cf[1 + a] = I.dv3 * (ubar[a] / rho - 2.0 * thbar * u[a] / (3.0 * rho));
  cf[4] = I.dv3 * 0.5 * Etil;
  const double dle = -al * I.a * s[5];
  dle_cells[cell] = accumulate ? dle_cells[cell] + dle : dle;
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

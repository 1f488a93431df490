// Coarse propagator G (Section 3.2) and the parareal correction sweep
// (Algorithm 2) for gfx950, FP64.
//
// G is the Euler system in conserved variables V = (rho, rho u, E) with
// Rusanov fluxes and adaptive CFL substeps.  It is cheap (5 Nx numbers) and
// inherently sequential in time, so one workgroup owns one propagation: it
// keeps the state in LDS (or an L2-resident global slab when it does not fit)
// and synchronises with workgroup barriers, and the whole sequential
// correction sweep of an
// iteration (N slices, each a G propagation plus the jump update) runs inside
// one single-workgroup kernel with no host round trip.
#include "bgk_internal.h"

namespace bgk {

namespace {

constexpr int kCoarseBlock = 512;      // most threads of a cell-per-thread workgroup
constexpr int kCompWaves = 5;          // grids of up to 64 cells: one wave per
constexpr int kCompThreads = 64 * kCompWaves;  // conserved component
constexpr int kMaxSubsteps = 1 << 20;  // hard cap: every loop ends

struct CoarseGeo {
  int nx, bc;
  double dx, cfl, gamma;
  const double* E;  // exterior force at the x centres (null: none)
  double eps;       // > 0: Navier-Stokes viscous and heat fluxes with this eps
};


__device__ __forceinline__ int gh(int i, int nx, int bc) {
  if (i < 0) return bc == 1 ? i + nx : 0;
  if (i >= nx) return bc == 1 ? i - nx : nx - 1;
  return i;
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_get(double v) {
  int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, true);
  int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, true);
  return __hiloint2double(hi, lo);
}

// Maximum over the block of non-negative values (lanes that read outside a
// DPP row see 0, which is neutral here).  One wave: DPP steps that leave
// the maximum in lane 63, no LDS and no barrier.  Several waves: one more
// exchange through LDS between two barriers.
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_get<0xb1, 0xf>(v));   // quad_perm [1,0,3,2]
  v = fmax(v, dpp_get<0x4e, 0xf>(v));   // quad_perm [2,3,0,1]
  v = fmax(v, dpp_get<0x114, 0xf>(v));  // row_shr:4
  v = fmax(v, dpp_get<0x118, 0xf>(v));  // row_shr:8 -> lane 15 of each row
  v = fmax(v, dpp_get<0x142, 0xa>(v));  // row_bcast:15 into rows 1, 3
  v = fmax(v, dpp_get<0x143, 0xc>(v));  // row_bcast:31 into rows 2, 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

__device__ double block_max(double v, double* red) {
  v = wave_max(v);
  if (blockDim.x == 64) return v;
  const int w = threadIdx.x / 64;
  __syncthreads();
  if (threadIdx.x % 64 == 0) red[w] = v;
  __syncthreads();
  double m = red[0];
  for (int k = 1; k < (int)(blockDim.x / 64); ++k) m = fmax(m, red[k]);
  return m;
}

// Navier-Stokes face flux between cells a (left) and b (right).
__device__ __forceinline__ void visc_flux(const CoarseGeo& G, const double* V,
                                          const double* prim, int a, int b, double* D) {
  const double* pa = prim + 4 * a;
  const double* pb = prim + 4 * b;
  const double mu = 0.5 * (V[5 * a] * pa[3] + V[5 * b] * pb[3]);
  const double kappa = 2.5 * mu;
  const double dux = pb[0] - pa[0], duy = pb[1] - pa[1], duz = pb[2] - pa[2];
  const double uxf = 0.5 * (pa[0] + pb[0]), uyf = 0.5 * (pa[1] + pb[1]),
               uzf = 0.5 * (pa[2] + pb[2]);
  const double k = G.eps / G.dx;
  D[0] = 0.0;
  D[1] = k * (4.0 / 3.0) * mu * dux;
  D[2] = k * mu * duy;
  D[3] = k * mu * duz;
  D[4] = k * (mu * ((4.0 / 3.0) * uxf * dux + uyf * duy + uzf * duz) + kappa * (pb[3] - pa[3]));
}

// euler_advance for grids of up to 64 cells on kCompWaves waves: wave c
// updates conserved component c of every cell (lane = cell).  Each wave
// computes the primitives, wave speeds and its component's flux of all cells
// (the same values and the same arithmetic in every wave, so the step size,
// the substep count and the exits agree), takes the neighbours' values by
// lane shuffles, and one workgroup barrier per substep publishes the new
// components.  Same results as the cell-per-thread loop below.
__device__ double* euler_advance_waves(const CoarseGeo& G, double* cur, double* nxt,
                                       double span, int* status, int* nsub_out) {
  const int nx = G.nx;
  const bool viscous = G.eps > 0.0;
  const int comp = threadIdx.x / 64, i = threadIdx.x % 64;
  const bool live = i < nx;
  const int ic = live ? i : 0;
  const int L = gh(ic - 1, nx, G.bc), R = gh(ic + 1, nx, G.bc);
  const double Ei = (G.E != nullptr) ? G.E[ic] : 0.0;
  const double kv = G.eps / G.dx;
  double t = 0.0;
  int nsub = 0;
  while (span - t > 1e-14 * span) {
    const double* V = cur + 5 * ic;
    const double v0 = V[0], v1 = V[1], v2 = V[2], v3 = V[3], v4 = V[4];
    const double rho = v0;
    const double irho = 1.0 / rho;
    const double ux = v1 * irho, uy = v2 * irho, uz = v3 * irho;
    const double usq = ux * ux + uy * uy + uz * uz;
    const double th = (2.0 * v4 * irho - usq) * (1.0 / 3.0);
    const bool bad = live && !(rho > 0.0 && th > 0.0 && isfinite(rho) && isfinite(th));
    const double cs = sqrt(G.gamma * th);
    const double pr = rho * th;
    const double spd = live ? fabs(ux) + cs : 0.0;
    const double hc = comp == 0 ? rho * ux
                    : comp == 1 ? rho * ux * ux + pr
                    : comp == 2 ? rho * ux * uy
                    : comp == 3 ? rho * ux * uz
                                : ux * (v4 + pr);
    const double vc = comp == 0 ? v0 : comp == 1 ? v1 : comp == 2 ? v2 : comp == 3 ? v3 : v4;
    if (bad) *status = 1;
    const double smax = wave_max(bad ? INFINITY : spd);
    if (!(smax > 0.0) || !isfinite(smax) || nsub >= kMaxSubsteps) {
      *status = 1;
      break;  // uniform: every wave sees the same smax and nsub
    }
    double dt = G.cfl * G.dx / smax;
    if (viscous) {
      const double tm = wave_max(bad ? INFINITY : (live ? th : 0.0));
      const double dt_visc = G.cfl * G.dx * G.dx / (2.0 * G.eps * (5.0 / 3.0) * tm);
      if (dt_visc < dt) dt = dt_visc;
    }
    if (dt > span - t) dt = span - t;
    const double r = dt / G.dx;
    const double spdL = __shfl(spd, L), spdR = __shfl(spd, R);
    const double hL = __shfl(hc, L), hR = __shfl(hc, R);
    const double cL = __shfl(vc, L), cR = __shfl(vc, R);
    const double SL = fmax(spdL, spd), SR = fmax(spd, spdR);
    const double Hr = 0.5 * (hc + hR) - 0.5 * SR * (cR - vc);
    const double Hl = 0.5 * (hL + hc) - 0.5 * SL * (vc - cL);
    double nv = vc - r * (Hr - Hl);
    if (viscous) {
      // face fluxes (L, i) and (i, R): mu = mean of rho theta, kappa = 5/2 mu
      const double rL = __shfl(rho, L), rR = __shfl(rho, R);
      const double xL = __shfl(ux, L), xR = __shfl(ux, R);
      const double yL = __shfl(uy, L), yR = __shfl(uy, R);
      const double zL = __shfl(uz, L), zR = __shfl(uz, R);
      const double tL = __shfl(th, L), tR = __shfl(th, R);
      auto face = [&](double ra, double xa, double ya, double za, double ta, double rb,
                      double xb, double yb, double zb, double tb) {
        const double mu = 0.5 * (ra * ta + rb * tb);
        const double kappa = 2.5 * mu;
        const double dux = xb - xa, duy = yb - ya, duz = zb - za;
        const double uxf = 0.5 * (xa + xb), uyf = 0.5 * (ya + yb), uzf = 0.5 * (za + zb);
        return comp == 1 ? kv * (4.0 / 3.0) * mu * dux
             : comp == 2 ? kv * mu * duy
             : comp == 3 ? kv * mu * duz
                         : kv * (mu * ((4.0 / 3.0) * uxf * dux + uyf * duy + uzf * duz) +
                                 kappa * (tb - ta));
      };
      if (comp > 0) {
        const double Dl = face(rL, xL, yL, zL, tL, rho, ux, uy, uz, th);
        const double Dr = face(rho, ux, uy, uz, th, rR, xR, yR, zR, tR);
        nv += r * (Dr - Dl);
      }
    }
    if (G.E != nullptr) {
      if (comp == 1) nv += dt * v0 * Ei;
      if (comp == 4) nv += dt * v1 * Ei;
    }
    if (live) nxt[5 * i + comp] = nv;
    __syncthreads();
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
    t += dt;
    ++nsub;
  }
  if (nsub_out) *nsub_out = nsub;
  return cur;
}

// Advances the state held in `cur` (5*nx doubles) over `span`, ping-ponging
// with `nxt`; h (5*nx), spd (nx) and prim (4*nx) are flux scratch.  With an
// exterior force each substep also adds the source (0, rho E, 0, 0,
// rho u_x E) of its initial state.  With G.eps > 0 it is the Navier-Stokes
// system of the BGK model (mu = rho theta, kappa = 5/2 rho theta): central
// viscous and heat face fluxes, and the diffusive step limit
// dt <= cfl dx^2 / (2 eps (5/3) max theta).  Returns the buffer that holds
// the final state (cur or nxt; identical in all threads) and the substep
// count.  Ends with a barrier after the last write of the state.
__device__ double* euler_advance(const CoarseGeo& G, double* cur, double* nxt, double* h,
                                 double* spd, double* prim, double span, double* red,
                                 int* status, int* nsub_out) {
  if (blockDim.x == kCompThreads) return euler_advance_waves(G, cur, nxt, span, status, nsub_out);
  const int nx = G.nx;
  const bool viscous = G.eps > 0.0;
  double t = 0.0;
  int nsub = 0;
  while (span - t > 1e-14 * span) {
    double lmax = 0.0, thmax = 0.0;
    int bad = 0;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
      const double* V = cur + 5 * i;
      const double rho = V[0];
      // one division per cell (the substep loop is one wave's instruction
      // stream for small grids)
      const double irho = 1.0 / rho;
      const double ux = V[1] * irho, uy = V[2] * irho, uz = V[3] * irho;
      const double usq = ux * ux + uy * uy + uz * uz;
      const double th = (2.0 * V[4] * irho - usq) * (1.0 / 3.0);
      if (!(rho > 0.0 && th > 0.0 && isfinite(rho) && isfinite(th))) bad = 1;
      const double c = sqrt(G.gamma * th);
      const double pr = rho * th;
      spd[i] = fabs(ux) + c;
      h[5 * i + 0] = rho * ux;
      h[5 * i + 1] = rho * ux * ux + pr;
      h[5 * i + 2] = rho * ux * uy;
      h[5 * i + 3] = rho * ux * uz;
      h[5 * i + 4] = ux * (V[4] + pr);
      lmax = fmax(lmax, spd[i]);
      if (viscous) {
        prim[4 * i + 0] = ux;
        prim[4 * i + 1] = uy;
        prim[4 * i + 2] = uz;
        prim[4 * i + 3] = th;
        thmax = fmax(thmax, th);
      }
    }
    if (bad) *status = 1;
    // block_max has barriers for several waves; one wave takes a barrier of
    // its own (cheap) so that the spd/h writes are ordered before the reads
    const double smax = block_max(bad ? INFINITY : lmax, red);
    if (blockDim.x == 64) __syncthreads();
    if (!(smax > 0.0) || !isfinite(smax) || nsub >= kMaxSubsteps) {
      *status = 1;
      break;  // uniform: every thread sees the same smax and nsub
    }
    double dt = G.cfl * G.dx / smax;
    if (viscous) {
      const double tm = block_max(bad ? INFINITY : thmax, red);
      const double dt_visc = G.cfl * G.dx * G.dx / (2.0 * G.eps * (5.0 / 3.0) * tm);
      if (dt_visc < dt) dt = dt_visc;
    }
    if (dt > span - t) dt = span - t;
    const double r = dt / G.dx;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
      const int L = gh(i - 1, nx, G.bc), R = gh(i + 1, nx, G.bc);
      const double SL = fmax(spd[L], spd[i]), SR = fmax(spd[i], spd[R]);
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        const double Hr = 0.5 * (h[5 * i + c] + h[5 * R + c]) -
                          0.5 * SR * (cur[5 * R + c] - cur[5 * i + c]);
        const double Hl = 0.5 * (h[5 * L + c] + h[5 * i + c]) -
                          0.5 * SL * (cur[5 * i + c] - cur[5 * L + c]);
        nxt[5 * i + c] = cur[5 * i + c] - r * (Hr - Hl);
      }
      if (viscous) {
        double Dl[5], Dr[5];
        visc_flux(G, cur, prim, L, i, Dl);
        visc_flux(G, cur, prim, i, R, Dr);
#pragma unroll
        for (int c = 1; c < 5; ++c) nxt[5 * i + c] += r * (Dr[c] - Dl[c]);
      }
      if (G.E != nullptr) {
        const double Ei = G.E[i];
        nxt[5 * i + 1] += dt * cur[5 * i + 0] * Ei;
        nxt[5 * i + 4] += dt * cur[5 * i + 1] * Ei;
      }
    }
    __syncthreads();
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
    t += dt;
    ++nsub;
  }
  if (nsub_out) *nsub_out = nsub;
  return cur;
}

// Propagates one state over `span`; scratch holds 16*nx doubles (in LDS
// when it fits, else an L2-resident global slab).  Returns the substep count
// (identical in all threads).
__device__ int euler_propagate(const CoarseGeo& G, const double* Vin,
                               double* Vout, double span, double* scratch,
                               double* red, int* status) {
  const int nx = G.nx;
  for (int k = threadIdx.x; k < 5 * nx; k += blockDim.x) scratch[k] = Vin[k];
  __syncthreads();
  int nsub = 0;
  const double* fin = euler_advance(G, scratch, scratch + 5 * nx, scratch + 10 * nx,
                                    scratch + 15 * nx, scratch + 16 * nx, span, red, status,
                                    &nsub);
  for (int k = threadIdx.x; k < 5 * nx; k += blockDim.x) Vout[k] = fin[k];
  __syncthreads();
  return nsub;
}

// Scratch of one workgroup: its dynamic LDS when use_lds, else the slab.
__device__ __forceinline__ double* coarse_scratch(bool use_lds, double* slab) {
  extern __shared__ double lds_scratch[];
  return use_lds ? lds_scratch : slab;
}

__global__ __launch_bounds__(kCoarseBlock) void k_euler(
    CoarseGeo G, const double* __restrict__ Vin, double* Vout, double span,
    int* nsub_out, double* scratch, int* status, int use_lds) {
  __shared__ double red[kCoarseBlock / 64];
  const long long m = blockIdx.x;
  const long long sl = 5LL * G.nx;
  double* sc = coarse_scratch(use_lds, scratch + m * (long long)kCoarseScratch * G.nx);
  int n = euler_propagate(G, Vin + m * sl, Vout + m * sl, span, sc, red, status);
  if (nsub_out != nullptr && threadIdx.x == 0) nsub_out[m] = n;
}

// U[0] = V(W0), U[n] = G(U[n-1]) for n = 1..N; Gc[n] = U[n].  The state
// stays in the workgroup's scratch from one slice to the next.
__global__ __launch_bounds__(kCoarseBlock) void k_parareal_init(
    CoarseGeo G, int n_slices, const double* __restrict__ W0, double* U,
    double* Gc, double span, double* scratch_slab, int* status, int use_lds) {
  __shared__ double red[kCoarseBlock / 64];
  double* scratch = coarse_scratch(use_lds, scratch_slab);
  const int nx = G.nx;
  const long long sl = 5LL * nx;
  double* cur = scratch;
  double* oth = scratch + 5 * nx;
  for (int i = threadIdx.x; i < nx; i += blockDim.x) {
    const double* w = W0 + 5 * i;
    const double rho = w[0];
    const double usq = w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
    double v[5] = {rho, rho * w[1], rho * w[2], rho * w[3], 0.5 * rho * usq + 1.5 * rho * w[4]};
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      U[5 * i + c] = v[c];
      cur[5 * i + c] = v[c];
    }
  }
  __syncthreads();
  for (int n = 1; n <= n_slices; ++n) {
    double* fin = euler_advance(G, cur, oth, scratch + 10 * nx, scratch + 15 * nx,
                                scratch + 16 * nx, span, red,
                                status, nullptr);
    for (long long q = threadIdx.x; q < sl; q += blockDim.x) {
      U[n * sl + q] = fin[q];
      Gc[n * sl + q] = fin[q];
    }
    oth = (fin == cur) ? oth : cur;
    cur = fin;
  }
}

// One correction sweep of iteration k: U_new[n] = U_old[n] for n <= k, then
// for n = k+1..N in order: g = G(U_new[n-1]); U_new[n] = g + (VF[n] - Gc[n]);
// Gc[n] = g.  *err = max over n, cells, components of |U_new - U_old|.
// The state stays in the workgroup's scratch from one slice to the next.
// R > 0: each thread owns R entries q = tid + r * blockDim of a slice and
// loads VF, Gc and U_old of slice n before propagating into it, so those
// reads overlap the propagation (requires R * blockDim >= 5 * nx).
template <int R>
__global__ __launch_bounds__(kCoarseBlock) void k_parareal_sweep(
    CoarseGeo G, int n_slices, int k, const double* __restrict__ U_old,
    double* U_new, const double* __restrict__ VF, double* Gc, double span,
    double* scratch_slab, double* err, int* status, int use_lds) {
  __shared__ double red[kCoarseBlock / 64];
  double* scratch = coarse_scratch(use_lds, scratch_slab);
  const int nx = G.nx;
  const long long sl = 5LL * nx;
  double* cur = scratch;
  double* oth = scratch + 5 * nx;
  // frozen slices n <= k: eight loads in flight per thread (one wave copies
  // up to a few thousand values here, so the copy is latency bound)
  const long long ncopy = (k + 1) * sl;
  for (long long q0 = threadIdx.x; q0 < ncopy; q0 += 8LL * blockDim.x) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const long long q = q0 + (long long)u * blockDim.x;
      if (q < ncopy) t[u] = U_old[q];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const long long q = q0 + (long long)u * blockDim.x;
      if (q < ncopy) U_new[q] = t[u];
    }
  }
  for (long long q = threadIdx.x; q < sl; q += blockDim.x) cur[q] = U_old[k * sl + q];
  __syncthreads();
  double lerr = 0.0;
  for (int n = k + 1; n <= n_slices; ++n) {
    const long long base = n * sl;
    double vf[R > 0 ? R : 1], gc[R > 0 ? R : 1], uo[R > 0 ? R : 1];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long long q = threadIdx.x + (long long)r * blockDim.x;
      if (q < sl) {
        vf[r] = VF[base + q];
        gc[r] = Gc[base + q];
        uo[r] = U_old[base + q];
      }
    }
    double* fin = euler_advance(G, cur, oth, scratch + 10 * nx, scratch + 15 * nx,
                                scratch + 16 * nx, span, red,
                                status, nullptr);
    auto update = [&](long long q, double v, double c, double o) {
      const double g = fin[q];
      const double un = g + (v - c);
      U_new[base + q] = un;
      Gc[base + q] = g;
      lerr = fmax(lerr, fabs(un - o));
      fin[q] = un;  // the next slice starts from U_new[n]
    };
    if (R > 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const long long q = threadIdx.x + (long long)r * blockDim.x;
        if (q < sl) update(q, vf[r], gc[r], uo[r]);
      }
    } else {
      for (long long q = threadIdx.x; q < sl; q += blockDim.x)
        update(q, VF[base + q], Gc[base + q], U_old[base + q]);
    }
    __syncthreads();
    oth = (fin == cur) ? oth : cur;
    cur = fin;
  }
  const double e = block_max(lerr, red);
  if (threadIdx.x == 0) *err = e;
}

CoarseGeo geo_of(const bgk_problem& p, const double* E, bool viscous) {
  CoarseGeo G;
  G.nx = p.nx;
  G.bc = p.bc;
  G.dx = dx_of(p);
  G.cfl = p.cfl;
  G.gamma = p.sound_gamma;
  G.E = E;
  G.eps = viscous ? p.eps : 0.0;
  return G;
}

// Threads per coarse workgroup: one wave per conserved component up to 64
// cells (scratch in LDS: kCoarseScratch nx doubles, at most 10 KB), else one
// per cell in whole waves up to 512 (several cells per thread beyond).
int coarse_threads(int nx) {
  if (nx <= 64) return kCompThreads;
  return nx <= kCoarseBlock ? (nx + 63) / 64 * 64 : kCoarseBlock;
}

// Dynamic LDS bytes for `doubles` of scratch (grids of up to 960 cells), or
// 0 if it must stay in an L2-resident global slab.
size_t coarse_lds(size_t doubles) {
  const size_t bytes = doubles * sizeof(double);
  return bytes <= 150 * 1024 ? bytes : 0;
}

}  // namespace

int launch_euler(const bgk_problem& p, int batch, const double* V_in,
                 double* V_out, double t_span, int* n_sub, double* scratch,
                 int* d_status, hipStream_t s, const double* E, bool viscous) {
  const size_t lds = coarse_lds(kCoarseScratch * (size_t)p.nx);
  hipLaunchKernelGGL(k_euler, dim3(batch), dim3(coarse_threads(p.nx)), lds, s, geo_of(p, E, viscous),
                     V_in, V_out, t_span, n_sub, scratch, d_status, lds ? 1 : 0);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

int launch_pararealsweep_init(const bgk_problem& p, int n_slices,
                              const double* W0, double* U, double* Gc,
                              double t_span, double* scratch, int* d_status,
                              hipStream_t s, const double* E, bool viscous) {
  const size_t lds = coarse_lds(kCoarseScratch * (size_t)p.nx);
  hipLaunchKernelGGL(k_parareal_init, dim3(1), dim3(coarse_threads(p.nx)), lds, s,
                     geo_of(p, E, viscous), n_slices, W0, U, Gc, t_span, scratch, d_status,
                     lds ? 1 : 0);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

int launch_parareal_sweep(const bgk_problem& p, int n_slices, int k,
                          const double* U_old, double* U_new, const double* VF,
                          double* Gc, double t_span, double* scratch,
                          double* d_err, int* d_status, hipStream_t s, const double* E,
                          bool viscous) {
  const size_t lds = coarse_lds(kCoarseScratch * (size_t)p.nx);
  const int threads = coarse_threads(p.nx);
  const long long per = (5LL * p.nx + threads - 1) / threads;  // entries per thread
  if (per <= 5) {
    hipLaunchKernelGGL(k_parareal_sweep<5>, dim3(1), dim3(threads), lds, s, geo_of(p, E, viscous),
                       n_slices, k, U_old, U_new, VF, Gc, t_span, scratch, d_err, d_status,
                       lds ? 1 : 0);
  } else if (per <= 10) {
    hipLaunchKernelGGL(k_parareal_sweep<10>, dim3(1), dim3(threads), lds, s, geo_of(p, E, viscous),
                       n_slices, k, U_old, U_new, VF, Gc, t_span, scratch, d_err, d_status,
                       lds ? 1 : 0);
  } else {
    hipLaunchKernelGGL(k_parareal_sweep<0>, dim3(1), dim3(threads), lds, s, geo_of(p, E, viscous),
                       n_slices, k, U_old, U_new, VF, Gc, t_span, scratch, d_err, d_status,
                       lds ? 1 : 0);
  }
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

}  // namespace bgk

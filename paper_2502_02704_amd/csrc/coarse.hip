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

constexpr int kCoarseBlock = 256;
constexpr int kMaxSubsteps = 1 << 20;  // hard cap: every loop ends

struct CoarseGeo {
  int nx, bc;
  double dx, cfl, gamma;
};

__device__ __forceinline__ int gh(int i, int nx, int bc) {
  if (i < 0) return bc == 1 ? i + nx : 0;
  if (i >= nx) return bc == 1 ? i - nx : nx - 1;
  return i;
}

__device__ double block_max(double v, double* red) {
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int w = threadIdx.x / 64;
  __syncthreads();
  if (threadIdx.x % 64 == 0) red[w] = v;
  __syncthreads();
  double m = red[0];
  for (int k = 1; k < (int)(blockDim.x / 64); ++k) m = fmax(m, red[k]);
  return m;
}

// Propagates one state over `span`; scratch holds 16*nx doubles (in LDS
// when it fits, else an L2-resident global slab).  Returns the substep count
// (identical in all threads).
__device__ int euler_propagate(const CoarseGeo& G, const double* Vin,
                               double* Vout, double span, double* scratch,
                               double* red, int* status) {
  const int nx = G.nx;
  double* cur = scratch;
  double* nxt = scratch + 5 * nx;
  double* h = scratch + 10 * nx;
  double* spd = scratch + 15 * nx;
  for (int k = threadIdx.x; k < 5 * nx; k += blockDim.x) cur[k] = Vin[k];
  __syncthreads();
  double t = 0.0;
  int nsub = 0;
  while (span - t > 1e-14 * span) {
    double lmax = 0.0;
    int bad = 0;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
      const double* V = cur + 5 * i;
      const double rho = V[0];
      const double ux = V[1] / rho, uy = V[2] / rho, uz = V[3] / rho;
      const double usq = ux * ux + uy * uy + uz * uz;
      const double th = (2.0 * V[4] / rho - usq) / 3.0;
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
    }
    if (bad) *status = 1;
    const double smax = block_max(bad ? INFINITY : lmax, red);  // includes a barrier
    if (!(smax > 0.0) || !isfinite(smax) || nsub >= kMaxSubsteps) {
      *status = 1;
      break;  // uniform: every thread sees the same smax and nsub
    }
    double dt = G.cfl * G.dx / smax;
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
    }
    __syncthreads();
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
    t += dt;
    ++nsub;
  }
  for (int k = threadIdx.x; k < 5 * nx; k += blockDim.x) Vout[k] = cur[k];
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
  double* sc = coarse_scratch(use_lds, scratch + m * 16LL * G.nx);
  int n = euler_propagate(G, Vin + m * sl, Vout + m * sl, span, sc, red, status);
  if (nsub_out != nullptr && threadIdx.x == 0) nsub_out[m] = n;
}

// U[0] = V(W0), U[n] = G(U[n-1]) for n = 1..N; Gc[n] = U[n].
__global__ __launch_bounds__(kCoarseBlock) void k_parareal_init(
    CoarseGeo G, int n_slices, const double* __restrict__ W0, double* U,
    double* Gc, double span, double* scratch_slab, int* status, int use_lds) {
  __shared__ double red[kCoarseBlock / 64];
  double* scratch = coarse_scratch(use_lds, scratch_slab);
  const int nx = G.nx;
  const long long sl = 5LL * nx;
  for (int i = threadIdx.x; i < nx; i += blockDim.x) {
    const double* w = W0 + 5 * i;
    const double rho = w[0];
    const double usq = w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
    double* v = U + 5 * i;
    v[0] = rho;
    v[1] = rho * w[1];
    v[2] = rho * w[2];
    v[3] = rho * w[3];
    v[4] = 0.5 * rho * usq + 1.5 * rho * w[4];
  }
  __syncthreads();
  for (int n = 1; n <= n_slices; ++n) {
    euler_propagate(G, U + (n - 1) * sl, U + n * sl, span, scratch, red, status);
    for (int k = threadIdx.x; k < sl; k += blockDim.x) Gc[n * sl + k] = U[n * sl + k];
    __syncthreads();
  }
}

// One correction sweep of iteration k: U_new[n] = U_old[n] for n <= k, then
// for n = k+1..N in order: g = G(U_new[n-1]); U_new[n] = g + (VF[n] - Gc[n]);
// Gc[n] = g.  *err = max over n, cells, components of |U_new - U_old|.
__global__ __launch_bounds__(kCoarseBlock) void k_parareal_sweep(
    CoarseGeo G, int n_slices, int k, const double* __restrict__ U_old,
    double* U_new, const double* __restrict__ VF, double* Gc, double span,
    double* scratch_slab, double* err, int* status, int use_lds) {
  __shared__ double red[kCoarseBlock / 64];
  double* scratch = coarse_scratch(use_lds, scratch_slab);
  const long long sl = 5LL * G.nx;
  for (long long q = threadIdx.x; q < (k + 1) * sl; q += blockDim.x) U_new[q] = U_old[q];
  __syncthreads();
  double* g = scratch + 16LL * G.nx;  // after the propagation scratch
  double lerr = 0.0;
  for (int n = k + 1; n <= n_slices; ++n) {
    euler_propagate(G, U_new + (n - 1) * sl, g, span, scratch, red, status);
    for (long long q = threadIdx.x; q < sl; q += blockDim.x) {
      const double jump = VF[n * sl + q] - Gc[n * sl + q];
      const double un = g[q] + jump;
      U_new[n * sl + q] = un;
      Gc[n * sl + q] = g[q];
      lerr = fmax(lerr, fabs(un - U_old[n * sl + q]));
    }
    __syncthreads();
  }
  const double e = block_max(lerr, red);
  if (threadIdx.x == 0) *err = e;
}

CoarseGeo geo_of(const bgk_problem& p) {
  CoarseGeo G;
  G.nx = p.nx;
  G.bc = p.bc;
  G.dx = dx_of(p);
  G.cfl = p.cfl;
  G.gamma = p.sound_gamma;
  return G;
}

// Threads per coarse workgroup: one per cell up to 256 (whole waves).
int coarse_threads(int nx) {
  return nx <= 64 ? 64 : (nx <= 128 ? 128 : kCoarseBlock);
}

// Dynamic LDS bytes for `doubles` of scratch, or 0 if it must stay in HBM.
size_t coarse_lds(size_t doubles) {
  const size_t bytes = doubles * sizeof(double);
  return bytes <= 60 * 1024 ? bytes : 0;
}

}  // namespace

int launch_euler(const bgk_problem& p, int batch, const double* V_in,
                 double* V_out, double t_span, int* n_sub, double* scratch,
                 int* d_status, hipStream_t s) {
  const size_t lds = coarse_lds(16 * (size_t)p.nx);
  hipLaunchKernelGGL(k_euler, dim3(batch), dim3(coarse_threads(p.nx)), lds, s, geo_of(p),
                     V_in, V_out, t_span, n_sub, scratch, d_status, lds ? 1 : 0);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

int launch_pararealsweep_init(const bgk_problem& p, int n_slices,
                              const double* W0, double* U, double* Gc,
                              double t_span, double* scratch, int* d_status,
                              hipStream_t s) {
  const size_t lds = coarse_lds(16 * (size_t)p.nx);
  hipLaunchKernelGGL(k_parareal_init, dim3(1), dim3(coarse_threads(p.nx)), lds, s,
                     geo_of(p), n_slices, W0, U, Gc, t_span, scratch, d_status,
                     lds ? 1 : 0);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

int launch_parareal_sweep(const bgk_problem& p, int n_slices, int k,
                          const double* U_old, double* U_new, const double* VF,
                          double* Gc, double t_span, double* scratch,
                          double* d_err, int* d_status, hipStream_t s) {
  const size_t lds = coarse_lds(21 * (size_t)p.nx);
  hipLaunchKernelGGL(k_parareal_sweep, dim3(1), dim3(coarse_threads(p.nx)), lds, s,
                     geo_of(p), n_slices, k, U_old, U_new, VF, Gc, t_span,
                     scratch, d_err, d_status, lds ? 1 : 0);
  BGK_HIP(hipGetLastError());
  return BGK_OK;
}

}  // namespace bgk

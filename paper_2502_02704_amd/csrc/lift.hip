// Lifting of order one (Definition 3 with L = 1) for gfx950, FP64.
//
// f = M[rho,u,theta] (1 - eps P), c = v - u, with P the first Chapman-Enskog
// correction of the BGK operator (relaxation rate 1/eps):
//   P = (u_x'/theta)(c_x^2 - |c|^2/3) + (u_y'/theta) c_x c_y
//       + (u_z'/theta) c_x c_z + (theta'/theta) c_x (|c|^2/(2 theta) - 5/2),
// ' the x-derivative by central differences of the primitive moments of the
// conserved input (ghost cells from the boundary condition).  Its stress and
// heat flux are the Navier-Stokes ones with mu = rho theta and kappa =
// 5/2 rho theta.  One block per (member, x cell, slab of 4 * kBlock
// velocities): the block forms the cell's separable Maxwellian factors in LDS
// (3 Nv exponentials) and writes its slab of f, which the first step then
// reads as its copy-mode source.
#include "bgk_internal.h"

namespace bgk {

namespace {

__device__ __forceinline__ int ghost_cell(int i, int nx, int bc) {
  if (i < 0) return bc == 1 ? i + nx : 0;
  if (i >= nx) return bc == 1 ? i - nx : nx - 1;
  return i;
}

// Primitive (u_x, u_y, u_z, theta) and density of conserved V.
__device__ __forceinline__ void prim_of(const double* V, double& rho, double w[4]) {
  rho = V[0];
  w[0] = V[1] / rho;
  w[1] = V[2] / rho;
  w[2] = V[3] / rho;
  const double usq = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  w[3] = (2.0 * V[4] / rho - usq) / 3.0;
}

__global__ __launch_bounds__(kBlock) void k_lift_ce(const Inst* __restrict__ insts,
                                                    double dx, double eps, int* status) {
  extern __shared__ double lds[];  // Ex (scaled by rho (2 pi theta)^-3/2), Ey, Ez
  const Inst& I = insts[0];
  const long long slabs = (I.nv3 + 4 * kBlock - 1) / (4 * kBlock);
  const long long cl = blockIdx.x / slabs;  // member * nx + x cell
  const int slab = (int)(blockIdx.x % slabs);
  const int nx = I.nx;
  const long long b = cl / nx;
  const int i = (int)(cl - b * nx);
  const double* vb = I.vin + b * nx * 5;
  double rho, w[4], rl, wl[4], rr, wr[4];
  prim_of(vb + 5 * i, rho, w);
  prim_of(vb + 5 * ghost_cell(i - 1, nx, I.bc), rl, wl);
  prim_of(vb + 5 * ghost_cell(i + 1, nx, I.bc), rr, wr);
  const double th = w[3];
  if (!(rho > 0.0 && th > 0.0 && isfinite(rho) && isfinite(th))) {
    if (threadIdx.x == 0) *status = 1;
  }
  double d[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) d[c] = (wr[c] - wl[c]) / (2.0 * dx);
  const double C0 = maxwell_norm(rho, th);
  const double inv2t = 1.0 / (2.0 * th);
  for (int k = threadIdx.x; k < I.nvs; k += kBlock) {
    const int ax = (k < I.nvx) ? 0 : (k < I.nvx + I.nvy ? 1 : 2);
    const int j = k - (ax == 0 ? 0 : (ax == 1 ? I.nvx : I.nvx + I.nvy));
    const double c = I.vlo[ax] + (j + 0.5) * I.dv[ax] - w[ax];
    const double e = exp(-c * c * inv2t);
    lds[k] = ax == 0 ? C0 * e : e;
  }
  __syncthreads();
  const int nyz = I.nvy * I.nvz;
  double* out = I.buf[1] + cl * I.nv3;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int jf = slab * 4 * kBlock + q * kBlock + threadIdx.x;
    if (jf >= I.nv3) break;
    const int jx = jf / nyz;
    const int rem = jf - jx * nyz;
    const int jy = rem / I.nvz;
    const int jz = rem - jy * I.nvz;
    const double cx = I.vlo[0] + (jx + 0.5) * I.dv[0] - w[0];
    const double cy = I.vlo[1] + (jy + 0.5) * I.dv[1] - w[1];
    const double cz = I.vlo[2] + (jz + 0.5) * I.dv[2] - w[2];
    const double c2 = cx * cx + cy * cy + cz * cz;
    const double P = d[0] / th * (cx * cx - c2 / 3.0) + d[1] / th * cx * cy +
                     d[2] / th * cx * cz + d[3] / th * cx * (c2 / (2.0 * th) - 2.5);
    const double M = lds[jx] * lds[I.nvx + jy] * lds[I.nvx + I.nvy + jz];
    out[jf] = M * (1.0 - eps * P);
  }
}

}  // namespace

int launch_lift_ce(const Inst* d_inst, const Inst& h, double dx, double eps, int* d_status,
                   hipStream_t s) {
  const long long slabs = (h.nv3 + 4 * kBlock - 1) / (4 * kBlock);
  const long long blocks = (long long)h.nbatch * h.nx * slabs;
  if (blocks <= 0) return BGK_OK;
  hipLaunchKernelGGL(k_lift_ce, dim3((unsigned)blocks), dim3(kBlock),
                     (size_t)h.nvs * sizeof(double), s, d_inst, dx, eps, d_status);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? BGK_OK : hip_fail(e, "k_lift_ce");
}

}  // namespace bgk

// Internal declarations of libbgk (HIP, gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "bgk.h"

namespace bgk {

constexpr int kWave = 64;            // CDNA wavefront
constexpr int kWavesPerBlock = 8;    // step kernels: independent waves
constexpr int kBlock = kWave * kWavesPerBlock;
constexpr int kMinElems = 2;         // smallest velocity elements per lane
constexpr int kPartElems = 32;       // fewest velocities behind one partial sum
constexpr int kMaxNv = 256;          // per velocity axis
constexpr int kMaxChunk = 64;        // x cells per work item
constexpr int kNumXcd = 8;           // MI355X: 8 accelerator complex dies
constexpr long long kLdsBytes = 163840;  // gfx950 LDS per workgroup (160 KB)

// One problem (or a batch of same-grid members) as the kernels see it.  All
// members b share the grid; member b's arrays start at b * (member stride).
struct Inst {
  int nx, nvx, nvy, nvz;
  int nv3, nvs, bc, nbatch;    // nvs = nvx + nvy + nvz (factor row length)
  int ntiles;                  // velocity tiles of kWave*E elements per x cell
  int ntg;                     // tile groups (kWavesPerBlock tiles) per x cell
  int nchunks;                 // x chunks of L cells
  int steps;                   // steps this instance takes (uneven batches)
  long long item_begin;        // first work item of this instance
  long long items;             // nbatch * ntg * nchunks
  long long cell_begin;        // first x cell (over all members) of this instance
  int part_tiles;              // partial-sum capacity of `part` per x cell
  int nparts;                  // partial sums per x cell the step writes
  int nsum;                    // values per partial: 5 moments, or 15 with the
                               // nu+ and nu- weighted moments (fused passes)
  int crec;                    // nonzero: compact records, 4 values per tile of
                               // crec velocities inside one v_x plane (the nu
                               // weights follow from the tile's v_x)
  double vlo[3], dv[3];        // v_a(j) = vlo[a] + (j + 1/2) dv[a]
  double dv3;                  // dv[0] dv[1] dv[2]
  double r;                    // dt / dx
  double a;                    // 1 / (1 + lambda)
  double al;                   // lambda / (1 + lambda)
  const double* fin;           // step-0 source in copy mode    [nbatch][nx][nv3]
  double* buf[2];              // ping-pong g = f* buffers      [nbatch][nx][nv3]
  double* fout;                // relaxed output                [nbatch][nx][nv3]
  double* part;                // wave partial sums    [nbatch][nx][part_tiles][5]
  double* fac;                 // Maxwellian factors            [nbatch][nx][nvs]
  double* vg;                  // conserved moments of g        [nbatch][nx][5]
  const double* vin;           // lift source moments (conserved)[nbatch][nx][5]
  double* vout;                // projected relaxed moments     [nbatch][nx][5]
  double* fac2;                // factors of the second step of a pass [..][nvs]
  double* aux;                 // per-cell weighted sums (fused passes) [..][nx][kAux]
  double* fac3;                // factors of the third step of a pass  [..][nvs]
  double* aux2;                // sums of the second step (three-step) [..][nx][kAux2]
  double* fac4;                // factors of the fourth step of a pass [..][nvs]
  double* aux3;                // sums of the third step (four-step)  [..][nx][kAux3]
  const double* efield;        // exterior force E_i at x centres [nx]; null = none
  double emax;                 // Rusanov coefficient of the v_x flux (>= max |E_i|)
  double rv;                   // dt / dv_x
  int order;                   // x transport: 1 upwind, 2 van Leer limited
  int nvz_live;                // v_z points that carry f: nvz, or nvz - 1 where
                               // each z row ends in one pad point whose
                               // Maxwellian factor is zero (f stays 0 there)
};

// Maxwellian normalisation rho (2 pi theta)^{-3/2} (Definition 2) as
// rho / (x sqrt(x)), x = 2 pi theta: a square root and a division (46
// instructions on gfx950 against 255 for the library's pow; relative error a
// few ulp); NaN for theta < 0 and +inf for theta = 0, as with pow.
__device__ __forceinline__ double maxwell_norm(double rho, double th) {
  const double x = 2.0 * M_PI * th;
  return rho / (x * sqrt(x));
}

// Bijective block -> work-item map that gives each XCD a contiguous range of
// work items (blocks are dispatched round-robin over the 8 XCDs), so x-chunk
// neighbours that share halo rows share an L2.
__device__ __forceinline__ long long xcd_item(unsigned b, unsigned n) {
  unsigned per = n / kNumXcd, rem = n % kNumXcd;
  unsigned x = b % kNumXcd, k = b / kNumXcd;
  return (x < rem) ? (long long)x * (per + 1) + k
                   : (long long)rem * (per + 1) + (long long)(x - rem) * per + k;
}

// Step-kernel source modes.
enum StepMode : int {
  kCopy = 0,   // f = fin (first step of a plain fine solve)
  kRelax = 1,  // f = a g + F  (relax-then-transport: g from the last step)
  kLift = 2,   // f = F        (Maxwellian lift fused into the first step)
};

// Reduce-kernel outputs.
enum ReduceMode : int {
  kRedRelaxFactors = 0,  // V(g) and relaxation factors al*M[U(g)]
  kRedProject = 1,       // V(g) and vout = a V(g) + al V(M[U(g)])
  kRedMomentsOnly = 2,   // V(g) into vg (and W into vout if set)
  kRedMaxwellFactors = 3,  // V(g) and unscaled factors M[U(g)] (adjoint)
  kRedW1 = 4,              // kRedRelaxFactors + the weighted sums in aux
  kRedW2 = 5,              // moments of the next transported field from aux
                           // of cells i-1, i, i+1 -> second-step factors fac2
  kRedW1x3 = 6,            // kRedW1 with the nu+^2, nu-^2 weighted sums too
  kRedW2x3 = 7,            // kRedW2 -> fac2, and the weighted sums of the
                           // second-step fields into aux2
  kRedW3x3 = 8,            // kRedW2 on aux2 -> third-step factors fac3
  kRedW2Project = 9,       // kRedW2's moments of the next field, projected:
                           // vout = a V + al V(M[U]) (a last step that is not
                           // written out)
  kRedW3x3Project = 10,    // the same from aux2: the second of two last steps
  kRedW1x4 = 11,           // kRedW1x3 with the nu+^3, nu-^3 weighted sums too
  kRedW2x4 = 12,           // kRedW2x3 to the second power: -> fac2, aux2
  kRedW3x4 = 13,           // from aux2: -> fac3, aux3 (first power)
  kRedW4x4 = 14,           // from aux3: -> fac4
  kRedW4x4Project = 15,    // from aux3, projected: the third of three last steps
};

// aux layout per x cell (conserved-moment units, 5 values each):
//   S, S+, S-    moments of g weighted by 1, nu+ = max(nu,0), nu- = max(-nu,0)
//   A, A+, A-    the same sums of the Maxwellian M[U(g)]
//   S++, S--     moments of g weighted by nu+^2, nu-^2   (three-step passes)
//   A++, A--     the same sums of M[U(g)]                (three-step passes)
//   S+3, S-3     moments of g weighted by nu+^3, nu-^3   (four-step passes)
//   A+3, A-3     the same sums of M[U(g)]                (four-step passes)
// A layout of highest power q holds its first 30 (q = 1), 50 (q = 2) or 70
// (q = 3) values.  aux2 holds the sums of a pass's second-step field
// g^{m+1} and its Maxwellian (to the first power in three-step passes, the
// second in four-step passes), aux3 those of the third-step field (first
// power, four-step passes).
constexpr int kAux = 70;
constexpr int kAux2 = 50;
constexpr int kAux3 = 30;

// ------------------------------------------------ global-memory pointers --
// The arrays an Inst points to live in device global memory, but a pointer
// loaded from a struct is generic to the compiler, and an access through it
// is a FLAT instruction.  FLAT accesses count against the LDS counter as well
// as the vector-memory one, so every wait for an LDS read would also wait for
// the HBM loads and stores still in flight.  Device code converts such a
// pointer once with gmem() and addresses through gptr<> from then on, which
// gives global_load / global_store.
#define BGK_GLOBAL __attribute__((address_space(1)))
template <class T>
using gptr = BGK_GLOBAL T*;
template <class T>
__device__ __forceinline__ gptr<T> gmem(T* p) {
  return (gptr<T>)p;
}
// 16-byte load and store of two doubles (p 16-byte aligned), through the
// compiler's native vector type: double2's members cannot bind to an object
// in the global address space.
typedef double bgk_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld2(gptr<const double> p) {
  const bgk_d2 t = *reinterpret_cast<gptr<const bgk_d2>>(p);
  return make_double2(t.x, t.y);
}
// The same load marked non-temporal (streamed, not kept in the caches).
__device__ __forceinline__ double2 ld2_nt(gptr<const double> p) {
  const bgk_d2 t = __builtin_nontemporal_load(reinterpret_cast<gptr<const bgk_d2>>(p));
  return make_double2(t.x, t.y);
}
__device__ __forceinline__ void st2(gptr<double> p, double x, double y) {
  bgk_d2 t;
  t.x = x;
  t.y = y;
  *reinterpret_cast<gptr<bgk_d2>>(p) = t;
}

// ---------------------------------------------------------------- errors --
void set_error(const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define BGK_HIP(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return ::bgk::hip_fail(e_, #call); \
  } while (0)

// --------------------------------------------------------- host helpers --
int check_problem(const bgk_problem* p);
double dx_of(const bgk_problem& p);
double dv_of(const bgk_problem& p, int a);
int n_steps_for(const bgk_problem& p, double t_span, int32_t* n, double* dt,
                double emax = 0.0);
size_t align_up(size_t n, size_t a = 256);

// Workspace header (first 256 bytes of every workspace).
struct WsHeader {
  int status;        // sticky non-physical flag
  int pad0;
  double err;        // parareal successive error
  double scratch[30];
};

// Workspace bytes of bgk_fine_propagate_moments for `batch` members, and
// that call itself (no force, Maxwellian lift, first-order transport) on a
// caller-chosen workspace.  propagate_ws_bytes expects a checked problem.
size_t propagate_ws_bytes(const bgk_problem& p, int batch);
int propagate_plain(const bgk_problem* prob, int32_t batch, const double* V_in,
                    double* V_out, double t_span, void* ws, size_t ws_bytes,
                    void* stream);

// ------------------------------------------------------------ launchers --
struct Tiles {
  int elems;   // velocity elements per lane
  int chunk;   // x cells per work item
  int pair;    // 1: lanes own pairs of adjacent velocities (needs even nv_z)
  int vcol;    // 1: lanes own (v_y, v_z) points, elements run along v_x
               //    (exterior-force step only; elems = v_x points per lane)
};

// generic: tiles for the generic lane mapping (no velocity pairs); force:
// the exterior-force step, on v_x columns where the grid allows; limited:
// the second-order x transport.
Tiles choose_tiles(const bgk_problem& p, int batch, bool generic = false,
                   bool force = false, bool limited = false);

// Fused relax-then-transport step over all instances in `d_insts`.
// ns: sums per partial, 5 (moments) or 15 (plus nu-weighted, paired only).
// force: one step with the exterior-force v_x transport (generic lanes, or
// the v_x-column mapping t.vcol).
// order 2: x transport with the van Leer limited Lax-Wendroff correction
// (generic lanes, 2 or 4 elements per lane, LDS rows for (chunk + 4) cells).
// uni: the limited step on tiles that each lie in one v_x plane (compact
// records; the descriptor's crec set).
int launch_step(const Inst* d_insts, int n_inst, long long total_items,
                int mode, int phase, Tiles t, int lds_doubles, int* d_status,
                hipStream_t s, int ns = 5, bool force = false, int order = 1,
                bool uni = false);
// Per-x-cell reduction of partial sums into moments and factors.
int launch_reduce(const Inst* d_insts, int n_inst, long long total_cells,
                  int mode, int phase, int* d_status, hipStream_t s);
// Lift factors from conserved (vin) or primitive moments.
int launch_lift_factors(const Inst* d_insts, int n_inst, long long total_cells,
                        const double* W, int* d_status, hipStream_t s,
                        int with_aux = 0);
// Two IMEX steps per pass (paired lanes): mode kRelax or kLift for the first.
// uni_only: every tile lies in one v_x plane (nvy*nvz a multiple of 64*elems).
int launch_step2x2(const Inst* d_insts, int n_inst, long long total_items,
                   int mode, int phase, Tiles t, int lds_doubles, bool uni_only,
                   hipStream_t s);
// Three IMEX steps per pass (paired lanes, every tile in one v_x plane,
// compact records, nx >= 3): mode kRelax or kLift for the first.
int launch_step3x(const Inst* d_insts, int n_inst, long long total_items, int mode,
                  int phase, Tiles t, int lds_doubles, hipStream_t s);
// Four IMEX steps per pass (one velocity pair per lane, every tile in one v_x
// plane, compact records, nx >= 4): mode kRelax or kLift for the first.
int launch_step4x(const Inst* d_insts, int n_inst, long long total_items, int mode,
                  int phase, Tiles t, int lds_doubles, hipStream_t s);
// Partial sums of an arbitrary f (source = fin), no transport.
int launch_partials(const Inst* d_insts, int n_inst, long long total_items,
                    int elems, int chunk, hipStream_t s);

// Scratch doubles per x cell of one coarse propagation: state and next state
// (5 + 5), physical flux (5), wave speed (1), primitive u and theta (4).
constexpr int kCoarseScratch = 20;

// Lifting of order one (first Chapman-Enskog correction) of the conserved
// moments h.vin of every member into h.buf[1] (device copy d_inst of h).
int launch_lift_ce(const Inst* d_inst, const Inst& h, double dx, double eps, int* d_status,
                   hipStream_t s);

// Coarse propagation, one workgroup per batch member.  E: exterior force at
// the x centres (device, nullable), added as a source term; viscous: the
// Navier-Stokes system of the BGK model instead of Euler's.
int launch_euler(const bgk_problem& p, int batch, const double* V_in,
                 double* V_out, double t_span, int* n_sub, double* scratch,
                 int* d_status, hipStream_t s, const double* E = nullptr,
                 bool viscous = false);
// Parareal initial coarse sweep and per-iteration correction sweep.
int launch_pararealsweep_init(const bgk_problem& p, int n_slices,
                              const double* W0, double* U, double* Gc,
                              double t_span, double* scratch, int* d_status,
                              hipStream_t s, const double* E = nullptr,
                              bool viscous = false);
int launch_parareal_sweep(const bgk_problem& p, int n_slices, int k,
                          const double* U_old, double* U_new, const double* VF,
                          double* Gc, double t_span, double* scratch,
                          double* d_err, int* d_status, hipStream_t s,
                          const double* E = nullptr, bool viscous = false);
int launch_prim_to_cons(const double* W, double* V, int n, hipStream_t s);

// f_out = a g + F from buf[src_sel], or f_out = F (pure lift) if src_sel < 0;
// with pad points (nvz_live < nvz) f_out holds only the live points.
int launch_relax_out_blocks(const Inst* d_insts, int n_inst, long long blocks,
                            int nvs_max, int src_sel, hipStream_t s);
// dst[rows][nz_live + 1] = src[rows][nz_live] with a zero pad point per row.
int launch_pad_rows(const double* src, double* dst, long long rows, int nz_live,
                    hipStream_t s);

// Adjoint kernels (single instance, nbatch = 1).  g is read from
// buf[g_sel]; factors in fac are the unscaled Maxwellian of U(g).
int launch_adjoint_sums(const Inst* d_inst, const Inst& h_inst, int g_sel,
                        const double* fbar_next, double* part6, hipStream_t s);
int launch_adjoint_reduce(const Inst* d_inst, const Inst& h_inst,
                          const double* part6, double* coef,
                          double* dle_cells, bool accumulate, hipStream_t s);
int launch_adjoint_transpose(const Inst* d_inst, const Inst& h_inst, int chunk,
                             const double* fbar_next, const double* coef,
                             double* fbar_prev, hipStream_t s);
int launch_sum_into(const double* cells, int n, double* acc, hipStream_t s);
// Whole-cell adjoint kernels (one block per x cell, the cell's velocities in
// the block's registers): elements per thread, 0 where a cell is too large.
int adj_cell_ept(const Inst& h_inst);
// backward false: fnext = a T f + al M[U(T f)] (the recomputation of a
// state); true: from f and fbar (of the next state), the cell coefficients
// of gbar into coef and the log-eps terms into dle_cells (added if
// accumulate).  The transposed stencil follows with launch_adjoint_transpose.
int launch_adj_cell(const Inst* d_inst, const Inst& h_inst, bool backward, const double* f,
                    double* fnext, const double* fbar, double* coef, double* dle_cells,
                    bool accumulate, int* status, hipStream_t s);
int launch_lift_adjoint_rho(const Inst* d_inst, const Inst& h_inst,
                            const double* W, const double* fbar, double* rhobar,
                            hipStream_t s);

constexpr int kAdjElems = 4;  // velocity elements per lane in adjoint kernels

// Timing of the step kernels; kind is one of the BGK_PROF_* tags.
// noalloc_mode(true): the calling thread's calls make no timing events and
// no workspace registry entries (the allocation-free entry point).
void noalloc_mode(bool on);
void prof_before(hipStream_t s);
void prof_after(hipStream_t s, double cells, double bytes_per_cell, int kind);

}  // namespace bgk

// Internal declarations of the hdsw library: complex arithmetic, geometry,
// schedule, context and kernel launchers.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <map>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/hdsw.h"

namespace hdsw {

// ---------------------------------------------------------------- complex
template <class T>
struct alignas(2 * sizeof(T)) cpx {
  T re, im;
};

// a[i] for a small array held in a kernel argument and a per-lane index i:
// a select over constant indices keeps the elements in scalar registers,
// where a[i] would become a dependent vector load from the argument
// segment in every lane.
template <int N>
__device__ __forceinline__ int pick(const int (&a)[N], int i) {
  int v = __builtin_amdgcn_readfirstlane(a[0]);
#pragma unroll
  for (int j = 1; j < N; ++j) v = i == j ? __builtin_amdgcn_readfirstlane(a[j]) : v;
  return v;
}

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also
// waits for every global load in flight, which would drain prefetches issued
// before it; kernels use this one where no global data passes between
// threads of the workgroup.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <class T>
__host__ __device__ inline cpx<T> mk(T r, T i) {
  cpx<T> z;
  z.re = r;
  z.im = i;
  return z;
}
template <class T>
__host__ __device__ inline cpx<T> operator+(cpx<T> a, cpx<T> b) {
  return mk<T>(a.re + b.re, a.im + b.im);
}
template <class T>
__host__ __device__ inline cpx<T> operator-(cpx<T> a, cpx<T> b) {
  return mk<T>(a.re - b.re, a.im - b.im);
}
template <class T>
__host__ __device__ inline cpx<T> operator*(cpx<T> a, cpx<T> b) {
  return mk<T>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <class T>
__host__ __device__ inline cpx<T> operator-(cpx<T> a) {
  return mk<T>(-a.re, -a.im);
}
// acc += a * b
template <class T>
__host__ __device__ inline void cfma(cpx<T>& acc, cpx<T> a, cpx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}
template <class T>
__host__ __device__ inline cpx<T> cinv(cpx<T> a) {
  // 1 / a with scaling against overflow (Smith's method)
  if (fabs(a.re) >= fabs(a.im)) {
    if (a.re == T(0)) return mk<T>(T(0), T(0));
    T r = a.im / a.re, d = a.re + a.im * r;
    return mk<T>(T(1) / d, -r / d);
  }
  T r = a.re / a.im, d = a.im + a.re * r;
  return mk<T>(r / d, T(-1) / d);
}
template <class T, class U>
__host__ __device__ inline cpx<T> ccast(cpx<U> a) {
  return mk<T>(T(a.re), T(a.im));
}

using c64 = cpx<float>;
using c128 = cpx<double>;

// ---------------------------------------------------------------- geometry
// Per-axis sizes of the problem and partition.  Axis 0 = x (fastest).
struct Geometry {
  int dim = 2;
  int N[3] = {1, 1, 1};    // interior nodes per axis
  int P[3] = {1, 1, 1};    // subdomains per axis
  int na[3] = {1, 1, 1};   // interior nodes per subdomain per axis
  int ne[3] = {1, 1, 1};   // extended nodes per subdomain per axis (na + 2W)
  int M[3] = {1, 1, 1};    // global nodes per axis (N + 2W)
  int W = 1;
  double h = 1.0;
  double s0 = 0.0;         // sigma0
  int nsub = 1;
  // 2D block structure: x-lines (n = ne[0]) indexed by y (K = ne[1]).
  // 3D block structure: xy-planes (n = ne[0] ne[1]) indexed by z (K = ne[2]).
  int n = 1, K = 1;
  int nP = 16;                 // n rounded up to a multiple of 16 (MFMA tiles)
  int mid = 0;                 // middle line of the twisted factorization
  int PL = 3;                  // panel lines per subdomain: K block lines + 2 scratch lines
  long long sub_nodes = 1;     // nodes of one extended subdomain
  long long glob_nodes = 1;    // nodes of the global grid
  long long int_nodes = 1;     // interior nodes
  // interface dofs: per side 2 layers x tangential extent
  int nsides = 4;
  int side_len[6] = {0};       // tangential extent of each side
  int side_off[6] = {0};       // offset of each side in the interface vector
  int NI = 0;                  // interface dofs per subdomain

  void sub_coords(int s, int c[3]) const {
    c[0] = s % P[0];
    c[1] = (s / P[0]) % P[1];
    c[2] = s / (P[0] * P[1]);
  }
  int sub_id(const int c[3]) const { return c[0] + P[0] * (c[1] + P[1] * c[2]); }
};

// Device-side view of the geometry (plain struct passed by value).
struct GeoDev {
  int dim, W, n, K, NI, nsub, nP, mid, PL;
  int N[3], P[3], na[3], ne[3], M[3];
  int side_len[6], side_off[6];
};

// Sweep schedule (eq. Sorder2D / Sorder3D, eq. step_subd / step_subd3) and
// trace routing (Rules 2.4/2.5, 4.1/4.2 over the extended sweep list).
struct Schedule {
  int nsweeps = 0;                       // rounds * 2^dim
  std::vector<std::array<int, 3>> dir;   // direction of each sweep
  int nsteps = 0;                        // steps per sweep
  // for every (sweep, step): offset into step_subs and count
  std::vector<int> step_off, step_cnt;
  std::vector<int> step_subs;            // concatenated subdomain ids
  // lprime[L * 6 + face] = sweep that uses a trace generated in sweep L
  // across face (0:-x,1:+x,2:-y,3:+y,4:-z,5:+z); -1 = dropped
  std::vector<int> lprime;
  // in_active[L * 6 + face] = 1 if the face can hold a received trace in
  // sweep L (some sweep L0 <= L routes a trace across it into slot L)
  std::vector<int> in_active;
  // Steps by level of the routing dependences (2D): launch i may run the
  // steps lsteps[lfirst[i] .. lfirst[i + 1]) (indices L * nsteps + st)
  // together, since none of them writes a slot another one reads or writes
  std::vector<int> lfirst, lsteps;
};

// ---------------------------------------------------------------- buffers
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Launch parameters of the autotuner's search space (0: built-in rule).
struct TuneParams {
  int solve_ng = 0;     // 2D complex64 block solve: 1 = 8, 2 = 16 columns per workgroup
  int sweep_rw = 0;     // 2D sweep step: 2 or 4 row tiles per workgroup
  int sweep_kb = 0;     // 2D sweep step: slices of T per register batch
                        // (complex64 6/8/10, complex128 3/4/5/6)
  int gemm_skinny = 0;  // 3D products with <= 8 columns: 1 streaming, 2 tiled
  int sweep_nw = 0;     // 2D sweep step: 4 or 8 waves per workgroup
  int sweep_sched = 0;  // 2D sweep steps: 1 one launch per step, 2 (rule)
                        // the steps of one level of the routing dependences
};

struct Timing {
  int mask = 0;                     // bit k: time kernel class k
  double ms[5] = {0, 0, 0, 0, 0};
  long long launches[5] = {0, 0, 0, 0, 0};
  double flops[5] = {0, 0, 0, 0, 0};
  double bytes[5] = {0, 0, 0, 0, 0};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

}  // namespace hdsw

struct hdsw_ctx {
  hdsw::Geometry g;
  hdsw::GeoDev gd;
  hdsw::Schedule sch;
  hdsw_options opt;
  hipStream_t stream = nullptr;
  int device = 0;
  std::vector<double> kappa;     // interior wavenumber (host copy)
  int nops = 0;
  std::vector<int> op_of_sub;    // subdomain -> distinct operator
  std::vector<int> rep_of_op;    // distinct operator -> representative subdomain
  bool factored = false;
  hdsw_status sticky = HDSW_OK;
  size_t alloc_bytes = 0;
  size_t factor_bytes = 0;
  std::vector<hdsw::DevBuf> bufs;   // every allocation, freed in destroy

  // device arrays (precision independent)
  int* d_op_of_sub = nullptr;
  int* d_step_subs = nullptr;
  int* d_all_subs = nullptr;        // 0..nsub-1
  int* d_all_ops = nullptr;         // 0..nops-1
  double* d_kappa = nullptr;        // interior kappa
  hdsw::c128* d_coef = nullptr;     // per op: operator coefficients (double)
  size_t coef_stride = 0;           // complex entries per op
  hdsw::c128* d_alpha_sub = nullptr;   // local alpha: node/half per axis
  hdsw::c128* d_alpha_glob = nullptr;  // global alpha: node/half per axis
  int alpha_sub_off[6] = {0};          // node_x, half_x, node_y, half_y, node_z, half_z
  int alpha_glob_off[6] = {0};
  double* d_kappa_sub = nullptr;    // per op: kappa on the extended grid
  int* d_flag = nullptr;            // device error flag (singular pivot)
  // plane-block (3D) solves: subdomains grouped by distinct operator
  int ngrp = 0, grp_maxcnt = 0;
  int* d_grp_op = nullptr;          // [ngrp] operator of the group
  int* d_grp_off = nullptr;         // [ngrp] first entry in d_grp_ids
  int* d_grp_cnt = nullptr;         // [ngrp] subdomains in the group
  int* d_grp_ids = nullptr;         // [nsub] subdomain ids, grouped
  int* d_zero_int = nullptr;        // {0}
  int* d_one_int = nullptr;         // {1}
  int* d_piv = nullptr;             // [nops][n] Gauss-Jordan row interchanges
  // plane-block (3D) sweep steps: T rows / columns of the active faces per
  // sweep, and the subdomains of every step grouped by operator
  int* d_sg_op = nullptr;
  int* d_sg_off = nullptr;
  int* d_sg_cnt = nullptr;
  int* d_sg_ids = nullptr;                     // step-local entry indices
  std::vector<int> sg_first, sg_n, sg_maxcnt;  // per (sweep, step)
  // 3D: T in tiles of 64 rows x t_tk columns, faces padded to whole tiles
  int t_tk = 32, t_nrt = 0, t_nkt = 0;
  int t_roff[6] = {0}, t_koff[6] = {0};         // padded face offsets
  int* d_tmap = nullptr;                        // per sweep: row tiles, k tiles, row map
  std::vector<int> tm_rt_off, tm_kt_off, tm_row_off, tm_nrt, tm_nkt, tm_mpad;
  // 3D split-sum partials per right-hand-side column (elements, one part):
  // the larger of the plane solves' and the step GEMMs' needs
  size_t gpart_per_col = 0;


  // precision-dependent factors: element type cpx<float> or cpx<double>
  void* d_X = nullptr;              // [nops][K][nP][nP] column-major blocks
                                    // (3D: [nops][K][n][n], no padding)
  void* d_T = nullptr;              // [nops][NI][NI] column-major (2D)
  void* d_coefT = nullptr;          // coefficients in working precision
  void* d_cface = nullptr;          // [nops][NI/2] face coupling per face and t

  // workspaces sized for Cmax columns
  int Cmax = 0;
  void* d_panel = nullptr;          // [nsub][PL][C][n], PL = K + 2 (lines K, K+1: scratch)
  void* d_slots = nullptr;          // [nsweeps][nsub][C][NI]
  void* d_g = nullptr;              // 3D: [nsub][Cp][padded k] sources of a step
  void* d_srcsum = nullptr;         // [nsub][C][NI] received sources, summed over sweeps
  void* d_y = nullptr;              // [nsub][C][NI] source-driven outputs
  void* d_out = nullptr;            // [nsub][C][NI] step outputs (3D)
  void* d_gpart = nullptr;          // split-sum partial products (3D plane solves)
  size_t gpart_bytes = 0;
  int* d_nzflag = nullptr;          // 2D: [nsub][ceil(C / 8)] nonzero right-hand side of
                                    // the source-driven block solve (0: skipped)
  hdsw::c128* d_xg = nullptr;       // [C][glob] iterate (FP64)
  hdsw::c128* d_rg = nullptr;       // [C][glob] residual (FP64)
  hdsw::c128* d_bg = nullptr;       // [C][glob] right-hand side (FP64)
  double* d_part = nullptr;         // partial norms
  double* d_norm = nullptr;         // [C] norms
  int part_blocks = 0;
  // GMRES workspace
  int gm_m = 0;
  int gm_cols = 0;                  // columns V, Z and dots are sized for
  hdsw::c128* d_V = nullptr;        // [m+1][C][glob]
  hdsw::c128* d_Z = nullptr;        // [m][C][glob]
  hdsw::c128* d_dots = nullptr;     // [m+1][C]
  hdsw::Timing tm;
  hdsw::TuneParams tune;
  bool factor_mfma = true;          // 2D blocks: blocked inversion on the matrix cores

  // continuous batching: occupied column slots, compacted to 0..nact-1
  int batch_cap = 0;
  int nact = 0;
  std::vector<int> slot_of_col;     // physical column -> caller slot id
  std::vector<int> col_of_slot;     // caller slot id -> physical column (-1 free)
  std::vector<double> bnorm_slot;   // ||b|| per slot
  double* h_norm = nullptr;         // pinned host copy of the step's norms
  hipEvent_t step_done = nullptr;
  int step_cols = 0;                // columns the in-flight step covers

  // captured DDM applications: (input, output, columns, accumulate) ->
  // executable graph; a key is captured the second time it is applied and
  // replayed from then on.  Cleared whenever the workspaces or the launch
  // parameters change.
  using GraphKey = std::tuple<const void*, const void*, int, int>;
  std::map<GraphKey, hipGraphExec_t> graphs;
  std::set<GraphKey> graph_seen;
  std::set<GraphKey> graph_bad;        // keys whose capture the runtime refused
  hipStream_t cap_stream = nullptr;    // private stream the captures record on
};

namespace hdsw {

// kernel classes for timing
// kernel classes of the timing API; KT_SOLVE_SRC is the source-driven 2D
// block solve, whose work depends on where the right-hand side is nonzero
// (timed without flops or bytes)
enum { KT_SOLVE = 0, KT_GEMM = 1, KT_FACTOR = 2, KT_RESID = 3, KT_SOLVE_SRC = 4 };

// Complex GEMM on the matrix cores (big.hip):
struct GemmArgs {
  int M, N, Kd;
  const void* A;
  long long lda, sAz;
  const void* B;
  long long ldb, sb, sBz;
  void* C;
  long long ldc, sc, sCz;
  int cpb;
  const int* ids;
  const int* grp_op;
  const int* grp_off;
  const int* grp_cnt;
  int neg;
  int beta;
  // tiled A (64-row x BK-deep tiles stored contiguously, k-major inside a
  // tile): row tile of workgroup x = a_rt[x], chunk ch = tile a_kt[ch], tile
  // (rt, kt) at A + (rt * a_tile_ld + kt) * 64 * BK; null = plain layout
  const int* a_rt;
  const int* a_kt;
  long long a_tile_ld;
  // output row r goes to row c_row[r] of C (-1: dropped); null = r
  const int* c_row;
  // split of the sum into ksplit parts (0 or 1: none); part holds the
  // partial products, ksplit * groups * columns * M elements
  int ksplit;
  void* part;
  int part_cols;
  // 1: products with at most 8 columns use the tiled kernel too (the
  // autotuner's choice); 0: they stream A through the skinny kernel
  int no_skinny;
};

template <class T>
hipError_t gemm(hipStream_t st, const GemmArgs& a, int maxcols, int ngroups);
template <class T>
int gemm_bk();
template <class T>
hipError_t launch_extract_tiled(hdsw_ctx* c, int C, int op, int col0);

// ----- launchers (kernels.hip) ------------------------------------------
hipError_t launch_assemble(hdsw_ctx* c);
template <class T>
hipError_t launch_cast_coef(hdsw_ctx* c);
template <class T>
hipError_t launch_factor_step(hdsw_ctx* c, int step, int middle);
template <class T>
hipError_t launch_fill_panel(hdsw_ctx* c, int mode, int nbatch, const int* d_ids,
                             int C, const c128* rglob, int unit_col0, int* nzflag = nullptr);
template <class T>
hipError_t launch_block_solve(hdsw_ctx* c, int nbatch, const int* d_ops_of_batch,
                              int C, const int* nzflag = nullptr);
template <class T>
hipError_t launch_extract_iface(hdsw_ctx* c, int nbatch, int C, void* dst,
                                long long dst_stride_batch, int dst_ld);
template <class T>
hipError_t launch_write_owned(hdsw_ctx* c, int C, c128* glob, int accumulate);
template <class T>
hipError_t launch_sweep_steps(hdsw_ctx* c, const int* sidx, int nst, int C);
template <class T>
hipError_t launch_face_coef(hdsw_ctx* c);
template <class T>
hipError_t launch_big_factor(hdsw_ctx* c, void* rbuf);
template <class T>
size_t big_factor_scratch_bytes(const hdsw_ctx* c);
hipError_t launch_rhs_from_f(hdsw_ctx* c, const c128* f, c128* b, int C);
hipError_t launch_residual(hdsw_ctx* c, const c128* b, const c128* x, c128* r,
                           int C);
hipError_t launch_norms(hdsw_ctx* c, const c128* v, int C, double* d_out);
hipError_t launch_extract_interior(hdsw_ctx* c, const c128* glob, c128* out,
                                   int C);
hipError_t launch_zero(hdsw_ctx* c, void* p, size_t bytes);
hipError_t launch_copy_cols(hdsw_ctx* c, c128* dst, const c128* src, size_t n);
// GMRES helpers (FP64)
hipError_t launch_dots(hdsw_ctx* c, const c128* V, int nv, const c128* w, int C,
                       c128* d_out);
hipError_t launch_axpy_multi(hdsw_ctx* c, c128* w, const c128* V, int nv,
                             const c128* coef, int C, double sign);
hipError_t launch_scale(hdsw_ctx* c, c128* dst, const c128* src, const double* inv,
                        int C);

}  // namespace hdsw

// HIP kernels of the hdsw library (gfx950).  Every kernel bounds-checks its
// indices against the sizes it is given; launchers check shapes on the host.
//
// Data layout in HBM (x fastest everywhere):
//   operator coefficients, per distinct subdomain operator (2D):
//     ax[K][n+1]  x-face coefficients a^x at the half-points between local
//                 x-nodes q-1 and q (q = 0..n, ghost faces included)
//     ay[K+1][n]  y-face coefficients a^y
//     dg[K][n]    diagonal h^2 k^2 J - (sum of the four face coefficients)
//   factors X[op][k][n][n]: X_k = D_k^{-1}, column-major (entry (r, j) at
//     j*n + r), so a thread per row reads consecutive addresses.
//   panels [batch][k][c][n]: right-hand sides / solutions of a batch of
//     subdomain solves, block k (grid line), column c, in-block index.
//   interface vectors [sub][c][NI]: the two layers next to each face, side
//     order -x, +x, -y, +y, layer 0 = the subdomain's own boundary layer,
//     layer 1 = the adjacent layer inside its own PML.
//   trace slots [sweep][sub][c][NI]: received pairs, in the receiver's
//     layer-0 / layer-1 convention.
//   global vectors [c][M_y][M_x] complex128.
#include "hdsw_internal.hpp"

namespace hdsw {

// ------------------------------------------------------------ helpers
// Local node coordinates (x, y, z) of an extended subdomain; a block is a
// grid line in 2D (in-block index p = x, block k = y) and a plane in 3D
// (p = y n_x + x, k = z).  Coordinates are kept in scalars: a small local
// array indexed by a run-time axis would live in scratch memory.
struct Loc {
  int x, y, z;
  __device__ int at(int a) const { return a == 0 ? x : (a == 1 ? y : z); }
  __device__ void set(int a, int v) {
    if (a == 0) x = v;
    else if (a == 1) y = v;
    else z = v;
  }
};
__device__ inline Loc block_node(const GeoDev& g, int p, int k) {
  Loc l;
  if (g.dim == 2) {
    l.x = p;
    l.y = k;
    l.z = 0;
  } else {
    l.y = p / g.ne[0];
    l.x = p - l.y * g.ne[0];
    l.z = k;
  }
  return l;
}
__device__ inline Loc sub_coords(const GeoDev& g, int s) {
  Loc c;
  c.x = s % g.P[0];
  c.y = (s / g.P[0]) % g.P[1];
  c.z = s / (g.P[0] * g.P[1]);
  return c;
}
// tangential index of a node on a face normal to `axis`: the other axes in
// increasing order, the first one fastest
__device__ inline int face_t(const GeoDev& g, int axis, const Loc& l) {
  if (g.dim == 2) return axis == 0 ? l.y : l.x;
  if (axis == 0) return l.z * g.ne[1] + l.y;
  if (axis == 1) return l.z * g.ne[0] + l.x;
  return l.y * g.ne[0] + l.x;
}
// face f, layer L and tangential index t of a local node on the faces
// normal to `axis` (layer 0: the subdomain's boundary layer, layer 1: the
// next one out); false if the node is on neither layer
__device__ inline bool iface_parts(const GeoDev& g, int axis, const Loc& l, int& f, int& L,
                                   int& t) {
  const int W = g.W, na = pick(g.na, axis), pa = l.at(axis);
  int s = -1;
  L = 0;
  if (pa == W) { s = 0; L = 0; }
  else if (pa == W - 1) { s = 0; L = 1; }
  else if (pa == W + na - 1) { s = 1; L = 0; }
  else if (pa == W + na) { s = 1; L = 1; }
  if (s < 0) return false;
  f = 2 * axis + s;
  t = face_t(g, axis, l);
  return true;
}
// interface dof of a local node on the faces normal to `axis`, -1 if none
__device__ inline int iface_dof(const GeoDev& g, int axis, const Loc& l) {
  int f, L, t;
  if (!iface_parts(g, axis, l, f, L, t)) return -1;
  return pick(g.side_off, f) + L * pick(g.side_len, f) + t;
}
// local node of interface dof i
__device__ inline Loc dof_node(const GeoDev& g, int i) {
  int f = 0;
#pragma unroll
  for (int j = 1; j < 6; ++j) f = (j < 2 * g.dim && i >= g.side_off[j]) ? j : f;
  const int len = pick(g.side_len, f);
  const int r = i - pick(g.side_off, f);
  const int L = r / len;
  const int t = r - L * len;
  const int axis = f >> 1, na = pick(g.na, axis);
  const int layer =
      (f & 1) == 0 ? (L == 0 ? g.W : g.W - 1) : (L == 0 ? g.W + na - 1 : g.W + na);
  Loc l;
  if (g.dim == 2) {
    if (axis == 0) { l.x = layer; l.y = t; }
    else { l.x = t; l.y = layer; }
    l.z = 0;
  } else if (axis == 0) {
    l.x = layer; l.z = t / g.ne[1]; l.y = t - l.z * g.ne[1];
  } else if (axis == 1) {
    l.y = layer; l.z = t / g.ne[0]; l.x = t - l.z * g.ne[0];
  } else {
    l.z = layer; l.y = t / g.ne[0]; l.x = t - l.y * g.ne[0];
  }
  return l;
}
__device__ inline bool owned_axis(const GeoDev& g, int a, int bc, int loc) {
  return (loc >= g.W || bc == 0) && (loc < g.W + g.na[a] || bc == g.P[a] - 1);
}
// global node index of a subdomain-local node, -1 if the subdomain does not
// own it
__device__ inline long long owned_global(const GeoDev& g, const Loc& sc, const Loc& l) {
  if (!owned_axis(g, 0, sc.x, l.x) || !owned_axis(g, 1, sc.y, l.y)) return -1;
  long long G = (long long)(sc.x * g.na[0] + l.x) + (long long)(sc.y * g.na[1] + l.y) * g.M[0];
  if (g.dim == 3) {
    if (!owned_axis(g, 2, sc.z, l.z)) return -1;
    G += (long long)(sc.z * g.na[2] + l.z) * g.M[0] * g.M[1];
  }
  return G;
}

// ------------------------------------------------------------ assembly
// Operator coefficients of every distinct subdomain operator (2D), from the
// local alpha profiles (identical for all subdomains: they depend only on
// the offset from the subdomain's own box) and the extended wavenumber.
__global__ void k_assemble2d(c128* coef, size_t stride, const c128* al, int o_nx,
                             int o_hx, int o_ny, int o_hy, const double* kap,
                             GeoDev g, double h2, int nops) {
  int op = blockIdx.y;
  if (op >= nops) return;
  int n = g.n, K = g.K;
  c128* ax = coef + (size_t)op * stride;
  c128* ay = ax + (size_t)K * (n + 1);
  c128* dg = ay + (size_t)(K + 1) * n;
  const double* kp = kap + (size_t)op * n * K;
  int tot1 = K * (n + 1), tot2 = (K + 1) * n;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < tot1 + tot2;
       idx += gridDim.x * blockDim.x) {
    if (idx < tot1) {
      int k = idx / (n + 1), q = idx - k * (n + 1);
      ax[idx] = al[o_ny + k] * cinv(al[o_hx + q]);
    } else {
      int j = idx - tot1;
      int q = j / n, p = j - q * n;
      ay[j] = al[o_nx + p] * cinv(al[o_hy + q]);
    }
  }
  __syncthreads();
  // diagonal needs the faces: recompute them locally (no cross-block sync)
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n * K;
       idx += gridDim.x * blockDim.x) {
    int k = idx / n, p = idx - k * n;
    c128 axl = al[o_ny + k] * cinv(al[o_hx + p]);
    c128 axr = al[o_ny + k] * cinv(al[o_hx + p + 1]);
    c128 ayl = al[o_nx + p] * cinv(al[o_hy + k]);
    c128 ayr = al[o_nx + p] * cinv(al[o_hy + k + 1]);
    double kk = kp[idx];
    c128 J = al[o_nx + p] * al[o_ny + k];
    c128 d = mk<double>(h2 * kk * kk * J.re, h2 * kk * kk * J.im);
    dg[idx] = d - axl - axr - ayl - ayr;
  }
}

// 3D: ax[n_z][n_y][n_x + 1], ay[n_z][n_y + 1][n_x], az[n_z + 1][n_y][n_x],
// dg[n_z][n_y][n_x]; a^x = alpha_y alpha_z / alpha_x(half), and so on
// (eq. (PML3)), dg = h^2 k^2 J - (sum of the six face coefficients).
struct AlphaOff {
  int o[6];
};
__global__ void k_assemble3d(c128* coef, size_t stride, const c128* al, AlphaOff ao,
                             const double* kap, GeoDev g, double h2, int nops) {
  const int* o = ao.o;
  const int op = blockIdx.y;
  if (op >= nops) return;
  const int nx = g.ne[0], ny = g.ne[1], nz = g.ne[2];
  const int onx = o[0], ohx = o[1], ony = o[2], ohy = o[3], onz = o[4], ohz = o[5];
  c128* ax = coef + (size_t)op * stride;
  c128* ay = ax + (size_t)nz * ny * (nx + 1);
  c128* az = ay + (size_t)nz * (ny + 1) * nx;
  c128* dg = az + (size_t)(nz + 1) * ny * nx;
  const double* kp = kap + (size_t)op * nx * ny * nz;
  const long long t1 = (long long)nz * ny * (nx + 1), t2 = (long long)nz * (ny + 1) * nx,
                  t3 = (long long)(nz + 1) * ny * nx, t4 = (long long)nz * ny * nx;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
       idx < t1 + t2 + t3 + t4; idx += (long long)gridDim.x * blockDim.x) {
    long long r = idx;
    if (r < t1) {
      int q = (int)(r % (nx + 1)), y = (int)((r / (nx + 1)) % ny), z = (int)(r / ((nx + 1) * (long long)ny));
      ax[r] = al[ony + y] * al[onz + z] * cinv(al[ohx + q]);
      continue;
    }
    r -= t1;
    if (r < t2) {
      int x = (int)(r % nx), q = (int)((r / nx) % (ny + 1)), z = (int)(r / (nx * (long long)(ny + 1)));
      ay[r] = al[onx + x] * al[onz + z] * cinv(al[ohy + q]);
      continue;
    }
    r -= t2;
    if (r < t3) {
      int x = (int)(r % nx), y = (int)((r / nx) % ny), q = (int)(r / (nx * (long long)ny));
      az[r] = al[onx + x] * al[ony + y] * cinv(al[ohz + q]);
      continue;
    }
    r -= t3;
    int x = (int)(r % nx), y = (int)((r / nx) % ny), z = (int)(r / (nx * (long long)ny));
    c128 axl = al[ony + y] * al[onz + z] * cinv(al[ohx + x]);
    c128 axr = al[ony + y] * al[onz + z] * cinv(al[ohx + x + 1]);
    c128 ayl = al[onx + x] * al[onz + z] * cinv(al[ohy + y]);
    c128 ayr = al[onx + x] * al[onz + z] * cinv(al[ohy + y + 1]);
    c128 azl = al[onx + x] * al[ony + y] * cinv(al[ohz + z]);
    c128 azr = al[onx + x] * al[ony + y] * cinv(al[ohz + z + 1]);
    double kk = kp[r];
    c128 J = al[onx + x] * al[ony + y] * al[onz + z];
    c128 d = mk<double>(h2 * kk * kk * J.re, h2 * kk * kk * J.im);
    dg[r] = d - axl - axr - ayl - ayr - azl - azr;
  }
}

hipError_t launch_assemble(hdsw_ctx* c) {
  const Geometry& g = c->g;
  if (g.dim == 3) {
    long long tot = (long long)g.ne[2] * g.ne[1] * (g.ne[0] + 1) +
                    (long long)g.ne[2] * (g.ne[1] + 1) * g.ne[0] +
                    (long long)(g.ne[2] + 1) * g.ne[1] * g.ne[0] + g.sub_nodes;
    dim3 grid((unsigned)std::min<long long>((tot + 255) / 256, 1 << 16), c->nops);
    AlphaOff ao;
    for (int i = 0; i < 6; ++i) ao.o[i] = c->alpha_sub_off[i];
    hipLaunchKernelGGL(k_assemble3d, grid, dim3(256), 0, c->stream, c->d_coef, c->coef_stride,
                       c->d_alpha_sub, ao, c->d_kappa_sub, c->gd, g.h * g.h, c->nops);
    return hipGetLastError();
  }
  int tot = g.K * (g.n + 1) + (g.K + 1) * g.n;
  dim3 grid((tot + 255) / 256, c->nops);
  hipLaunchKernelGGL(k_assemble2d, grid, dim3(256), 0, c->stream, c->d_coef,
                     c->coef_stride, c->d_alpha_sub, c->alpha_sub_off[0],
                     c->alpha_sub_off[1], c->alpha_sub_off[2], c->alpha_sub_off[3],
                     c->d_kappa_sub, c->gd, g.h * g.h, c->nops);
  return hipGetLastError();
}

template <class T>
__global__ void k_cast_coef(cpx<T>* dst, const c128* src, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = ccast<T>(src[i]);
}
template <class T>
hipError_t launch_cast_coef(hdsw_ctx* c) {
  size_t n = c->coef_stride * c->nops;
  int blocks = (int)std::min<size_t>((n + 255) / 256, 65535);
  hipLaunchKernelGGL(k_cast_coef<T>, dim3(blocks), dim3(256), 0, c->stream,
                     (cpx<T>*)c->d_coefT, c->d_coef, n);
  return hipGetLastError();
}

// (factorization kernels: mfma.hip)

// ------------------------------------------------------------ panels
// Sources received over the sweeps of one DDM application: for every face,
// the sweeps whose slot can hold a trace across it (bit L of mask[face]).
struct TraceSum {
  int nsweeps;
  int mask[6];
};

// mode 0: owned part of a global FP64 vector, cast to the working precision
// mode 1: mode 0 plus the interface sources received in every sweep
//         (scatter P_I^T of sum_L g_L, g_L = [S_r, chi_r] of the pairs in
//         slot L), summed in sweep order
// mode 2: unit vectors of interface dofs unit_col0 .. unit_col0 + C - 1
// batch entry b is subdomain ids[b] (modes 0, 1) or operator ids[b] (mode 2)
// Sources received over the sweeps of one DDM application, per interface
// dof: srcsum[s][c][d] = sum over the sweeps L whose slot can hold a trace
// across the face of d of g_L[d], g = [S_r, chi_r] v~ of the pairs in slot L
// (g[layer 1] = c pair[layer 0], g[layer 0] = -c pair[layer 1]), summed in
// sweep order.
template <class T>
__global__ void k_source_sum(cpx<T>* srcsum, const cpx<T>* __restrict__ slots,
                             const cpx<T>* __restrict__ cface, const int* __restrict__ op_of,
                             int C, TraceSum ts, GeoDev g) {
  const int NI = g.NI;
  const unsigned per = (unsigned)C * NI;
  const int s = blockIdx.y;
  const size_t slot_stride = (size_t)g.nsub * C * NI;
  for (unsigned r = blockIdx.x * blockDim.x + threadIdx.x; r < per; r += gridDim.x * blockDim.x) {
    const int col = (int)(r / (unsigned)NI), d = (int)(r - (unsigned)col * NI);
    int f = 0;
#pragma unroll
    for (int j = 1; j < 6; ++j) f = (j < 2 * g.dim && d >= g.side_off[j]) ? j : f;
    const int len = pick(g.side_len, f), so = pick(g.side_off, f);
    const int L = (d - so) >= len, t = d - so - L * len;
    const int partner = so + (1 - L) * len + t, mask = pick(ts.mask, f);
    const cpx<T> cf = cface[(size_t)op_of[s] * (NI / 2) + so / 2 + t];
    const cpx<T>* recv = slots + ((size_t)s * C + col) * NI + partner;
    cpx<T> a = mk<T>(T(0), T(0));
    for (int sw = 0; sw < ts.nsweeps; ++sw) {
      if (!((mask >> sw) & 1)) continue;
      cpx<T> gv = cf * recv[sw * slot_stride];
      if (L == 0) gv = -gv;
      a = a + gv;
    }
    srcsum[(size_t)s * per + r] = a;
  }
}

// Entries per thread of the panel fill and the owned-node write: their
// global loads are issued together (unconditionally, clamped indices) before
// any entry is written, so each thread keeps several loads in flight.
constexpr int kFillEPT = 4;

// nzflag (mode 0, may be null): nzflag[b * ceil(C / 8) + col / 8] is set
// to 1 where batch entry b has a nonzero right-hand side entry in one of
// the 8 columns; the block solve skips the pairs left at 0.  Each thread
// marks the groups of its nonzero entries in a 64-bit mask relative to the
// group of the span's first entry (the host passes nzflag only when a span
// of blockDim * kFillEPT entries cannot reach 64 groups), the masks are
// ORed across each wave by shuffles and across the workgroup in LDS, and
// one lane sets the flags.
template <class T>
__global__ void k_fill_panel(cpx<T>* __restrict__ panel, int mode, const int* __restrict__ ids,
                             int C, const c128* __restrict__ rg,
                             const cpx<T>* __restrict__ srcsum, GeoDev g, long long glob,
                             int col0, int* __restrict__ nzflag) {
  // grid: x over the entries (k, column, p) of one batch entry, flat so that
  // every lane works, y over the batch entry b (its subdomain is uniform per
  // workgroup); 32-bit index arithmetic
  const int n = g.n, K = g.K, b = blockIdx.y;
  const unsigned per = (unsigned)K * C * n, cn = (unsigned)C * n;
  cpx<T>* pb = panel + (size_t)b * g.PL * C * n;
  if (mode == 2) {
    for (unsigned r = blockIdx.x * blockDim.x + threadIdx.x; r < per; r += gridDim.x * blockDim.x) {
      const int k = (int)(r / cn), rem = (int)(r - (unsigned)k * cn);
      const int col = rem / n, p = rem - col * n;
      const Loc loc = block_node(g, p, k);
      cpx<T> v = mk<T>(T(0), T(0));
      for (int a = 0; a < g.dim; ++a)
        if (iface_dof(g, a, loc) == col0 + col) v.re = T(1);
      pb[r] = v;
    }
    return;
  }
  const int s = ids[b];
  const Loc sc = sub_coords(g, s);
  const unsigned span = blockDim.x * kFillEPT;
  const bool flags = mode == 0 && nzflag != nullptr;
  const int ng8 = (C + 7) / 8;
  __shared__ unsigned long long nzm;
  // uniform loop bounds: every thread runs every span (the reductions below)
  for (unsigned base = blockIdx.x * span; base < per; base += gridDim.x * span) {
    const unsigned r0 = base + threadIdx.x;
    c128 gv[kFillEPT];
    long long gi[kFillEPT];                     // index into rg, -1: not owned / past the end
#pragma unroll
    for (int j = 0; j < kFillEPT; ++j) {
      const unsigned r = r0 + j * blockDim.x;
      gi[j] = -1;
      if (r < per) {
        const int k = (int)(r / cn), rem = (int)(r - (unsigned)k * cn);
        const int col = rem / n, p = rem - col * n;
        const long long G = owned_global(g, sc, block_node(g, p, k));
        if (G >= 0) gi[j] = (long long)col * glob + G;
      }
      gv[j] = rg[gi[j] >= 0 ? gi[j] : 0];
    }
    // column group of the span's first entry
    const int ga = (int)((base % cn) / n) / 8;
    unsigned long long m = 0;
#pragma unroll
    for (int j = 0; j < kFillEPT; ++j) {
      const unsigned r = r0 + j * blockDim.x;
      if (r < per) {
        cpx<T> v = mk<T>(T(0), T(0));
        if (gi[j] >= 0) v = ccast<T>(gv[j]);
        if (flags && (v.re != T(0) || v.im != T(0))) {
          const int gq = (int)((r % cn) / n) / 8;
          m |= 1ull << ((gq - ga + ng8) % ng8);
        }
        if (mode == 1) {
          const int k = (int)(r / cn), rem = (int)(r - (unsigned)k * cn);
          const int col = rem / n, p = rem - col * n;
          const Loc loc = block_node(g, p, k);
          const cpx<T>* a = srcsum + ((size_t)s * C + col) * g.NI;
          for (int ax = 0; ax < g.dim; ++ax) {
            int d = iface_dof(g, ax, loc);
            if (d >= 0) v = v + a[d];
          }
        }
        pb[r] = v;
      }
    }
    if (flags) {
      if (threadIdx.x == 0) nzm = 0;
      __syncthreads();
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) m |= __shfl_xor(m, o);
      if ((threadIdx.x & 63) == 0 && m) atomicOr(&nzm, m);
      __syncthreads();
      if (threadIdx.x == 0) {
        for (unsigned long long mm = nzm; mm; mm &= mm - 1) {
          const int d = __builtin_ctzll(mm);
          atomicOr(nzflag + (size_t)b * ng8 + (ga + d) % ng8, 1);
        }
      }
      __syncthreads();   // nzm is cleared by the next span
    }
  }
}

template <class T>
hipError_t launch_fill_panel(hdsw_ctx* c, int mode, int nbatch, const int* d_ids,
                             int C, const c128* rglob, int unit_col0, int* nzflag) {
  const Geometry& g = c->g;
  if (nbatch > 65535) return hipErrorInvalidValue;
  const long long per = (long long)g.K * C * g.n;
  if (per >= (1LL << 31)) return hipErrorInvalidValue;
  const long long span = mode == 2 ? 256 : 256 * kFillEPT;
  dim3 grid((unsigned)std::min<long long>((per + span - 1) / span, 1 << 20), nbatch);
  if (mode == 1) {
    // the received sources of every interface dof, summed over the sweeps
    TraceSum ts{};
    ts.nsweeps = c->sch.nsweeps;
    for (int L = 0; L < c->sch.nsweeps; ++L)
      for (int f = 0; f < 6; ++f)
        if (c->sch.in_active[L * 6 + f]) ts.mask[f] |= (int)(1u << L);   // nsweeps <= 32
    const long long ps = (long long)C * g.NI;
    if (nbatch != g.nsub || ps >= (1LL << 31)) return hipErrorInvalidValue;
    dim3 sgrid((unsigned)std::min<long long>((ps + 255) / 256, 1 << 20), g.nsub);
    hipLaunchKernelGGL(k_source_sum<T>, sgrid, dim3(256), 0, c->stream, (cpx<T>*)c->d_srcsum,
                       (const cpx<T>*)c->d_slots, (const cpx<T>*)c->d_cface, c->d_op_of_sub, C,
                       ts, c->gd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // the column-group flags: a span of 256 kFillEPT entries covers at most
  // span / (8 n) + 3 groups, which must stay below the 64 bits of a mask
  if (mode == 0 && nzflag && 256 * kFillEPT / (8 * g.n) + 3 >= 64) nzflag = nullptr;
  hipLaunchKernelGGL(k_fill_panel<T>, grid, dim3(256), 0, c->stream,
                     (cpx<T>*)c->d_panel, mode, d_ids, C, rglob,
                     (const cpx<T>*)c->d_srcsum, c->gd, g.glob_nodes, unit_col0, nzflag);
  return hipGetLastError();
}

// (block solve kernels: mfma.hip)

// ------------------------------------------------------------ interface I/O
// dst[b][col][i] = panel[b][k_i][col][p_i]  (restriction P_I)
template <class T>
__global__ void k_extract_iface(const cpx<T>* panel, int nbatch, int C, cpx<T>* dst,
                                long long dst_sb, int dst_ld, GeoDev g) {
  long long tot = (long long)nbatch * C * g.NI;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    int b = (int)(idx / ((long long)C * g.NI));
    int r = (int)(idx - (long long)b * C * g.NI);
    int col = r / g.NI, i = r - col * g.NI;
    const Loc loc = dof_node(g, i);
    const int p = g.dim == 2 ? loc.x : loc.y * g.ne[0] + loc.x;
    const int k = g.dim == 2 ? loc.y : loc.z;
    dst[b * dst_sb + (long long)col * dst_ld + i] =
        panel[(((long long)b * g.PL + k) * C + col) * g.n + p];
  }
}
template <class T>
hipError_t launch_extract_iface(hdsw_ctx* c, int nbatch, int C, void* dst,
                                long long dst_sb, int dst_ld) {
  long long tot = (long long)nbatch * C * c->g.NI;
  int blocks = (int)std::min<long long>((tot + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_extract_iface<T>, dim3(blocks), dim3(256), 0, c->stream,
                     (const cpx<T>*)c->d_panel, nbatch, C, (cpx<T>*)dst, dst_sb,
                     dst_ld, c->gd);
  return hipGetLastError();
}

// glob[col][G] (+)= panel on owned nodes (every global node has exactly one
// owner, so no two threads touch the same element)
template <class T>
__global__ void k_write_owned(const cpx<T>* __restrict__ panel, int C, c128* __restrict__ glob,
                              long long gn, int accumulate, GeoDev g) {
  // grid: x over the entries (k, column, p) of one subdomain (flat), y over
  // the subdomain; 32-bit index arithmetic
  const int n = g.n, K = g.K, s = blockIdx.y;
  const unsigned per = (unsigned)K * C * n, cn = (unsigned)C * n;
  const Loc sc = sub_coords(g, s);
  const cpx<T>* ps = panel + (size_t)s * g.PL * C * n;
  const unsigned span = blockDim.x * kFillEPT;
  for (unsigned r0 = blockIdx.x * span + threadIdx.x; r0 < per; r0 += gridDim.x * span) {
    cpx<T> pv[kFillEPT];
    c128 dv[kFillEPT];
    long long gi[kFillEPT];                     // index into glob, -1: not owned / past the end
#pragma unroll
    for (int j = 0; j < kFillEPT; ++j) {
      const unsigned r = r0 + j * blockDim.x;
      gi[j] = -1;
      if (r < per) {
        const int k = (int)(r / cn), rem = (int)(r - (unsigned)k * cn);
        const int col = rem / n, p = rem - col * n;
        const long long G = owned_global(g, sc, block_node(g, p, k));
        if (G >= 0) gi[j] = (long long)col * gn + G;
      }
      pv[j] = ps[gi[j] >= 0 ? r : 0];
      dv[j] = mk<double>(0.0, 0.0);
      if (accumulate) dv[j] = glob[gi[j] >= 0 ? gi[j] : 0];
    }
#pragma unroll
    for (int j = 0; j < kFillEPT; ++j)
      if (gi[j] >= 0) glob[gi[j]] = accumulate ? dv[j] + ccast<double>(pv[j]) : ccast<double>(pv[j]);
  }
}
template <class T>
hipError_t launch_write_owned(hdsw_ctx* c, int C, c128* glob, int accumulate) {
  const Geometry& g = c->g;
  if (g.nsub > 65535) return hipErrorInvalidValue;
  const long long per = (long long)g.K * C * g.n;
  if (per >= (1LL << 31)) return hipErrorInvalidValue;
  dim3 grid((unsigned)std::min<long long>((per + 256 * kFillEPT - 1) / (256 * kFillEPT), 1 << 20),
            g.nsub);
  hipLaunchKernelGGL(k_write_owned<T>, grid, dim3(256), 0, c->stream,
                     (const cpx<T>*)c->d_panel, C, glob, g.glob_nodes, accumulate, c->gd);
  return hipGetLastError();
}

// ------------------------------------------------------------ FP64 global
// b = h^2 J f on the global grid (J = 1 inside B, f = 0 in the layer)
__global__ void k_rhs_from_f(const c128* f, c128* b, int C, GeoDev g, double h2,
                             long long gn) {
  long long tot = (long long)C * gn;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    int col = (int)(idx / gn);
    long long G = idx - col * gn;
    long long I = 0, istride = 1, ni = 1;
    bool inside = true;
    for (int a = 0; a < g.dim; ++a) {
      int ga = (int)(G % g.M[a]);
      G /= g.M[a];
      int ia = ga - g.W;
      inside = inside && ia >= 0 && ia < g.N[a];
      I += (long long)ia * istride;
      istride *= g.N[a];
      ni *= g.N[a];
    }
    c128 v = mk<double>(0.0, 0.0);
    if (inside) {
      c128 fv = f[(long long)col * ni + I];
      v = mk<double>(h2 * fv.re, h2 * fv.im);
    }
    b[idx] = v;
  }
}
hipError_t launch_rhs_from_f(hdsw_ctx* c, const c128* f, c128* b, int C) {
  long long tot = (long long)C * c->g.glob_nodes;
  int blocks = (int)std::min<long long>((tot + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_rhs_from_f, dim3(blocks), dim3(256), 0, c->stream, f, b, C,
                     c->gd, c->g.h * c->g.h, c->g.glob_nodes);
  return hipGetLastError();
}

// r = b - S x with the global operator's coefficients formed on the fly,
// once per node for all C columns (thread per node, columns in a loop; the
// pointers are restrict-qualified).  Unrolling the column loop with
// unconditional neighbour loads measured slower.
__global__ void k_residual2d(const c128* __restrict__ b, const c128* __restrict__ x,
                             c128* __restrict__ r, int C,
                             const c128* al, int o_nx, int o_hx, int o_ny, int o_hy,
                             const double* kap, GeoDev g, double h2, long long gn) {
  const int Mx = g.M[0], My = g.M[1];
  for (long long G = blockIdx.x * (long long)blockDim.x + threadIdx.x; G < gn;
       G += (long long)gridDim.x * blockDim.x) {
    int gy = (int)(G / Mx), gx = (int)(G - (long long)gy * Mx);
    c128 anx = al[o_nx + gx], any = al[o_ny + gy];
    c128 axl = any * cinv(al[o_hx + gx]);
    c128 axr = any * cinv(al[o_hx + gx + 1]);
    c128 ayl = anx * cinv(al[o_hy + gy]);
    c128 ayr = anx * cinv(al[o_hy + gy + 1]);
    int ix = min(max(gx - g.W, 0), g.N[0] - 1);
    int iy = min(max(gy - g.W, 0), g.N[1] - 1);
    double kk = kap[(long long)iy * g.N[0] + ix];
    c128 J = anx * any;
    c128 d = mk<double>(h2 * kk * kk * J.re, h2 * kk * kk * J.im);
    const bool hl = gx > 0, hr = gx < Mx - 1, hd = gy > 0, hu = gy < My - 1;
    for (int col = 0; col < C; ++col) {
      const c128* xc = x + (long long)col * gn;
      c128 u = xc[G];
      c128 z = mk<double>(0.0, 0.0);
      c128 ul = z, ur = z, ud = z, uu = z;
      if (hl) ul = xc[G - 1];
      if (hr) ur = xc[G + 1];
      if (hd) ud = xc[G - Mx];
      if (hu) uu = xc[G + Mx];
      c128 su = d * u;
      su = su + axr * (ur - u) - axl * (u - ul) + ayr * (uu - u) - ayl * (u - ud);
      long long idx = (long long)col * gn + G;
      r[idx] = b ? (b[idx] - su) : su;
    }
  }
}

// 3D: 7-point operator of eq. (PML3) on the global grid
__global__ void k_residual3d(const c128* __restrict__ b, const c128* __restrict__ x,
                             c128* __restrict__ r, int C, const c128* al,
                             AlphaOff ao, const double* kap, GeoDev g, double h2,
                             long long gn) {
  const int* o = ao.o;
  const int Mx = g.M[0], My = g.M[1], Mz = g.M[2];
  const long long Mxy = (long long)Mx * My;
  const int onx = o[0], ohx = o[1], ony = o[2], ohy = o[3], onz = o[4], ohz = o[5];
  for (long long G = blockIdx.x * (long long)blockDim.x + threadIdx.x; G < gn;
       G += (long long)gridDim.x * blockDim.x) {
    int gz = (int)(G / Mxy);
    long long rem = G - gz * Mxy;
    int gy = (int)(rem / Mx), gx = (int)(rem - (long long)gy * Mx);
    c128 anx = al[onx + gx], any = al[ony + gy], anz = al[onz + gz];
    c128 axl = any * anz * cinv(al[ohx + gx]);
    c128 axr = any * anz * cinv(al[ohx + gx + 1]);
    c128 ayl = anx * anz * cinv(al[ohy + gy]);
    c128 ayr = anx * anz * cinv(al[ohy + gy + 1]);
    c128 azl = anx * any * cinv(al[ohz + gz]);
    c128 azr = anx * any * cinv(al[ohz + gz + 1]);
    int ix = min(max(gx - g.W, 0), g.N[0] - 1);
    int iy = min(max(gy - g.W, 0), g.N[1] - 1);
    int iz = min(max(gz - g.W, 0), g.N[2] - 1);
    double kk = kap[((long long)iz * g.N[1] + iy) * g.N[0] + ix];
    c128 J = anx * any * anz;
    c128 d = mk<double>(h2 * kk * kk * J.re, h2 * kk * kk * J.im);
    const bool hl = gx > 0, hr = gx < Mx - 1, hd = gy > 0, hu = gy < My - 1, hb = gz > 0,
               hf = gz < Mz - 1;
    for (int col = 0; col < C; ++col) {
      const c128* xc = x + (long long)col * gn;
      c128 u = xc[G];
      c128 z = mk<double>(0.0, 0.0);
      c128 ul = z, ur = z, ud = z, uu = z, ub = z, uf = z;
      if (hl) ul = xc[G - 1];
      if (hr) ur = xc[G + 1];
      if (hd) ud = xc[G - Mx];
      if (hu) uu = xc[G + Mx];
      if (hb) ub = xc[G - Mxy];
      if (hf) uf = xc[G + Mxy];
      c128 su = d * u;
      su = su + axr * (ur - u) - axl * (u - ul) + ayr * (uu - u) - ayl * (u - ud) +
           azr * (uf - u) - azl * (u - ub);
      long long idx = (long long)col * gn + G;
      r[idx] = b ? (b[idx] - su) : su;
    }
  }
}

hipError_t launch_residual(hdsw_ctx* c, const c128* b, const c128* x, c128* r, int C) {
  long long tot = c->g.glob_nodes;
  int blocks = (int)std::min<long long>((tot + 255) / 256, 1 << 20);
  if (c->g.dim == 3) {
    AlphaOff ao;
    for (int i = 0; i < 6; ++i) ao.o[i] = c->alpha_glob_off[i];
    hipLaunchKernelGGL(k_residual3d, dim3(blocks), dim3(256), 0, c->stream, b, x, r, C,
                       c->d_alpha_glob, ao, c->d_kappa, c->gd, c->g.h * c->g.h,
                       c->g.glob_nodes);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_residual2d, dim3(blocks), dim3(256), 0, c->stream, b, x, r, C,
                     c->d_alpha_glob, c->alpha_glob_off[0], c->alpha_glob_off[1],
                     c->alpha_glob_off[2], c->alpha_glob_off[3], c->d_kappa, c->gd,
                     c->g.h * c->g.h, c->g.glob_nodes);
  return hipGetLastError();
}


// per-column 2-norms, deterministic two-pass reduction
__global__ void k_norm_part(const c128* v, long long gn, int nblk, double* part) {
  __shared__ double sh[256];
  int col = blockIdx.y;
  const c128* vc = v + (long long)col * gn;
  double s = 0.0;
  long long chunk = (gn + nblk - 1) / nblk;
  long long lo = (long long)blockIdx.x * chunk, hi = min(gn, lo + chunk);
  for (long long i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    c128 z = vc[i];
    s += z.re * z.re + z.im * z.im;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long long)col * nblk + blockIdx.x] = sh[0];
}
__global__ void k_norm_final(const double* part, int nblk, double* out) {
  __shared__ double sh[256];
  int col = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) s += part[(long long)col * nblk + i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[col] = sqrt(sh[0]);
}
hipError_t launch_norms(hdsw_ctx* c, const c128* v, int C, double* d_out) {
  int nblk = c->part_blocks;
  hipLaunchKernelGGL(k_norm_part, dim3(nblk, C), dim3(256), 0, c->stream, v,
                     c->g.glob_nodes, nblk, c->d_part);
  hipLaunchKernelGGL(k_norm_final, dim3(C), dim3(256), 0, c->stream, c->d_part, nblk,
                     d_out);
  return hipGetLastError();
}

__global__ void k_extract_interior(const c128* glob, c128* out, int C, GeoDev g,
                                   long long gn) {
  long long ni = 1;
  for (int a = 0; a < g.dim; ++a) ni *= g.N[a];
  long long tot = (long long)C * ni;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    int col = (int)(idx / ni);
    long long r = idx - col * ni;
    long long G = 0, stride = 1;
    for (int a = 0; a < g.dim; ++a) {
      int ia = (int)(r % g.N[a]);
      r /= g.N[a];
      G += (long long)(ia + g.W) * stride;
      stride *= g.M[a];
    }
    out[idx] = glob[(long long)col * gn + G];
  }
}
hipError_t launch_extract_interior(hdsw_ctx* c, const c128* glob, c128* out, int C) {
  long long tot = (long long)C * c->g.int_nodes;
  int blocks = (int)std::min<long long>((tot + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_extract_interior, dim3(blocks), dim3(256), 0, c->stream, glob,
                     out, C, c->gd, c->g.glob_nodes);
  return hipGetLastError();
}

__global__ void k_zero(uint32_t* p, size_t nwords) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nwords;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}
hipError_t launch_zero(hdsw_ctx* c, void* p, size_t bytes) {
  size_t nw = bytes / 4;
  if (nw == 0) return hipSuccess;
  int blocks = (int)std::min<size_t>((nw + 255) / 256, 1 << 16);
  hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, c->stream, (uint32_t*)p, nw);
  return hipGetLastError();
}

__global__ void k_copy(c128* dst, const c128* src, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}
hipError_t launch_copy_cols(hdsw_ctx* c, c128* dst, const c128* src, size_t n) {
  if (n == 0) return hipSuccess;
  int blocks = (int)std::min<size_t>((n + 255) / 256, 1 << 16);
  hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, c->stream, dst, src, n);
  return hipGetLastError();
}

// ------------------------------------------------------------ GMRES (FP64)
// dots[j][col] = sum_G conj(V_j[col][G]) w[col][G], two-pass deterministic
__global__ void k_dots_part(const c128* V, int nv, const c128* w, int C, long long gn,
                            int nblk, double* part) {
  __shared__ double sr[256], si[256];
  int col = blockIdx.y, j = blockIdx.z;
  const c128* vj = V + ((long long)j * C + col) * gn;
  const c128* wc = w + (long long)col * gn;
  long long chunk = (gn + nblk - 1) / nblk;
  long long lo = (long long)blockIdx.x * chunk, hi = min(gn, lo + chunk);
  double ar = 0.0, ai = 0.0;
  for (long long i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    c128 a = vj[i], b = wc[i];
    ar += a.re * b.re + a.im * b.im;
    ai += a.re * b.im - a.im * b.re;
  }
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    long long o = (((long long)j * C + col) * nblk + blockIdx.x) * 2;
    part[o] = sr[0];
    part[o + 1] = si[0];
  }
}
__global__ void k_dots_final(const double* part, int nblk, c128* out) {
  __shared__ double sr[256], si[256];
  long long jc = blockIdx.x;
  double ar = 0.0, ai = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
    ar += part[(jc * nblk + i) * 2];
    ai += part[(jc * nblk + i) * 2 + 1];
  }
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[jc] = mk<double>(sr[0], si[0]);
}
hipError_t launch_dots(hdsw_ctx* c, const c128* V, int nv, const c128* w, int C,
                       c128* d_out) {
  int nblk = c->part_blocks;
  hipLaunchKernelGGL(k_dots_part, dim3(nblk, C, nv), dim3(256), 0, c->stream, V, nv, w,
                     C, c->g.glob_nodes, nblk, c->d_part);
  hipLaunchKernelGGL(k_dots_final, dim3(nv * C), dim3(256), 0, c->stream, c->d_part,
                     nblk, d_out);
  return hipGetLastError();
}
// w[col] += sign * sum_j coef[j][col] V_j[col]
__global__ void k_axpy_multi(c128* w, const c128* V, int nv, const c128* coef, int C,
                             long long gn, double sign) {
  long long tot = (long long)C * gn;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    int col = (int)(idx / gn);
    long long G = idx - col * gn;
    c128 acc = mk<double>(0.0, 0.0);
    for (int j = 0; j < nv; ++j)
      cfma(acc, coef[(long long)j * C + col], V[((long long)j * C + col) * gn + G]);
    c128 v = w[idx];
    w[idx] = mk<double>(v.re + sign * acc.re, v.im + sign * acc.im);
  }
}
hipError_t launch_axpy_multi(hdsw_ctx* c, c128* w, const c128* V, int nv,
                             const c128* coef, int C, double sign) {
  long long tot = (long long)C * c->g.glob_nodes;
  int blocks = (int)std::min<long long>((tot + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_axpy_multi, dim3(blocks), dim3(256), 0, c->stream, w, V, nv, coef,
                     C, c->g.glob_nodes, sign);
  return hipGetLastError();
}
// dst[col] = src[col] * inv[col]
__global__ void k_scale(c128* dst, const c128* src, const double* inv, int C,
                        long long gn) {
  long long tot = (long long)C * gn;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    int col = (int)(idx / gn);
    double s = inv[col];
    c128 v = src[idx];
    dst[idx] = mk<double>(v.re * s, v.im * s);
  }
}
hipError_t launch_scale(hdsw_ctx* c, c128* dst, const c128* src, const double* inv,
                        int C) {
  long long tot = (long long)C * c->g.glob_nodes;
  int blocks = (int)std::min<long long>((tot + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_scale, dim3(blocks), dim3(256), 0, c->stream, dst, src, inv, C,
                     c->g.glob_nodes);
  return hipGetLastError();
}

// ------------------------------------------------------------ instantiation
#define HDSW_INST(T)                                                                  \
  template hipError_t launch_cast_coef<T>(hdsw_ctx*);                                \
  template hipError_t launch_fill_panel<T>(hdsw_ctx*, int, int, const int*, int,     \
                                           const c128*, int, int*);                  \
  template hipError_t launch_extract_iface<T>(hdsw_ctx*, int, int, void*, long long, \
                                              int);                                  \
  template hipError_t launch_write_owned<T>(hdsw_ctx*, int, c128*, int);
HDSW_INST(float)
HDSW_INST(double)

}  // namespace hdsw

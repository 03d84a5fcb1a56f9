// Factorization, batched block solve and interface GEMM of the hdsw library.
//
// Twisted ("from both ends") block-tridiagonal LU of a subdomain operator
// with K grid lines and coupling B_k = diag(ay[k]) between lines k-1 and k,
// middle line m = K / 2:
//   top     D_0 = A_0,          D_k = A_k - B_k D_{k-1}^{-1} B_k          (k < m)
//   bottom  E_{K-1} = A_{K-1},  E_k = A_k - B_{k+1} E_{k+1}^{-1} B_{k+1}  (k > m)
//   middle  F_m = A_m - B_m D_{m-1}^{-1} B_m - B_{m+1} E_{m+1}^{-1} B_{m+1}
// X_k is the inverse of the block of line k (D, E or F), stored column-major
// in an nP x nP tile (nP = n rounded up to 16, zero padded).  The two chains
// are independent, which halves the dependent chain of both the
// factorization and every solve.
//
// Solve with the stored inverses, two launches:
//   A: top     w_k = X_k (f_k - B_k w_{k-1})          k = 0 .. m-1
//      bottom  v_k = X_k (f_k - B_{k+1} v_{k+1})      k = K-1 .. m+1
//      (the top chain leaves f_m - B_m w_{m-1} in a scratch line)
//   B: middle  x_m = X_m (f_m - B_m w_{m-1} - B_{m+1} v_{m+1})
//      top     x_k = w_k - X_k B_{k+1} x_{k+1}        k = m-1 .. 0
//      bottom  x_k = v_k - X_k B_k x_{k-1}            k = m+1 .. K-1
// Every block product is a complex matrix times 8 complex columns on the
// matrix cores: with X = Xr + i Xi and V = Vr + i Vi,
//   [Yr | Yi] = Xr [Vr | Vi] + Xi [-Vi | Vr],
// two real 16x16x4 MFMAs per 16-row tile and 4-deep slice of the sum.
#include "hdsw_internal.hpp"

namespace hdsw {

template <class T>
struct MF;
template <>
struct MF<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 mfma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator register i of lane l holds row 4 (l / 16) + i, column l % 16
  static __device__ inline int row(int l, int i) { return 4 * (l >> 4) + i; }
};
template <>
struct MF<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 mfma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator register i of lane l holds row l / 16 + 4 i, column l % 16
  static __device__ inline int row(int l, int i) { return (l >> 4) + 4 * i; }
};

// ------------------------------------------------------------ matvec
// yb[c][r] = sum_j Xb(r, j) vb[c][j] for 8 columns c (LDS vectors of length
// nP, zero beyond n).  Waves split the rows in two halves of 16-row tiles
// and the sum in KS = NW / 2 slices; the slices are added in a fixed order,
// so results do not depend on timing.  Ends with the block synchronized.
template <class T, int MAXT, int NW>
__device__ inline void mfma_matvec(const cpx<T>* __restrict__ Xb, int nP, const cpx<T>* vb,
                                   cpx<T>* yb, cpx<T>* red, int wave, int lane) {
  typedef typename MF<T>::v4 v4;
  constexpr int KS = NW / 2;
  const int nMt = nP >> 4, nK = nP >> 2;
  const int mh = wave & 1, kq = wave >> 1;
  const int th = (nMt + 1) >> 1;
  const int t0 = mh ? th : 0, nt = mh ? nMt - th : th;
  const int kchunk = (nK + KS - 1) / KS;
  const int k0 = kq * kchunk, k1 = min(nK, k0 + kchunk);
  v4 acc[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) acc[t] = v4{T(0), T(0), T(0), T(0)};
  const int jc = lane & 15, cc = jc & 7, part = jc >> 3, kk = lane >> 4, rr = lane & 15;
  const cpx<T>* xbase = Xb + (size_t)(t0 * 16 + rr);
#pragma unroll 2
  for (int ks = k0; ks < k1; ++ks) {
    const int j = 4 * ks + kk;
    const cpx<T> vv = vb[cc * nP + j];
    const T b1 = part ? vv.im : vv.re;
    const T b2 = part ? vv.re : -vv.im;
    const cpx<T>* xc = xbase + (size_t)j * nP;
    cpx<T> xa[MAXT];
#pragma unroll
    for (int t = 0; t < MAXT; ++t)
      if (t < nt) xa[t] = xc[t * 16];
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
      if (t < nt) {
        acc[t] = MF<T>::mfma(xa[t].re, b1, acc[t]);
        acc[t] = MF<T>::mfma(xa[t].im, b2, acc[t]);
      }
    }
  }
  if (kq > 0) {
    T* dst = reinterpret_cast<T*>(red + (size_t)(kq - 1) * 8 * nP);
#pragma unroll
    for (int t = 0; t < MAXT; ++t)
      if (t < nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          int row = 16 * (t0 + t) + MF<T>::row(lane, i);
          dst[2 * (cc * nP + row) + part] = acc[t][i];
        }
  }
  __syncthreads();
  if (kq == 0) {
    T* y = reinterpret_cast<T*>(yb);
    const T* rd = reinterpret_cast<const T*>(red);
#pragma unroll
    for (int t = 0; t < MAXT; ++t)
      if (t < nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          int row = 16 * (t0 + t) + MF<T>::row(lane, i);
          int idx = 2 * (cc * nP + row) + part;
          T s = acc[t][i];
          for (int q = 0; q < KS - 1; ++q) s += rd[(size_t)q * 16 * nP + idx];
          y[idx] = s;
        }
  }
  __syncthreads();
}

// ------------------------------------------------------------ solve A
template <class T, int MAXT, int NW>
__global__ __launch_bounds__(NW * 64) void k_solve_fwd(const cpx<T>* __restrict__ X,
                                                       size_t xstride,
                                                       const cpx<T>* __restrict__ coefT,
                                                       size_t cstride, cpx<T>* panel,
                                                       const int* __restrict__ ops, GeoDev g,
                                                       int C, int nbatch) {
  extern __shared__ unsigned char smem_raw[];
  constexpr int NT = NW * 64;
  const int n = g.n, nP = g.nP, K = g.K, mid = g.mid;
  const int b = blockIdx.y, half = blockIdx.z;
  if (b >= nbatch) return;
  const int c0 = blockIdx.x * 8, nc = min(8, C - c0);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  cpx<T>* vb0 = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* vb1 = vb0 + 8 * nP;
  cpx<T>* yb = vb1 + 8 * nP;
  cpx<T>* red = yb + 8 * nP;
  const int op = ops[b];
  const cpx<T>* Xo = X + (size_t)op * xstride;
  const cpx<T>* ay = coefT + (size_t)op * cstride + (size_t)K * (n + 1);
  cpx<T>* pb = panel + (size_t)b * (K + 1) * C * n;
  for (int idx = tid; idx < 16 * nP; idx += NT) vb0[idx] = mk<T>(T(0), T(0));
  __syncthreads();
  int k = half ? K - 1 : 0;
  const int nsteps = half ? K - 1 - mid : mid;
  for (int idx = tid; idx < 8 * n; idx += NT) {
    int c = idx / n, r = idx - c * n;
    if (c < nc) vb0[c * nP + r] = pb[((size_t)k * C + c0 + c) * n + r];
  }
  __syncthreads();
  cpx<T>* vc = vb0;
  cpx<T>* vn = vb1;
  for (int s = 0; s < nsteps; ++s) {
    mfma_matvec<T, MAXT, NW>(Xo + (size_t)k * nP * nP, nP, vc, yb, red, wave, lane);
    const bool more = s + 1 < nsteps;
    const int kn = half ? k - 1 : k + 1;
    const int face = half ? k : k + 1;
    for (int idx = tid; idx < 8 * n; idx += NT) {
      int c = idx / n, r = idx - c * n;
      if (c < nc) {
        cpx<T> y = yb[c * nP + r];
        pb[((size_t)k * C + c0 + c) * n + r] = y;
        cpx<T> nxt = pb[((size_t)kn * C + c0 + c) * n + r] - ay[(size_t)face * n + r] * y;
        if (more) vn[c * nP + r] = nxt;
        else if (half == 0)   // scratch line K: f_m - B_m w_{m-1}
          pb[((size_t)K * C + c0 + c) * n + r] = nxt;
      }
    }
    __syncthreads();
    k = kn;
    cpx<T>* t = vc;
    vc = vn;
    vn = t;
  }
}

// ------------------------------------------------------------ solve B
template <class T, int MAXT, int NW>
__global__ __launch_bounds__(NW * 64) void k_solve_bwd(const cpx<T>* __restrict__ X,
                                                       size_t xstride,
                                                       const cpx<T>* __restrict__ coefT,
                                                       size_t cstride, cpx<T>* panel,
                                                       const int* __restrict__ ops, GeoDev g,
                                                       int C, int nbatch) {
  extern __shared__ unsigned char smem_raw[];
  constexpr int NT = NW * 64;
  const int n = g.n, nP = g.nP, K = g.K, mid = g.mid;
  const int b = blockIdx.y, half = blockIdx.z;
  if (b >= nbatch) return;
  const int c0 = blockIdx.x * 8, nc = min(8, C - c0);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  cpx<T>* vb0 = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* vb1 = vb0 + 8 * nP;
  cpx<T>* yb = vb1 + 8 * nP;
  cpx<T>* red = yb + 8 * nP;
  const int op = ops[b];
  const cpx<T>* Xo = X + (size_t)op * xstride;
  const cpx<T>* ay = coefT + (size_t)op * cstride + (size_t)K * (n + 1);
  cpx<T>* pb = panel + (size_t)b * (K + 1) * C * n;
  for (int idx = tid; idx < 16 * nP; idx += NT) vb0[idx] = mk<T>(T(0), T(0));
  __syncthreads();
  // middle line: v = (f_m - B_m w_{m-1}) - B_{m+1} v_{m+1}
  for (int idx = tid; idx < 8 * n; idx += NT) {
    int c = idx / n, r = idx - c * n;
    if (c < nc)
      vb0[c * nP + r] = pb[((size_t)K * C + c0 + c) * n + r] -
                        ay[(size_t)(mid + 1) * n + r] * pb[((size_t)(mid + 1) * C + c0 + c) * n + r];
  }
  __syncthreads();
  cpx<T>* vc = vb0;
  cpx<T>* vn = vb1;
  mfma_matvec<T, MAXT, NW>(Xo + (size_t)mid * nP * nP, nP, vc, yb, red, wave, lane);
  {
    const int face = half ? mid + 1 : mid;
    for (int idx = tid; idx < 8 * n; idx += NT) {
      int c = idx / n, r = idx - c * n;
      if (c < nc) {
        cpx<T> x = yb[c * nP + r];
        if (half == 0) pb[((size_t)mid * C + c0 + c) * n + r] = x;
        vn[c * nP + r] = ay[(size_t)face * n + r] * x;
      }
    }
    __syncthreads();
    cpx<T>* t = vc;
    vc = vn;
    vn = t;
  }
  int k = half ? mid + 1 : mid - 1;
  const int nsteps = half ? K - 1 - mid : mid;
  for (int s = 0; s < nsteps; ++s) {
    mfma_matvec<T, MAXT, NW>(Xo + (size_t)k * nP * nP, nP, vc, yb, red, wave, lane);
    const bool more = s + 1 < nsteps;
    const int face = half ? k + 1 : k;
    for (int idx = tid; idx < 8 * n; idx += NT) {
      int c = idx / n, r = idx - c * n;
      if (c < nc) {
        size_t o = ((size_t)k * C + c0 + c) * n + r;
        cpx<T> x = pb[o] - yb[c * nP + r];
        pb[o] = x;
        if (more) vn[c * nP + r] = ay[(size_t)face * n + r] * x;
      }
    }
    __syncthreads();
    k += half ? 1 : -1;
    cpx<T>* t = vc;
    vc = vn;
    vn = t;
  }
}

template <class T>
static int solve_nw(int nP) {
  // 8 waves (sum split in 4 slices) when the LDS fits, else 4 waves
  size_t e = sizeof(cpx<T>);
  return (6 * 8 * (size_t)nP * e <= 160 * 1024) ? 8 : 4;
}

template <class T, int MAXT, int NW>
static hipError_t launch_solve_t(hdsw_ctx* c, int nbatch, const int* d_ops, int C) {
  const Geometry& g = c->g;
  dim3 grid((C + 7) / 8, nbatch, 2);
  size_t lds = (size_t)(2 + NW / 2) * 8 * g.nP * sizeof(cpx<T>);
  size_t xstride = (size_t)g.K * g.nP * g.nP;
  hipLaunchKernelGGL((k_solve_fwd<T, MAXT, NW>), grid, dim3(NW * 64), lds, c->stream,
                     (const cpx<T>*)c->d_X, xstride, (const cpx<T>*)c->d_coefT,
                     c->coef_stride, (cpx<T>*)c->d_panel, d_ops, c->gd, C, nbatch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_solve_bwd<T, MAXT, NW>), grid, dim3(NW * 64), lds, c->stream,
                     (const cpx<T>*)c->d_X, xstride, (const cpx<T>*)c->d_coefT,
                     c->coef_stride, (cpx<T>*)c->d_panel, d_ops, c->gd, C, nbatch);
  return hipGetLastError();
}

template <class T>
hipError_t launch_block_solve(hdsw_ctx* c, int nbatch, const int* d_ops, int C) {
  const int nMt = c->g.nP / 16;
  const int half = (nMt + 1) / 2;
  const int nw = solve_nw<T>(c->g.nP);
  if ((size_t)(2 + nw / 2) * 8 * c->g.nP * sizeof(cpx<T>) > 160 * 1024) return hipErrorInvalidValue;
  if (half <= 4)
    return nw == 8 ? launch_solve_t<T, 4, 8>(c, nbatch, d_ops, C)
                   : launch_solve_t<T, 4, 4>(c, nbatch, d_ops, C);
  if (half <= 8)
    return nw == 8 ? launch_solve_t<T, 8, 8>(c, nbatch, d_ops, C)
                   : launch_solve_t<T, 8, 4>(c, nbatch, d_ops, C);
  if (half <= 16)
    return nw == 8 ? launch_solve_t<T, 16, 8>(c, nbatch, d_ops, C)
                   : launch_solve_t<T, 16, 4>(c, nbatch, d_ops, C);
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------ factor
// One step of the twisted factorization for every distinct operator:
// blockIdx.y = 0 builds top line `step`, = 1 bottom line K-1-step; with
// `middle` set, blockIdx.y = 0 builds the middle line.  The Schur update
// uses the previous inverse(s), then the block is inverted in place by
// Gauss-Jordan elimination with partial pivoting (largest |re|+|im| in the
// pivot column, lowest row on ties).  The block is handled as its transpose
// in row-major form (leading dimension nP), so the inverse lands
// column-major.  One workgroup per (operator, chain).
template <class T>
__global__ __launch_bounds__(1024) void k_factor_step(cpx<T>* X, size_t xstride,
                                                      const cpx<T>* coefT, size_t cstride,
                                                      GeoDev g, int step, int middle,
                                                      int* flag, int nops) {
  extern __shared__ unsigned char smem_raw[];
  const int op = blockIdx.x, half = blockIdx.y;
  if (op >= nops) return;
  const int n = g.n, nP = g.nP, K = g.K, mid = g.mid;
  int k, pa = -1, fa = 0, pb2 = -1, fb = 0;
  if (middle) {
    if (half) return;
    k = mid;
    pa = mid - 1;
    fa = mid;
    pb2 = mid + 1;
    fb = mid + 1;
  } else if (half == 0) {
    k = step;
    if (k >= mid) return;
    if (k > 0) { pa = k - 1; fa = k; }
  } else {
    k = K - 1 - step;
    if (k <= mid) return;
    if (k < K - 1) { pa = k + 1; fa = k + 1; }
  }
  const int tid = threadIdx.x, bs = blockDim.x;
  cpx<T>* rowv = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* colv = rowv + n;
  int* perm = reinterpret_cast<int*>(colv + n);
  T* redv = reinterpret_cast<T*>(perm + ((n + 3) & ~3));
  int* redi = reinterpret_cast<int*>(redv + bs);

  const cpx<T>* Xo = X + (size_t)op * xstride;
  cpx<T>* M = X + (size_t)op * xstride + (size_t)k * nP * nP;
  const cpx<T>* co = coefT + (size_t)op * cstride;
  const cpx<T>* ax = co + (size_t)k * (n + 1);
  const cpx<T>* ay = co + (size_t)K * (n + 1);
  const cpx<T>* dg = co + (size_t)K * (n + 1) + (size_t)(K + 1) * n + (size_t)k * n;
  const cpx<T>* PA = pa >= 0 ? Xo + (size_t)pa * nP * nP : nullptr;
  const cpx<T>* PB = pb2 >= 0 ? Xo + (size_t)pb2 * nP * nP : nullptr;
  for (int idx = tid; idx < nP * nP; idx += bs) {
    int i = idx / nP, j = idx - i * nP;
    cpx<T> v = mk<T>(T(0), T(0));
    if (i < n && j < n) {
      if (i == j) v = dg[i];
      else if (j == i + 1) v = ax[j];
      else if (i == j + 1) v = ax[i];
      if (PA) v = v - ay[(size_t)fa * n + i] * ay[(size_t)fa * n + j] * PA[idx];
      if (PB) v = v - ay[(size_t)fb * n + i] * ay[(size_t)fb * n + j] * PB[idx];
    }
    M[idx] = v;
  }
  __threadfence_block();
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    T best = T(-1);
    int bi = n;
    for (int i = j + tid; i < n; i += bs) {
      cpx<T> a = M[(size_t)i * nP + j];
      T m = fabs(a.re) + fabs(a.im);
      if (m > best) { best = m; bi = i; }
    }
    redv[tid] = best;
    redi[tid] = bi;
    __syncthreads();
    for (int s = bs / 2; s > 0; s >>= 1) {
      if (tid < s) {
        T ob = redv[tid + s];
        int oi = redi[tid + s];
        if (ob > redv[tid] || (ob == redv[tid] && oi < redi[tid])) {
          redv[tid] = ob;
          redi[tid] = oi;
        }
      }
      __syncthreads();
    }
    int p = redi[0];
    if (p >= n) p = j;
    if (tid == 0) perm[j] = p;
    if (p != j) {
      for (int jj = tid; jj < n; jj += bs) {
        cpx<T> a = M[(size_t)j * nP + jj];
        M[(size_t)j * nP + jj] = M[(size_t)p * nP + jj];
        M[(size_t)p * nP + jj] = a;
      }
    }
    __threadfence_block();
    __syncthreads();
    cpx<T> piv = M[(size_t)j * nP + j];
    if (piv.re == T(0) && piv.im == T(0)) {
      if (tid == 0) atomicExch(flag, 1);
    }
    cpx<T> inv = cinv(piv);
    for (int jj = tid; jj < n; jj += bs) rowv[jj] = (jj == j) ? inv : M[(size_t)j * nP + jj] * inv;
    for (int i = tid; i < n; i += bs) colv[i] = M[(size_t)i * nP + j];
    __syncthreads();
    for (int idx = tid; idx < n * n; idx += bs) {
      int i = idx / n, jj = idx - i * n;
      size_t o = (size_t)i * nP + jj;
      if (i == j) {
        M[o] = rowv[jj];
      } else if (jj == j) {
        M[o] = -(colv[i] * inv);
      } else {
        cpx<T> m = M[o];
        cpx<T> cv = colv[i], rv = rowv[jj];
        m.re = fma(-cv.re, rv.re, m.re);
        m.re = fma(cv.im, rv.im, m.re);
        m.im = fma(-cv.re, rv.im, m.im);
        m.im = fma(-cv.im, rv.re, m.im);
        M[o] = m;
      }
    }
    __threadfence_block();
    __syncthreads();
  }
  for (int j = n - 1; j >= 0; --j) {
    int p = perm[j];
    if (p != j) {
      for (int i = tid; i < n; i += bs) {
        cpx<T> a = M[(size_t)i * nP + j];
        M[(size_t)i * nP + j] = M[(size_t)i * nP + p];
        M[(size_t)i * nP + p] = a;
      }
    }
    __threadfence_block();
    __syncthreads();
  }
}

template <class T>
hipError_t launch_factor_step(hdsw_ctx* c, int step, int middle) {
  const Geometry& g = c->g;
  int bs = 1024;
  size_t lds = 2 * g.n * sizeof(cpx<T>) + ((g.n + 3) & ~3) * sizeof(int) +
               bs * (sizeof(T) + sizeof(int));
  size_t xstride = (size_t)g.K * g.nP * g.nP;
  hipLaunchKernelGGL(k_factor_step<T>, dim3(c->nops, 2), dim3(bs), lds, c->stream,
                     (cpx<T>*)c->d_X, xstride, (const cpx<T>*)c->d_coefT, c->coef_stride,
                     c->gd, step, middle, c->d_flag, c->nops);
  return hipGetLastError();
}

// ------------------------------------------------------------ interface GEMM
// out[s][col][:] = T_op(s) g[s][col][:] (+ y[s][col][:]): the subdomain
// solve of one sweep step restricted to its interface layers.  One
// workgroup per (64 output rows, 8 columns, subdomain); each wave owns one
// 16-row tile over the whole sum; the step's sources are staged in LDS.
template <class T>
__global__ __launch_bounds__(256) void k_iface_gemm(const cpx<T>* __restrict__ Tm,
                                                    const cpx<T>* __restrict__ gbuf,
                                                    const cpx<T>* __restrict__ ybuf,
                                                    cpx<T>* __restrict__ out,
                                                    const int* __restrict__ op_of,
                                                    const int* __restrict__ subs, int C, int NI,
                                                    int NIc, int add_y) {
  typedef typename MF<T>::v4 v4;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* gs = reinterpret_cast<cpx<T>*>(smem_raw);   // [8][NIc]; reused for output
  const int s = subs[blockIdx.z];
  const int c0 = blockIdx.y * 8, nc = min(8, C - c0);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int row0 = blockIdx.x * 64 + wave * 16;
  const cpx<T>* Top = Tm + (size_t)op_of[s] * NI * NI;
  const cpx<T>* gb = gbuf + ((size_t)s * C + c0) * NI;
  const int jc = lane & 15, cc = jc & 7, part = jc >> 3, kk = lane >> 4, rr = lane & 15;
  const int myrow = row0 + rr;
  v4 acc = v4{T(0), T(0), T(0), T(0)};
  for (int jb = 0; jb < NI; jb += NIc) {
    const int jn = min(NIc, NI - jb);
    __syncthreads();
    for (int idx = tid; idx < 8 * NIc; idx += 256) {
      int cq = idx / NIc, j = idx - cq * NIc;
      gs[idx] = (cq < nc && j < jn) ? gb[(size_t)cq * NI + jb + j] : mk<T>(T(0), T(0));
    }
    __syncthreads();
    const cpx<T>* xc = Top + (size_t)jb * NI + myrow;
    const bool rowok = myrow < NI;
#pragma unroll 4
    for (int ks = 0; ks < (jn >> 2); ++ks) {
      const int j = 4 * ks + kk;
      const cpx<T> vv = gs[cc * NIc + j];
      const T b1 = part ? vv.im : vv.re;
      const T b2 = part ? vv.re : -vv.im;
      cpx<T> xa = rowok ? xc[(size_t)j * NI] : mk<T>(T(0), T(0));
      acc = MF<T>::mfma(xa.re, b1, acc);
      acc = MF<T>::mfma(xa.im, b2, acc);
    }
  }
  __syncthreads();
  // stage the 64 x 8 output tile in LDS, then write rows coalesced
  T* st = reinterpret_cast<T*>(gs);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int row = wave * 16 + MF<T>::row(lane, i);
    st[2 * (cc * 64 + row) + part] = acc[i];
  }
  __syncthreads();
  for (int idx = tid; idx < 8 * 64; idx += 256) {
    int cq = idx / 64, r = idx - cq * 64;
    int row = blockIdx.x * 64 + r;
    if (cq < nc && row < NI) {
      size_t o = ((size_t)s * C + c0 + cq) * NI + row;
      cpx<T> v = gs[cq * 64 + r];
      if (add_y) v = v + ybuf[o];
      out[o] = v;
    }
  }
}

template <class T>
hipError_t launch_iface_gemm(hdsw_ctx* c, int off, int cnt, int C, int add_y) {
  int NI = c->g.NI;
  int NIc = sizeof(T) == 4 ? 1024 : 512;
  NIc = std::min(NIc, (NI + 3) / 4 * 4);
  dim3 grid((NI + 63) / 64, (C + 7) / 8, cnt);
  size_t lds = std::max<size_t>((size_t)8 * NIc, 8 * 64) * sizeof(cpx<T>);
  hipLaunchKernelGGL(k_iface_gemm<T>, grid, dim3(256), lds, c->stream, (const cpx<T>*)c->d_T,
                     (const cpx<T>*)c->d_g, (const cpx<T>*)c->d_y, (cpx<T>*)c->d_out,
                     c->d_op_of_sub, c->d_step_subs + off, C, NI, NIc, add_y);
  return hipGetLastError();
}

#define HDSW_INST2(T)                                                          \
  template hipError_t launch_block_solve<T>(hdsw_ctx*, int, const int*, int);  \
  template hipError_t launch_factor_step<T>(hdsw_ctx*, int, int);              \
  template hipError_t launch_iface_gemm<T>(hdsw_ctx*, int, int, int, int);
HDSW_INST2(float)
HDSW_INST2(double)

}  // namespace hdsw

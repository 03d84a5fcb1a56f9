// Factorization, batched block solve and fused sweep step of the hdsw library.
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
// Every barrier of the solve and sweep kernels orders LDS only: no global
// data passes between threads of a workgroup within one launch (each thread
// reads back only the panel entries it wrote), so prefetched loads stay in
// flight across barriers.
//
// Solve with the stored inverses, two launches:
//   A: top     w_k = X_k (f_k - B_k w_{k-1})          k = 0 .. m-1
//      bottom  v_k = X_k (f_k - B_{k+1} v_{k+1})      k = K-1 .. m+1
//      (the top chain leaves f_m - B_m w_{m-1} in scratch line K, the
//      bottom chain B_{m+1} v_{m+1} in scratch line K + 1, so launch B never
//      reads a line that one of its chains overwrites)
//   B: middle  x_m = X_m (f_m - B_m w_{m-1} - B_{m+1} v_{m+1})
//      top     x_k = w_k - X_k B_{k+1} x_{k+1}        k = m-1 .. 0
//      bottom  x_k = v_k - X_k B_k x_{k-1}            k = m+1 .. K-1
// Every block product is a complex matrix times groups of 8 complex columns
// on the matrix cores (one group per workgroup, two for complex64 batches
// with many workgroups): with X = Xr + i Xi and V = Vr + i Vi,
//   [Yr | Yi] = Xr [Vr | Vi] + Xi [-Vi | Vr],
// two real 16x16x4 MFMAs per 16-row tile, column group and 4-deep slice of
// the sum.
#include "hdsw_internal.hpp"
#include "mfma_ops.hpp"

namespace hdsw {

// ------------------------------------------------------------ matvec
// y[r][c] = sum_j Xb(r, j) vb[j][c] for 8 columns c (LDS, row-major with the
// 8 columns contiguous so one 4-row slice is 64 distinct banks; zero beyond
// n).  Waves split the rows in two halves of 16-row tiles and the sum in
// KS = NW / 2 slices; the slices are added in a fixed order, so results do
// not depend on timing.
//
// A wave's X tiles are loaded in batches of KSB 4-deep slices; the first
// batch of the next block is loaded while the current block is reduced and
// its epilogue runs, so the load latency is hidden behind LDS work.
template <class T, int MAXT, int KSB>
struct WaveTiles {
  cpx<T> x[KSB][MAXT];
};

// Loads under a branch make the compiler wait for every load in flight
// before the first use; unconditional loads let it count them.  For the X
// tiles the counted form is faster for complex128 blocks and slower for
// complex64 ones (measured on the 1024^2 workload: 0.91 vs 1.00 ms and 1.37
// vs 1.20 ms per block solve), so the form follows the precision; the
// epilogue prefetch is unconditional in both (1.20 -> 1.14 ms for
// complex64).  Unconditionally, a slice past k1 re-reads slice k1 - 1 and a
// tile past nt reads past the block's last row (at most MAXT - nt tiles,
// kept in bounds by the spare block after the inverses); neither value
// reaches a result.
//
// complex64 with 8-column workgroups double-buffers the batches instead: the
// second batch is loaded while the first one's MFMAs run, with counted loads
// and unconditional MFMAs (a slice past k1 gets a zero vector operand), 1.14
// -> 1.09 ms per block solve on the 1024^2 workload; the other forms would
// spill with a second buffer.
template <class T, int NG>
struct DoubleBuf { static constexpr bool v = sizeof(T) == 4 && NG == 1; };
template <class T, int NG>
struct CountedLoads { static constexpr bool v = sizeof(T) == 8 || DoubleBuf<T, NG>::v; };

template <class T, int MAXT, int KSB, int NG>
__device__ __forceinline__ void mv_load(WaveTiles<T, MAXT, KSB>& w, const cpx<T>* __restrict__ Xb,
                                        int nP, int t0, int nt, int kb0, int k1, int kk, int rr) {
  const cpx<T>* base = Xb + (size_t)(t0 * 16 + rr);
#pragma unroll
  for (int q = 0; q < KSB; ++q) {
    if constexpr (CountedLoads<T, NG>::v) {
      const int ks = max(0, min(kb0 + q, k1 - 1));
      const cpx<T>* xc = base + (size_t)(4 * ks + kk) * nP;
#pragma unroll
      for (int t = 0; t < MAXT; ++t) w.x[q][t] = xc[t * 16];
    } else {
      const int ks = kb0 + q;
      if (ks < k1) {
        const cpx<T>* xc = base + (size_t)(4 * ks + kk) * nP;
#pragma unroll
        for (int t = 0; t < MAXT; ++t)
          if (t < nt) w.x[q][t] = xc[t * 16];
      }
    }
  }
}

// NG groups of 8 columns: every X tile loaded feeds NG pairs of MFMAs
template <class T, int MAXT, int KSB, int NG>
__device__ __forceinline__ void mv_mfma(const WaveTiles<T, MAXT, KSB>& w,
                                        typename MF<T>::v4 (&acc)[MAXT][NG], const cpx<T>* vb,
                                        int kb0, int k1, int nt, int kk, int cc, int part) {
#pragma unroll
  for (int q = 0; q < KSB; ++q) {
    const int ks = kb0 + q;
    if (ks < k1) {
#pragma unroll
      for (int gq = 0; gq < NG; ++gq) {
        const cpx<T> vv = vb[(4 * ks + kk) * 8 * NG + gq * 8 + cc];
        const T b1 = part ? vv.im : vv.re;
        const T b2 = part ? vv.re : -vv.im;
#pragma unroll
        for (int t = 0; t < MAXT; ++t) {
          if (t < nt) {
            acc[t][gq] = MF<T>::mfma(w.x[q][t].re, b1, acc[t][gq]);
            acc[t][gq] = MF<T>::mfma(w.x[q][t].im, b2, acc[t][gq]);
          }
        }
      }
    }
  }
}

// The same with every MFMA issued (double-buffered form): slices past k1
// multiply a zero vector operand, tiles past nt accumulate rows never stored
template <class T, int MAXT, int KSB, int NG>
__device__ __forceinline__ void mv_mfma_all(const WaveTiles<T, MAXT, KSB>& w,
                                            typename MF<T>::v4 (&acc)[MAXT][NG],
                                            const cpx<T>* vb, int kb0, int k1, int kk, int cc,
                                            int part) {
#pragma unroll
  for (int q = 0; q < KSB; ++q) {
    const int ks = kb0 + q;
    const bool ok = ks < k1;
    const int ksc = ok ? ks : k1 - 1;
#pragma unroll
    for (int gq = 0; gq < NG; ++gq) {
      const cpx<T> vv = vb[(4 * ksc + kk) * 8 * NG + gq * 8 + cc];
      const T b1 = ok ? (part ? vv.im : vv.re) : T(0);
      const T b2 = ok ? (part ? vv.re : -vv.im) : T(0);
#pragma unroll
      for (int t = 0; t < MAXT; ++t) {
        acc[t][gq] = MF<T>::mfma(w.x[q][t].re, b1, acc[t][gq]);
        acc[t][gq] = MF<T>::mfma(w.x[q][t].im, b2, acc[t][gq]);
      }
    }
  }
}

// Wave geometry of the matvec
struct WaveGeo {
  int t0, nt, k0, k1, cc, part, kk, rr, kq;
};
template <int NW>
__device__ inline WaveGeo wave_geo(int nP, int wave, int lane) {
  constexpr int KS = NW / 2;
  WaveGeo w;
  const int nMt = nP >> 4, nK = nP >> 2;
  const int mh = wave & 1;
  w.kq = wave >> 1;
  const int th = (nMt + 1) >> 1;
  w.t0 = mh ? th : 0;
  w.nt = mh ? nMt - th : th;
  const int kchunk = (nK + KS - 1) / KS;
  w.k0 = min(nK, w.kq * kchunk);
  w.k1 = min(nK, w.k0 + kchunk);
  const int jc = lane & 15;
  w.cc = jc & 7;
  w.part = jc >> 3;
  w.kk = lane >> 4;
  w.rr = lane & 15;
  return w;
}

// One block product y = X_k vc.  On entry `tiles` holds the first batch of
// X_k; on exit it holds the first batch of Xnext (if not null).  Every wave
// leaves its part of the sum (rows of its half, a quarter of the columns of
// X_k) in red[kq]; ends with the block synchronized, the parts complete.
template <class T, int MAXT, int KSB, int NW, int NG>
__device__ __forceinline__ void block_product(WaveTiles<T, MAXT, KSB>& tiles, const WaveGeo& wg,
                                              const cpx<T>* __restrict__ Xk,
                                              const cpx<T>* __restrict__ Xnext, int nP,
                                              const cpx<T>* vc, cpx<T>* red, int lane) {
  typedef typename MF<T>::v4 v4;
  v4 acc[MAXT][NG];
#pragma unroll
  for (int t = 0; t < MAXT; ++t)
#pragma unroll
    for (int gq = 0; gq < NG; ++gq) acc[t][gq] = v4{T(0), T(0), T(0), T(0)};
  if constexpr (DoubleBuf<T, NG>::v) {
    WaveTiles<T, MAXT, KSB> tb;
    for (int kb = wg.k0; kb < wg.k1; kb += 2 * KSB) {
      const bool second = kb + KSB < wg.k1;
      if (second)
        mv_load<T, MAXT, KSB, NG>(tb, Xk, nP, wg.t0, wg.nt, kb + KSB, wg.k1, wg.kk, wg.rr);
      mv_mfma_all<T, MAXT, KSB, NG>(tiles, acc, vc, kb, wg.k1, wg.kk, wg.cc, wg.part);
      if (kb + 2 * KSB < wg.k1)
        mv_load<T, MAXT, KSB, NG>(tiles, Xk, nP, wg.t0, wg.nt, kb + 2 * KSB, wg.k1, wg.kk, wg.rr);
      if (second)
        mv_mfma_all<T, MAXT, KSB, NG>(tb, acc, vc, kb + KSB, wg.k1, wg.kk, wg.cc, wg.part);
    }
  } else {
    mv_mfma<T, MAXT, KSB, NG>(tiles, acc, vc, wg.k0, wg.k1, wg.nt, wg.kk, wg.cc, wg.part);
    for (int kb = wg.k0 + KSB; kb < wg.k1; kb += KSB) {
      mv_load<T, MAXT, KSB, NG>(tiles, Xk, nP, wg.t0, wg.nt, kb, wg.k1, wg.kk, wg.rr);
      mv_mfma<T, MAXT, KSB, NG>(tiles, acc, vc, kb, wg.k1, wg.nt, wg.kk, wg.cc, wg.part);
    }
  }
  if (Xnext)
    mv_load<T, MAXT, KSB, NG>(tiles, Xnext, nP, wg.t0, wg.nt, wg.k0, wg.k1, wg.kk, wg.rr);
  T* dst = reinterpret_cast<T*>(red + (size_t)wg.kq * 8 * NG * nP);
#pragma unroll
  for (int t = 0; t < MAXT; ++t)
    if (t < wg.nt)
#pragma unroll
      for (int gq = 0; gq < NG; ++gq)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          int row = 16 * (wg.t0 + t) + MF<T>::row(lane, i);
          dst[2 * (row * 8 * NG + gq * 8 + wg.cc) + wg.part] = acc[t][gq][i];
        }
  lds_barrier();
}

// Entry rc = row * 8 NG + column of the last block product: its NW / 2 parts
// added in a fixed order, so the result does not depend on timing.
template <class T, int NW, int NG>
__device__ __forceinline__ cpx<T> prod_y(const cpx<T>* red, int nP, int rc) {
  cpx<T> y = red[rc];
#pragma unroll
  for (int q = 1; q < NW / 2; ++q) y = y + red[(size_t)q * 8 * NG * nP + rc];
  return y;
}

// ------------------------------------------------------------ solve A
// EPT epilogue elements per thread have their global operands prefetched
// before the block product (EPT * threads >= 8 NG n is checked at launch).
// A workgroup owns 8 NG columns of one batch entry and one chain.  Entry
// idx of the epilogue is row idx / 8 NG, column idx % 8 NG: the lanes of a
// wave read the partial sums and write the next vector at consecutive LDS
// addresses (row-major [row][8 NG]), free of bank conflicts (with the row
// fastest, the lanes of a wave would all meet in two banks).
template <class T, int MAXT, int KSB, int NW, int EPT, int NG>
__global__ __launch_bounds__(NW * 64) void k_solve_fwd(const cpx<T>* __restrict__ X,
                                                       size_t xstride,
                                                       const cpx<T>* __restrict__ coefT,
                                                       size_t cstride, cpx<T>* panel,
                                                       const int* __restrict__ ops, GeoDev g,
                                                       int C, int nbatch,
                                                       const int* __restrict__ nzflag) {
  extern __shared__ unsigned char smem_raw[];
  constexpr int NT = NW * 64;
  const int n = g.n, nP = g.nP, K = g.K, mid = g.mid;
  const int b = blockIdx.y, half = blockIdx.z;
  if (b >= nbatch) return;
  constexpr int NCOL = 8 * NG;                    // columns of the workgroup
  const int c0 = blockIdx.x * NCOL, nc = min(NCOL, C - c0);
  if (nzflag) {
    // a right-hand side that is zero in all of the workgroup's columns
    // solves to zero, which the panel already holds (both chains and both
    // passes skip alike, so the scratch lines are never read)
    const int* fl = nzflag + (size_t)b * ((C + 7) / 8) + c0 / 8;
    int any = 0;
#pragma unroll
    for (int q = 0; q < NG; ++q)
      if (c0 + 8 * q < C) any |= fl[q];
    if (!any) return;
  }
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  cpx<T>* vb0 = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* vb1 = vb0 + NCOL * nP;
  cpx<T>* red = vb1 + NCOL * nP;                  // NW / 2 parts of a product
  const int op = ops[b];
  const cpx<T>* Xo = X + (size_t)op * xstride;
  const cpx<T>* ay = coefT + (size_t)op * cstride + (size_t)K * (n + 1);
  cpx<T>* pb = panel + (size_t)b * g.PL * C * n;
  const WaveGeo wg = wave_geo<NW>(nP, wave, lane);
  for (int idx = tid; idx < 2 * NCOL * nP; idx += NT) vb0[idx] = mk<T>(T(0), T(0));
  lds_barrier();
  int k = half ? K - 1 : 0;
  const int nsteps = half ? K - 1 - mid : mid;
  for (int idx = tid; idx < NCOL * n; idx += NT) {
    int c = idx / n, r = idx - c * n;
    if (c < nc) vb0[r * NCOL + c] = pb[((size_t)k * C + c0 + c) * n + r];
  }
  WaveTiles<T, MAXT, KSB> tiles;
  mv_load<T, MAXT, KSB, NG>(tiles, Xo + (size_t)k * nP * nP, nP, wg.t0, wg.nt, wg.k0, wg.k1, wg.kk,
                        wg.rr);
  lds_barrier();
  cpx<T>* vc = vb0;
  cpx<T>* vn = vb1;
  for (int s = 0; s < nsteps; ++s) {
    const bool more = s + 1 < nsteps;
    const int kn = half ? k - 1 : k + 1;
    const int face = half ? k : k + 1;
    // prefetch the epilogue operands: f of the next line and the coupling
    cpx<T> fpre[EPT], apre[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      int idx = tid + q * NT;
      int r = idx / NCOL, c = idx - r * NCOL;
      if (!(idx < NCOL * n && c < nc)) c = r = 0;   // unused value: the load stays unconditional
      fpre[q] = pb[((size_t)kn * C + c0 + c) * n + r];
      apre[q] = ay[(size_t)face * n + r];
    }
    block_product<T, MAXT, KSB, NW, NG>(tiles, wg, Xo + (size_t)k * nP * nP,
                                    more ? Xo + (size_t)kn * nP * nP : nullptr, nP, vc, red,
                                    lane);
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      int idx = tid + q * NT;
      int r = idx / NCOL, c = idx - r * NCOL;
      if (idx < NCOL * n && c < nc) {
        cpx<T> y = prod_y<T, NW, NG>(red, nP, r * NCOL + c);
        pb[((size_t)k * C + c0 + c) * n + r] = y;
        cpx<T> nxt = fpre[q] - apre[q] * y;
        if (more) vn[r * NCOL + c] = nxt;
        else if (half == 0)   // scratch line K: f_m - B_m w_{m-1}
          pb[((size_t)K * C + c0 + c) * n + r] = nxt;
        else                  // scratch line K + 1: B_{m+1} v_{m+1}
          pb[((size_t)(K + 1) * C + c0 + c) * n + r] = apre[q] * y;
      }
    }
    lds_barrier();
    k = kn;
    cpx<T>* t = vc;
    vc = vn;
    vn = t;
  }
}

// ------------------------------------------------------------ solve B
template <class T, int MAXT, int KSB, int NW, int EPT, int NG>
__global__ __launch_bounds__(NW * 64) void k_solve_bwd(const cpx<T>* __restrict__ X,
                                                       size_t xstride,
                                                       const cpx<T>* __restrict__ coefT,
                                                       size_t cstride, cpx<T>* panel,
                                                       const int* __restrict__ ops, GeoDev g,
                                                       int C, int nbatch,
                                                       const int* __restrict__ nzflag) {
  extern __shared__ unsigned char smem_raw[];
  constexpr int NT = NW * 64;
  const int n = g.n, nP = g.nP, K = g.K, mid = g.mid;
  const int b = blockIdx.y, half = blockIdx.z;
  if (b >= nbatch) return;
  constexpr int NCOL = 8 * NG;                    // columns of the workgroup
  const int c0 = blockIdx.x * NCOL, nc = min(NCOL, C - c0);
  if (nzflag) {
    // a right-hand side that is zero in all of the workgroup's columns
    // solves to zero, which the panel already holds (both chains and both
    // passes skip alike, so the scratch lines are never read)
    const int* fl = nzflag + (size_t)b * ((C + 7) / 8) + c0 / 8;
    int any = 0;
#pragma unroll
    for (int q = 0; q < NG; ++q)
      if (c0 + 8 * q < C) any |= fl[q];
    if (!any) return;
  }
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  cpx<T>* vb0 = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* vb1 = vb0 + NCOL * nP;
  cpx<T>* red = vb1 + NCOL * nP;                  // NW / 2 parts of a product
  const int op = ops[b];
  const cpx<T>* Xo = X + (size_t)op * xstride;
  const cpx<T>* ay = coefT + (size_t)op * cstride + (size_t)K * (n + 1);
  cpx<T>* pb = panel + (size_t)b * g.PL * C * n;
  const WaveGeo wg = wave_geo<NW>(nP, wave, lane);
  for (int idx = tid; idx < 2 * NCOL * nP; idx += NT) vb0[idx] = mk<T>(T(0), T(0));
  lds_barrier();
  // middle line: v = (f_m - B_m w_{m-1}) - B_{m+1} v_{m+1}, both terms from
  // the scratch lines the forward launch left.  Line m + 1 itself is not
  // read: the bottom chain of this launch overwrites it with x_{m+1}, and
  // nothing orders the two chains' workgroups.
  for (int idx = tid; idx < NCOL * n; idx += NT) {
    int c = idx / n, r = idx - c * n;
    if (c < nc)
      vb0[r * NCOL + c] = pb[((size_t)K * C + c0 + c) * n + r] -
                          pb[((size_t)(K + 1) * C + c0 + c) * n + r];
  }
  WaveTiles<T, MAXT, KSB> tiles;
  mv_load<T, MAXT, KSB, NG>(tiles, Xo + (size_t)mid * nP * nP, nP, wg.t0, wg.nt, wg.k0, wg.k1,
                        wg.kk, wg.rr);
  lds_barrier();
  cpx<T>* vc = vb0;
  cpx<T>* vn = vb1;
  const int nsteps = half ? K - 1 - mid : mid;
  int k = half ? mid + 1 : mid - 1;
  {
    const int face = half ? mid + 1 : mid;
    cpx<T> apre[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      int idx = tid + q * NT;
      int r = idx / NCOL, c = idx - r * NCOL;
      if (!(idx < NCOL * n && c < nc)) r = 0;
      apre[q] = ay[(size_t)face * n + r];
    }
    block_product<T, MAXT, KSB, NW, NG>(tiles, wg, Xo + (size_t)mid * nP * nP,
                                    nsteps > 0 ? Xo + (size_t)k * nP * nP : nullptr, nP, vc,
                                    red, lane);
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      int idx = tid + q * NT;
      int r = idx / NCOL, c = idx - r * NCOL;
      if (idx < NCOL * n && c < nc) {
        cpx<T> x = prod_y<T, NW, NG>(red, nP, r * NCOL + c);
        if (half == 0) pb[((size_t)mid * C + c0 + c) * n + r] = x;
        vn[r * NCOL + c] = apre[q] * x;
      }
    }
    lds_barrier();
    cpx<T>* t = vc;
    vc = vn;
    vn = t;
  }
  for (int s = 0; s < nsteps; ++s) {
    const bool more = s + 1 < nsteps;
    const int kn = half ? k + 1 : k - 1;
    const int face = half ? k + 1 : k;
    cpx<T> wpre[EPT], apre[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      int idx = tid + q * NT;
      int r = idx / NCOL, c = idx - r * NCOL;
      if (!(idx < NCOL * n && c < nc)) c = r = 0;
      wpre[q] = pb[((size_t)k * C + c0 + c) * n + r];
      apre[q] = ay[(size_t)face * n + r];
    }
    block_product<T, MAXT, KSB, NW, NG>(tiles, wg, Xo + (size_t)k * nP * nP,
                                    more ? Xo + (size_t)kn * nP * nP : nullptr, nP, vc, red,
                                    lane);
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      int idx = tid + q * NT;
      int r = idx / NCOL, c = idx - r * NCOL;
      if (idx < NCOL * n && c < nc) {
        cpx<T> x = wpre[q] - prod_y<T, NW, NG>(red, nP, r * NCOL + c);
        pb[((size_t)k * C + c0 + c) * n + r] = x;
        if (more) vn[r * NCOL + c] = apre[q] * x;
      }
    }
    lds_barrier();
    k = kn;
    cpx<T>* t = vc;
    vc = vn;
    vn = t;
  }
}

template <class T>
static int solve_nw(int nP, int NG) {
  // as many waves as the LDS allows: (2 + NW/2) vectors of 8 NG x nP complex
  size_t e = sizeof(cpx<T>);
  auto fits = [&](int nw) { return (size_t)(2 + nw / 2) * 8 * NG * nP * e <= 160 * 1024; };
  if (fits(8)) return 8;
  if (fits(4)) return 4;
  return 0;
}

// 4-deep slices loaded per batch: as many as fit in registers without spills
// (checked in the register report of the build for every instantiation)
template <class T, int MAXT>
struct SolveKSB {
  static constexpr int v =
      sizeof(T) == 4 ? (MAXT <= 5 ? 5 : MAXT <= 8 ? 2 : 1) : (MAXT == 5 ? 3 : 2);
};

template <class T, int MAXT, int NW, int NG>
static hipError_t launch_solve_t(hdsw_ctx* c, int nbatch, const int* d_ops, int C,
                                 const int* nzflag) {
  // epilogue entries per thread: 8 NG columns of up to 256 rows (up to 384
  // with 12 tiles per half)
  constexpr int EPT = (MAXT <= 8 ? 2048 : 3072) * NG / (NW * 64);
  const Geometry& g = c->g;
  if (8 * NG * g.n > EPT * NW * 64) return hipErrorInvalidValue;
  dim3 grid((C + 8 * NG - 1) / (8 * NG), nbatch, 2);
  size_t lds = (size_t)(2 + NW / 2) * 8 * NG * g.nP * sizeof(cpx<T>);
  size_t xstride = (size_t)g.K * g.nP * g.nP;
  hipLaunchKernelGGL((k_solve_fwd<T, MAXT, SolveKSB<T, MAXT>::v, NW, EPT, NG>), grid, dim3(NW * 64), lds,
                     c->stream, (const cpx<T>*)c->d_X, xstride, (const cpx<T>*)c->d_coefT,
                     c->coef_stride, (cpx<T>*)c->d_panel, d_ops, c->gd, C, nbatch, nzflag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_solve_bwd<T, MAXT, SolveKSB<T, MAXT>::v, NW, EPT, NG>), grid, dim3(NW * 64), lds,
                     c->stream, (const cpx<T>*)c->d_X, xstride, (const cpx<T>*)c->d_coefT,
                     c->coef_stride, (cpx<T>*)c->d_panel, d_ops, c->gd, C, nbatch, nzflag);
  return hipGetLastError();
}

template <class T, int NW, int NG>
static hipError_t launch_solve_nw(hdsw_ctx* c, int nbatch, const int* d_ops, int C,
                                  const int* nz) {
  const int nMt = c->g.nP / 16;
  const int th = (nMt + 1) / 2;
  if (th <= 2) return launch_solve_t<T, 2, NW, NG>(c, nbatch, d_ops, C, nz);
  if (th <= 3) return launch_solve_t<T, 3, NW, NG>(c, nbatch, d_ops, C, nz);
  if (th <= 5) return launch_solve_t<T, 5, NW, NG>(c, nbatch, d_ops, C, nz);
  if (th <= 8) return launch_solve_t<T, 8, NW, NG>(c, nbatch, d_ops, C, nz);
  // complex64 lines of up to 384 nodes (8 columns: the LDS holds the
  // vectors of eight waves; setup refuses longer lines and complex128
  // beyond 256)
  if constexpr (sizeof(T) == 4 && NW == 8 && NG == 1)
    if (th <= 12) return launch_solve_t<T, 12, NW, NG>(c, nbatch, d_ops, C, nz);
  return hipErrorInvalidValue;
}

template <class T>
hipError_t launch_big_solve(hdsw_ctx* c, int nbatch, const int* d_ops, const int* grp_op,
                            const int* grp_off, const int* grp_cnt, const int* ids,
                            int ngroups, int maxcnt, int C);

// nzflag (2D, may be null): per (batch entry, 8 columns), 0 where the
// right-hand side in the panel is zero; those workgroups return at once.
template <class T>
hipError_t launch_block_solve(hdsw_ctx* c, int nbatch, const int* d_ops, int C,
                              const int* nzflag) {
  if (c->g.dim == 3) {
    // plane blocks: one GEMM per plane and operator group; the batch is
    // either every subdomain (grouped by operator) or one operator's panel
    if (nbatch == c->g.nsub && d_ops == c->d_op_of_sub)
      return launch_big_solve<T>(c, nbatch, d_ops, c->d_grp_op, c->d_grp_off, c->d_grp_cnt,
                                 c->d_grp_ids, c->ngrp, c->grp_maxcnt, C);
    if (nbatch == 1)
      return launch_big_solve<T>(c, 1, d_ops, d_ops, c->d_zero_int, c->d_one_int,
                                 c->d_zero_int, 1, 1, C);
    return hipErrorInvalidValue;
  }
  // complex64: 16 columns per workgroup once 8-column workgroups would take
  // more than two rounds of the 256 CUs (throughput-bound: every X tile then
  // feeds twice the MFMAs); 8 while the chain latency dominates, unless the
  // autotuner chose (solve_ng; columns of an MFMA product are independent,
  // so the choice does not change results).  complex128 keeps 8 (16 would
  // not fit the register file)
  if constexpr (sizeof(T) == 4) {
    const long long wg8 = (long long)((C + 7) / 8) * nbatch * 2;
    const bool wide = c->tune.solve_ng ? c->tune.solve_ng == 2 : (C >= 16 && wg8 > 2 * 256);
    if (wide && C > 8 && solve_nw<T>(c->g.nP, 2) == 8)
      return launch_solve_nw<T, 8, 2>(c, nbatch, d_ops, C, nzflag);
  }
  const int nw = solve_nw<T>(c->g.nP, 1);
  if (nw == 8) return launch_solve_nw<T, 8, 1>(c, nbatch, d_ops, C, nzflag);
  if (nw == 4) return launch_solve_nw<T, 4, 1>(c, nbatch, d_ops, C, nzflag);
  return hipErrorInvalidValue;
}

// Swaps two complex entries of global memory field by field (a struct copy
// between two entries of one array goes through a private temporary).
template <class T>
__device__ __forceinline__ void swap_fields(cpx<T>* x, cpx<T>* y) {
  const T xr = x->re, xi = x->im, yr = y->re, yi = y->im;
  x->re = yr;
  x->im = yi;
  y->re = xr;
  y->im = xi;
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
      // the source is chosen as a pointer and read field by field: a struct
      // copy under a condition would keep v in private memory
      const cpx<T>* src = i == j ? dg + i : j == i + 1 ? ax + j : i == j + 1 ? ax + i : nullptr;
      if (src) v = mk<T>(src->re, src->im);
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
      for (int jj = tid; jj < n; jj += bs) swap_fields(M + (size_t)j * nP + jj, M + (size_t)p * nP + jj);
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
      for (int i = tid; i < n; i += bs) swap_fields(M + (size_t)i * nP + j, M + (size_t)i * nP + p);
    }
    __threadfence_block();
    __syncthreads();
  }
}

// Register-resident variant for blocks of n <= 32 B: a 32 x 32 grid of
// threads, thread (tr, tc) = (tid % 32, tid / 32) holding the B x B
// sub-block of rows B tr.., columns B tc.. in registers (zero beyond n).
// Per pivot: the search in column j and the interchanged column j are
// formed within the 32 threads of column group j / B (one half-wave,
// shuffles), the old rows j and p go through LDS (buffers double-buffered
// by pivot parity, so two barriers per pivot), and every thread updates
// its own sub-block.  Same
// arithmetic and pivot rule as k_factor_step.  Register arrays are indexed
// by unrolled compile-time loops only (a run-time index would spill them).
template <class T, int B>
__global__ __launch_bounds__(1024) void k_factor_reg(cpx<T>* X, size_t xstride,
                                                     const cpx<T>* coefT, size_t cstride,
                                                     GeoDev g, int step, int middle, int* flag,
                                                     int nops) {
  constexpr int NB = 32 * B;
  __shared__ cpx<T> rowj[2][NB], rowp[2][NB], colv[2][NB];
  __shared__ int pivs[2];
  __shared__ int perm[NB];
  __shared__ int place[NB];
  __shared__ int src[NB];
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
  const int tid = threadIdx.x, tr = tid & 31, tc = tid >> 5;
  const int r0 = B * tr, c0 = B * tc;
  const cpx<T>* Xo = X + (size_t)op * xstride;
  cpx<T>* M = X + (size_t)op * xstride + (size_t)k * nP * nP;
  const cpx<T>* co = coefT + (size_t)op * cstride;
  const cpx<T>* ax = co + (size_t)k * (n + 1);
  const cpx<T>* ay = co + (size_t)K * (n + 1);
  const cpx<T>* dg = co + (size_t)K * (n + 1) + (size_t)(K + 1) * n + (size_t)k * n;
  const cpx<T>* PA = pa >= 0 ? Xo + (size_t)pa * nP * nP : nullptr;
  const cpx<T>* PB = pb2 >= 0 ? Xo + (size_t)pb2 * nP * nP : nullptr;
  cpx<T> m[B][B];
#pragma unroll
  for (int a = 0; a < B; ++a)
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int i = r0 + a, j = c0 + b;
      cpx<T> v = mk<T>(T(0), T(0));
      if (i < n && j < n) {
        if (i == j) v = dg[i];
        else if (j == i + 1) v = ax[j];
        else if (i == j + 1) v = ax[i];
        const size_t idx = (size_t)i * nP + j;
        if (PA) v = v - ay[(size_t)fa * n + i] * ay[(size_t)fa * n + j] * PA[idx];
        if (PB) v = v - ay[(size_t)fb * n + i] * ay[(size_t)fb * n + j] * PB[idx];
      }
      m[a][b] = v;
    }
  for (int j = 0; j < n; ++j) {
    const int par = j & 1;
    // 1. column group j / B: pivot search (largest |Re| + |Im| at or below
    //    the diagonal, lowest row on ties) and column j after the
    //    interchange of rows j and p, both within the half-wave
    if (tc == j / B) {
      T best = T(-1);
      int bi = n;
      cpx<T> cj[B];
#pragma unroll
      for (int a = 0; a < B; ++a) {
        cj[a] = mk<T>(T(0), T(0));
#pragma unroll
        for (int b = 0; b < B; ++b)
          if (c0 + b == j) {
            cj[a] = m[a][b];
            if (r0 + a >= j && r0 + a < n) {
              const T v = fabs(m[a][b].re) + fabs(m[a][b].im);
              if (v > best) { best = v; bi = r0 + a; }
            }
          }
      }
#pragma unroll
      for (int o = 16; o > 0; o >>= 1) {
        const T ob = __shfl_xor(best, o, 32);
        const int oi = __shfl_xor(bi, o, 32);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      const int p = bi < n ? bi : j;
      // entries (j, j) and (p, j) from the threads holding rows j and p
      cpx<T> vj = mk<T>(T(0), T(0)), vp = vj;
#pragma unroll
      for (int a = 0; a < B; ++a) {
        if (r0 + a == j) vj = cj[a];
        if (r0 + a == p) vp = cj[a];
      }
      const int sj = j / B, sp = p / B;
      cpx<T> aj, ap;
      aj.re = __shfl(vj.re, sj, 32);
      aj.im = __shfl(vj.im, sj, 32);
      ap.re = __shfl(vp.re, sp, 32);
      ap.im = __shfl(vp.im, sp, 32);
#pragma unroll
      for (int a = 0; a < B; ++a) {
        const int i = r0 + a;
        cpx<T> v = cj[a];
        if (i == j) v = ap;
        else if (i == p) v = aj;
        colv[par][i] = v;
      }
      if (tr == 0) pivs[par] = p;
    }
    __syncthreads();
    const int p = pivs[par];
    if (tid == 0) perm[j] = p;
    // 2. the old rows j and p
#pragma unroll
    for (int a = 0; a < B; ++a) {
      if (r0 + a == j)
#pragma unroll
        for (int b = 0; b < B; ++b) rowj[par][c0 + b] = m[a][b];
      if (r0 + a == p)
#pragma unroll
        for (int b = 0; b < B; ++b) rowp[par][c0 + b] = m[a][b];
    }
    __syncthreads();
    const cpx<T> piv = colv[par][j];
    if (piv.re == T(0) && piv.im == T(0) && tid == 0) atomicExch(flag, 1);
    const cpx<T> inv = cinv(piv);
    // 3. Gauss-Jordan update of the own sub-block
    cpx<T> rv[B], cv[B];
#pragma unroll
    for (int b = 0; b < B; ++b) rv[b] = rowp[par][c0 + b] * inv;
#pragma unroll
    for (int a = 0; a < B; ++a) cv[a] = colv[par][r0 + a];
#pragma unroll
    for (int a = 0; a < B; ++a)
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int i = r0 + a, jj = c0 + b;
        if (i >= n || jj >= n) continue;
        if (i == j) {
          m[a][b] = jj == j ? inv : rv[b];
        } else if (jj == j) {
          m[a][b] = -(cv[a] * inv);
        } else {
          cpx<T> cur = i == p ? rowj[par][jj] : m[a][b];
          cur.re = fma(-cv[a].re, rv[b].re, cur.re);
          cur.re = fma(cv[a].im, rv[b].im, cur.re);
          cur.im = fma(-cv[a].re, rv[b].im, cur.im);
          cur.im = fma(-cv[a].im, rv[b].re, cur.im);
          m[a][b] = cur;
        }
      }
  }
  // undo the interchanges on the columns: the column j of the eliminated
  // block ends at place[j]
  __syncthreads();
  if (tid == 0) {
    // src[pos] = eliminated column found at result position pos after the
    // column interchanges j <-> perm[j], last first
    for (int c = 0; c < n; ++c) src[c] = c;
    for (int j = n - 1; j >= 0; --j) {
      const int q = perm[j];
      if (q != j) {
        int t = src[j];
        src[j] = src[q];
        src[q] = t;
      }
    }
    for (int c = 0; c < n; ++c) place[src[c]] = c;
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < B; ++a)
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int i = r0 + a, jj = c0 + b;
      if (i >= nP || jj >= nP) continue;
      const int col = jj < n ? place[jj] : jj;
      M[(size_t)i * nP + col] = (i < n && jj < n) ? m[a][b] : mk<T>(T(0), T(0));
    }
}

// Blocked Gauss-Jordan inversion of a line block on the matrix cores.
// Block formation and pivot rule as in k_factor_reg (partial pivoting: for
// column j the largest |re| + |im| among the rows not yet used as a pivot,
// lowest row on ties; columns in natural order), with three differences:
//  * rows are never interchanged: the pivot row p(j) of every column is
//    recorded, and the permutations are applied when the inverse is written
//    out, X[q(a)][p(b)] = M[a][b] with q the inverse of p;
//  * the block lives in MFMA accumulator tiles in registers: tile (rt, ct)
//    holds rows 16 rt.. and complex columns 8 ct.. as 16 real columns
//    [Re | Im]; 8 waves form a 2 x 4 grid, wave (wr, wc) owning row tiles
//    wr, wr + 2, .. and column tiles wc, wc + 4, ..;
//  * columns are eliminated in panels of 16.  A panel's columns are
//    gathered to LDS and eliminated in registers, two threads per row
//    (in-place Gauss-Jordan restricted to the panel, one barrier per
//    pivot).  The panel column pivoted at
//    row p_k then holds T e_{p_k}, T the product of the panel's elementary
//    eliminations; T differs from the identity only in the columns p_k, so
//    T = I + W S^T with W = (eliminated panel) - (unit vectors e_{p_k}),
//    and every other column is updated by one rank-16 complex product,
//      M[:, rest] += W R,   R = rows p_1..p_16 of M[:, rest] before the
//    update, as two real MFMAs per 4-deep slice with R staged as the pairs
//    ([Re r | Im r], [-Im r | Re r]).
// The update order differs from the unblocked kernels, so results agree
// with them to rounding.
// The value of the neighbouring lane of a lane pair (lane ^ 1), by a DPP
// quad permutation (no LDS round trip).
__device__ __forceinline__ float swap_pair_f(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double swap_pair_f(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// The value of lane l (wave-uniform) of v, into a scalar register.
__device__ __forceinline__ float rdlane(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double rdlane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <class T>
__device__ __forceinline__ cpx<T> swap_pair(cpx<T> v) {
  return mk<T>(swap_pair_f(v.re), swap_pair_f(v.im));
}

template <class T, int RA, int CB>
__global__ __launch_bounds__(512) void k_factor_mfma(cpx<T>* X, size_t xstride,
                                                     const cpx<T>* coefT, size_t cstride,
                                                     GeoDev g, int step, int middle, int* flag,
                                                     int nops, int ld) {
  typedef typename MF<T>::v4 v4;
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
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave & 1, wc = wave >> 1;        // 2 x 4 grid of waves
  const int nMt = nP >> 4, nCt = nP >> 3;
  const int jc = lane & 15, cc = jc & 7, part = jc >> 3;
  cpx<T>* PJ = reinterpret_cast<cpx<T>*>(smem_raw);   // [16][nP] panel columns
  T* Wr = reinterpret_cast<T*>(PJ + 16 * nP);         // [16][ld] W, planar
  T* Wi = Wr + 16 * ld;
  T* Rr = Wi + 16 * ld;                               // [16][ld] R, planar
  T* Ri = Rr + 16 * ld;
  int* pivr = reinterpret_cast<int*>(Ri + 16 * ld);   // [nP] column -> pivot row
  int* invp = pivr + nP;                              // [nP] row -> column it pivots
  cpx<T>* rsb = reinterpret_cast<cpx<T>*>(invp + nP + (nP & 1));   // [16] pivot row
  cpx<T>* candrow = rsb + 16;                         // [2][8][16] offered pivot rows
  unsigned* candk = reinterpret_cast<unsigned*>(candrow + 2 * 8 * 16);   // [2][8] their keys
                                                      // (16-byte aligned: offsets are
                                                      // multiples of 16 bytes)
  T* spare = reinterpret_cast<T*>(candk + 16);        // [64 + nP] target of unused stores
  for (int i = tid; i < nP; i += 512) {
    pivr[i] = i;
    invp[i] = i < n ? (1 << 20) : i;                  // padding rows keep their place
  }
  const cpx<T>* Xo = X + (size_t)op * xstride;
  // distinct blocks of X: the output block and the neighbours' inverses do
  // not overlap, so their loads and stores may be reordered
  cpx<T>* __restrict__ Mout = X + (size_t)op * xstride + (size_t)k * nP * nP;
  const cpx<T>* co = coefT + (size_t)op * cstride;
  const cpx<T>* __restrict__ ax = co + (size_t)k * (n + 1);
  const cpx<T>* __restrict__ ay = co + (size_t)K * (n + 1);
  const cpx<T>* __restrict__ dg = co + (size_t)K * (n + 1) + (size_t)(K + 1) * n + (size_t)k * n;
  const cpx<T>* __restrict__ PA = pa >= 0 ? Xo + (size_t)pa * nP * nP : nullptr;
  const cpx<T>* __restrict__ PB = pb2 >= 0 ? Xo + (size_t)pb2 * nP * nP : nullptr;
  // D_k = A_k - B X_{k-1} B (- B X_{k+1} B for the middle line), formed
  // column-major in the output block, then read into the accumulators
  // Four entries per thread per pass, every load of the four issued before
  // the first use (indices clamped into the block, results masked), so the
  // loads of a pass are in flight together instead of one entry's at a time.
  // The operands of the neighbour's term come from a valid block even where
  // it does not exist (PA, PB null); the term is then not applied.
  const cpx<T>* PAs = PA ? PA : Mout;   // (may alias the output: not restrict)
  const cpx<T>* PBs = PB ? PB : Mout;
  const int fa0 = PA ? fa : 0, fb0 = PB ? fb : 0;
  constexpr int FU = 4;
  for (int i0 = tid; i0 < nP * nP; i0 += FU * 512) {
    cpx<T> e0[FU], ar[FU], ac[FU], xa[FU], br[FU], bc[FU], xb[FU];
    int rw[FU], cl[FU];
#pragma unroll
    for (int u = 0; u < FU; ++u) {
      const int idx = min(i0 + u * 512, nP * nP - 1);
      const int col = idx / nP, row = idx - col * nP;
      rw[u] = row;
      cl[u] = col;
      const int r1 = min(row, n - 1), c1 = min(col, n - 1);
      // the diagonal entry or the coupling to the neighbouring node, read
      // field by field from a pointer (a struct copy under a condition
      // would keep the value in private memory)
      const cpx<T>* src = row == col ? dg + r1 : ax + max(r1, c1);
      e0[u] = mk<T>(src->re, src->im);
      ar[u] = ay[(size_t)fa0 * n + r1];
      ac[u] = ay[(size_t)fa0 * n + c1];
      xa[u] = PAs[(size_t)c1 * nP + r1];
      br[u] = ay[(size_t)fb0 * n + r1];
      bc[u] = ay[(size_t)fb0 * n + c1];
      xb[u] = PBs[(size_t)c1 * nP + r1];
    }
#pragma unroll
    for (int u = 0; u < FU; ++u) {
      const int row = rw[u], col = cl[u];
      if (i0 + u * 512 >= nP * nP) continue;
      cpx<T> v = mk<T>(T(0), T(0));
      if (row < n && col < n) {
        const bool nb = row == col || col == row + 1 || row == col + 1;
        if (nb) v = e0[u];
        if (PA) v = v - ar[u] * ac[u] * xa[u];
        if (PB) v = v - br[u] * bc[u] * xb[u];
      }
      Mout[(size_t)col * nP + row] = v;
    }
  }
  __threadfence_block();
  __syncthreads();
  v4 acc[RA][CB];
#pragma unroll
  for (int a = 0; a < RA; ++a)
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      const int rt = wr + 2 * a, ct = wc + 4 * b;
      // unconditional loads (a tile past the block reads entry 0; its
      // accumulators are never written out)
      const unsigned base = (rt < nMt && ct < nCt) ? (unsigned)(8 * ct + cc) * nP + 16 * rt : 0u;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const cpx<T> v = Mout[base + MF<T>::row(lane, i)];
        acc[a][b][i] = part ? v.im : v.re;
      }
    }
  __syncthreads();
  for (int q = 0; 16 * q < n; ++q) {
    const int j0 = 16 * q;
    // the lane index, opaque to the compiler in every iteration: the tiles'
    // row and column offsets are recomputed per panel instead of being
    // hoisted out of the loop into registers the accumulators need
    int ln = lane;
    asm volatile("" : "+v"(ln));
    const int cq = ln & 7, pq = (ln >> 3) & 1, rq = ln & 15;
    // a. the panel's tiles to LDS
#pragma unroll
    for (int a = 0; a < RA; ++a)
#pragma unroll
      for (int b = 0; b < CB; ++b) {
        const int rt = wr + 2 * a, ct = wc + 4 * b;
        if (rt < nMt && (ct >> 1) == q) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int row = 16 * rt + MF<T>::row(ln, i);
            T* dst = reinterpret_cast<T*>(PJ + (size_t)(8 * (ct - 2 * q) + cq) * nP + row);
            dst[pq] = acc[a][b][i];
          }
        }
      }
    lds_barrier();
    // c. the panel's columns are eliminated with threads 2 r and 2 r + 1
    //    holding row r of the panel in registers (8 columns each, r < nP).
    //    Per pivot, one barrier: every wave finds its best candidate row by
    //    cross-lane moves (the key: |re| + |im| with its exponent and leading
    //    15 mantissa bits, then the lowest row) and offers it, key and row,
    //    in LDS; after the barrier every thread takes the best of the eight
    //    offers as the pivot row.  Offers alternate between two buffers by
    //    pivot parity, so a pivot's offers never overwrite ones still read.
    {
      const bool has = tid < 2 * nP;
      const int row = has ? tid >> 1 : 0, h = tid & 1;
      bool used = !has || row >= n || invp[row] < n;
      cpx<T> pr[8];
#pragma unroll
      for (int c2 = 0; c2 < 8; ++c2) pr[c2] = PJ[(size_t)(8 * h + c2) * nP + row];
      int mykk = -1;                                // panel column this row pivots
      int anybad = 0;                               // a zero or NaN pivot in the panel
      const int kend = min(16, n - j0);             // padding columns: no pivot
#pragma unroll 1
      for (int kk = 0; kk < kend; ++kk) {
        const int j = j0 + kk, slot = kk & 1, k7 = kk & 7;
        // column kk of this row, from the thread of the row that holds it
        // (the neighbouring lane: a DPP swap within lane pairs); the entry is
        // picked by a select tree over the bits of kk (depth 3, not a chain
        // of 7 dependent selects)
        const bool b0 = k7 & 1, b1 = (k7 & 2) != 0, b2 = (k7 & 4) != 0;
        const T s01r = b0 ? pr[1].re : pr[0].re, s01i = b0 ? pr[1].im : pr[0].im;
        const T s23r = b0 ? pr[3].re : pr[2].re, s23i = b0 ? pr[3].im : pr[2].im;
        const T s45r = b0 ? pr[5].re : pr[4].re, s45i = b0 ? pr[5].im : pr[4].im;
        const T s67r = b0 ? pr[7].re : pr[6].re, s67i = b0 ? pr[7].im : pr[6].im;
        const T s03r = b1 ? s23r : s01r, s03i = b1 ? s23i : s01i;
        const T s47r = b1 ? s67r : s45r, s47i = b1 ? s67i : s45i;
        const cpx<T> own = mk<T>(b2 ? s47r : s03r, b2 ? s47i : s03i);
        const cpx<T> oth = swap_pair(own);
        const cpx<T> f = h == (kk >> 3) ? own : oth;
        unsigned key = 0u;
        if (!used && h == (kk >> 3)) {
          float m = (float)(fabs(f.re) + fabs(f.im));
          if (!(m == m)) m = 0.f;                   // NaN: the row stays a candidate
          key = ((__float_as_uint(m) >> 8) << 8) | (unsigned)(255 - row);
        }
        const unsigned wk = wave_max_u32(key);
        if (wk && has && row == 255 - (int)(wk & 255u)) {
#pragma unroll
          for (int c2 = 0; c2 < 8; ++c2) candrow[(slot * 8 + wave) * 16 + 8 * h + c2] = pr[c2];
        }
        if (lane == 0) candk[slot * 8 + wave] = wk;
        lds_barrier();
        // the eight offers' keys in two 16-byte reads.  Offered keys are
        // distinct (each carries its row) and the best one is positive (an
        // unused row below n exists for every column j < n; padding rows
        // start out used), so the pivot row p is a row below n and the
        // largest key; the wave that offered it is the one holding row p
        // (rows 32 w .. 32 w + 31, two threads per row), so no search over
        // the offers is needed.
        const uint4* ck = reinterpret_cast<const uint4*>(candk + slot * 8);
        const uint4 k0 = ck[0], k1 = ck[1];
        const unsigned best = max(max(max(k0.x, k0.y), max(k0.z, k0.w)),
                                  max(max(k1.x, k1.y), max(k1.z, k1.w)));
        const int p = 255 - (int)(best & 255u), bw = p >> 5;
        const cpx<T>* prow = candrow + (slot * 8 + bw) * 16;
        // this thread's half of the pivot row and the pivot entry in one
        // batch of reads, ahead of the reciprocal
        cpx<T> ph[8];
#pragma unroll
        for (int c2 = 0; c2 < 8; ++c2) ph[c2] = prow[8 * h + c2];
        const cpx<T> piv = prow[kk];
        anybad |= (piv.re == T(0) && piv.im == T(0)) || !(piv.re == piv.re) ||
                  !(piv.im == piv.im);
        const cpx<T> inv = cinv(piv);
        // complex64: both branches read ph (the pivot row's thread finds
        // its own row there, as it offered it), so its reads stay ahead of
        // the reciprocal instead of sinking into one branch; complex128
        // keeps them after it (holding them across the reciprocal would
        // spill).  The column kk of the other rows is taken by a select,
        // not a branch per column.
        if (has && row == p) {
#pragma unroll
          for (int c2 = 0; c2 < 8; ++c2)
            pr[c2] = 8 * h + c2 == kk ? inv : (sizeof(T) == 4 ? ph[c2] : pr[c2]) * inv;
          used = true;
          mykk = kk;
          if (h == 0) {
            pivr[j] = p;
            invp[p] = j;
          }
        } else {
          const cpx<T> nfi = -(f * inv);
#pragma unroll
          for (int c2 = 0; c2 < 8; ++c2) {
            const cpx<T> r2 = ph[c2] * inv;
            cpx<T> m = pr[c2];
            m.re = fma(-f.re, r2.re, m.re);
            m.re = fma(f.im, r2.im, m.re);
            m.im = fma(-f.re, r2.im, m.im);
            m.im = fma(-f.im, r2.re, m.im);
            const bool isk = 8 * h + c2 == kk;
            pr[c2] = mk<T>(isk ? nfi.re : m.re, isk ? nfi.im : m.im);
          }
        }
      }
      if (anybad && tid == 0) atomicExch(flag, 1);
      // eliminated panel back to LDS; W = panel - unit vectors at the pivot
      // rows; R rows of panel columns without a pivot (padding) are zero
      if (has) {
#pragma unroll
        for (int c2 = 0; c2 < 8; ++c2) {
          const int kc = 8 * h + c2;
          PJ[(size_t)kc * nP + row] = pr[c2];
          Wr[kc * ld + row] = kc == mykk ? pr[c2].re - T(1) : pr[c2].re;
          Wi[kc * ld + row] = pr[c2].im;
        }
      }
      for (int idx = tid; idx < 16 * nP; idx += 512) {
        const int kk = idx / nP, col = idx - kk * nP;
        if (j0 + kk >= n) {
          Rr[kk * ld + col] = T(0);
          Ri[kk * ld + col] = T(0);
        }
      }
    }
    lds_barrier();
    // e. the panel's tiles take the eliminated panel; the pivot rows of the
    //    other tiles, before their update, go to R.  Where each of this
    //    lane's rows goes in R (if its pivot column lies in this panel) is
    //    found once per row tile; every store is then issued, a row without
    //    a place in R writing the lane's own spare slot (spare + lane + the
    //    tile's column offset), so an entry's store is its base plus the
    //    tile's column offset, with no branch or select of its own.
    T* const rbase = (pq ? Ri : Rr) + cq;
#pragma unroll
    for (int a = 0; a < RA; ++a) {
      T* rp[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int j = invp[16 * min(wr + 2 * a, nMt - 1) + MF<T>::row(ln, i)];
        rp[i] = ((j >> 4) == q && j < n) ? rbase + (j & 15) * ld : spare + ln;
      }
#pragma unroll
      for (int b = 0; b < CB; ++b) {
        const int rt = wr + 2 * a, ct = wc + 4 * b;
        if (rt >= nMt || ct >= nCt) continue;
        if ((ct >> 1) == q) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int row = 16 * rt + MF<T>::row(ln, i);
            const T* srcp = reinterpret_cast<const T*>(PJ + (size_t)(8 * (ct - 2 * q) + cq) * nP + row);
            acc[a][b][i] = srcp[pq];
          }
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i) rp[i][8 * ct] = acc[a][b][i];
        }
      }
    }
    lds_barrier();
    // g. M[:, rest] += W R on the matrix cores
#pragma unroll 1
    for (int sl = 0; sl < 4; ++sl) {
      const int kq = 4 * sl + (ln >> 4);
      T a1[RA], a2[RA], b1[CB], b2[CB];
#pragma unroll
      for (int a = 0; a < RA; ++a) {
        const int rt = min(wr + 2 * a, nMt - 1);
        a1[a] = Wr[kq * ld + 16 * rt + rq];
        a2[a] = Wi[kq * ld + 16 * rt + rq];
      }
      // every MFMA is issued (a conditional one would keep a copy of its
      // accumulator for the select): the panel's own tiles and tiles past
      // the block get a zero B operand, which leaves them unchanged
#pragma unroll
      for (int b = 0; b < CB; ++b) {
        const int ct = wc + 4 * b;
        const int ctc = min(ct, nCt - 1);
        const bool upd = ct < nCt && (ct >> 1) != q;
        const T rr = Rr[kq * ld + 8 * ctc + cq], ri = Ri[kq * ld + 8 * ctc + cq];
        b1[b] = upd ? (pq ? ri : rr) : T(0);
        b2[b] = upd ? (pq ? rr : -ri) : T(0);
      }
#pragma unroll
      for (int a = 0; a < RA; ++a)
#pragma unroll
        for (int b = 0; b < CB; ++b) {
          acc[a][b] = MF<T>::mfma(a1[a], b1[b], acc[a][b]);
          acc[a][b] = MF<T>::mfma(a2[a], b2[b], acc[a][b]);
        }
      // one slice's operands at a time (registers)
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  __syncthreads();
  // write out X[q(a)][p(b)] = M[a][b] column-major; padding rows and columns
  // (which keep their places) are zero
#pragma unroll
  for (int a = 0; a < RA; ++a)
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      const int rt = wr + 2 * a, ct = wc + 4 * b;
      if (rt >= nMt || ct >= nCt) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * rt + MF<T>::row(lane, i), col = 8 * ct + cc;
        const bool in = row < n && col < n;
        // (clamped: every index is in range by construction)
        const int r = min(max(in ? invp[row] : row, 0), nP - 1);
        const int cl = min(max(in ? pivr[col] : col, 0), nP - 1);
        T* dst = reinterpret_cast<T*>(Mout + (size_t)cl * nP + r);
        dst[part] = in ? acc[a][b][i] : T(0);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
}

template <class T, int RA, int CB>
static hipError_t launch_factor_mfma_t(hdsw_ctx* c, int step, int middle) {
  const Geometry& g = c->g;
  int ld = g.nP;
  while (ld % 64 != 16 && ld % 64 != 48) ld += 16;   // conflict-free operand reads
  const size_t lds = (size_t)16 * g.nP * sizeof(cpx<T>) + (size_t)4 * 16 * ld * sizeof(T) +
                     (size_t)(2 * g.nP + 2) * sizeof(int) + (16 + 256) * sizeof(cpx<T>) +
                     16 * sizeof(unsigned) + (size_t)(64 + g.nP) * sizeof(T);
  const size_t xs = (size_t)g.K * g.nP * g.nP;
  hipLaunchKernelGGL((k_factor_mfma<T, RA, CB>), dim3(c->nops, 2), dim3(512), lds, c->stream,
                     (cpx<T>*)c->d_X, xs, (const cpx<T>*)c->d_coefT, c->coef_stride, c->gd,
                     step, middle, c->d_flag, c->nops, ld);
  return hipGetLastError();
}

// Line blocks up to 160 (complex64) or 96 (complex128) nodes: the blocked
// inversion on the matrix cores (larger tile sets would not fit the
// registers of two waves per SIMD); larger ones on the unblocked kernels.
template <class T>
static bool factor_on_mfma(hdsw_ctx* c, int step, int middle, hipError_t* e) {
  const int nP = c->g.nP;
  if (!c->factor_mfma) return false;
  if (nP <= 64) { *e = launch_factor_mfma_t<T, 2, 2>(c, step, middle); return true; }
  if (nP <= 96) { *e = launch_factor_mfma_t<T, 3, 3>(c, step, middle); return true; }
  if constexpr (sizeof(T) == 4) {
    if (nP <= 128) { *e = launch_factor_mfma_t<T, 4, 4>(c, step, middle); return true; }
    if (nP <= 160) { *e = launch_factor_mfma_t<T, 5, 5>(c, step, middle); return true; }
  }
  return false;
}

template <class T>
hipError_t launch_factor_step(hdsw_ctx* c, int step, int middle) {
  const Geometry& g = c->g;
  {
    hipError_t e = hipSuccess;
    if (factor_on_mfma<T>(c, step, middle, &e)) return e;
  }
  const size_t xs = (size_t)g.K * g.nP * g.nP;
#define HDSW_FREG(B)                                                                        \
  if (g.nP <= 32 * (B)) {                                                                   \
    hipLaunchKernelGGL((k_factor_reg<T, B>), dim3(c->nops, 2), dim3(1024), 0, c->stream,    \
                       (cpx<T>*)c->d_X, xs, (const cpx<T>*)c->d_coefT, c->coef_stride, c->gd, \
                       step, middle, c->d_flag, c->nops);                                   \
    return hipGetLastError();                                                               \
  }
  HDSW_FREG(2)
  HDSW_FREG(3)
  // complex128 sub-blocks of 4 x 4 and more exceed the registers of a
  // 1024-thread workgroup: those blocks stay on k_factor_step below
  if constexpr (sizeof(T) == 4) {
    HDSW_FREG(4)
    HDSW_FREG(5)
  }
#undef HDSW_FREG
  int bs = 1024;
  size_t lds = 2 * g.n * sizeof(cpx<T>) + ((g.n + 3) & ~3) * sizeof(int) +
               bs * (sizeof(T) + sizeof(int));
  size_t xstride = (size_t)g.K * g.nP * g.nP;
  hipLaunchKernelGGL(k_factor_step<T>, dim3(c->nops, 2), dim3(bs), lds, c->stream,
                     (cpx<T>*)c->d_X, xstride, (const cpx<T>*)c->d_coefT, c->coef_stride,
                     c->gd, step, middle, c->d_flag, c->nops);
  return hipGetLastError();
}

// ------------------------------------------------------------ sweep step
// One step of a sweep for the subdomains of one anti-diagonal, one launch
// (2D; the 3D step below is a GEMM between two small kernels):
//   1. trace -> source: g = [S_r, chi_r] v~ from the pairs in the step's
//      sweep slot (g[layer 1] = c pair[layer 0], g[layer 0] = -c pair[layer 1],
//      c = the face coefficient of the receiver), formed while the B operand
//      is staged in LDS;
//   2. the subdomain solve restricted to the interface layers,
//      out = T g (+ y in the sweep that carries the sources f_ij);
//   3. in the epilogue, the routing: each output pair goes into slot l' of
//      the neighbour across its face, taken as the limit from the receiver's
//      side (the layer on the sender's side loses the pair the sender
//      received there).
// The sources of the final owned-node solve are summed from the slots after
// the sweeps (k_source_sum).  Only faces that can hold a trace in this sweep
// enter the sum, and only faces whose traces have a destination are
// computed.  One workgroup of 8 waves per (RW 16-row output tiles, 16
// columns, subdomain); the waves split the sum into 8/RW parts that are
// added in a fixed order.
struct FaceSet {
  int n;                 // active faces
  int face[6];           // face ids (0:-x, 1:+x, 2:-y, 3:+y, 4:-z, 5:+z)
  int start[6];          // first row (or sum index) of the face
  int lq[6];             // destination sweep per face (outputs only)
};
// Subdomains of one launch of a step and their operators, as a kernel
// argument: a workgroup reads its own entry with a scalar load, so every
// address of the step is known at the start instead of after a chain of
// dependent memory loads.  Longer anti-diagonals take several launches (the
// 16 x 16 partitions of the benchmarks take one per step; 32 x 32 ones, in
// the tests, two on their longer steps).
constexpr int kStepListMax = 16;
// One or two steps of one launch (steps that no slot dependence orders, in
// different sweeps): each a group with its own faces, chunking and
// subdomains sub[first .. first + n)
constexpr int kStepGroups = 2;
struct StepGroup {
  int L, nout, add_y, LMAX, nsub_chunks, first, n;
  FaceSet fin, fout;
};
struct StepLaunch {
  int ng;
  StepGroup g[kStepGroups];
  int sub[kStepGroups * kStepListMax], op[kStepGroups * kStepListMax];
};
__device__ inline int fs_find(const FaceSet& fs, int idx) {
  // the last active face that starts at or before idx (starts increase)
  int q = 0;
#pragma unroll
  for (int j = 1; j < 6; ++j) q = (j < fs.n && idx >= fs.start[j]) ? j : q;
  return q;
}

// Epilogue of the sweep step for one output element: where its value goes.
struct StepOut {
  long long dst;     // slot element to add to (-1: none)
  long long yo;      // y element (source-driven part), -1 if not added
  long long ino;     // incoming pair element to subtract, -1 if none
};
__device__ inline StepOut step_out(const GeoDev& g, const FaceSet& fout, int s, int orow,
                                   int col, int C, int L, size_t slot_stride, int add_y) {
  StepOut o{-1, -1, -1};
  const int NI = g.NI;
  int q = fs_find(fout, orow);
  int f = pick(fout.face, q);
  int lq = pick(fout.lq, q);
  int len = pick(g.side_len, f), so = pick(g.side_off, f);
  int rq = orow - pick(fout.start, q);
  int lay = rq / len, t = rq - lay * len;
  int d = so + rq;
  int c0 = s % g.P[0], c1 = (s / g.P[0]) % g.P[1], c2 = s / (g.P[0] * g.P[1]);
  const int axis = f >> 1, step = (f & 1) ? 1 : -1;
  if (axis == 0) c0 += step;
  else if (axis == 1) c1 += step;
  else c2 += step;
  if (c0 < 0 || c0 >= g.P[0] || c1 < 0 || c1 >= g.P[1] || c2 < 0 || c2 >= g.P[2]) return o;
  int recv = c0 + g.P[0] * (c1 + g.P[1] * c2);
  const int sofo = pick(g.side_off, f ^ 1);
  size_t rb = (size_t)lq * slot_stride + ((size_t)recv * C + col) * NI;
  if (add_y) o.yo = (long long)(((size_t)s * C + col) * NI + d);
  if (lay == 1) {
    o.dst = (long long)(rb + sofo + t);
  } else {
    o.dst = (long long)(rb + sofo + len + t);
    o.ino = (long long)((size_t)L * slot_stride + ((size_t)s * C + col) * NI + so + t);
  }
  return o;
}

// Longest face chunk of the sum staged in LDS at once (a multiple of 64):
// 2 tiles x lcap rows of kSweepRS operand pairs, 136 KB for eight-wave
// workgroups (one per CU), at most 80 KB for four-wave workgroups (two per
// CU).  Rows hold 16 pairs and one of padding, so that the staging stores
// (one row per lane) and the operand reads (four rows per wave) are free of
// bank conflicts.
template <class T, int NWV>
__host__ __device__ constexpr int sweep_lcap() {
  return NWV == 8 ? (sizeof(T) == 4 ? 512 : 256) : (sizeof(T) == 4 ? 256 : 128);
}
constexpr int kSweepRS = 17;
// Two-tile workgroups per 16-column group of a step above which the
// four-tile form is used (the 1024^2 workload's largest steps, 8 subdomains
// of 40 row-tile workgroups, stay at two tiles)
constexpr int kSweepRows = 320;

// The sum runs face by face over the active input faces.  For each face the
// B operand is staged in LDS already split for the two real MFMAs of the
// complex product: for column c < 8 of a tile, lane column jc = c carries
// (Re v, -Im v) and jc = c + 8 carries (Im v, Re v), so every lane reads one
// pair per 4-deep slice.  Four accumulators (two tiles x real/imaginary part
// of X) keep dependent MFMAs apart; the T columns of a face are contiguous,
// so its operand is walked by pointer increments.
template <class T, int KB, int RW, int NWV>
__global__ __launch_bounds__(NWV * 64) void k_sweep_step(
    const cpx<T>* __restrict__ Tm, const cpx<T>* __restrict__ cface, cpx<T>* slots,
    const cpx<T>* __restrict__ ybuf, StepLaunch sl, int C, GeoDev g) {
  typedef typename MF<T>::v4 v4;
  // RW 16-row tiles per workgroup; the NWV waves split the sum in KH parts
  static_assert(NWV % RW == 0 && 8 % NWV == 0, "waves and row tiles");
  constexpr int NT = NWV * 64;
  constexpr int KH = NWV / RW, RWS = 16 * RW, NQ = (RWS * 16 + NT - 1) / NT;
  extern __shared__ unsigned char smem_raw[];
  cpx<T>* bp = reinterpret_cast<cpx<T>*>(smem_raw);        // [2 tiles][LMAX][kSweepRS] pairs
  const int NI = g.NI;
  // XCD-aware mapping: workgroups are dispatched round-robin over the 8
  // XCDs (id % 8), each with its own L2.  The (row tile, subdomain) pairs
  // of the launch, group by group and row tile major, are cut into 8
  // contiguous runs of equal length, one per XCD: every XCD gets the same
  // number of tiles, and the subdomains of one row tile (which read the
  // same slice of T when they share an operator) sit on at most two XCDs.
  const int np0 = (sl.g[0].nout + RWS - 1) / RWS * sl.g[0].n;
  const int np = np0 + (sl.ng > 1 ? (sl.g[1].nout + RWS - 1) / RWS * sl.g[1].n : 0);
  const int xcd = blockIdx.x & 7, loc = blockIdx.x >> 3;
  const int pair = xcd * np / 8 + loc;
  if (pair >= (xcd + 1) * np / 8) return;
  const int gi = pair >= np0 ? 1 : 0;
  const StepGroup& G = sl.g[gi];
  const int L = G.L, nout = G.nout, add_y = G.add_y, LMAX = G.LMAX;
  const int nsub_chunks = G.nsub_chunks, cnt = G.n;
  const FaceSet& fin = G.fin;
  const FaceSet& fout = G.fout;
  const int lp = pair - (gi ? np0 : 0);
  const int rtile = lp / cnt, si = lp - rtile * cnt;
  const int s = sl.sub[G.first + si], op = sl.op[G.first + si];
  const int cg = blockIdx.y;                               // 16-column group
  const int c0 = cg * 16;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int rw = wave % RW, kh = wave / RW;                // row tile, part of the sum
  const cpx<T>* Top = Tm + (size_t)op * NI * NI;
  const size_t slot_stride = (size_t)g.nsub * C * NI;
  const cpx<T>* recv = slots + (size_t)L * slot_stride + (size_t)s * C * NI;
  const cpx<T>* cf_op = cface + (size_t)op * (NI / 2);
  const int jc = lane & 15, kk = lane >> 4, rr = lane & 15;
  // The B operand, g = [S_r, chi_r] v~ of the pairs received in slot L
  // (g[layer 1] = c pair[layer 0], g[layer 0] = -c pair[layer 1], c the
  // receiver's face coefficient), is formed while it is staged in LDS, one
  // face chunk at a time.  Each thread holds its share of a chunk in
  // registers: the loads of the next chunk are issued before the current
  // chunk's sum.  Wave w stages columns w + NWV j (j < CPW) of both
  // 8-column tiles, lane l the sum indices k = l + 64 i: the loads of a
  // wave read 64 consecutive sources of one column.  SK blocks of 64
  // indices cover the longest chunk.
  constexpr int SK = sweep_lcap<T, NWV>() / 64, CPW = 8 / NWV;
  cpx<T> sv[2 * CPW * SK], cv[SK];
  const int nqc = fin.n * nsub_chunks;
  auto chunk_len = [&](int q) {                // sum length of chunk q (0: none)
    const int qf = q / nsub_chunks, sc = q - qf * nsub_chunks;
    return max(0, min(LMAX, 2 * pick(g.side_len, pick(fin.face, qf)) - sc * LMAX));
  };
  // staged column j of tile t: c0 + 8 t + wave + NWV j
  bool sok[2 * CPW];
  const cpx<T>* rcol[2 * CPW];
#pragma unroll
  for (int j = 0; j < 2 * CPW; ++j) {
    const int col = c0 + 8 * (j & 1) + wave + NWV * (j >> 1);
    sok[j] = col < C;
    rcol[j] = recv + (size_t)(sok[j] ? col : 0) * NI;
  }
  cpx<T>* lds_st = bp + (size_t)lane * kSweepRS + wave;
  auto stage_load = [&](int q) {
    const int qf = q / nsub_chunks, sc = q - qf * nsub_chunks;
    const int f = pick(fin.face, qf);
    const int len = pick(g.side_len, f), so = pick(g.side_off, f);
    const int kn = chunk_len(q), kb = sc * LMAX;
#pragma unroll
    for (int i = 0; i < SK; ++i) {
      // unconditional loads (indices past the chunk re-read its first
      // source and are masked at the store), so they stay in flight together
      const int k = lane + 64 * i;
      const int kf = kb + (k < kn ? k : 0);    // index within the face's 2 len sources
      const bool lay1 = kf >= len;
      const int partner = so + kf + (lay1 ? -len : len);   // the pair's other layer
#pragma unroll
      for (int j = 0; j < 2 * CPW; ++j) sv[2 * CPW * i + j] = rcol[j][partner];
      cv[i] = cf_op[so / 2 + kf - (lay1 ? len : 0)];
    }
  };
  auto stage_store = [&](int q) {
    const int qf = q / nsub_chunks, sc = q - qf * nsub_chunks;
    const int len = pick(g.side_len, pick(fin.face, qf));
    const int kn = chunk_len(q), k4 = (kn + 3) & ~3, kb = sc * LMAX;
#pragma unroll
    for (int i = 0; i < SK; ++i) {
      const int k = lane + 64 * i;
      if (k < k4) {
#pragma unroll
        for (int j = 0; j < 2 * CPW; ++j) {
          const int t = j & 1;
          cpx<T> gv = cv[i] * sv[2 * CPW * i + j];
          if (kb + k < len) gv = -gv;          // layer 0 receives -c pair[layer 1]
          if (!(k < kn && sok[j])) gv = mk<T>(T(0), T(0));
          cpx<T>* row = lds_st + ((size_t)t * LMAX + 64 * i) * kSweepRS + NWV * (j >> 1);
          row[0] = mk<T>(gv.re, -gv.im);
          row[8] = mk<T>(gv.im, gv.re);
        }
      }
    }
  };
  // output dof of this lane's A row
  const int row = rtile * RWS + rw * 16 + rr;
  int dout = -1;
  if (row < nout) {
    int q = fs_find(fout, row);
    dout = pick(g.side_off, pick(fout.face, q)) + (row - pick(fout.start, q));
  }
  const unsigned arow = dout >= 0 ? dout : 0;
  // this wave's share of chunk q: T columns, sum length, slice range
  struct ChunkGeo {
    const cpx<T>* abase;                       // uniform base, 32-bit lane offsets
    int kn, nks, ksb, kse;
  };
  auto cgeo = [&](int q) {
    ChunkGeo c;
    const int qf = q / nsub_chunks, sc = q - qf * nsub_chunks;
    c.kn = chunk_len(q);                       // sum length of the chunk
    c.nks = (c.kn + 3) >> 2;                   // 4-deep slices, last one padded
    const int hh = (c.nks + KH - 1) / KH;
    c.ksb = kh * hh;
    c.kse = min(c.nks, c.ksb + hh);
    c.abase = Top + (size_t)(pick(g.side_off, pick(fin.face, qf)) + sc * LMAX) * NI;
    return c;
  };
  // unconditional loads: a slice past this wave's range is never used, a
  // sum index past the chunk meets a zero operand in LDS, and a row past
  // nout is not written out
  auto load = [&](cpx<T>(&a)[KB], const ChunkGeo& c, int ks0) {
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const int ks = max(0, min(ks0 + u, c.kse - 1));
      a[u] = c.abase[(unsigned)min(4 * ks + kk, c.kn - 1) * (unsigned)NI + arow];
    }
  };
  const cpx<T>* b0 = bp + (size_t)kk * kSweepRS + jc;
  const cpx<T>* b1 = bp + (size_t)(LMAX + kk) * kSweepRS + jc;
  v4 aR0 = v4{T(0), T(0), T(0), T(0)}, aI0 = aR0, aR1 = aR0, aI1 = aR0;
  // each slice's B operand is read from LDS next to its MFMAs (a batch's
  // worth read ahead held 2 KB complex registers, which with the epilogue
  // operands cost the second workgroup per CU)
  auto compute = [&](const cpx<T>(&a)[KB], const ChunkGeo& c, int ks0) {
    if (ks0 + KB <= c.kse) {
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        const cpx<T> p0 = b0[(size_t)(ks0 + u) * 4 * kSweepRS];
        const cpx<T> p1 = b1[(size_t)(ks0 + u) * 4 * kSweepRS];
        aR0 = MF<T>::mfma(a[u].re, p0.re, aR0);
        aR1 = MF<T>::mfma(a[u].re, p1.re, aR1);
        aI0 = MF<T>::mfma(a[u].im, p0.im, aI0);
        aI1 = MF<T>::mfma(a[u].im, p1.im, aI1);
      }
    } else {
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        if (ks0 + u < c.kse) {
          const cpx<T> p0 = b0[(size_t)(ks0 + u) * 4 * kSweepRS];
          const cpx<T> p1 = b1[(size_t)(ks0 + u) * 4 * kSweepRS];
          aR0 = MF<T>::mfma(a[u].re, p0.re, aR0);
          aR1 = MF<T>::mfma(a[u].re, p1.re, aR1);
          aI0 = MF<T>::mfma(a[u].im, p0.im, aI0);
          aI1 = MF<T>::mfma(a[u].im, p1.im, aI1);
        }
      }
    }
  };
  // The A operand (rows of T) streams through two register batches, one
  // batch ahead across chunk boundaries: the first batch is requested
  // before anything else, and the last prefetch of a chunk fetches the
  // first batch of the next one.
  cpx<T> a0[KB], a1[KB];
  int qc = 0;
  while (qc < nqc && chunk_len(qc) == 0) ++qc;
  ChunkGeo cur{};
  if (qc < nqc) {
    cur = cgeo(qc);
    load(a0, cur, cur.ksb);
    stage_load(qc);
  }
  // The epilogue operands do not depend on the product.  They are fetched
  // once the first chunk is staged (after the loop when there is none), so
  // that a workgroup's first requests are only those its first chunk waits
  // for: at the start of a launch every workgroup asks at once, and the
  // epilogue operands in the same burst held the first chunk back about
  // 5 us.  No workgroup of the launch writes what another reads, so when
  // they are read does not matter.  Only the destination index stays live.
  long long dsti[NQ];
  cpx<T> ey[NQ], ein[NQ], edst[NQ];
  auto epi_fetch = [&]() {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      int idx = tid + q * NT;
      int col = idx / RWS, r = idx % RWS;
      int orow = rtile * RWS + r;
      StepOut o{-1, -1, -1};
      if (idx < RWS * 16 && orow < nout && c0 + col < C)
        o = step_out(g, fout, s, orow, c0 + col, C, L, slot_stride, add_y);
      dsti[q] = o.dst;
      ey[q] = mk<T>(T(0), T(0));
      ein[q] = ey[q];
      edst[q] = ey[q];
      if (o.yo >= 0) ey[q] = ybuf[o.yo];
      if (o.ino >= 0) ein[q] = slots[o.ino];
      if (o.dst >= 0) edst[q] = slots[o.dst];
    }
  };
  bool fetched = false;
  while (qc < nqc) {
    int qn = qc + 1;
    while (qn < nqc && chunk_len(qn) == 0) ++qn;
    const ChunkGeo nxt = qn < nqc ? cgeo(qn) : cur;
    lds_barrier();
    stage_store(qc);
    lds_barrier();
    if (qn < nqc) stage_load(qn);              // in flight during this chunk's sum
    if (!fetched) {
      epi_fetch();
      fetched = true;
    }
    if (cur.ksb >= cur.kse) load(a0, nxt, nxt.ksb);   // no slices here: move on
    for (int ks0 = cur.ksb; ks0 < cur.kse; ks0 += 2 * KB) {
      load(a1, cur, ks0 + KB);
      compute(a0, cur, ks0);
      if (ks0 + 2 * KB < cur.kse) load(a0, cur, ks0 + 2 * KB);
      else load(a0, nxt, nxt.ksb);
      if (ks0 + KB < cur.kse) compute(a1, cur, ks0 + KB);
    }
    qc = qn;
    cur = nxt;
  }
  if (!fetched) epi_fetch();
  lds_barrier();
  // add the KH parts in a fixed order and stage the RWS x 16 tile:
  // part p of the sum at st + p * (2 * 16 * RWS) floats, p = 0 the final tile
  T* st = reinterpret_cast<T*>(bp);
  const int cc = jc & 7, part = jc >> 3;
  if (kh > 0) {
    T* pp = st + (size_t)kh * 2 * 16 * RWS;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int r = rw * 16 + MF<T>::row(lane, i);
      pp[2 * (cc * RWS + r) + part] = aR0[i] + aI0[i];
      pp[2 * ((cc + 8) * RWS + r) + part] = aR1[i] + aI1[i];
    }
  }
  lds_barrier();
  if (kh == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int r = rw * 16 + MF<T>::row(lane, i);
      int i0 = 2 * (cc * RWS + r) + part, i1 = 2 * ((cc + 8) * RWS + r) + part;
      T v0 = aR0[i] + aI0[i], v1 = aR1[i] + aI1[i];
#pragma unroll
      for (int p = 1; p < KH; ++p) {
        v0 += st[(size_t)p * 2 * 16 * RWS + i0];
        v1 += st[(size_t)p * 2 * 16 * RWS + i1];
      }
      st[i0] = v0;
      st[i1] = v1;
    }
  }
  lds_barrier();
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (dsti[q] < 0) continue;
    int idx = tid + q * NT;
    int col = idx / RWS, r = idx % RWS;
    cpx<T> v = bp[col * RWS + r] + ey[q];
    slots[dsti[q]] = edst[q] + (v - ein[q]);
  }
}

// Plane-block (3D) sweep step as three launches: the trace sources in plain
// column layout gplain[bi][col][k] (k over the active input faces, each
// face padded to whole tiles), one grouped GEMM out = T[out rows, in
// columns] g per distinct operator on the tiled T (the row-tile and k-tile
// maps select the active faces), and the routing epilogue below.
template <class T>
__global__ void k_trace_src_plain(const cpx<T>* __restrict__ cface,
                                  const cpx<T>* __restrict__ slots, cpx<T>* gplain,
                                  const int* __restrict__ op_of, const int* __restrict__ subs,
                                  int cnt, int L, int C, FaceSet fin, int nin, GeoDev g) {
  const int NI = g.NI;
  const size_t slot_stride = (size_t)g.nsub * C * NI;
  long long tot = (long long)cnt * C * nin;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    int k = (int)(idx % nin);
    long long bc = idx / nin;
    int col = (int)(bc % C), bi = (int)(bc / C);
    int s = subs[bi];
    int q = fs_find(fin, k);
    int f = pick(fin.face, q);
    int len = pick(g.side_len, f), so = pick(g.side_off, f);
    int rq = k - pick(fin.start, q);
    if (rq >= 2 * len) {             // padding of the face to whole tiles
      gplain[idx] = mk<T>(T(0), T(0));
      continue;
    }
    int lay = rq / len, t = rq - lay * len;
    int partner = so + (1 - lay) * len + t;
    const cpx<T>* sl = slots + (size_t)L * slot_stride + ((size_t)s * C + col) * NI;
    cpx<T> gv = cface[(size_t)op_of[s] * (NI / 2) + so / 2 + t] * sl[partner];
    if (lay == 0) gv = -gv;
    gplain[idx] = gv;
  }
}

template <class T>
__global__ void k_step_scatter(const cpx<T>* __restrict__ out, cpx<T>* slots,
                               const cpx<T>* __restrict__ ybuf, const int* __restrict__ subs,
                               int cnt, int L, int C, FaceSet fout, int nout, int add_y,
                               GeoDev g) {
  const size_t slot_stride = (size_t)g.nsub * C * g.NI;
  long long tot = (long long)cnt * C * nout;
  const cpx<T> z = mk<T>(T(0), T(0));
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    int r = (int)(idx % nout);
    long long bc = idx / nout;
    int col = (int)(bc % C), bi = (int)(bc / C);
    StepOut eo = step_out(g, fout, subs[bi], r, col, C, L, slot_stride, add_y);
    if (eo.dst < 0) continue;
    cpx<T> v = out[idx];
    if (eo.yo >= 0) v = v + ybuf[eo.yo];
    cpx<T> in = z;
    if (eo.ino >= 0) in = slots[eo.ino];
    slots[eo.dst] = slots[eo.dst] + (v - in);
  }
}

// face coefficients c(face, t) of every distinct operator, contiguous per
// face: [op][side_off[f] / 2 + t]
template <class T>
__global__ void k_face_coef(cpx<T>* cface, const cpx<T>* coefT, size_t cstride, GeoDev g,
                            int nops) {
  const int half = g.NI / 2;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < nops * half;
       idx += gridDim.x * blockDim.x) {
    int op = idx / half, i = idx - op * half;
    int f = 0;
#pragma unroll
    for (int j = 1; j < 6; ++j) f = (j < 2 * g.dim && i >= g.side_off[j] / 2) ? j : f;
    int t = i - pick(g.side_off, f) / 2;
    const cpx<T>* co = coefT + (size_t)op * cstride;
    const int axis = f >> 1;
    // half-point index across the face, between layer 0 and layer 1
    const int q = (f & 1) ? g.W + pick(g.na, axis) : g.W;
    cpx<T> v;
    if (g.dim == 2) {
      if (f < 2) v = co[(size_t)t * (g.n + 1) + q];
      else v = co[(size_t)g.K * (g.n + 1) + (size_t)q * g.n + t];
    } else {
      // faces: x t = z n_y + y, y t = z n_x + x, z t = y n_x + x
      const int nx = g.ne[0], ny = g.ne[1], nz = g.ne[2];
      const size_t o_ay = (size_t)nz * ny * (nx + 1);
      const size_t o_az = o_ay + (size_t)nz * (ny + 1) * nx;
      if (axis == 0) {
        v = co[(size_t)t * (nx + 1) + q];
      } else if (axis == 1) {
        int z = t / nx, x = t - z * nx;
        v = co[o_ay + ((size_t)z * (ny + 1) + q) * nx + x];
      } else {
        v = co[o_az + (size_t)q * ny * nx + t];
      }
    }
    cface[idx] = v;
  }
}
template <class T>
hipError_t launch_face_coef(hdsw_ctx* c) {
  int tot = c->nops * c->g.NI / 2;
  hipLaunchKernelGGL(k_face_coef<T>, dim3((tot + 255) / 256), dim3(256), 0, c->stream,
                     (cpx<T>*)c->d_cface, (const cpx<T>*)c->d_coefT, c->coef_stride, c->gd,
                     c->nops);
  return hipGetLastError();
}

// Active faces of sweep L: inputs are the faces that can hold a received
// trace, outputs the faces whose trace some sweep uses (Rules 2.4/2.5,
// 4.1/4.2); returns the output rows, nin the input sum length.
static int step_faces(const hdsw_ctx* c, int L, FaceSet& fin, FaceSet& fout, int* nin) {
  const Geometry& g = c->g;
  fin = FaceSet{};
  fout = FaceSet{};
  int ni = 0, nout = 0;
  for (int f = 0; f < 2 * g.dim; ++f) {
    if (c->sch.in_active[L * 6 + f]) {
      fin.face[fin.n] = f;
      fin.start[fin.n] = ni;
      fin.lq[fin.n] = -1;
      fin.n++;
      ni += 2 * g.side_len[f];
    }
    int lq = c->sch.lprime[L * 6 + f];
    if (lq >= 0) {
      fout.face[fout.n] = f;
      fout.start[fout.n] = nout;
      fout.lq[fout.n] = lq;
      fout.n++;
      nout += 2 * g.side_len[f];
    }
  }
  *nin = ni;
  return nout;
}

template <class T>
static hipError_t launch_sweep_step3(hdsw_ctx* c, int L, int st, int off, int cnt, int C) {
  const Geometry& g = c->g;
  FaceSet fin{}, fout{};
  int nin = 0;
  const int nout = step_faces(c, L, fin, fout, &nin);
  if (nout == 0) return hipSuccess;
  const int* subs = c->d_step_subs + off;
  // input faces in the padded k space of the tiled T
  const int tk = c->t_tk;
  FaceSet finp = fin;
  int ninp = 0;
  for (int q = 0; q < fin.n && nin > 0; ++q) {
    finp.start[q] = ninp;
    ninp += (2 * g.side_len[fin.face[q]] + tk - 1) / tk * tk;
  }
  if (nin > 0) {
    long long tot = (long long)cnt * C * ninp;
    int blocks = (int)std::min<long long>((tot + 255) / 256, 1 << 20);
    hipLaunchKernelGGL(k_trace_src_plain<T>, dim3(blocks), dim3(256), 0, c->stream,
                       (const cpx<T>*)c->d_cface, (const cpx<T>*)c->d_slots,
                       (cpx<T>*)c->d_g, c->d_op_of_sub, subs, cnt, L, C,
                       finp, ninp, c->gd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int sidx = L * c->sch.nsteps + st;
  GemmArgs a{};
  a.M = c->tm_mpad[L];
  a.N = 0;
  a.Kd = ninp;
  a.A = c->d_T;
  a.lda = 0;
  a.sAz = (long long)c->t_nrt * 64 * (long long)c->t_nkt * tk;
  a.a_rt = c->d_tmap + c->tm_rt_off[L];
  a.a_kt = c->d_tmap + c->tm_kt_off[L];
  a.a_tile_ld = c->t_nkt;
  a.c_row = c->d_tmap + c->tm_row_off[L];
  a.B = c->d_g;
  a.ldb = ninp;
  a.sb = (long long)C * ninp;
  a.sBz = 0;
  a.C = c->d_out;
  a.ldc = nout;
  a.sc = (long long)C * nout;
  a.sCz = 0;
  a.cpb = C;
  a.ids = c->d_sg_ids;
  a.grp_op = c->d_sg_op + c->sg_first[sidx];
  a.grp_off = c->d_sg_off + c->sg_first[sidx];
  a.grp_cnt = c->d_sg_cnt + c->sg_first[sidx];
  a.neg = 0;
  a.beta = 0;
  if (nin == 0) {
    // nothing received yet: the outputs are the source-driven part alone
    hipError_t e = launch_zero(c, c->d_out, (size_t)cnt * C * nout * sizeof(cpx<T>));
    if (e != hipSuccess) return e;
  } else {
    if (tk != gemm_bk<T>()) return hipErrorInvalidValue;
    a.no_skinny = c->tune.gemm_skinny == 2;
    // fewer row tiles than the CUs hold workgroups (four each): split the
    // sum, from the step's shape only (rows and operator groups); the
    // streaming kernel of narrow products keeps one part
    const int maxcols = c->sg_maxcnt[sidx] * C;
    const bool skinny = maxcols <= 8 && !a.no_skinny;
    const long long rtiles = (long long)(a.M / 64) * c->sg_n[sidx];
    int ks = skinny ? 1 : (int)std::min<long long>(4, std::max<long long>(1, (1024 + rtiles - 1) / rtiles));
    while (ks > 1 && (size_t)ks * c->sg_n[sidx] * maxcols * a.M * sizeof(cpx<T>) > c->gpart_bytes)
      --ks;
    a.ksplit = ks;
    a.part = c->d_gpart;
    hipError_t e = gemm<T>(c->stream, a, maxcols, c->sg_n[sidx]);
    if (e != hipSuccess) return e;
  }
  long long tot = (long long)cnt * C * nout;
  int blocks = (int)std::min<long long>((tot + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_step_scatter<T>, dim3(blocks), dim3(256), 0, c->stream,
                     (const cpx<T>*)c->d_out, (cpx<T>*)c->d_slots, (const cpx<T>*)c->d_y, subs,
                     cnt, L, C, fout, nout, L == 0 ? 1 : 0, c->gd);
  return hipGetLastError();
}

// Sweep steps sidx[0 .. nst) (indices L * nsteps + st) that no slot
// dependence orders: in 2D one launch of k_sweep_step takes up to two of
// them (or two groups of kStepListMax subdomains of one step); 3D steps run
// one after another.
template <class T>
hipError_t launch_sweep_steps(hdsw_ctx* c, const int* sidx, int nst, int C) {
  const Geometry& g = c->g;
  const Schedule& sc = c->sch;
  if (g.dim == 3) {
    for (int i = 0; i < nst; ++i) {
      const int cnt = sc.step_cnt[sidx[i]];
      if (cnt == 0) continue;
      hipError_t e = launch_sweep_step3<T>(c, sidx[i] / sc.nsteps, sidx[i] % sc.nsteps,
                                           sc.step_off[sidx[i]], cnt, C);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const int Cp = (C + 15) / 16 * 16;
  // the steps' subdomains in groups of at most kStepListMax, each with the
  // longest input face (its chunking) and its row-tile count.  RW 16-row
  // tiles per workgroup, the sum split in NWV / RW parts.  The split fixes
  // the order in which a column's partial sums are added, so it is chosen
  // from the step's shape only (rows and subdomains), never from the column
  // count: a column's result is then the same whichever columns share the
  // launch.  Two tiles while one column group of two-tile workgroups fits
  // in kSweepRows workgroups, four on larger steps (measured: two tiles
  // best at 1024^2 with 16 RHS, four on the large steps at 2048^2 with 64
  // RHS)
  struct HostGroup {
    StepGroup d;
    int flen, rw;
  };
  std::vector<HostGroup> hg;
  for (int i = 0; i < nst; ++i) {
    const int L = sidx[i] / sc.nsteps;
    const int off = sc.step_off[sidx[i]], cnt = sc.step_cnt[sidx[i]];
    if (cnt == 0) continue;
    FaceSet fin{}, fout{};
    int nin = 0;
    const int nout = step_faces(c, L, fin, fout, &nin);
    if (nout == 0) continue;
    int flen = 0;
    for (int q = 0; q < fin.n; ++q) flen = std::max(flen, 2 * g.side_len[fin.face[q]]);
    for (int b0 = 0; b0 < cnt; b0 += kStepListMax) {
      HostGroup h{};
      h.d.L = L;
      h.d.nout = nout;
      h.d.add_y = L == 0 ? 1 : 0;
      h.d.n = std::min(kStepListMax, cnt - b0);
      h.d.first = off + b0;              // into step_subs until packed
      h.d.fin = fin;
      h.d.fout = fout;
      h.flen = flen;
      const long long wg2 = 8LL * (((nout + 31) / 32 + 7) / 8) * h.d.n;
      h.rw = c->tune.sweep_rw ? c->tune.sweep_rw : (wg2 > kSweepRows ? 4 : 2);
      hg.push_back(h);
    }
  }
  const int nhg = (int)hg.size();
  // 4-deep slices of T per register batch (two batches in flight): by
  // default a wave's 20 (complex64) or 10 (complex128) slices of a 1024^2
  // face chunk in two batches (measured: complex64 8 -> 10 shortens the step
  // by 5%, 12 is slower again; complex128 4 -> 5 by 4%); the autotuner may
  // choose another compiled depth (sweep_kb).  The depth does not change
  // the order of the sum.
  const int kb_sel = c->tune.sweep_kb ? c->tune.sweep_kb : (sizeof(T) == 4 ? 10 : 5);
  for (int i = 0; i < nhg;) {
    // the next group shares the launch when its row-tile count agrees
    const int j = (i + 1 < nhg && hg[i + 1].rw == hg[i].rw) ? i + 2 : i + 1;
    StepLaunch sl{};
    sl.ng = j - i;
    int pos = 0;
    for (int k = i; k < j; ++k) {
      StepGroup d = hg[k].d;
      for (int t = 0; t < d.n; ++t) {
        sl.sub[pos + t] = sc.step_subs[d.first + t];
        sl.op[pos + t] = c->op_of_sub[sl.sub[pos + t]];
      }
      d.first = pos;
      pos += d.n;
      sl.g[k - i] = d;
    }
    // NWV waves per workgroup: eight (one workgroup per CU, the LDS holds
    // long face chunks) or four (two workgroups per CU, shorter chunks),
    // chosen per shape by the autotuner
    auto launch_kb = [&](auto rw, auto kbc, auto nwv) -> hipError_t {
      constexpr int RW = decltype(rw)::value;
      constexpr int KB = decltype(kbc)::value;
      constexpr int NWV = decltype(nwv)::value;
      // LDS chunks of one input face (or a part of it): 2 tiles x LMAX rows
      // of kSweepRS operand pairs, LMAX a multiple of 4 no larger than lcap
      const int lcap = sweep_lcap<T, NWV>();
      size_t lds_pairs = (size_t)(NWV / RW) * 16 * 16 * RW;   // the KH partial tiles
      int np = 0;
      for (int k = 0; k < sl.ng; ++k) {
        StepGroup& d = sl.g[k];
        const int flen = hg[i + k].flen;
        d.nsub_chunks = std::max(1, (flen + lcap - 1) / lcap);
        d.LMAX = std::max(4, ((flen + d.nsub_chunks - 1) / d.nsub_chunks + 3) / 4 * 4);
        lds_pairs = std::max(lds_pairs, (size_t)2 * d.LMAX * kSweepRS);
        np += (d.nout + 16 * RW - 1) / (16 * RW) * d.n;
      }
      dim3 grid(8 * ((np + 7) / 8), Cp / 16, 1);
      hipLaunchKernelGGL((k_sweep_step<T, KB, RW, NWV>), grid, dim3(NWV * 64),
                         lds_pairs * sizeof(cpx<T>), c->stream, (const cpx<T>*)c->d_T,
                         (const cpx<T>*)c->d_cface, (cpx<T>*)c->d_slots,
                         (const cpx<T>*)c->d_y, sl, C, c->gd);
      return hipGetLastError();
    };
    auto launch_nw = [&](auto rw, auto nwv) -> hipError_t {
      if constexpr (sizeof(T) == 4) {
        if (kb_sel == 6) return launch_kb(rw, std::integral_constant<int, 6>{}, nwv);
        if (kb_sel == 8) return launch_kb(rw, std::integral_constant<int, 8>{}, nwv);
        if (kb_sel == 10) return launch_kb(rw, std::integral_constant<int, 10>{}, nwv);
      } else {
        if (kb_sel == 3) return launch_kb(rw, std::integral_constant<int, 3>{}, nwv);
        if (kb_sel == 4) return launch_kb(rw, std::integral_constant<int, 4>{}, nwv);
        if (kb_sel == 5) return launch_kb(rw, std::integral_constant<int, 5>{}, nwv);
        if (kb_sel == 6) return launch_kb(rw, std::integral_constant<int, 6>{}, nwv);
      }
      return hipErrorInvalidValue;   // not a compiled depth (checked when set)
    };
    auto launch = [&](auto rw) -> hipError_t {
      if (c->tune.sweep_nw == 4) return launch_nw(rw, std::integral_constant<int, 4>{});
      return launch_nw(rw, std::integral_constant<int, 8>{});
    };
    hipError_t e = hg[i].rw == 4 ? launch(std::integral_constant<int, 4>{})
                                 : launch(std::integral_constant<int, 2>{});
    if (e != hipSuccess) return e;
    i = j;
  }
  return hipSuccess;
}

#define HDSW_INST2(T)                                                          \
  template hipError_t launch_block_solve<T>(hdsw_ctx*, int, const int*, int, const int*); \
  template hipError_t launch_factor_step<T>(hdsw_ctx*, int, int);              \
  template hipError_t launch_sweep_steps<T>(hdsw_ctx*, const int*, int, int);\
  template hipError_t launch_face_coef<T>(hdsw_ctx*);
HDSW_INST2(float)
HDSW_INST2(double)

}  // namespace hdsw

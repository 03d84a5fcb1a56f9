// Dense-block path of the hdsw library, used when one block of the
// subdomain operator is a whole grid plane (3D: n = n_x n_y, K = n_z).
//
// Block-tridiagonal LU with the coupling B_k = diag(a^z) between planes
// k-1 and k (the operator is complex symmetric, so the coupling is the same
// on both sides of the diagonal):
//   D_0 = A_0,   D_k = A_k - B_k D_{k-1}^{-1} B_k,   X_k = D_k^{-1}
// and, for every right-hand side,
//   forward   w_0 = X_0 f_0,   w_k = X_k (f_k - B_k w_{k-1})
//   backward  x_{K-1} = w_{K-1},   x_k = w_k - X_k (B_{k+1} x_{k+1}).
// X_k is formed by blocked Gauss-Jordan elimination with partial pivoting
// (largest |Re| + |Im| in the column, lowest row index on ties): a panel of
// nb columns is eliminated by one workgroup (in registers for blocks up to
// 2048 nodes), the rest of the matrix takes the panel's row interchanges
// and is updated by one complex GEMM, and the column order is restored at
// the end.
// Every product with a dense block is a complex GEMM on the matrix cores
// (k_cgemm).
#include "hdsw_internal.hpp"
#include "mfma_ops.hpp"

namespace hdsw {

// ------------------------------------------------------------ complex GEMM
// C_z = beta C_z + s A_z B_z  (s = +1 or -1, beta = 0 or 1), complex, all
// column-major.  z indexes a group of columns that share one A:
//   A_z        = A + op_z * sAz,            op_z = grp_op ? grp_op[z] : z
//   column j of B_z (j < ncols_z): B + z * sBz + e * sb + (j % cpb) * ldb,
//     e = ids ? ids[off_z + j / cpb] : j / cpb,  off_z = grp_off ? grp_off[z] : 0
//   C the same with sCz, sc, ldc,
//   ncols_z = grp_cnt ? grp_cnt[z] * cpb : N.
// A workgroup computes a 64 x 32 tile of C with four waves, one 16-row
// strip each; the sum runs in chunks of 16 staged in LDS.  A complex
// product takes two real MFMAs per 16 x 16 x 4 step: B is staged as pairs
// (Re b, -Im b) and (Im b, Re b) in the two halves of a 16-wide operand, so
// that Re(A) x first + Im(A) x second gives [Re(AB) | Im(AB)] for 8 complex
// columns.
constexpr int GM = 64, GN = 32, GPAD = 80;

// BK-deep chunks of the sum, double-buffered in LDS (one barrier per
// chunk): the next chunk's global loads are in flight while the current one
// is multiplied.  BK = 16 (complex64) or 8 (complex128) keeps the LDS of a
// workgroup at 40 KB, so four workgroups (four waves per SIMD) share a CU
// and hide each other's load and barrier latency; the tiled A layout keeps
// its 64 x TK tiles (TK = 32 or 16), a chunk reading half of one.
// Workgroups are dispatched round-robin over the 8 XCDs (id % 8), each with
// its own L2: all column tiles of a row tile are given the same XCD, so the
// row slab of A is fetched from HBM once.  With ksplit > 1 the sum is cut
// into ksplit parts whose raw products go to a.part and are added in a
// fixed order by k_gemm_combine (results do not depend on timing).
template <class T>
constexpr int gemm_tk() { return sizeof(T) == 4 ? 32 : 16; }

template <class T, int BK, bool TILED>
__global__ __launch_bounds__(256) void k_cgemm(GemmArgs a, int nrt, int nct) {
  constexpr int TK = gemm_tk<T>();
  static_assert(TK % BK == 0, "a chunk lies inside one A tile");
  typedef typename MF<T>::v4 v4;
  constexpr int AL = BK / 4;                 // A elements per thread
  constexpr int BL = BK / 8;                 // B elements per thread
  // A chunks [buf][k][row] and B operand pairs [buf][k][4 groups x 16
  // operand columns], then the output tile staged over both
  __shared__ cpx<T> smem[4 * BK * GPAD];
  cpx<T>(*As)[BK][GPAD] = reinterpret_cast<cpx<T>(*)[BK][GPAD]>(smem);
  cpx<T>(*Bp)[BK][GPAD] = reinterpret_cast<cpx<T>(*)[BK][GPAD]>(smem + 2 * BK * GPAD);
  const int z = blockIdx.z / a.ksplit, kpart = blockIdx.z - z * a.ksplit;
  const int xcd = blockIdx.x & 7, pos = blockIdx.x >> 3;
  const int rtile = xcd + 8 * (pos / nct), ctile = pos - (pos / nct) * nct;
  if (rtile >= nrt) return;
  const int ncols = a.grp_cnt ? a.grp_cnt[z] * a.cpb : a.N;
  const int col0 = ctile * GN;
  if (col0 >= ncols) return;
  const int row0 = rtile * GM;
  const int opz = a.grp_op ? a.grp_op[z] : z;
  const int off = a.grp_off ? a.grp_off[z] : 0;
  const cpx<T>* A = reinterpret_cast<const cpx<T>*>(a.A) + (long long)opz * a.sAz;
  const cpx<T>* B = reinterpret_cast<const cpx<T>*>(a.B) + (long long)z * a.sBz;
  cpx<T>* C = reinterpret_cast<cpx<T>*>(a.C) + (long long)z * a.sCz;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;

  // B: column bc, k = bk .. bk + BL - 1
  const int bc = tid >> 3, bk = (tid & 7) * BL;
  const cpx<T>* bcol = nullptr;
  {
    int j = col0 + bc;
    if (j < ncols) {
      int e = j / a.cpb, jj = j - e * a.cpb;
      int eid = a.ids ? a.ids[off + e] : e;
      bcol = B + (long long)eid * a.sb + (long long)jj * a.ldb;
    }
  }
  // A: row ar, k = ak .. ak + AL - 1
  const int ar = tid & 63, ak = (tid >> 6) * AL;
  const bool arow_ok = row0 + ar < a.M;
  const cpx<T>* acol = A + (arow_ok ? row0 + ar : 0);
  const cpx<T>* atile = TILED ? A + (long long)a.a_rt[rtile] * a.a_tile_ld * (GM * TK) : nullptr;

  cpx<T> ra[AL], rb[BL];
  v4 accR[4], accI[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    accR[g] = v4{T(0), T(0), T(0), T(0)};
    accI[g] = accR[g];
  }
  const int mr = wave * 16 + (lane & 15), mk4 = lane >> 4, mc = lane & 15;
  const int nch_all = (a.Kd + BK - 1) / BK;
  const int ch0 = (int)((long long)nch_all * kpart / a.ksplit);
  const int ch1 = (int)((long long)nch_all * (kpart + 1) / a.ksplit);

#define HDSW_GEMM_LOAD(k0)                                                       \
  {                                                                              \
    if (TILED) {                                                                 \
      const cpx<T>* tp = atile + (long long)a.a_kt[(k0) / TK] * (GM * TK) +      \
                         ((k0) % TK) * GM + ar;                                  \
      /* field by field: a complex128 struct copy goes through private */      \
      /* memory here */                                                          \
      _Pragma("unroll") for (int u = 0; u < AL; ++u) {                           \
        ra[u].re = tp[(ak + u) * GM].re;                                         \
        ra[u].im = tp[(ak + u) * GM].im;                                         \
      }                                                                          \
    } else {                                                                     \
      _Pragma("unroll") for (int u = 0; u < AL; ++u) {                           \
        int k = (k0) + ak + u;                                                   \
        ra[u].re = T(0);                                                         \
        ra[u].im = T(0);                                                         \
        if (arow_ok && k < a.Kd) ra[u] = acol[(long long)k * a.lda];             \
      }                                                                          \
    }                                                                            \
    _Pragma("unroll") for (int u = 0; u < BL; ++u) {                             \
      int k = (k0) + bk + u;                                                     \
      rb[u].re = T(0);                                                           \
      rb[u].im = T(0);                                                           \
      if (bcol && k < a.Kd) rb[u] = bcol[k];                                     \
    }                                                                            \
  }
#define HDSW_GEMM_STORE(buf)                                                     \
  {                                                                              \
    _Pragma("unroll") for (int u = 0; u < AL; ++u)                               \
      As[buf][ak + u][ar] = mk<T>(ra[u].re, ra[u].im);                           \
    const int g_ = bc >> 3, cc_ = bc & 7;                                        \
    _Pragma("unroll") for (int u = 0; u < BL; ++u) {                             \
      Bp[buf][bk + u][g_ * 16 + cc_] = mk<T>(rb[u].re, -rb[u].im);               \
      Bp[buf][bk + u][g_ * 16 + cc_ + 8] = mk<T>(rb[u].im, rb[u].re);            \
    }                                                                            \
  }

  if (ch0 < ch1) {
    HDSW_GEMM_LOAD(ch0 * BK);
    HDSW_GEMM_STORE(0);
  }
  __syncthreads();
  for (int ch = ch0; ch < ch1; ++ch) {
    const int buf = (ch - ch0) & 1;
    if (ch + 1 < ch1) HDSW_GEMM_LOAD((ch + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const cpx<T> av = As[buf][ks * 4 + mk4][mr];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const cpx<T> p = Bp[buf][ks * 4 + mk4][g * 16 + mc];
        accR[g] = MF<T>::mfma(av.re, p.re, accR[g]);
        accI[g] = MF<T>::mfma(av.im, p.im, accI[g]);
      }
    }
    if (ch + 1 < ch1) HDSW_GEMM_STORE(buf ^ 1);
    __syncthreads();
  }
#undef HDSW_GEMM_LOAD
#undef HDSW_GEMM_STORE

  // stage [Re | Im] halves as complex columns (reusing the operand buffers)
  cpx<T>(*Cs)[GM] = reinterpret_cast<cpx<T>(*)[GM]>(smem);
  static_assert(sizeof(smem) >= sizeof(cpx<T>) * GN * GM, "staging does not fit");
  T* cs = reinterpret_cast<T*>(smem);
  const int part = mc >> 3, cc = mc & 7;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int r = wave * 16 + MF<T>::row(lane, i);
      cs[2 * ((g * 8 + cc) * GM + r) + part] = accR[g][i] + accI[g][i];
    }
  }
  __syncthreads();
  const int orow = tid & 63, oc = tid >> 6;
  if (row0 + orow >= a.M) return;
  if (a.ksplit > 1) {
    // raw partial product: part[kpart][z][j][row], j < column tiles x GN
    cpx<T>* P = reinterpret_cast<cpx<T>*>(a.part) +
                ((long long)kpart * gridDim.z / a.ksplit + z) * a.part_cols * a.M;
#pragma unroll
    for (int q = 0; q < GN / 4; ++q) {
      int c = oc * (GN / 4) + q;
      int j = col0 + c;
      if (j >= ncols) break;
      P[(long long)j * a.M + row0 + orow] = Cs[c][orow];
    }
    return;
  }
  const int crow = a.c_row ? a.c_row[row0 + orow] : row0 + orow;
  if (crow < 0) return;
#pragma unroll
  for (int q = 0; q < GN / 4; ++q) {
    int c = oc * (GN / 4) + q;
    int j = col0 + c;
    if (j >= ncols) break;
    int e = j / a.cpb, jj = j - e * a.cpb;
    int eid = a.ids ? a.ids[off + e] : e;
    cpx<T>* dst = C + (long long)eid * a.sc + (long long)jj * a.ldc + crow;
    cpx<T> v = Cs[c][orow];
    if (a.neg) v = -v;
    if (a.beta) v = *dst + v;
    *dst = v;
  }
}

// k extent of one tile of a tiled A operand
template <class T>
int gemm_bk() {
  return gemm_tk<T>();
}

// Skinny product (at most 8 columns per group), HBM-bound: each wave
// streams a 16-row strip of A straight from memory into the MFMA operand
// registers, a batch of SB 4-deep slices ahead of the multiplication; B is
// staged in LDS in chunks of KC rows shared by the workgroup's 4 waves.
constexpr int SK_KC = 256, SK_SB = 16;

template <class T, bool TILED>
__global__ __launch_bounds__(256) void k_cgemm_skinny(GemmArgs a, int nrt) {
  typedef typename MF<T>::v4 v4;
  __shared__ cpx<T> Bs[2][SK_KC][8];          // [buf][k][column]
  __shared__ cpx<T> Cs[8][GM];
  const int z = blockIdx.y;
  const int xcd = blockIdx.x & 7, pos = blockIdx.x >> 3;
  const int rtile = xcd + 8 * pos;
  if (rtile >= nrt) return;
  const int ncols = a.grp_cnt ? a.grp_cnt[z] * a.cpb : a.N;
  if (ncols <= 0) return;
  const int row0 = rtile * GM;
  const int opz = a.grp_op ? a.grp_op[z] : z;
  const int off = a.grp_off ? a.grp_off[z] : 0;
  const cpx<T>* A = reinterpret_cast<const cpx<T>*>(a.A) + (long long)opz * a.sAz;
  const cpx<T>* B = reinterpret_cast<const cpx<T>*>(a.B) + (long long)z * a.sBz;
  cpx<T>* C = reinterpret_cast<cpx<T>*>(a.C) + (long long)z * a.sCz;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  // this lane's A operand: row r, k = 4 s + kq
  const int r = row0 + wave * 16 + (lane & 15), kq = lane >> 4;
  const bool rok = r < a.M;
  const cpx<T>* arow = TILED ? nullptr : A + (rok ? r : 0);
  const cpx<T>* atile = TILED ? A + (long long)a.a_rt[rtile] * a.a_tile_ld * (GM * 32) : nullptr;
  const int rt_in = wave * 16 + (lane & 15);
  // B columns of this group (thread c < 8 of each staging pass)
  const int mc = lane & 15, cc = mc & 7;
  const bool hi = mc >= 8;
  v4 accR = v4{T(0), T(0), T(0), T(0)}, accI = accR;
  const int nkc = (a.Kd + SK_KC - 1) / SK_KC;
  auto stageB = [&](int kc, int buf) {
    const int k0 = kc * SK_KC;
    for (int idx = tid; idx < SK_KC * 8; idx += 256) {
      const int j = idx / SK_KC, kk = idx - j * SK_KC;   // consecutive threads: consecutive k
      const int k = k0 + kk;
      cpx<T> v;
      v.re = T(0);
      v.im = T(0);
      if (j < ncols && k < a.Kd) {
        const int e = j / a.cpb, jj = j - e * a.cpb;
        const int eid = a.ids ? a.ids[off + e] : e;
        v = B[(long long)eid * a.sb + (long long)jj * a.ldb + k];
      }
      Bs[buf][kk][j] = v;
    }
  };
  stageB(0, 0);
  __syncthreads();
  for (int kc = 0; kc < nkc; ++kc) {
    const int buf = kc & 1;
    if (kc + 1 < nkc) stageB(kc + 1, buf ^ 1);
    const int k0 = kc * SK_KC;
    const int ns = min(SK_KC, a.Kd - k0 + 3) / 4;          // slices in this chunk
    cpx<T> av[SK_SB];
    for (int s0 = 0; s0 < ns; s0 += SK_SB) {
#pragma unroll
      for (int u = 0; u < SK_SB; ++u) {
        const int k = k0 + 4 * (s0 + u) + kq;
        av[u].re = T(0);
        av[u].im = T(0);
        if (rok && s0 + u < ns && k < a.Kd) {
          if (TILED)
            av[u] = atile[(long long)a.a_kt[k >> 5] * (GM * 32) + (k & 31) * GM + rt_in];
          else
            av[u] = arow[(long long)k * a.lda];
        }
      }
#pragma unroll
      for (int u = 0; u < SK_SB; ++u) {
        if (s0 + u >= ns) break;
        const cpx<T> v = Bs[buf][4 * (s0 + u) + kq][cc];
        const T p_re = hi ? v.im : v.re;
        const T p_im = hi ? v.re : -v.im;
        accR = MF<T>::mfma(av[u].re, p_re, accR);
        accI = MF<T>::mfma(av[u].im, p_im, accI);
      }
    }
    __syncthreads();
  }
  T* cs = reinterpret_cast<T*>(&Cs[0][0]);
  const int part = mc >> 3;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int rr = wave * 16 + MF<T>::row(lane, i);
    cs[2 * (cc * GM + rr) + part] = accR[i] + accI[i];
  }
  __syncthreads();
  const int orow = tid & 63, oc = tid >> 6;
  if (row0 + orow >= a.M) return;
  const int crow = a.c_row ? a.c_row[row0 + orow] : row0 + orow;
  if (crow < 0) return;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int c = oc * 2 + q;
    if (c >= ncols) break;
    const int e = c / a.cpb, jj = c - e * a.cpb;
    const int eid = a.ids ? a.ids[off + e] : e;
    cpx<T>* dst = C + (long long)eid * a.sc + (long long)jj * a.ldc + crow;
    cpx<T> v = Cs[c][orow];
    if (a.neg) v = -v;
    if (a.beta) v = *dst + v;
    *dst = v;
  }
}

// C = beta C + s (sum of the partial products), in a fixed order
template <class T>
__global__ void k_gemm_combine(GemmArgs a, int ngroups, int maxcols) {
  const long long per = (long long)maxcols * a.M;
  const long long tot = per * ngroups;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    int z = (int)(idx / per);
    long long r = idx - z * per;
    int j = (int)(r / a.M), row = (int)(r - (long long)j * a.M);
    const int ncols = a.grp_cnt ? a.grp_cnt[z] * a.cpb : a.N;
    if (j >= ncols) continue;
    const int crow = a.c_row ? a.c_row[row] : row;
    if (crow < 0) continue;
    const cpx<T>* P = reinterpret_cast<const cpx<T>*>(a.part);
    cpx<T> v = P[((long long)z * a.part_cols + j) * a.M + row];
    for (int p = 1; p < a.ksplit; ++p)
      v = v + P[(((long long)p * ngroups + z) * a.part_cols + j) * a.M + row];
    const int off = a.grp_off ? a.grp_off[z] : 0;
    int e = j / a.cpb, jj = j - e * a.cpb;
    int eid = a.ids ? a.ids[off + e] : e;
    cpx<T>* C = reinterpret_cast<cpx<T>*>(a.C) + (long long)z * a.sCz;
    cpx<T>* dst = C + (long long)eid * a.sc + (long long)jj * a.ldc + crow;
    if (a.neg) v = -v;
    if (a.beta) v = *dst + v;
    *dst = v;
  }
}

// a.ksplit > 1 needs a.part with ksplit * ngroups * maxcols * M elements
template <class T>
hipError_t gemm(hipStream_t st, const GemmArgs& a_in, int maxcols, int ngroups) {
  if (a_in.M <= 0 || maxcols <= 0 || ngroups <= 0) return hipSuccess;
  GemmArgs a = a_in;
  if (a.ksplit < 1) a.ksplit = 1;
  if (a.ksplit > 1 && !a.part) return hipErrorInvalidValue;
  a.part_cols = maxcols;
  constexpr int BK = sizeof(T) == 4 ? 16 : 8;
  constexpr int TK = gemm_tk<T>();
  const int nrt = (a.M + GM - 1) / GM, nct = (maxcols + GN - 1) / GN;
  // at most 8 columns per group: the product streams A (HBM-bound)
  if (maxcols <= 8 && a.ksplit == 1 && !a.no_skinny && (!a.a_rt || TK == 32)) {
    dim3 g2(8 * ((nrt + 7) / 8), ngroups, 1);
    if (a.a_rt) {
      if (a.M % GM != 0) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_cgemm_skinny<T, true>), g2, dim3(256), 0, st, a, nrt);
    } else {
      hipLaunchKernelGGL((k_cgemm_skinny<T, false>), g2, dim3(256), 0, st, a, nrt);
    }
    return hipGetLastError();
  }
  dim3 grid(8 * ((nrt + 7) / 8) * nct, 1, ngroups * a.ksplit);
  if (a.a_rt) {
    // tiled A: whole tiles only
    if (a.M % GM != 0 || a.Kd % TK != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_cgemm<T, BK, true>), grid, dim3(256), 0, st, a, nrt, nct);
  } else {
    hipLaunchKernelGGL((k_cgemm<T, BK, false>), grid, dim3(256), 0, st, a, nrt, nct);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.ksplit == 1) return e;
  long long tot = (long long)ngroups * maxcols * a.M;
  int blocks = (int)std::min<long long>((tot + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_gemm_combine<T>, dim3(blocks), dim3(256), 0, st, a, ngroups, maxcols);
  return hipGetLastError();
}

// ------------------------------------------------------------ Gauss-Jordan
// One workgroup per matrix z (X + z * sz, n x n column-major) eliminates the
// pivots j0 .. j0 + nbr - 1, touching whole rows for the swaps and the
// panel columns for the elimination.  piv[z * n + kc] records the row
// swapped into position kc.
template <class T>
__global__ __launch_bounds__(1024) void k_gj_panel(cpx<T>* X, long long sz, int n, int j0,
                                                   int nbr, int* piv, int* flag) {
  __shared__ float bestv[1024];
  __shared__ int besti[1024];
  __shared__ cpx<T> prow[64];
  const int tid = threadIdx.x;
  cpx<T>* A = X + (long long)blockIdx.x * sz;
  for (int kc = j0; kc < j0 + nbr; ++kc) {
    // pivot: largest |Re| + |Im| at or below the diagonal, lowest index on ties
    float bv = -1.f;
    int bi = n;
    for (int i = kc + tid; i < n; i += 1024) {
      cpx<T> v = A[(long long)kc * n + i];
      float m = (float)(fabs(v.re) + fabs(v.im));
      if (m > bv) { bv = m; bi = i; }
    }
    bestv[tid] = bv;
    besti[tid] = bi;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
      if (tid < w) {
        float ov = bestv[tid + w];
        int oi = besti[tid + w];
        if (ov > bestv[tid] || (ov == bestv[tid] && oi < besti[tid])) {
          bestv[tid] = ov;
          besti[tid] = oi;
        }
      }
      __syncthreads();
    }
    const int r = besti[0];
    const bool singular = !(bestv[0] > 0.f) || r >= n;
    __syncthreads();
    if (tid == 0) {
      piv[(long long)blockIdx.x * n + kc] = singular ? kc : r;
      if (singular) flag[0] = 1;
    }
    if (!singular && r != kc) {
      for (int j = tid; j < n; j += 1024) {
        cpx<T> t = A[(long long)j * n + kc];
        A[(long long)j * n + kc] = A[(long long)j * n + r];
        A[(long long)j * n + r] = t;
      }
    }
    __syncthreads();
    const cpx<T> pv = A[(long long)kc * n + kc];
    const cpx<T> ip = singular ? mk<T>(T(0), T(0)) : cinv(pv);
    if (tid < nbr) {
      int j = j0 + tid;
      cpx<T> v = A[(long long)j * n + kc];
      prow[tid] = j == kc ? ip : v * ip;
    }
    __syncthreads();
    for (int i = tid; i < n; i += 1024) {
      if (i == kc) continue;
      cpx<T> f = A[(long long)kc * n + i];
      for (int q = 0; q < nbr; ++q) {
        int j = j0 + q;
        if (j == kc) {
          A[(long long)j * n + i] = -(f * ip);
        } else {
          cpx<T> v = A[(long long)j * n + i];
          A[(long long)j * n + i] = v - f * prow[q];
        }
      }
    }
    __syncthreads();
    if (tid < nbr) A[(long long)(j0 + tid) * n + kc] = prow[tid];
    __syncthreads();
  }
}

// R_z[q][j] = A_z[j0 + q][j] for j outside the panel (0 inside), those
// entries of A_z set to zero, and E_z = the eliminated panel columns: the
// rest of the matrix is then A += E R.  R is nbr x n (leading dimension
// nbr), E is n x nbr (leading dimension n); they sit at R + z sR and
// R + z sR + n nbr_max.
template <class T>
__global__ void k_gj_take_rows(cpx<T>* X, long long sz, int n, int j0, int nbr, cpx<T>* R,
                               long long sR, long long eoff) {
  cpx<T>* A = X + (long long)blockIdx.y * sz;
  cpx<T>* Rz = R + (long long)blockIdx.y * sR;
  cpx<T>* Ez = Rz + eoff;
  long long tot = (long long)n * nbr;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    int j = (int)(idx / nbr), q = (int)(idx - (long long)j * nbr);
    cpx<T>* src = A + (long long)j * n + j0 + q;
    if (j >= j0 && j < j0 + nbr) {
      Rz[idx] = mk<T>(T(0), T(0));
    } else {
      Rz[idx] = *src;
      *src = mk<T>(T(0), T(0));
    }
    // panel column j0 + q, row j (rows of the panel columns are not zeroed)
    Ez[(long long)q * n + j] = A[(long long)(j0 + q) * n + j];
  }
}

// undo the row interchanges on the columns of the inverse, last first
template <class T>
__global__ void k_gj_colperm(cpx<T>* X, long long sz, int n, const int* piv) {
  cpx<T>* A = X + (long long)blockIdx.y * sz;
  const int* pz = piv + (long long)blockIdx.y * n;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int kc = n - 1; kc >= 0; --kc) {
    int r = pz[kc];
    if (r != kc) {
      cpx<T> t = A[(long long)kc * n + i];
      A[(long long)kc * n + i] = A[(long long)r * n + i];
      A[(long long)r * n + i] = t;
    }
  }
}

// Register-resident panel (n <= 1024 S): one workgroup of 1024 threads per
// matrix z eliminates the pivots j0 .. j0 + nbr - 1 (nbr <= NB) on the panel
// columns only, thread t holding rows t + 1024 s (s < S) of the NB panel
// columns in registers.  Rows are not moved while the panel is eliminated:
// the pivot of column j0 + q is the row with the largest |Re| + |Im| (its
// exponent and leading 10 mantissa bits, then the lowest row) among the rows
// at positions >= j0 not chosen yet, which are exactly the candidate
// positions of the row-swapping algorithm.  One barrier per pivot: every
// wave finds its best row by cross-lane moves and offers it (key and the
// row's NB entries) in LDS; every thread then takes the best of the 16
// offers.  Offers alternate between two buffers by pivot parity, so a
// pivot's offers never overwrite ones still being read.
// At the end the chosen rows are turned into the interchanges of the
// swapping algorithm (position j0 + q with position piv[j0 + q]) and the
// panel is written back with every row at its interchanged position.  The
// interchanges' net effect on any other column is a set of at most 2 NB
// moves (row at position src goes to position dst), written to mv for the
// kernels that bring the other columns along.
template <int NB>
__host__ __device__ constexpr int gj_mv_stride() { return 1 + 4 * NB; }

// Applies the moves of one panel (list m: count, destinations, sources) to a
// column: every source is read before any destination is written.
template <class T, int NB>
__device__ __forceinline__ void gj_apply_moves(cpx<T>* col, const int* m) {
  // field by field: a conditional complex128 struct copy would go through
  // private memory
  const int cnt = m[0];
  T vr[2 * NB], vi[2 * NB];
#pragma unroll
  for (int e = 0; e < 2 * NB; ++e) {
    vr[e] = T(0);
    vi[e] = T(0);
    if (e < cnt) {
      const cpx<T>* s = col + m[1 + 2 * NB + e];
      vr[e] = s->re;
      vi[e] = s->im;
    }
  }
#pragma unroll
  for (int e = 0; e < 2 * NB; ++e)
    if (e < cnt) {
      cpx<T>* d = col + m[1 + e];
      d->re = vr[e];
      d->im = vi[e];
    }
}

template <class T, int NB, int S>
__global__ __launch_bounds__(1024) void k_gj_panel_reg(cpx<T>* X, long long sz, int n, int j0,
                                                       int nbr, int* piv, int* flag, int* mv,
                                                       long long mvso) {
  __shared__ cpx<T> offer[2][16][NB];
  __shared__ __align__(16) unsigned okey[2][16];
  __shared__ int obad[2][16];                  // the offered pivot is zero or NaN
  __shared__ int prow_of[NB];                  // row chosen for column j0 + q
  __shared__ int mrow[2 * NB], mpos[2 * NB];   // moved rows and their positions
  __shared__ int mcnt;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  cpx<T>* A = X + (long long)blockIdx.x * sz;
  cpx<T> pr[S][NB];
  bool cand[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int i = tid + 1024 * s;
    cand[s] = i < n && i >= j0;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      pr[s][c] = mk<T>(T(0), T(0));
      if (i < n && c < nbr) pr[s][c] = A[(long long)(j0 + c) * n + i];
    }
  }
  int anybad = 0;                              // thread 0: a zero or NaN pivot
  // the pivot loop is unrolled: column q of the panel is a static register
  // index in every step
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    if (q >= nbr) continue;
    const int slot = q & 1;
    unsigned key = 0u;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if (cand[s]) {
        float m = (float)(fabs(pr[s][q].re) + fabs(pr[s][q].im));
        if (!(m == m)) m = 0.f;                  // NaN: the row stays a candidate
        const unsigned k = (__float_as_uint(m) & ~8191u) | (unsigned)(8191 - (tid + 1024 * s));
        key = k > key ? k : key;
      }
    }
    const unsigned wk = wave_max_u32(key);
    // the wave's best row offers itself already scaled as the pivot row
    // (entry q: the inverse of the pivot, the others: entry x inverse)
    if (wk) {
      const int wrow = 8191 - (int)(wk & 8191u);
#pragma unroll
      for (int s = 0; s < S; ++s)
        if (wrow == tid + 1024 * s) {
          const cpx<T> pv = pr[s][q];
          const bool bad = (pv.re == T(0) && pv.im == T(0)) || !(pv.re == pv.re) ||
                           !(pv.im == pv.im);
          const cpx<T> inv = bad ? mk<T>(T(0), T(0)) : cinv(pv);
#pragma unroll
          for (int c = 0; c < NB; ++c) offer[slot][wave][c] = c == q ? inv : pr[s][c] * inv;
          obad[slot][wave] = bad ? 1 : 0;
        }
    }
    if (lane == 0) okey[slot][wave] = wk;
    lds_barrier();
    // the sixteen offers' keys: they are distinct (each carries its row)
    // and the best is positive (a candidate exists for every column: n - j0
    // - q rows), so the pivot row p is the one in the largest key, found by
    // a max tree, and the wave that offered it is the one holding row p
    // (row i lives in thread i mod 1024)
    const uint4* ok4 = reinterpret_cast<const uint4*>(okey[slot]);
    const uint4 k0 = ok4[0], k1 = ok4[1], k2 = ok4[2], k3 = ok4[3];
    const unsigned best =
        max(max(max(max(k0.x, k0.y), max(k0.z, k0.w)), max(max(k1.x, k1.y), max(k1.z, k1.w))),
            max(max(max(k2.x, k2.y), max(k2.z, k2.w)), max(max(k3.x, k3.y), max(k3.z, k3.w))));
    const int p = 8191 - (int)(best & 8191u), bw = (p & 1023) >> 6;
    const cpx<T>* ph = offer[slot][bw];
    if (tid == 0) {
      anybad |= obad[slot][bw];
      prow_of[q] = p;
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int i = tid + 1024 * s;
      if (i == p) {
#pragma unroll
        for (int c = 0; c < NB; ++c) pr[s][c] = ph[c];
        cand[s] = false;
      } else if (i < n) {
        const cpx<T> f = pr[s][q];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
          const cpx<T> r2 = ph[c];
          if (c == q) {
            pr[s][c] = -(f * r2);
          } else {
            cpx<T> m = pr[s][c];
            m.re = fma(-f.re, r2.re, m.re);
            m.re = fma(f.im, r2.im, m.re);
            m.im = fma(-f.re, r2.im, m.im);
            m.im = fma(-f.im, r2.re, m.im);
            pr[s][c] = m;
          }
        }
      }
    }
  }
  if (tid == 0 && anybad) atomicExch(flag, 1);
  lds_barrier();
  // the interchanges: position j0 + q swaps with the position its pivot
  // row holds at that point; only the rows of the swaps move
  if (tid == 0) {
    int cnt = 0;
    for (int q = 0; q < nbr; ++q) {
      const int pr_ = prow_of[q], a = j0 + q;
      int rq = pr_, y = a, ip = -1, iy = -1;
      for (int e = 0; e < cnt; ++e) {
        if (mrow[e] == pr_) { rq = mpos[e]; ip = e; }
        if (mpos[e] == a) { y = mrow[e]; iy = e; }
      }
      piv[(long long)blockIdx.x * n + a] = rq;
      if (rq != a) {
        if (ip < 0) { ip = cnt++; mrow[ip] = pr_; }
        mpos[ip] = a;
        if (iy < 0) { iy = cnt++; mrow[iy] = y; }
        mpos[iy] = rq;
      }
    }
    mcnt = cnt;
    // the moves for the other columns: [count, destinations, sources]
    int* m = mv + (long long)blockIdx.x * mvso;
    m[0] = cnt;
    for (int e = 0; e < cnt; ++e) {
      m[1 + e] = mpos[e];
      m[1 + 2 * NB + e] = mrow[e];
    }
  }
  lds_barrier();
  const int cnt = mcnt;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int i = tid + 1024 * s;
    if (i >= n) continue;
    int pos = i;
    for (int e = 0; e < cnt; ++e)
      if (mrow[e] == i) pos = mpos[e];
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < nbr) A[(long long)(j0 + c) * n + pos] = pr[s][c];
  }
}

// Inner update of a two-level panel: after the register panel of columns
// j0 .. j0 + nbr - 1, every other column j of the outer panel J0 .. J0 +
// OBr - 1 takes the panel's moves, its rows j0 .. j0 + nbr - 1 (r) are
// taken out and zeroed, and the column is updated by the eliminated panel
// E (those columns of X): col += E r.  One workgroup per (column, matrix);
// a plain sum over the panel's nbr columns per row.
template <class T, int NB>
__global__ __launch_bounds__(256) void k_gj_inner(cpx<T>* X, long long sz, int n, int J0, int j0,
                                                  int nbr, const int* mv, long long mvso) {
  __shared__ cpx<T> r[NB];
  const int z = blockIdx.y, j = J0 + blockIdx.x, tid = threadIdx.x;
  if (j >= j0 && j < j0 + nbr) return;
  cpx<T>* A = X + (long long)z * sz;
  cpx<T>* col = A + (long long)j * n;
  const cpx<T>* E = A + (long long)j0 * n;
  if (tid == 0) gj_apply_moves<T, NB>(col, mv + (long long)z * mvso);
  __syncthreads();
  if (tid < nbr) {
    r[tid] = col[j0 + tid];
    col[j0 + tid] = mk<T>(T(0), T(0));
  }
  __syncthreads();
  for (int i = tid; i < n; i += 256) {
    cpx<T> acc = col[i];
    for (int q = 0; q < nbr; ++q) acc = acc + E[(long long)q * n + i] * r[q];
    col[i] = acc;
  }
}

// Outer rows of a two-level panel: thread j of matrix z (blockIdx.y), for a
// column j outside the outer panel J0 .. J0 + OBr - 1, applies the moves of
// the npan inner panels in order, moves its rows J0 .. J0 + OBr - 1 to R_z
// (OBr x n, leading dimension OBr) and zeroes them.  The rest of the matrix
// is then A += E R with E the outer panel's columns.
template <class T, int NB>
__global__ void k_gj_outer_rows(cpx<T>* X, long long sz, int n, int J0, int OBr, int npan,
                                const int* mv, long long mvso, cpx<T>* R, long long sR) {
  const int z = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n || (j >= J0 && j < J0 + OBr)) return;
  cpx<T>* col = X + (long long)z * sz + (long long)j * n;
  const int* mz = mv + (long long)z * mvso;
  for (int p = 0; p < npan; ++p) gj_apply_moves<T, NB>(col, mz + p * gj_mv_stride<NB>());
  cpx<T>* Rz = R + (long long)z * sR + (long long)j * OBr;
  for (int q = 0; q < OBr; ++q) {
    Rz[q] = col[J0 + q];
    col[J0 + q] = mk<T>(T(0), T(0));
  }
}

// ------------------------------------------------------------ factor
// Dense D_k of every distinct operator (3D, plane k) written into its X_k
// slot: the in-plane 5-point part of the operator minus
// B_k X_{k-1} B_k (k > 0).  Coefficients per operator:
//   ax[n_z][n_y][n_x + 1], ay[n_z][n_y + 1][n_x], az[n_z + 1][n_y][n_x], dg[n_z][n_y][n_x]
template <class T>
__global__ void k_form_plane(cpx<T>* X, const cpx<T>* coefT, size_t cstride, GeoDev g,
                             int k, int nops) {
  const int nx = g.ne[0], ny = g.ne[1], nz = g.ne[2];
  const int n = g.n;
  const long long nn = (long long)n * n;
  const size_t o_ay = (size_t)nz * ny * (nx + 1);
  const size_t o_az = o_ay + (size_t)nz * (ny + 1) * nx;
  const size_t o_dg = o_az + (size_t)(nz + 1) * ny * nx;
  const int op = blockIdx.y;
  if (op >= nops) return;
  const cpx<T>* co = coefT + (size_t)op * cstride;
  cpx<T>* Xk = X + ((long long)op * g.K + k) * nn;
  const cpx<T>* Xp = Xk - nn;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < nn;
       idx += (long long)gridDim.x * blockDim.x) {
    int j = (int)(idx / n), i = (int)(idx - (long long)j * n);
    int yi = i / nx, xi = i - yi * nx;
    int yj = j / nx, xj = j - yj * nx;
    cpx<T> v = mk<T>(T(0), T(0));
    if (i == j) v = co[o_dg + ((size_t)k * ny + yi) * nx + xi];
    else if (yi == yj && xj == xi + 1) v = co[((size_t)k * ny + yi) * (nx + 1) + xi + 1];
    else if (yi == yj && xj == xi - 1) v = co[((size_t)k * ny + yi) * (nx + 1) + xi];
    else if (xi == xj && yj == yi + 1) v = co[o_ay + ((size_t)k * (ny + 1) + yi + 1) * nx + xi];
    else if (xi == xj && yj == yi - 1) v = co[o_ay + ((size_t)k * (ny + 1) + yi) * nx + xi];
    if (k > 0) {
      cpx<T> bi = co[o_az + ((size_t)k * ny + yi) * nx + xi];
      cpx<T> bj = co[o_az + ((size_t)k * ny + yj) * nx + xj];
      v = v - bi * Xp[idx] * bj;
    }
    Xk[idx] = v;
  }
}

// rbuf: 2 n 32 elements per distinct operator (panel rows R and columns E)
// Two-level panels for blocks up to 2048 nodes: outer panels of OB = 128
// columns, each eliminated as inner panels of NBR columns in registers
// (k_gj_panel_reg) whose updates reach only the outer panel's other
// columns (k_gj_inner); the rest of the matrix then takes the outer panel's
// moves and one rank-128 complex GEMM (measured at 96^3 with 27 operators:
// rank 64 1.78 s, 128 1.61 s, 256 1.66 s).  Larger blocks: 32-column
// panels eliminated in global memory (k_gj_panel) and a rank-32 GEMM each.
constexpr int kGjOuter = 128;
template <class T>
constexpr int gj_inner_nb() { return sizeof(T) == 4 ? 16 : 8; }
static bool gj_two_level(int n) { return n <= 2048; }

// Scratch of launch_big_factor: the R rows of every operator, then (two
// levels) the inner panels' move lists.
template <class T>
size_t big_factor_scratch_bytes(const hdsw_ctx* c) {
  const size_t n = c->g.n, nops = c->nops;
  if (!gj_two_level((int)n)) return nops * 2 * n * 32 * sizeof(cpx<T>);
  constexpr int NBR = gj_inner_nb<T>();
  const size_t mvso = (size_t)(kGjOuter / NBR) * gj_mv_stride<NBR>();
  return nops * kGjOuter * n * sizeof(cpx<T>) + nops * mvso * sizeof(int) + 256;
}

template <class T>
hipError_t launch_big_factor(hdsw_ctx* c, void* rbuf) {
  const Geometry& g = c->g;
  const int n = g.n, nops = c->nops;
  const long long nn = (long long)n * n;
  const long long sz = (long long)g.K * nn;     // operator stride in X
  cpx<T>* X = (cpx<T>*)c->d_X;
  cpx<T>* R = (cpx<T>*)rbuf;
  constexpr int NBR = gj_inner_nb<T>();
  const bool two = gj_two_level(n);
  const long long sR = two ? (long long)kGjOuter * n : 2LL * n * 32;   // R per operator
  const long long mvso = (long long)(kGjOuter / NBR) * gj_mv_stride<NBR>();
  int* mv = reinterpret_cast<int*>(R + (size_t)nops * sR);
  for (int k = 0; k < g.K; ++k) {
    int blocks = (int)std::min<long long>((nn + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(k_form_plane<T>, dim3(blocks, nops), dim3(256), 0, c->stream, X,
                       (const cpx<T>*)c->d_coefT, c->coef_stride, c->gd, k, nops);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    cpx<T>* Xk = X + (long long)k * nn;
    int* piv = c->d_piv;
    const int ob = two ? kGjOuter : 32;
    for (int J0 = 0; J0 < n; J0 += ob) {
      const int OBr = std::min(ob, n - J0);
      if (two) {
        const int npan = (OBr + NBR - 1) / NBR;
        for (int p = 0; p < npan; ++p) {
          const int j0 = J0 + p * NBR, nbr = std::min(NBR, J0 + OBr - j0);
          int* mvp = mv + p * gj_mv_stride<NBR>();
          if (n <= 1024)
            hipLaunchKernelGGL((k_gj_panel_reg<T, NBR, 1>), dim3(nops), dim3(1024), 0,
                               c->stream, Xk, sz, n, j0, nbr, piv, c->d_flag, mvp, mvso);
          else
            hipLaunchKernelGGL((k_gj_panel_reg<T, NBR, 2>), dim3(nops), dim3(1024), 0,
                               c->stream, Xk, sz, n, j0, nbr, piv, c->d_flag, mvp, mvso);
          if (OBr > nbr)
            hipLaunchKernelGGL((k_gj_inner<T, NBR>), dim3(OBr, nops), dim3(256), 0, c->stream,
                               Xk, sz, n, J0, j0, nbr, (const int*)mvp, mvso);
        }
        hipLaunchKernelGGL((k_gj_outer_rows<T, NBR>), dim3((n + 255) / 256, nops), dim3(256),
                           0, c->stream, Xk, sz, n, J0, OBr, npan, (const int*)mv, mvso, R, sR);
      } else {
        hipLaunchKernelGGL(k_gj_panel<T>, dim3(nops), dim3(1024), 0, c->stream, Xk, sz, n, J0,
                           OBr, piv, c->d_flag);
        long long tot = (long long)n * OBr;
        int tb = (int)std::min<long long>((tot + 255) / 256, 1 << 16);
        hipLaunchKernelGGL(k_gj_take_rows<T>, dim3(tb, nops), dim3(256), 0, c->stream, Xk, sz,
                           n, J0, OBr, R, sR, (long long)n * 32);
      }
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      // rest of the matrix += E R (two levels: E = the outer panel's
      // columns of X, and the columns left and right of it; one level: E
      // copied beside R, every column, R zero in the panel's columns)
      auto update = [&](int c0, int ncols) -> hipError_t {
        if (ncols <= 0) return hipSuccess;
        GemmArgs a{};
        a.M = n;
        a.N = ncols;
        a.Kd = OBr;
        if (two) {
          a.A = Xk + (long long)J0 * n;
          a.sAz = sz;
          a.B = R + (long long)c0 * OBr;
          a.ldb = OBr;
        } else {
          a.A = R + (long long)n * 32;
          a.sAz = sR;
          a.B = R;
          a.ldb = OBr;
        }
        a.lda = n;
        a.sb = 0;
        a.sBz = sR;
        a.C = Xk + (long long)c0 * n;
        a.ldc = n;
        a.sc = 0;
        a.sCz = sz;
        a.cpb = ncols;
        a.neg = 0;
        a.beta = 1;
        return gemm<T>(c->stream, a, ncols, nops);
      };
      if (two) {
        e = update(0, J0);
        if (e == hipSuccess) e = update(J0 + OBr, n - J0 - OBr);
      } else {
        e = update(0, n);
      }
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_gj_colperm<T>, dim3((n + 255) / 256, nops), dim3(256), 0, c->stream,
                       Xk, sz, n, piv);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ------------------------------------------------------------ tiled T
// T(i, j) of operator op into its tile: face f of a row dof i starts at the
// padded row t_roff[f], face of the column dof j at the padded column
// t_koff[f]; tiles are 64 rows x TK columns, k-major inside, row tiles
// outermost.  Padding stays zero (the buffer is cleared first).
struct TileGeo {
  int roff[6], koff[6], nkt, tk;
};
__device__ inline int face_of(const GeoDev& g, int i) {
  int f = 0;
#pragma unroll
  for (int j = 1; j < 6; ++j) f = (j < 2 * g.dim && i >= g.side_off[j]) ? j : f;
  return f;
}
template <class T>
__global__ void k_extract_tiled(const cpx<T>* panel, int C, cpx<T>* Tt, int col0, GeoDev g,
                                TileGeo tg) {
  long long tot = (long long)C * g.NI;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    int col = (int)(idx / g.NI), i = (int)(idx - (long long)col * g.NI);
    // node of dof i: plane k, in-plane p (3D)
    int f = face_of(g, i);
    int r = i - pick(g.side_off, f);
    const int len = pick(g.side_len, f);
    int L = r / len, t = r - L * len;
    int axis = f >> 1, na = pick(g.na, axis);
    int layer = (f & 1) == 0 ? (L == 0 ? g.W : g.W - 1) : (L == 0 ? g.W + na - 1 : g.W + na);
    int x, y, z;
    if (axis == 0) { x = layer; z = t / g.ne[1]; y = t - z * g.ne[1]; }
    else if (axis == 1) { y = layer; z = t / g.ne[0]; x = t - z * g.ne[0]; }
    else { z = layer; y = t / g.ne[0]; x = t - y * g.ne[0]; }
    cpx<T> v = panel[((long long)z * C + col) * g.n + (long long)y * g.ne[0] + x];
    int j = col0 + col;
    int fj = face_of(g, j);
    int prow = pick(tg.roff, f) + r;
    int pcol = pick(tg.koff, fj) + (j - pick(g.side_off, fj));
    long long tile = (long long)(prow >> 6) * tg.nkt + pcol / tg.tk;
    Tt[tile * 64 * tg.tk + (long long)(pcol % tg.tk) * 64 + (prow & 63)] = v;
  }
}

template <class T>
hipError_t launch_extract_tiled(hdsw_ctx* c, int C, int op, int col0) {
  const Geometry& g = c->g;
  TileGeo tg;
  for (int f = 0; f < 6; ++f) {
    tg.roff[f] = c->t_roff[f];
    tg.koff[f] = c->t_koff[f];
  }
  tg.nkt = c->t_nkt;
  tg.tk = c->t_tk;
  cpx<T>* Tt = (cpx<T>*)c->d_T + (long long)op * c->t_nrt * 64 * (long long)c->t_nkt * c->t_tk;
  long long tot = (long long)C * g.NI;
  int blocks = (int)std::min<long long>((tot + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_extract_tiled<T>, dim3(blocks), dim3(256), 0, c->stream,
                     (const cpx<T>*)c->d_panel, C, Tt, col0, c->gd, tg);
  return hipGetLastError();
}

// ------------------------------------------------------------ solve
// scratch line K of each panel entry b (operator ops[b]):
//   forward  t = f_k - B_k w_{k-1}  (k > 0),  t = f_0
//   backward t = B_{k+1} x_{k+1}
template <class T>
__global__ void k_plane_rhs(cpx<T>* panel, int nbatch, int C, int k, int fwd,
                            const int* ops, const cpx<T>* coefT, size_t cstride, GeoDev g) {
  const int n = g.n, K = g.K;
  const int nx = g.ne[0], ny = g.ne[1], nz = g.ne[2];
  const size_t o_az = (size_t)nz * ny * (nx + 1) + (size_t)nz * (ny + 1) * nx;
  const long long per = (long long)C * n;
  const long long tot = per * nbatch;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < tot;
       idx += (long long)gridDim.x * blockDim.x) {
    int b = (int)(idx / per);
    long long r = idx - b * per;
    int p = (int)(r % n);
    cpx<T>* base = panel + (long long)b * g.PL * per;
    const cpx<T>* az = coefT + (size_t)ops[b] * cstride + o_az;
    cpx<T> v;
    if (fwd) {
      v = base[(long long)k * per + r];
      if (k > 0) v = v - az[(size_t)k * n + p] * base[(long long)(k - 1) * per + r];
    } else {
      v = az[(size_t)(k + 1) * n + p] * base[(long long)(k + 1) * per + r];
    }
    base[(long long)K * per + r] = v;
  }
}

template <class T>
hipError_t launch_big_solve(hdsw_ctx* c, int nbatch, const int* d_ops, const int* grp_op,
                            const int* grp_off, const int* grp_cnt, const int* ids,
                            int ngroups, int maxcnt, int C) {
  const Geometry& g = c->g;
  const int n = g.n, K = g.K;
  const long long nn = (long long)n * n;
  const long long per = (long long)C * n;
  cpx<T>* P = (cpx<T>*)c->d_panel;
  long long tot = per * nbatch;
  int blocks = (int)std::min<long long>((tot + 255) / 256, 1 << 20);
  for (int pass = 0; pass < 2; ++pass) {
    const int fwd = pass == 0;
    for (int s = 0; s < (fwd ? K : K - 1); ++s) {
      const int k = fwd ? s : K - 2 - s;
      hipLaunchKernelGGL(k_plane_rhs<T>, dim3(blocks), dim3(256), 0, c->stream, P, nbatch, C,
                         k, fwd, d_ops, (const cpx<T>*)c->d_coefT, c->coef_stride, c->gd);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      GemmArgs a{};
      a.M = n;
      a.N = 0;
      a.Kd = n;
      a.A = (const cpx<T>*)c->d_X + (long long)k * nn;
      a.lda = n;
      a.sAz = (long long)K * nn;
      a.B = P + (long long)K * per;
      a.ldb = n;
      a.sb = (long long)g.PL * per;
      a.sBz = 0;
      a.C = P + (long long)k * per;
      a.ldc = n;
      a.sc = (long long)g.PL * per;
      a.sCz = 0;
      a.cpb = C;
      a.ids = ids;
      a.grp_op = grp_op;
      a.grp_off = grp_off;
      a.grp_cnt = grp_cnt;
      a.neg = fwd ? 0 : 1;
      a.beta = fwd ? 0 : 1;
      // too few output tiles to fill the chip: split the sum
      const long long tiles = (long long)((n + 63) / 64) * ((maxcnt * C + 31) / 32) * ngroups;
      int ks = (int)std::min<long long>(4, std::max<long long>(1, (512 + tiles - 1) / tiles));
      while (ks > 1 && (size_t)ks * ngroups * maxcnt * C * n * sizeof(cpx<T>) > c->gpart_bytes)
        --ks;
      a.ksplit = ks;
      a.part = c->d_gpart;
      a.no_skinny = c->tune.gemm_skinny == 2;
      e = gemm<T>(c->stream, a, maxcnt * C, ngroups);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

#define HDSW_INST3(T)                                                                      \
  template hipError_t gemm<T>(hipStream_t, const GemmArgs&, int, int);                     \
  template int gemm_bk<T>();                                                               \
  template hipError_t launch_extract_tiled<T>(hdsw_ctx*, int, int, int);                   \
  template hipError_t launch_big_factor<T>(hdsw_ctx*, void*);                              \
  template size_t big_factor_scratch_bytes<T>(const hdsw_ctx*);                             \
  template hipError_t launch_big_solve<T>(hdsw_ctx*, int, const int*, const int*,          \
                                          const int*, const int*, const int*, int, int, int);
HDSW_INST3(float)
HDSW_INST3(double)

}  // namespace hdsw

// Right-preconditioned restarted GMRES(m) in FP64 with the DDM as
// preconditioner (the paper's use of the method, Sec. 5.2), batched over
// RHS columns.  Orthogonalisation is classical Gram-Schmidt applied twice
// (the dots of one pass are independent, so each pass is one batched
// reduction on the device); the small Hessenberg least-squares problem of
// every column is reduced by Givens rotations on the host.  A column whose
// residual estimate meets the tolerance inside a cycle takes its update from
// the Arnoldi steps up to that point only (later steps, run for the other
// columns, do not enter it), so its result and iteration count are those of
// the same column solved alone.
#include <cmath>
#include <complex>
#include <vector>

#include "hdsw_internal.hpp"

namespace hdsw {

hdsw_status ddm_dispatch(hdsw_ctx* c, const c128* r, c128* out, int C, int accumulate);

#define HCHK(expr)                \
  do {                            \
    if ((expr) != hipSuccess) {   \
      c->sticky = HDSW_EDEVICE;   \
      return HDSW_EDEVICE;        \
    }                             \
  } while (0)
#define ACHK(expr)                \
  do {                            \
    hdsw_status s_ = (expr);      \
    if (s_ != HDSW_OK) return s_; \
  } while (0)

using cd = std::complex<double>;

hdsw_status gmres_cols(hdsw_ctx* c, int C, std::vector<int>& iters, std::vector<double>& rel,
                       const std::vector<double>& bn) {
  const Geometry& g = c->g;
  const int m = c->opt.gmres_m;
  const long long gn = g.glob_nodes;
  const size_t vec = (size_t)C * gn;
  if (C > c->gm_cols || C > c->Cmax) return HDSW_EINVAL;   // basis sized for fewer columns
  c128* V = c->d_V;
  c128* Z = c->d_Z;
  c128* dots = c->d_dots;                          // [(m+1)][C]
  c128* coef = c->d_dots + (size_t)(m + 1) * C;    // [(m+1)][C]
  iters.assign(C, -1);
  rel.assign(C, 0.0);
  HCHK(launch_zero(c, c->d_xg, vec * sizeof(c128)));
  std::vector<double> nrm(C), inv(C);
  std::vector<cd> H((size_t)C * (m + 1) * m), cs((size_t)C * m), sn((size_t)C * m),
      gv((size_t)C * (m + 1));
  std::vector<c128> hbuf((size_t)(m + 1) * C), cbuf((size_t)(m + 1) * C);
  int total = 0;
  // per column: Arnoldi steps of the current cycle that enter its update,
  // and the iteration count at which its estimate met the tolerance
  std::vector<int> kcol(C, 0), done_at(C, -1);
  auto h_at = [&](int col, int i, int j) -> cd& { return H[((size_t)col * (m + 1) + i) * m + j]; };
  while (true) {
    HCHK(launch_residual(c, c->d_bg, c->d_xg, c->d_rg, C));
    HCHK(launch_norms(c, c->d_rg, C, c->d_norm));
    HCHK(hipMemcpyAsync(nrm.data(), c->d_norm, C * sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
    HCHK(hipStreamSynchronize(c->stream));
    bool all = true;
    std::vector<char> active(C, 0);
    for (int j = 0; j < C; ++j) {
      rel[j] = bn[j] > 0 ? nrm[j] / bn[j] : 0.0;
      if (iters[j] < 0 && rel[j] <= c->opt.tol) iters[j] = done_at[j] >= 0 ? done_at[j] : total;
      if (iters[j] < 0) {
        all = false;
        active[j] = 1;
      }
    }
    if (all || total >= c->opt.max_iter) break;
    for (int j = 0; j < C; ++j) {
      inv[j] = nrm[j] > 0 ? 1.0 / nrm[j] : 0.0;
      for (int i = 0; i <= m; ++i) gv[(size_t)j * (m + 1) + i] = 0.0;
      gv[(size_t)j * (m + 1)] = nrm[j];
    }
    HCHK(hipMemcpyAsync(c->d_norm, inv.data(), C * sizeof(double), hipMemcpyHostToDevice,
                        c->stream));
    HCHK(launch_scale(c, V, c->d_rg, c->d_norm, C));
    int kused = 0;
    std::vector<char> done(C, 0);
    for (int j = 0; j < C; ++j) done_at[j] = -1;
    for (int k = 0; k < m; ++k) {
      c128* Vk = V + (size_t)k * vec;
      c128* Zk = Z + (size_t)k * vec;
      ACHK(ddm_dispatch(c, Vk, Zk, C, 0));
      HCHK(launch_residual(c, nullptr, Zk, c->d_rg, C));   // w = S z_k
      std::vector<cd> hsum((size_t)(k + 1) * C, 0.0);
      for (int pass = 0; pass < 2; ++pass) {
        HCHK(launch_dots(c, V, k + 1, c->d_rg, C, dots));
        HCHK(hipMemcpyAsync(hbuf.data(), dots, (size_t)(k + 1) * C * sizeof(c128),
                            hipMemcpyDeviceToHost, c->stream));
        HCHK(hipStreamSynchronize(c->stream));
        for (size_t i = 0; i < (size_t)(k + 1) * C; ++i)
          hsum[i] += cd(hbuf[i].re, hbuf[i].im);
        HCHK(hipMemcpyAsync(coef, hbuf.data(), (size_t)(k + 1) * C * sizeof(c128),
                            hipMemcpyHostToDevice, c->stream));
        HCHK(launch_axpy_multi(c, c->d_rg, V, k + 1, coef, C, -1.0));
      }
      HCHK(launch_norms(c, c->d_rg, C, c->d_norm));
      HCHK(hipMemcpyAsync(nrm.data(), c->d_norm, C * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
      HCHK(hipStreamSynchronize(c->stream));
      for (int j = 0; j < C; ++j) inv[j] = nrm[j] > 0 ? 1.0 / nrm[j] : 0.0;
      HCHK(hipMemcpyAsync(c->d_norm, inv.data(), C * sizeof(double), hipMemcpyHostToDevice,
                          c->stream));
      HCHK(launch_scale(c, V + (size_t)(k + 1) * vec, c->d_rg, c->d_norm, C));
      ++total;
      kused = k + 1;
      bool all_done = true;
      for (int j = 0; j < C; ++j) {
        for (int i = 0; i <= k; ++i) h_at(j, i, k) = hsum[(size_t)i * C + j];
        h_at(j, k + 1, k) = nrm[j];
        for (int i = 0; i < k; ++i) {     // previous rotations
          cd a = h_at(j, i, k), b = h_at(j, i + 1, k);
          cd cc = cs[(size_t)j * m + i], ss = sn[(size_t)j * m + i];
          h_at(j, i, k) = cc * a + ss * b;
          h_at(j, i + 1, k) = -std::conj(ss) * a + std::conj(cc) * b;
        }
        cd a = h_at(j, k, k), b = h_at(j, k + 1, k);
        double den = std::sqrt(std::norm(a) + std::norm(b));
        cd cc = 1.0, ss = 0.0;
        if (den > 0) {
          cc = std::conj(a / den);
          ss = std::conj(b / den);
        }
        cs[(size_t)j * m + k] = cc;
        sn[(size_t)j * m + k] = ss;
        h_at(j, k, k) = cc * a + ss * b;
        h_at(j, k + 1, k) = 0.0;
        cd gk = gv[(size_t)j * (m + 1) + k];
        gv[(size_t)j * (m + 1) + k + 1] = -std::conj(ss) * gk;
        gv[(size_t)j * (m + 1) + k] = cc * gk;
        double est = std::abs(gv[(size_t)j * (m + 1) + k + 1]);
        if (active[j] && !done[j] && (est <= c->opt.tol * bn[j] || nrm[j] == 0.0)) {
          done[j] = 1;
          kcol[j] = k + 1;
          done_at[j] = total;
        }
        if (active[j] && !done[j]) all_done = false;
      }
      if (all_done || total >= c->opt.max_iter) break;
    }
    // x += Z y, y = H^{-1} g (upper triangular, per column)
    for (int j = 0; j < C; ++j) {
      std::vector<cd> y(kused, 0.0);
      const int kj = done[j] ? kcol[j] : kused;
      if (active[j]) {
        for (int i = kj - 1; i >= 0; --i) {
          cd s = gv[(size_t)j * (m + 1) + i];
          for (int l = i + 1; l < kj; ++l) s -= h_at(j, i, l) * y[l];
          cd d = h_at(j, i, i);
          y[i] = std::abs(d) > 0 ? s / d : 0.0;
        }
      }
      for (int i = 0; i < kused; ++i) cbuf[(size_t)i * C + j] = mk<double>(y[i].real(), y[i].imag());
    }
    HCHK(hipMemcpyAsync(coef, cbuf.data(), (size_t)kused * C * sizeof(c128),
                        hipMemcpyHostToDevice, c->stream));
    HCHK(launch_axpy_multi(c, c->d_xg, Z, kused, coef, C, 1.0));
  }
  return HDSW_OK;
}

}  // namespace hdsw

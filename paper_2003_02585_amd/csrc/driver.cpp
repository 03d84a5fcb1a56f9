// Host runtime of the hdsw library: validation, partition, sweep schedule and
// trace routing, operator deduplication, device memory, factorization, the
// DDM application (Algorithm 2.1) and the FP64 refinement / GMRES drivers.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <map>
#include <mutex>
#include <new>
#include <unordered_map>

#include "hdsw_internal.hpp"

namespace hdsw {

hdsw_status scratch_init(int device);

#define HCHK(expr)                                   \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) {                          \
      c->sticky = HDSW_EDEVICE;                      \
      return HDSW_EDEVICE;                           \
    }                                                \
  } while (0)

// ------------------------------------------------------------ schedule
// Sweep order: eq. (Sorder2D) / (Sorder3D).
static void sweep_dirs(int dim, std::vector<std::array<int, 3>>& out) {
  out.clear();
  if (dim == 2) {
    out.push_back({1, 1, 0});
    out.push_back({-1, 1, 0});
    out.push_back({1, -1, 0});
    out.push_back({-1, -1, 0});
  } else {
    for (int dz : {1, -1})
      for (int dy : {1, -1})
        for (int dx : {1, -1}) out.push_back({dx, dy, dz});
  }
}

// Rule 2.4 / 4.1: similar directions
static bool similar(const int* e, const int* d, int dim) {
  int dot = 0;
  for (int a = 0; a < dim; ++a) dot += e[a] * d[a];
  if (dot <= 0) return false;
  if (dim == 3)
    for (int a = 0; a < 3; ++a)
      if (e[a] * d[a] < 0) return false;
  return true;
}

// Rule 2.5 / 4.2: may a trace of direction e generated in a sweep dg be used
// in the later sweep du?
static bool opposite_blocked(const int* e, const int* dg, const int* du, int dim) {
  if (dim == 2) return du[0] == -dg[0] && du[1] == -dg[1];
  static const int planes[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  for (auto& pl : planes) {
    int a = pl[0], b = pl[1];
    int zeros = (e[a] == 0) + (e[b] == 0);
    if (zeros != 1) continue;
    if (du[a] == -dg[a] && du[b] == -dg[b]) return true;
  }
  return false;
}

// Levels of the sweep steps in the routing dependences.  Subdomain s in
// sweep L reads its slot L, which every neighbour s' fills across the shared
// face in each sweep L' <= L that routes that face to L (L' = L: the
// neighbour's earlier step of the same sweep); and it adds into the slots
// of its neighbours, which the same neighbour-sweep pairs also add into.
// Taking (L, s) after all of those writers and after (L - 1, s) orders
// every slot's additions by sweep, as the step-by-step order does, so the
// results do not change.  level(L, s) = 1 + the largest level of those
// predecessors; the steps whose subdomains share a level go to one launch
// (at most two steps of consecutive sweeps on the partitions tried).  A step
// whose subdomains would land on several levels is not merged.
static void build_levels(const Geometry& g, Schedule& s) {
  s.lfirst.clear();
  s.lsteps.clear();
  const int nst = s.nsweeps * s.nsteps;
  std::vector<int> lev((size_t)s.nsweeps * g.nsub, 0), slev(nst, -1);
  bool uniform = g.dim == 2;
  for (int L = 0; L < s.nsweeps && uniform; ++L)
    for (int st = 0; st < s.nsteps && uniform; ++st) {
      const int off = s.step_off[L * s.nsteps + st], cnt = s.step_cnt[L * s.nsteps + st];
      for (int i = 0; i < cnt; ++i) {
        const int sub = s.step_subs[off + i];
        int cc[3], v = L > 0 ? lev[(size_t)(L - 1) * g.nsub + sub] + 1 : 0;
        g.sub_coords(sub, cc);
        for (int f = 0; f < 2 * g.dim; ++f) {
          int nc[3] = {cc[0], cc[1], cc[2]};
          nc[f >> 1] += (f & 1) ? 1 : -1;
          if (nc[f >> 1] < 0 || nc[f >> 1] >= g.P[f >> 1]) continue;
          const int nb = g.sub_id(nc);
          for (int L0 = 0; L0 <= L; ++L0)   // the neighbour sends across face f ^ 1
            if (s.lprime[L0 * 6 + (f ^ 1)] == L)
              v = std::max(v, lev[(size_t)L0 * g.nsub + nb] + 1);
        }
        lev[(size_t)L * g.nsub + sub] = v;
        if (i == 0) slev[L * s.nsteps + st] = v;
        else if (slev[L * s.nsteps + st] != v) uniform = false;
      }
    }
  if (!uniform) return;          // one launch per step
  int nlev = 0;
  for (int v : slev) nlev = std::max(nlev, v + 1);
  std::vector<std::vector<int>> by(nlev);
  for (int i = 0; i < nst; ++i)
    if (slev[i] >= 0) by[slev[i]].push_back(i);
  for (auto& v : by) {
    if (v.empty()) continue;
    s.lfirst.push_back((int)s.lsteps.size());
    s.lsteps.insert(s.lsteps.end(), v.begin(), v.end());
  }
  s.lfirst.push_back((int)s.lsteps.size());
}

static void build_schedule(hdsw_ctx* c) {
  Geometry& g = c->g;
  Schedule& s = c->sch;
  std::vector<std::array<int, 3>> base;
  sweep_dirs(g.dim, base);
  int per = (int)base.size();
  s.nsweeps = c->opt.rounds * per;
  s.dir.resize(s.nsweeps);
  for (int L = 0; L < s.nsweeps; ++L) s.dir[L] = base[L % per];
  s.nsteps = 1;
  for (int a = 0; a < g.dim; ++a) s.nsteps += g.P[a] - 1;
  s.step_off.assign(s.nsweeps * s.nsteps, 0);
  s.step_cnt.assign(s.nsweeps * s.nsteps, 0);
  s.step_subs.clear();
  for (int L = 0; L < s.nsweeps; ++L) {
    const auto& d = s.dir[L];
    std::vector<std::vector<int>> groups(s.nsteps);
    for (int sub = 0; sub < g.nsub; ++sub) {
      int cc[3];
      g.sub_coords(sub, cc);
      int st = 0;  // 0-based step: sum of ihat (eq. step_subd_ij / step_subd_k)
      for (int a = 0; a < g.dim; ++a) st += d[a] == 1 ? cc[a] : g.P[a] - 1 - cc[a];
      groups[st].push_back(sub);
    }
    for (int st = 0; st < s.nsteps; ++st) {
      s.step_off[L * s.nsteps + st] = (int)s.step_subs.size();
      s.step_cnt[L * s.nsteps + st] = (int)groups[st].size();
      s.step_subs.insert(s.step_subs.end(), groups[st].begin(), groups[st].end());
    }
  }
  // routing: smallest l' >= L allowed by the rules over the extended list
  s.lprime.assign(s.nsweeps * 6, -1);
  for (int L = 0; L < s.nsweeps; ++L) {
    for (int f = 0; f < 2 * g.dim; ++f) {
      int e[3] = {0, 0, 0};
      e[f >> 1] = (f & 1) ? 1 : -1;
      for (int lp = L; lp < s.nsweeps; ++lp) {
        if (!similar(e, s.dir[lp].data(), g.dim)) continue;
        if (lp > L && opposite_blocked(e, s.dir[L].data(), s.dir[lp].data(), g.dim))
          continue;
        s.lprime[L * 6 + f] = lp;
        break;
      }
    }
  }
  s.in_active.assign(s.nsweeps * 6, 0);
  for (int L0 = 0; L0 < s.nsweeps; ++L0)
    for (int f = 0; f < 2 * g.dim; ++f) {
      int lq = s.lprime[L0 * 6 + f];
      if (lq >= 0) s.in_active[lq * 6 + (f ^ 1)] = 1;
    }
  build_levels(g, s);
}

// ------------------------------------------------------------ PML profile
// alpha = 1 + i sigma0 (dist / W)^2, dist = distance outside the box in
// units of h (quadratic profile of eq. (sigma), translation invariant).
static c128 alpha_of(double dist, double s0, int W) {
  double t = dist / W;
  return mk<double>(1.0, s0 * t * t);
}
// node p (local 0..ne-1) and half-point q (0..ne) of a box of na interior
// nodes preceded and followed by W layer nodes
static double node_dist(int p, int W, int na) {
  if (p < W) return W - p - 0.5;
  if (p >= W + na) return p - (W + na) + 0.5;
  return 0.0;
}
static double half_dist(int q, int W, int na) {
  if (q < W) return double(W - q);
  if (q > W + na) return double(q - W - na);
  return 0.0;
}

static uint64_t fnv1a(const void* data, size_t n) {
  const unsigned char* p = (const unsigned char*)data;
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

// ------------------------------------------------------------ runtime lock
// Runtime calls that may wait on other streams or on the whole device
// (allocation and free, blocking copies, creation and destruction of
// streams, events and graphs) fail while another thread records a graph,
// and a graph being recorded can be invalidated by them.  Contexts may be
// driven from several threads (a serving loop factors new operators on a
// worker thread while the main thread records DDM applications), so these
// calls and the recording of an application hold one process-wide lock.
static std::recursive_mutex& rt_mu() {
  static std::recursive_mutex m;
  return m;
}
typedef std::lock_guard<std::recursive_mutex> RtGuard;

// ------------------------------------------------------------ memory
// Every device allocation of a context goes through these two: the caller's
// allocator hooks when hdsw_options sets them (so a framework's caching
// allocator can own the memory), hipMalloc / hipFree otherwise.
static void raw_free(const hdsw_ctx* c, void* p) {
  RtGuard lk(rt_mu());
  if (c->opt.dev_free) c->opt.dev_free(p, c->opt.alloc_ctx);
  else (void)hipFree(p);
}
static hdsw_status dev_alloc(hdsw_ctx* c, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  if (c->opt.hbm_budget && c->alloc_bytes + bytes > c->opt.hbm_budget) return HDSW_ENOMEM;
  RtGuard lk(rt_mu());
  if (c->opt.dev_alloc) {
    *p = c->opt.dev_alloc(bytes, c->opt.alloc_ctx);
    if (!*p) return HDSW_ENOMEM;
  } else if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return HDSW_ENOMEM;
  }
  c->alloc_bytes += bytes;
  c->bufs.push_back({*p, bytes});
  return HDSW_OK;
}
static void dev_free(hdsw_ctx* c, void* p) {
  if (!p) return;
  for (size_t i = 0; i < c->bufs.size(); ++i) {
    if (c->bufs[i].p == p) {
      c->alloc_bytes -= c->bufs[i].bytes;
      raw_free(c, p);
      c->bufs.erase(c->bufs.begin() + i);
      return;
    }
  }
}
static void free_all(hdsw_ctx* c) {
  for (auto& b : c->bufs) raw_free(c, b.p);
  c->bufs.clear();
  c->alloc_bytes = 0;
}

// A caller's array: device memory of the context's device (hipMalloc or an
// allocator on top of it, or managed memory) that holds `bytes` from p.
// Host memory, pinned or not, and other devices' memory are rejected before
// any kernel sees the pointer.  The size is checked against the allocation
// that contains p (a caching allocator's block: the bound is that block).
hdsw_status check_dev_ptr(const hdsw_ctx* c, const void* p, size_t bytes) {
  if (!p) return HDSW_EINVAL;
  hipPointerAttribute_t a;
  std::memset(&a, 0, sizeof(a));
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();   // not known to the runtime: plain host memory
    return HDSW_EINVAL;
  }
  if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged) return HDSW_EINVAL;
  if (a.device != c->device) return HDSW_EINVAL;
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) == hipSuccess) {
    const char* lo = (const char*)base;
    if ((const char*)p < lo || (size_t)((const char*)p - lo) + bytes > size) return HDSW_EINVAL;
  } else {
    (void)hipGetLastError();
  }
  return HDSW_OK;
}
#define PCHK(ptr, bytes)                                   \
  do {                                                     \
    hdsw_status s_ = check_dev_ptr(c, (ptr), (bytes));     \
    if (s_ != HDSW_OK) return s_;                          \
  } while (0)
#define ACHK(expr)                         \
  do {                                     \
    hdsw_status s_ = (expr);               \
    if (s_ != HDSW_OK) return s_;          \
  } while (0)

static size_t elt(const hdsw_ctx* c) {
  return c->opt.precision == HDSW_MIXED ? sizeof(c64) : sizeof(c128);
}

// ------------------------------------------------------------ timing
// Pairs of HIP events from a pool created once per context bracket the
// timed launches on the context's stream; they are resolved when the
// timings are read.
struct PendingEv {
  int cls;
  int slot;
  double flops, bytes;
};
struct EvPool {
  std::vector<hipEvent_t> ev;      // 2 per slot
  std::vector<PendingEv> pending;
  size_t next = 0;
};
static std::unordered_map<const hdsw_ctx*, EvPool>& pools() {
  static std::unordered_map<const hdsw_ctx*, EvPool> m;
  return m;
}
static void resolve_timing(hdsw_ctx* c);
struct TimedScope {
  hdsw_ctx* c;
  int cls;
  double flops, bytes;
  int slot = -1;
  TimedScope(hdsw_ctx* c_, int cls_, double f, double b) : c(c_), cls(cls_), flops(f), bytes(b) {
    if (!((c->tm.mask >> cls) & 1)) return;
    EvPool& p = pools()[c];
    if (p.ev.empty()) {
      RtGuard lk(rt_mu());
      p.ev.resize(2 * 8192, nullptr);
      for (auto& e : p.ev)
        if (hipEventCreate(&e) != hipSuccess) e = nullptr;
    }
    if (p.next >= p.ev.size() / 2) resolve_timing(c);
    slot = (int)p.next++;
    if (p.ev[2 * slot]) (void)hipEventRecord(p.ev[2 * slot], c->stream);
  }
  ~TimedScope() {
    if (slot < 0) return;
    EvPool& p = pools()[c];
    if (p.ev[2 * slot + 1]) (void)hipEventRecord(p.ev[2 * slot + 1], c->stream);
    p.pending.push_back({cls, slot, flops, bytes});
  }
};

static void resolve_timing(hdsw_ctx* c) {
  auto it = pools().find(c);
  if (it == pools().end()) return;
  EvPool& p = it->second;
  for (auto& e : p.pending) {
    hipEvent_t a = p.ev[2 * e.slot], b = p.ev[2 * e.slot + 1];
    float ms = 0.f;
    if (a && b && hipEventSynchronize(b) == hipSuccess &&
        hipEventElapsedTime(&ms, a, b) == hipSuccess) {
      c->tm.ms[e.cls] += ms;
      c->tm.launches[e.cls] += 1;
      c->tm.flops[e.cls] += e.flops;
      c->tm.bytes[e.cls] += e.bytes;
    } else {
      (void)hipGetLastError();   // a failed read must not reach the next launch check
    }
  }
  p.pending.clear();
  p.next = 0;
}

// ------------------------------------------------------------ setup
hdsw_status setup_impl(const hdsw_grid* grid, const double* kappa, const hdsw_partition* part,
                       int W, const hdsw_options* opt, void* stream, hdsw_ctx** out) {
  if (!grid || !kappa || !part || !opt || !out) return HDSW_EINVAL;
  if (grid->dim != 2 && grid->dim != 3) return HDSW_EINVAL;
  if (!(grid->h > 0) || !std::isfinite(grid->h) || W < 1) return HDSW_EINVAL;
  if (opt->precision != HDSW_FP64 && opt->precision != HDSW_MIXED) return HDSW_EINVAL;
  if (opt->rounds < 1 || opt->rounds > 4 || !(opt->pml_R > 0 && opt->pml_R < 1) ||
      !(opt->tol > 0) || opt->max_iter < 0 || opt->gmres_m < 0 || opt->gmres_m > 200)
    return HDSW_EINVAL;
  if (!opt->dev_alloc != !opt->dev_free) return HDSW_EINVAL;   // both hooks or neither
  hdsw_ctx* c = new (std::nothrow) hdsw_ctx();
  if (!c) return HDSW_ENOMEM;
  Geometry& g = c->g;
  g.dim = grid->dim;
  g.W = W;
  g.h = grid->h;
  long long nint = 1;
  for (int a = 0; a < g.dim; ++a) {
    g.N[a] = grid->n[a];
    g.P[a] = part->nsub[a];
    if (g.N[a] < 1 || g.P[a] < 1 || g.N[a] % g.P[a] != 0 || g.N[a] / g.P[a] < 2) {
      delete c;
      return HDSW_EINVAL;
    }
    g.na[a] = g.N[a] / g.P[a];
    g.ne[a] = g.na[a] + 2 * W;
    g.M[a] = g.N[a] + 2 * W;
    nint *= g.N[a];
  }
  g.nsub = 1;
  g.sub_nodes = 1;
  g.glob_nodes = 1;
  for (int a = 0; a < g.dim; ++a) {
    g.nsub *= g.P[a];
    g.sub_nodes *= g.ne[a];
    g.glob_nodes *= g.M[a];
  }
  g.int_nodes = nint;
  if (g.dim == 2) {
    g.n = g.ne[0];
    g.K = g.ne[1];
  } else {
    g.n = g.ne[0] * g.ne[1];
    g.K = g.ne[2];
  }
  g.nP = (g.n + 15) / 16 * 16;
  g.mid = g.K / 2;
  g.PL = g.K + 2;
  // the 2D block solver keeps nP-long vectors per column in LDS and up to
  // 12 row tiles per half chain in registers: complex64 lines of up to 384
  // nodes, complex128 up to 256; 3D plane blocks go through the dense-block
  // path
  if (g.dim == 2 && (g.nP > 384 || (g.nP > 256 && opt->precision != HDSW_MIXED))) {
    delete c;
    return HDSW_EINVAL;
  }
  if (g.dim == 3 && (long long)g.n * 6 * 2 * g.n > (1LL << 31)) {
    delete c;
    return HDSW_EINVAL;  // interface response too large for 32-bit offsets
  }
  g.nsides = 2 * g.dim;
  if (g.dim == 2) {
    g.side_len[0] = g.side_len[1] = g.ne[1];
    g.side_len[2] = g.side_len[3] = g.ne[0];
  } else {
    g.side_len[0] = g.side_len[1] = g.ne[1] * g.ne[2];
    g.side_len[2] = g.side_len[3] = g.ne[0] * g.ne[2];
    g.side_len[4] = g.side_len[5] = g.ne[0] * g.ne[1];
  }
  int off = 0;
  for (int s = 0; s < g.nsides; ++s) {
    g.side_off[s] = off;
    off += 2 * g.side_len[s];
  }
  g.NI = off;
  double kmin = 1e300;
  for (long long i = 0; i < nint; ++i) {
    double k = kappa[i];
    if (!std::isfinite(k) || !(k > 0)) {
      delete c;
      return HDSW_EINVAL;
    }
    kmin = std::min(kmin, k);
  }
  c->opt = *opt;
  g.s0 = 3.0 * std::log(1.0 / opt->pml_R) / (kmin * W * g.h);
  c->stream = (hipStream_t)stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return HDSW_EDEVICE;
  }
  // device address of this device's allocation-free workspace array (once
  // per device, with the device current); a failure here only disables
  // hdsw_apply_precond_noalloc, which then returns EDEVICE
  (void)scratch_init(c->device);
  c->kappa.assign(kappa, kappa + nint);

  GeoDev& d = c->gd;
  d.dim = g.dim;
  d.W = g.W;
  d.n = g.n;
  d.K = g.K;
  d.NI = g.NI;
  d.nsub = g.nsub;
  d.nP = g.nP;
  d.mid = g.mid;
  d.PL = g.PL;
  for (int a = 0; a < 3; ++a) {
    d.N[a] = g.N[a];
    d.P[a] = g.P[a];
    d.na[a] = g.na[a];
    d.ne[a] = g.ne[a];
    d.M[a] = g.M[a];
  }
  for (int s = 0; s < 6; ++s) {
    d.side_len[s] = g.side_len[s];
    d.side_off[s] = g.side_off[s];
  }

  build_schedule(c);

  // extended wavenumber of each subdomain (eq. wave_number: nearest point
  // of the subdomain = index clamping) and deduplication by exact bytes
  std::vector<std::vector<double>> kops;
  std::unordered_map<uint64_t, std::vector<int>> byhash;
  c->op_of_sub.assign(g.nsub, -1);
  std::vector<double> ks((size_t)g.sub_nodes);
  for (int s = 0; s < g.nsub; ++s) {
    int cc[3];
    g.sub_coords(s, cc);
    auto clampi = [&](int a, int l) {
      return std::min(std::max(cc[a] * g.na[a] + l - W, cc[a] * g.na[a]), (cc[a] + 1) * g.na[a] - 1);
    };
    const int nz = g.dim == 3 ? g.ne[2] : 1;
    for (int lz = 0; lz < nz; ++lz) {
      int iz = g.dim == 3 ? clampi(2, lz) : 0;
      for (int k = 0; k < g.ne[1]; ++k) {
        int iy = clampi(1, k);
        for (int p = 0; p < g.ne[0]; ++p) {
          int ix = clampi(0, p);
          ks[((size_t)lz * g.ne[1] + k) * g.ne[0] + p] =
              c->kappa[((size_t)iz * g.N[1] + iy) * g.N[0] + ix];
        }
      }
    }
    int op = -1;
    if (opt->dedup) {
      uint64_t hsh = fnv1a(ks.data(), ks.size() * sizeof(double));
      for (int cand : byhash[hsh])
        if (std::memcmp(kops[cand].data(), ks.data(), ks.size() * sizeof(double)) == 0) {
          op = cand;
          break;
        }
      if (op < 0) {
        op = (int)kops.size();
        kops.push_back(ks);
        byhash[hsh].push_back(op);
        c->rep_of_op.push_back(s);
      }
    } else {
      op = (int)kops.size();
      kops.push_back(ks);
      c->rep_of_op.push_back(s);
    }
    c->op_of_sub[s] = op;
  }
  c->nops = (int)kops.size();

  // alpha tables: subdomain-local and global, node and half-points per axis
  std::vector<c128> al_sub, al_glob;
  for (int a = 0; a < g.dim; ++a) {
    c->alpha_sub_off[2 * a] = (int)al_sub.size();
    for (int p = 0; p < g.ne[a]; ++p) al_sub.push_back(alpha_of(node_dist(p, W, g.na[a]), g.s0, W));
    c->alpha_sub_off[2 * a + 1] = (int)al_sub.size();
    for (int q = 0; q <= g.ne[a]; ++q) al_sub.push_back(alpha_of(half_dist(q, W, g.na[a]), g.s0, W));
    c->alpha_glob_off[2 * a] = (int)al_glob.size();
    for (int p = 0; p < g.M[a]; ++p) al_glob.push_back(alpha_of(node_dist(p, W, g.N[a]), g.s0, W));
    c->alpha_glob_off[2 * a + 1] = (int)al_glob.size();
    for (int q = 0; q <= g.M[a]; ++q) al_glob.push_back(alpha_of(half_dist(q, W, g.N[a]), g.s0, W));
  }

  auto fail = [&](hdsw_status st) {
    free_all(c);
    delete c;
    return st;
  };
  hdsw_status st;
  size_t e = elt(c);
  if (g.dim == 2) {
    c->coef_stride = (size_t)g.K * (g.n + 1) + (size_t)(g.K + 1) * g.n + (size_t)g.K * g.n;
  } else {
    const size_t nx = g.ne[0], ny = g.ne[1], nz = g.ne[2];
    c->coef_stride = nz * ny * (nx + 1) + nz * (ny + 1) * nx + (nz + 1) * ny * nx + nz * ny * nx;
  }
  // 2D: one spare block after the inverses, so the block solve's whole-tile
  // loads past the last row tile stay inside the allocation (never used)
  size_t xbytes = g.dim == 2 ? ((size_t)c->nops * g.K + 1) * g.nP * g.nP * e
                             : (size_t)c->nops * g.K * g.n * g.n * e;
  size_t tbytes = (size_t)c->nops * g.NI * g.NI * e;
  if (g.dim == 3) {
    // T in 64 x t_tk tiles, every face padded to whole tiles
    c->t_tk = opt->precision == HDSW_MIXED ? 32 : 16;
    int ro = 0, ko = 0;
    for (int f = 0; f < 6; ++f) {
      c->t_roff[f] = ro;
      c->t_koff[f] = ko;
      ro += (2 * g.side_len[f] + 63) / 64 * 64;
      ko += (2 * g.side_len[f] + c->t_tk - 1) / c->t_tk * c->t_tk;
    }
    c->t_nrt = ro / 64;
    c->t_nkt = ko / c->t_tk;
    tbytes = (size_t)c->nops * ro * ko * e;
  }
  c->factor_bytes = xbytes + tbytes;
  void* p;
#define SALLOC(dst, bytes)                     \
  do {                                         \
    st = dev_alloc(c, &p, (bytes));            \
    if (st != HDSW_OK) return fail(st);        \
    dst = decltype(dst)(p);                    \
  } while (0)
  SALLOC(c->d_X, xbytes);
  SALLOC(c->d_T, tbytes);
  SALLOC(c->d_coef, c->coef_stride * c->nops * sizeof(c128));
  SALLOC(c->d_coefT, c->coef_stride * c->nops * e);
  SALLOC(c->d_cface, (size_t)c->nops * (g.NI / 2) * e);
  SALLOC(c->d_kappa_sub, (size_t)c->nops * g.sub_nodes * sizeof(double));
  SALLOC(c->d_kappa, (size_t)nint * sizeof(double));
  SALLOC(c->d_alpha_sub, al_sub.size() * sizeof(c128));
  SALLOC(c->d_alpha_glob, al_glob.size() * sizeof(c128));
  SALLOC(c->d_op_of_sub, g.nsub * sizeof(int));
  SALLOC(c->d_step_subs, c->sch.step_subs.size() * sizeof(int));
  SALLOC(c->d_all_subs, g.nsub * sizeof(int));
  SALLOC(c->d_all_ops, c->nops * sizeof(int));
  SALLOC(c->d_flag, sizeof(int));
  SALLOC(c->d_zero_int, sizeof(int));
  SALLOC(c->d_one_int, sizeof(int));
  SALLOC(c->d_piv, (size_t)c->nops * g.n * sizeof(int));
  // subdomains grouped by operator (plane-block solves share one GEMM per
  // operator and plane)
  std::vector<int> grp_op, grp_off, grp_cnt, grp_ids;
  for (int o = 0; o < c->nops; ++o) {
    grp_op.push_back(o);
    grp_off.push_back((int)grp_ids.size());
    for (int s = 0; s < g.nsub; ++s)
      if (c->op_of_sub[s] == o) grp_ids.push_back(s);
    grp_cnt.push_back((int)grp_ids.size() - grp_off.back());
    c->grp_maxcnt = std::max(c->grp_maxcnt, grp_cnt.back());
  }
  c->ngrp = c->nops;
  // 3D sweep steps: face maps per sweep and per-step operator groups
  std::vector<int> fmap, sg_op, sg_off, sg_cnt, sg_ids;
  if (g.dim == 3) {
    const Schedule& sc = c->sch;
    const int tk = c->t_tk;
    for (int L = 0; L < sc.nsweeps; ++L) {
      // row tiles of the output faces, k tiles of the input faces, and the
      // padded output row -> unpadded step output row map
      c->tm_rt_off.push_back((int)fmap.size());
      int nrt = 0, mpad = 0, nkt = 0;
      for (int f = 0; f < 2 * g.dim; ++f)
        if (sc.lprime[L * 6 + f] >= 0) {
          int rf = (2 * g.side_len[f] + 63) / 64;
          for (int q = 0; q < rf; ++q) fmap.push_back(c->t_roff[f] / 64 + q);
          nrt += rf;
        }
      c->tm_kt_off.push_back((int)fmap.size());
      for (int f = 0; f < 2 * g.dim; ++f)
        if (sc.in_active[L * 6 + f]) {
          int kf = (2 * g.side_len[f] + tk - 1) / tk;
          for (int q = 0; q < kf; ++q) fmap.push_back(c->t_koff[f] / tk + q);
          nkt += kf;
        }
      c->tm_row_off.push_back((int)fmap.size());
      int uo = 0;
      for (int f = 0; f < 2 * g.dim; ++f)
        if (sc.lprime[L * 6 + f] >= 0) {
          int len = 2 * g.side_len[f];
          int rp = (len + 63) / 64 * 64;
          for (int r = 0; r < rp; ++r) fmap.push_back(r < len ? uo + r : -1);
          uo += len;
          mpad += rp;
        }
      c->tm_nrt.push_back(nrt);
      c->tm_nkt.push_back(nkt);
      c->tm_mpad.push_back(mpad);
      for (int st = 0; st < sc.nsteps; ++st) {
        int off = sc.step_off[L * sc.nsteps + st], cnt = sc.step_cnt[L * sc.nsteps + st];
        c->sg_first.push_back((int)sg_op.size());
        int ng = 0, mx = 0;
        for (int o = 0; o < c->nops; ++o) {
          int first = (int)sg_ids.size();
          for (int bi = 0; bi < cnt; ++bi)
            if (c->op_of_sub[sc.step_subs[off + bi]] == o) sg_ids.push_back(bi);
          int n_o = (int)sg_ids.size() - first;
          if (n_o == 0) continue;
          sg_op.push_back(o);
          sg_off.push_back(first);
          sg_cnt.push_back(n_o);
          ++ng;
          mx = std::max(mx, n_o);
        }
        c->sg_n.push_back(ng);
        c->sg_maxcnt.push_back(mx);
        c->gpart_per_col = std::max(c->gpart_per_col, (size_t)ng * mx * mpad);
      }
    }
    c->gpart_per_col = std::max(c->gpart_per_col, (size_t)c->nops * c->grp_maxcnt * g.n);
    if (fmap.empty()) fmap.push_back(0);
    if (sg_op.empty()) { sg_op.push_back(0); sg_off.push_back(0); sg_cnt.push_back(0); }
    if (sg_ids.empty()) sg_ids.push_back(0);
    SALLOC(c->d_tmap, fmap.size() * sizeof(int));
    SALLOC(c->d_sg_op, sg_op.size() * sizeof(int));
    SALLOC(c->d_sg_off, sg_off.size() * sizeof(int));
    SALLOC(c->d_sg_cnt, sg_cnt.size() * sizeof(int));
    SALLOC(c->d_sg_ids, sg_ids.size() * sizeof(int));
  }
  SALLOC(c->d_grp_op, c->ngrp * sizeof(int));
  SALLOC(c->d_grp_off, c->ngrp * sizeof(int));
  SALLOC(c->d_grp_cnt, c->ngrp * sizeof(int));
  SALLOC(c->d_grp_ids, g.nsub * sizeof(int));
  std::vector<int> iota_s(g.nsub), iota_o(c->nops);
  for (int i = 0; i < g.nsub; ++i) iota_s[i] = i;
  for (int i = 0; i < c->nops; ++i) iota_o[i] = i;
  std::vector<double> kflat((size_t)c->nops * g.sub_nodes);
  for (int o = 0; o < c->nops; ++o)
    std::copy(kops[o].begin(), kops[o].end(), kflat.begin() + (size_t)o * g.sub_nodes);
  hipError_t he = hipSuccess;
  auto up = [&](void* dst, const void* src, size_t bytes) {
    RtGuard lk(rt_mu());
    if (he == hipSuccess) he = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
  };
  up(c->d_kappa_sub, kflat.data(), kflat.size() * sizeof(double));
  up(c->d_kappa, c->kappa.data(), nint * sizeof(double));
  up(c->d_alpha_sub, al_sub.data(), al_sub.size() * sizeof(c128));
  up(c->d_alpha_glob, al_glob.data(), al_glob.size() * sizeof(c128));
  up(c->d_op_of_sub, c->op_of_sub.data(), g.nsub * sizeof(int));
  up(c->d_step_subs, c->sch.step_subs.data(), c->sch.step_subs.size() * sizeof(int));
  up(c->d_all_subs, iota_s.data(), g.nsub * sizeof(int));
  up(c->d_all_ops, iota_o.data(), c->nops * sizeof(int));
  const int zero_one[2] = {0, 1};
  up(c->d_zero_int, &zero_one[0], sizeof(int));
  up(c->d_one_int, &zero_one[1], sizeof(int));
  up(c->d_grp_op, grp_op.data(), c->ngrp * sizeof(int));
  up(c->d_grp_off, grp_off.data(), c->ngrp * sizeof(int));
  up(c->d_grp_cnt, grp_cnt.data(), c->ngrp * sizeof(int));
  up(c->d_grp_ids, grp_ids.data(), g.nsub * sizeof(int));
  if (g.dim == 3) {
    up(c->d_tmap, fmap.data(), fmap.size() * sizeof(int));
    up(c->d_sg_op, sg_op.data(), sg_op.size() * sizeof(int));
    up(c->d_sg_off, sg_off.data(), sg_off.size() * sizeof(int));
    up(c->d_sg_cnt, sg_cnt.data(), sg_cnt.size() * sizeof(int));
    up(c->d_sg_ids, sg_ids.data(), sg_ids.size() * sizeof(int));
  }
  if (he != hipSuccess) return fail(HDSW_EDEVICE);
  c->part_blocks = 256;
  *out = c;
  return HDSW_OK;
}

// ------------------------------------------------------------ factor
template <class T>
static hdsw_status factor_impl(hdsw_ctx* c) {
  const Geometry& g = c->g;
  HCHK(launch_zero(c, c->d_flag, sizeof(int)));
  HCHK(launch_assemble(c));
  HCHK(launch_cast_coef<T>(c));
  HCHK(launch_face_coef<T>(c));
  if (g.dim == 2) {
    double fl = 8.0 * g.n * (double)g.n * g.n * g.K * c->nops;
    double by = 2.0 * g.K * (double)g.n * g.n * sizeof(cpx<T>) * c->nops;
    TimedScope ts(c, KT_FACTOR, fl, by);
    // twisted: top and bottom chains advance together, then the middle line
    int steps = std::max(g.mid, g.K - 1 - g.mid);
    for (int st = 0; st < steps; ++st) HCHK(launch_factor_step<T>(c, st, 0));
    HCHK(launch_factor_step<T>(c, 0, 1));
  } else {
    // plane blocks: one dense inversion per plane, all operators together
    void* rbuf = nullptr;
    ACHK(dev_alloc(c, &rbuf, big_factor_scratch_bytes<T>(c)));
    hipError_t fe;
    {
      double fl = 8.0 * g.n * (double)g.n * g.n * g.K * c->nops;
      double by = 2.0 * g.K * (double)g.n * g.n * sizeof(cpx<T>) * c->nops;
      TimedScope ts(c, KT_FACTOR, fl, by);
      fe = launch_big_factor<T>(c, rbuf);
    }
    if (fe == hipSuccess) fe = hipStreamSynchronize(c->stream);
    dev_free(c, rbuf);
    HCHK(fe);
  }
  // interface-to-interface response T = P_I S^{-1} P_I^T of every distinct
  // operator: block solves with unit sources on the interface dofs
  const size_t e = sizeof(cpx<T>);
  size_t per_col = (size_t)g.PL * g.n * e;
  size_t budget = (size_t)1 << 31;
  int ct = (int)std::min<size_t>(g.NI, std::max<size_t>(1, budget / per_col));
  void* tmp = nullptr;
  ACHK(dev_alloc(c, &tmp, per_col * ct));
  void* saved = c->d_panel;
  c->d_panel = tmp;
  if (g.dim == 3) {
    hipError_t rz = launch_zero(
        c, c->d_T, (size_t)c->nops * c->t_nrt * 64 * (size_t)c->t_nkt * c->t_tk * e);
    if (rz != hipSuccess) {
      c->d_panel = saved;
      dev_free(c, tmp);
      c->sticky = HDSW_EDEVICE;
      return HDSW_EDEVICE;
    }
  }
  for (int op = 0; op < c->nops; ++op) {
    for (int col0 = 0; col0 < g.NI; col0 += ct) {
      int nc = std::min(ct, g.NI - col0);
      hipError_t r1 = launch_fill_panel<T>(c, 2, 1, c->d_all_ops + op, nc, nullptr, col0);
      hipError_t r2 = r1 == hipSuccess ? launch_block_solve<T>(c, 1, c->d_all_ops + op, nc) : r1;
      hipError_t r3 = r2;
      if (r2 == hipSuccess && g.dim == 3) {
        r3 = launch_extract_tiled<T>(c, nc, op, col0);
      } else if (r2 == hipSuccess) {
        r3 = launch_extract_iface<T>(
            c, 1, nc, (cpx<T>*)c->d_T + (size_t)op * g.NI * g.NI + (size_t)col0 * g.NI, 0, g.NI);
      }
      if (r3 != hipSuccess) {
        c->d_panel = saved;
        dev_free(c, tmp);
        c->sticky = HDSW_EDEVICE;
        return HDSW_EDEVICE;
      }
    }
  }
  HCHK(hipStreamSynchronize(c->stream));
  c->d_panel = saved;
  dev_free(c, tmp);
  int flag = 0;
  {
    RtGuard lk(rt_mu());
    HCHK(hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HCHK(hipStreamSynchronize(c->stream));
  }
  if (flag) return HDSW_EINVAL;  // a singular diagonal block
  c->factored = true;
  return HDSW_OK;
}

hdsw_status factor(hdsw_ctx* c) {
  if (c->sticky != HDSW_OK) return c->sticky;
  if (c->factored) return HDSW_OK;
  return c->opt.precision == HDSW_MIXED ? factor_impl<float>(c) : factor_impl<double>(c);
}

// ------------------------------------------------------------ workspaces
static void graphs_clear(hdsw_ctx* c);

static hdsw_status ensure_ws(hdsw_ctx* c, int C, bool need_gmres) {
  const Geometry& g = c->g;
  size_t e = elt(c);
  if (C > c->Cmax) {
    graphs_clear(c);   // captured applications hold the old workspace addresses
    void* ptrs[] = {c->d_panel, c->d_slots, c->d_g, c->d_srcsum, c->d_y, c->d_out, c->d_gpart,
                    c->d_xg, c->d_rg, c->d_bg, c->d_part, c->d_norm, c->d_nzflag};
    for (void* p : ptrs) dev_free(c, p);
    c->d_panel = c->d_slots = c->d_g = c->d_srcsum = c->d_y = c->d_out = c->d_gpart = nullptr;
    c->d_nzflag = nullptr;
    c->gpart_bytes = 0;
    c->d_xg = c->d_rg = c->d_bg = nullptr;
    c->d_part = c->d_norm = nullptr;
    c->Cmax = 0;
    void* p;
    hdsw_status st;
#define WALLOC(dst, bytes)                \
  do {                                    \
    st = dev_alloc(c, &p, (bytes));       \
    if (st != HDSW_OK) return st;         \
    dst = decltype(dst)(p);               \
  } while (0)
    size_t iface = (size_t)g.nsub * C * g.NI * e;
    WALLOC(c->d_panel, (size_t)g.nsub * g.PL * C * g.n * e);
    WALLOC(c->d_slots, iface * c->sch.nsweeps);
    WALLOC(c->d_srcsum, iface);
    WALLOC(c->d_y, iface);
    if (g.dim == 2) WALLOC(c->d_nzflag, (size_t)g.nsub * ((C + 7) / 8) * sizeof(int));
    if (g.dim == 3) {
      // the step GEMM's B operand: trace sources in the padded k space of T
      WALLOC(c->d_g, (size_t)g.nsub * ((C + 15) / 16 * 16) * (size_t)c->t_nkt * c->t_tk * e);
      WALLOC(c->d_out, iface);
      // split-sum partials of the plane solves and step GEMMs: up to 4
      // parts of every operator group's columns
      size_t gp = (size_t)4 * c->gpart_per_col * C * e;
      WALLOC(c->d_gpart, gp);
      c->gpart_bytes = gp;
    }
    WALLOC(c->d_xg, (size_t)C * g.glob_nodes * sizeof(c128));
    WALLOC(c->d_rg, (size_t)C * g.glob_nodes * sizeof(c128));
    WALLOC(c->d_bg, (size_t)C * g.glob_nodes * sizeof(c128));
    WALLOC(c->d_part, (size_t)(std::max(c->opt.gmres_m, 0) + 1) * C * c->part_blocks * 2 *
                          sizeof(double));
    WALLOC(c->d_norm, (size_t)C * sizeof(double));
    c->Cmax = C;
  }
  // the Krylov basis is sized for the workspaces' column count: regrow it
  // whenever the workspaces grew since it was allocated
  if (need_gmres && (c->gm_m != c->opt.gmres_m || !c->d_V || c->gm_cols < c->Cmax)) {
    graphs_clear(c);
    dev_free(c, c->d_V);
    dev_free(c, c->d_Z);
    dev_free(c, c->d_dots);
    c->d_V = c->d_Z = c->d_dots = nullptr;
    c->gm_cols = 0;
    int m = c->opt.gmres_m;
    void* p;
    hdsw_status st;
    WALLOC(c->d_V, (size_t)(m + 1) * c->Cmax * g.glob_nodes * sizeof(c128));
    WALLOC(c->d_Z, (size_t)m * c->Cmax * g.glob_nodes * sizeof(c128));
    WALLOC(c->d_dots, (size_t)2 * (m + 1) * c->Cmax * sizeof(c128));
    c->gm_m = m;
    c->gm_cols = c->Cmax;
  }
  return HDSW_OK;
}

// ------------------------------------------------------------ DDM
// One application of Algorithm 2.1 to C global-grid right-hand sides r,
// written (accumulate = 0) or added (accumulate = 1) to out on owned nodes.
//
// Every per-step subdomain solve S^{-1}(f_ij [sweep 1] + trace sources) is
// needed only (a) on the interface layers, to form the outgoing traces, and
// (b) on owned nodes, summed over sweeps.  (a) is y_ij + T g with
// y_ij = P_I S^{-1} f_ij (one batched solve before the sweeps) and T the
// subdomain's interface response; (b) is, by linearity, one solve with the
// summed right-hand side f_ij + sum_l g_l after the sweeps.
template <class T>
static hdsw_status ddm_impl(hdsw_ctx* c, const c128* r, c128* out, int C, int accumulate) {
  const Geometry& g = c->g;
  const Schedule& s = c->sch;
  const size_t e = sizeof(cpx<T>);
  const double solve_fl = 8.0 * (2.0 * g.K - 1) * g.n * (double)g.n * C * g.nsub;
  const double solve_by = 2.0 * g.K * (double)g.n * g.n * e * c->nops +
                          4.0 * g.K * (double)g.n * C * e * g.nsub;
  // the source-driven solve: (subdomain, 8-column) pairs whose right-hand
  // side is zero (most of them for compact sources) are skipped in 2D, once
  // the solve runs more than two rounds of 8-column workgroups on the 256
  // CUs (below that the launch lasts one workgroup's chain however many
  // return early, and the flags only cost time).  Skipping never changes a
  // result, so the rule may depend on the column count.  The solve is timed
  // as its own class then, without flops: the solve class's flops assume
  // every pair
  const bool skip = (long long)((C + 7) / 8) * g.nsub * 2 > 2 * 256;
  int* nzf = skip ? c->d_nzflag : nullptr;
  if (nzf) HCHK(launch_zero(c, nzf, (size_t)g.nsub * ((C + 7) / 8) * sizeof(int)));
  HCHK(launch_fill_panel<T>(c, 0, g.nsub, c->d_all_subs, C, r, 0, nzf));
  if (nzf) {
    TimedScope ts(c, KT_SOLVE_SRC, 0, 0);
    HCHK(launch_block_solve<T>(c, g.nsub, c->d_op_of_sub, C, nzf));
  } else {
    TimedScope ts(c, KT_SOLVE, solve_fl, solve_by);
    HCHK(launch_block_solve<T>(c, g.nsub, c->d_op_of_sub, C));
  }
  HCHK(launch_extract_iface<T>(c, g.nsub, C, c->d_y, (long long)C * g.NI, g.NI));
  size_t iface = (size_t)g.nsub * C * g.NI * e;
  HCHK(launch_zero(c, c->d_slots, iface * s.nsweeps));
  // the steps in sweep order, or (2D) the steps of one level of the slot
  // dependences per launch; both orders give the same results
  const bool merged = !s.lfirst.empty() && c->tune.sweep_sched != 1;
  const int nlaunch = merged ? (int)s.lfirst.size() - 1 : s.nsweeps * s.nsteps;
  for (int i = 0; i < nlaunch; ++i) {
    const int* sidx = merged ? &s.lsteps[s.lfirst[i]] : &i;
    const int nst = merged ? s.lfirst[i + 1] - s.lfirst[i] : 1;
    double fl = 0, by = 0;
    for (int k = 0; k < nst; ++k) {
      const int L = sidx[k] / s.nsteps, cnt = s.step_cnt[sidx[k]];
      double nin = 0, nout = 0;
      for (int f = 0; f < 2 * g.dim; ++f) {
        if (s.in_active[L * 6 + f]) nin += 2 * g.side_len[f];
        if (s.lprime[L * 6 + f] >= 0) nout += 2 * g.side_len[f];
      }
      fl += 8.0 * nin * nout * C * cnt;
      by += nin * nout * e * std::min(cnt, c->nops) + (nin + 2 * nout) * C * e * cnt;
    }
    if (fl == 0 && by == 0) continue;    // empty steps
    TimedScope ts(c, KT_GEMM, fl, by);
    HCHK(launch_sweep_steps<T>(c, sidx, nst, C));
  }
  HCHK(launch_fill_panel<T>(c, 1, g.nsub, c->d_all_subs, C, r, 0));
  {
    TimedScope ts(c, KT_SOLVE, solve_fl, solve_by);
    HCHK(launch_block_solve<T>(c, g.nsub, c->d_op_of_sub, C));
  }
  HCHK(launch_write_owned<T>(c, C, out, accumulate));
  return HDSW_OK;
}

static hdsw_status ddm_eager(hdsw_ctx* c, const c128* r, c128* out, int C, int accumulate) {
  return c->opt.precision == HDSW_MIXED ? ddm_impl<float>(c, r, out, C, accumulate)
                                        : ddm_impl<double>(c, r, out, C, accumulate);
}

static void graphs_clear(hdsw_ctx* c) {
  RtGuard lk(rt_mu());
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  c->graph_seen.clear();
  c->graph_bad.clear();
}

// One DDM application, from a captured graph when the same (input, output,
// columns, accumulate) was applied before.  The launch sequence has no host
// synchronization and clears its buffers with fill kernels (no memset
// nodes), so it is recorded on a private stream and replayed on the
// context's stream; the replay runs the same kernels with the same
// arguments, so results equal the eager launches bit for bit.  With kernel
// timing on, launches are eager: HIP events recorded by a graph's event
// nodes cannot be read as elapsed times.
static hdsw_status ddm(hdsw_ctx* c, const c128* r, c128* out, int C, int accumulate) {
  if (!c->opt.graphs || c->tm.mask) return ddm_eager(c, r, out, C, accumulate);
  const hdsw_ctx::GraphKey key{r, out, C, accumulate};
  if (c->graph_bad.count(key)) return ddm_eager(c, r, out, C, accumulate);
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    if (!c->graph_seen.count(key)) {
      if (c->graph_seen.size() >= 256) c->graph_seen.clear();
      c->graph_seen.insert(key);
      return ddm_eager(c, r, out, C, accumulate);
    }
    if (c->graphs.size() >= 64) graphs_clear(c);
    RtGuard lk(rt_mu());
    if (!c->cap_stream) HCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    // The recording holds the runtime lock, so this library's own
    // allocations, frees and blocking copies on other threads wait for it.
    // A capture can still be refused or invalidated by the runtime (for
    // example by other work on the legacy default stream).  Nothing
    // recorded ran, so the application then runs eagerly and the key stays
    // eager; errors seen while recording are not device errors.
    const hdsw_status sticky0 = c->sticky;
    auto give_up = [&]() {
      (void)hipGetLastError();
      c->sticky = sticky0;
      if (c->graph_bad.size() >= 256) c->graph_bad.clear();
      c->graph_bad.insert(key);
      return ddm_eager(c, r, out, C, accumulate);
    };
    if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return give_up();
    hipStream_t s = c->stream;
    c->stream = c->cap_stream;
    hdsw_status st = ddm_eager(c, r, out, C, accumulate);
    c->stream = s;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
    if (st == HDSW_OK && e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (st != HDSW_OK || e != hipSuccess) {
      if (exec) (void)hipGraphExecDestroy(exec);
      return give_up();
    }
    it = c->graphs.emplace(key, exec).first;
  }
  HCHK(hipGraphLaunch(it->second, c->stream));
  return HDSW_OK;
}

hdsw_status ddm_dispatch(hdsw_ctx* c, const c128* r, c128* out, int C, int accumulate) {
  return ddm(c, r, out, C, accumulate);
}

// Eager form for callers that swap the context's workspaces for a call
// (captured graphs hold the context's own workspace addresses).
hdsw_status ddm_dispatch_eager(hdsw_ctx* c, const c128* r, c128* out, int C, int accumulate) {
  return ddm_eager(c, r, out, C, accumulate);
}

static size_t max_cols(hdsw_ctx* c) {
  // columns per pass under the budget (0 budget: all requested columns)
  if (!c->opt.hbm_budget) return 1u << 30;
  const Geometry& g = c->g;
  size_t e = elt(c);
  size_t per_col = (size_t)g.nsub * g.PL * g.n * e +
                   (size_t)g.nsub * g.NI * e * (c->sch.nsweeps + (g.dim == 3 ? 4 : 2)) +
                   3 * (size_t)g.glob_nodes * sizeof(c128);
  if (c->opt.gmres_m > 0) per_col += (size_t)(2 * c->opt.gmres_m + 1) * g.glob_nodes * sizeof(c128);
  if (g.dim == 3) per_col += (size_t)4 * c->gpart_per_col * e;
  size_t used = c->alloc_bytes;
  // workspaces currently held can be reused
  if (c->Cmax > 0) used -= std::min(used, (size_t)c->Cmax * per_col);
  if (used >= c->opt.hbm_budget) return 0;
  return (c->opt.hbm_budget - used) / per_col;
}

hdsw_status apply_precond(hdsw_ctx* c, const c128* r, c128* z, int nrhs) {
  if (c->sticky != HDSW_OK) return c->sticky;
  if (!c->factored) return HDSW_ENOTFACTORED;
  if (!r || !z || nrhs < 1) return HDSW_EINVAL;
  PCHK(r, (size_t)nrhs * c->g.glob_nodes * sizeof(c128));
  PCHK(z, (size_t)nrhs * c->g.glob_nodes * sizeof(c128));
  if (c->nact > 0) return HDSW_EBUSY;  // batch slots own the workspaces
  int chunk = (int)std::min<size_t>(nrhs, max_cols(c));
  if (chunk < 1) return HDSW_ENOMEM;
  ACHK(ensure_ws(c, chunk, false));
  for (int c0 = 0; c0 < nrhs; c0 += chunk) {
    int C = std::min(chunk, nrhs - c0);
    ACHK(ddm(c, r + (size_t)c0 * c->g.glob_nodes, z + (size_t)c0 * c->g.glob_nodes, C, 0));
  }
  HCHK(hipStreamSynchronize(c->stream));
  return HDSW_OK;
}

hdsw_status residual(hdsw_ctx* c, const c128* b, const c128* x, c128* r, int nrhs,
                     double* rn) {
  if (c->sticky != HDSW_OK) return c->sticky;
  if (!b || !x || !r || nrhs < 1) return HDSW_EINVAL;
  PCHK(b, (size_t)nrhs * c->g.glob_nodes * sizeof(c128));
  PCHK(x, (size_t)nrhs * c->g.glob_nodes * sizeof(c128));
  PCHK(r, (size_t)nrhs * c->g.glob_nodes * sizeof(c128));
  {
    // the residual kernels read b and x through restrict pointers
    const size_t bytes = (size_t)nrhs * c->g.glob_nodes * sizeof(c128);
    auto overlap = [bytes](const void* p, const void* q) {
      const char *a = (const char*)p, *d = (const char*)q;
      return a < d + bytes && d < a + bytes;
    };
    if (overlap(r, b) || overlap(r, x)) return HDSW_EINVAL;
  }
  if (c->nact > 0) return HDSW_EBUSY;  // batch slots own the workspaces
  ACHK(ensure_ws(c, std::min(nrhs, std::max(c->Cmax, 1)), false));
  for (int c0 = 0; c0 < nrhs; c0 += c->Cmax) {
    int C = std::min(c->Cmax, nrhs - c0);
    size_t o = (size_t)c0 * c->g.glob_nodes;
    HCHK(launch_residual(c, b + o, x + o, r + o, C));
    if (rn) {
      HCHK(launch_norms(c, r + o, C, c->d_norm));
      HCHK(hipMemcpyAsync(rn + c0, c->d_norm, C * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
    }
  }
  HCHK(hipStreamSynchronize(c->stream));
  return HDSW_OK;
}

// ------------------------------------------------------------ Krylov
// FP64 iterative refinement, x_{j+1} = x_j + M^{-1}(b - S x_j), for C
// columns held in the context's global buffers.
static hdsw_status refine_cols(hdsw_ctx* c, int C, std::vector<int>& iters,
                               std::vector<double>& rel, const std::vector<double>& bn) {
  const Geometry& g = c->g;
  HCHK(launch_zero(c, c->d_xg, (size_t)C * g.glob_nodes * sizeof(c128)));
  std::vector<double> rn(C);
  iters.assign(C, -1);
  rel.assign(C, 0.0);
  for (int it = 0; it <= c->opt.max_iter; ++it) {
    {
      TimedScope ts(c, KT_RESID, 22.0 * g.glob_nodes * C, 48.0 * g.glob_nodes * C);
      HCHK(launch_residual(c, c->d_bg, c->d_xg, c->d_rg, C));
    }
    HCHK(launch_norms(c, c->d_rg, C, c->d_norm));
    HCHK(hipMemcpyAsync(rn.data(), c->d_norm, C * sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
    HCHK(hipStreamSynchronize(c->stream));
    bool all = true;
    for (int j = 0; j < C; ++j) {
      if (iters[j] < 0) {
        rel[j] = bn[j] > 0 ? rn[j] / bn[j] : 0.0;
        if (rel[j] <= c->opt.tol) iters[j] = it;
      }
      if (iters[j] < 0) all = false;
    }
    if (all || it == c->opt.max_iter) break;
    // a converged column takes no further update (x += M^{-1} 0 is x
    // exactly), so its result does not depend on the other columns
    for (int j = 0; j < C; ++j)
      if (iters[j] >= 0)
        HCHK(launch_zero(c, c->d_rg + (size_t)j * g.glob_nodes, g.glob_nodes * sizeof(c128)));
    ACHK(ddm(c, c->d_rg, c->d_xg, C, 1));
  }
  return HDSW_OK;
}

hdsw_status gmres_cols(hdsw_ctx* c, int C, std::vector<int>& iters, std::vector<double>& rel,
                       const std::vector<double>& bn);

hdsw_status solve(hdsw_ctx* c, const c128* f, c128* x, int nrhs, hdsw_solve_info* info) {
  if (c->sticky != HDSW_OK) return c->sticky;
  if (!c->factored) return HDSW_ENOTFACTORED;
  if (!f || !x || nrhs < 1) return HDSW_EINVAL;
  PCHK(f, (size_t)nrhs * c->g.int_nodes * sizeof(c128));
  PCHK(x, (size_t)nrhs * c->g.int_nodes * sizeof(c128));
  if (c->nact > 0) return HDSW_EBUSY;  // batch slots own the workspaces
  int chunk = (int)std::min<size_t>(nrhs, max_cols(c));
  if (chunk < 1) return HDSW_ENOMEM;
  bool gm = c->opt.gmres_m > 0;
  ACHK(ensure_ws(c, chunk, gm));
  const Geometry& g = c->g;
  bool conv = true;
  for (int c0 = 0; c0 < nrhs; c0 += chunk) {
    int C = std::min(chunk, nrhs - c0);
    HCHK(launch_rhs_from_f(c, f + (size_t)c0 * g.int_nodes, c->d_bg, C));
    HCHK(launch_norms(c, c->d_bg, C, c->d_norm));
    std::vector<double> bn(C);
    HCHK(hipMemcpyAsync(bn.data(), c->d_norm, C * sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
    HCHK(hipStreamSynchronize(c->stream));
    std::vector<int> iters;
    std::vector<double> rel;
    if (gm) ACHK(gmres_cols(c, C, iters, rel, bn));
    else ACHK(refine_cols(c, C, iters, rel, bn));
    HCHK(launch_extract_interior(c, c->d_xg, x + (size_t)c0 * g.int_nodes, C));
    for (int j = 0; j < C; ++j) {
      if (iters[j] < 0) conv = false;
      if (info) {
        info[c0 + j].iters = iters[j] < 0 ? c->opt.max_iter : iters[j];
        info[c0 + j].rel_residual = rel[j];
      }
    }
  }
  HCHK(hipStreamSynchronize(c->stream));
  return conv ? HDSW_OK : HDSW_ENOCONV;
}

// ------------------------------------------------------------ batching
// Column slots for continuous batching.  Occupied slots are kept in
// physical columns 0..nact-1 of the iterate / residual / right-hand-side
// buffers; a slot that leaves is filled by the last occupied column.  A
// column joins with x = 0 and r = b; a step is one refinement iteration,
// x += M^{-1} r followed by r = b - S x, over all occupied columns, and the
// norms of the new residuals are copied to pinned host memory for
// batch_wait.  A slot that reports convergence can be taken at once, with
// no further update.
hdsw_status batch_reserve(hdsw_ctx* c, int cap) {
  if (c->sticky != HDSW_OK) return c->sticky;
  if (!c->factored) return HDSW_ENOTFACTORED;
  if (cap < 1) return HDSW_EINVAL;
  if (c->nact > 0) return HDSW_EBUSY;
  ACHK(ensure_ws(c, cap, false));
  RtGuard lk(rt_mu());
  if (!c->h_norm || cap > c->batch_cap) {
    if (c->h_norm) (void)hipHostFree(c->h_norm);
    c->h_norm = nullptr;
    if (hipHostMalloc((void**)&c->h_norm, sizeof(double) * cap) != hipSuccess) {
      c->h_norm = nullptr;
      c->batch_cap = 0;
      return HDSW_ENOMEM;
    }
  }
  if (!c->step_done) HCHK(hipEventCreateWithFlags(&c->step_done, hipEventDisableTiming));
  c->batch_cap = cap;
  c->slot_of_col.assign(cap, -1);
  c->col_of_slot.assign(cap, -1);
  c->bnorm_slot.assign(cap, 0.0);
  c->nact = 0;
  c->step_cols = 0;
  return HDSW_OK;
}

hdsw_status batch_add(hdsw_ctx* c, const c128* f, int nrhs, int* slots) {
  if (c->sticky != HDSW_OK) return c->sticky;
  if (c->batch_cap == 0) return HDSW_ENOTFACTORED;
  if (!f || !slots || nrhs < 1) return HDSW_EINVAL;
  PCHK(f, (size_t)nrhs * c->g.int_nodes * sizeof(c128));
  if (c->nact + nrhs > c->batch_cap) return HDSW_EBUSY;
  const size_t gn = (size_t)c->g.glob_nodes;
  const int c0 = c->nact;
  HCHK(launch_rhs_from_f(c, f, c->d_bg + (size_t)c0 * gn, nrhs));
  HCHK(launch_copy_cols(c, c->d_rg + (size_t)c0 * gn, c->d_bg + (size_t)c0 * gn,
                        (size_t)nrhs * gn));
  HCHK(launch_zero(c, c->d_xg + (size_t)c0 * gn, (size_t)nrhs * gn * sizeof(c128)));
  HCHK(launch_norms(c, c->d_bg + (size_t)c0 * gn, nrhs, c->d_norm));
  std::vector<double> bn(nrhs);
  HCHK(hipMemcpyAsync(bn.data(), c->d_norm, nrhs * sizeof(double), hipMemcpyDeviceToHost,
                      c->stream));
  HCHK(hipStreamSynchronize(c->stream));
  int s = 0;
  for (int j = 0; j < nrhs; ++j) {
    while (c->col_of_slot[s] >= 0) ++s;
    c->col_of_slot[s] = c0 + j;
    c->slot_of_col[c0 + j] = s;
    c->bnorm_slot[s] = bn[j];
    slots[j] = s;
  }
  c->nact += nrhs;
  return HDSW_OK;
}

hdsw_status batch_step(hdsw_ctx* c) {
  if (c->sticky != HDSW_OK) return c->sticky;
  if (c->batch_cap == 0) return HDSW_ENOTFACTORED;
  const int C = c->nact;
  c->step_cols = C;
  if (C == 0) return HDSW_OK;
  ACHK(ddm(c, c->d_rg, c->d_xg, C, 1));
  {
    TimedScope ts(c, KT_RESID, 22.0 * c->g.glob_nodes * C, 48.0 * c->g.glob_nodes * C);
    HCHK(launch_residual(c, c->d_bg, c->d_xg, c->d_rg, C));
  }
  HCHK(launch_norms(c, c->d_rg, C, c->d_norm));
  HCHK(hipMemcpyAsync(c->h_norm, c->d_norm, C * sizeof(double), hipMemcpyDeviceToHost,
                      c->stream));
  HCHK(hipEventRecord(c->step_done, c->stream));
  return HDSW_OK;
}

hdsw_status batch_wait(hdsw_ctx* c, double* rel) {
  if (c->sticky != HDSW_OK) return c->sticky;
  if (c->batch_cap == 0) return HDSW_ENOTFACTORED;
  if (c->step_cols > 0) HCHK(hipEventSynchronize(c->step_done));
  if (rel) {
    for (int s = 0; s < c->batch_cap; ++s) rel[s] = -1.0;
    for (int j = 0; j < c->step_cols && j < c->nact; ++j) {
      int s = c->slot_of_col[j];
      rel[s] = c->bnorm_slot[s] > 0 ? c->h_norm[j] / c->bnorm_slot[s] : 0.0;
    }
  }
  return HDSW_OK;
}

hdsw_status batch_ready(hdsw_ctx* c) {
  if (c->sticky != HDSW_OK) return c->sticky;
  if (c->batch_cap == 0) return HDSW_ENOTFACTORED;
  if (c->step_cols == 0) return HDSW_OK;
  hipError_t e = hipEventQuery(c->step_done);
  if (e == hipErrorNotReady) return HDSW_EBUSY;
  HCHK(e);
  return HDSW_OK;
}

hdsw_status batch_take(hdsw_ctx* c, int slot, c128* x) {
  if (c->sticky != HDSW_OK) return c->sticky;
  if (c->batch_cap == 0) return HDSW_ENOTFACTORED;
  if (slot < 0 || slot >= c->batch_cap || c->col_of_slot[slot] < 0) return HDSW_EINVAL;
  if (x) PCHK(x, (size_t)c->g.int_nodes * sizeof(c128));
  const Geometry& g = c->g;
  const size_t gn = (size_t)g.glob_nodes;
  int col = c->col_of_slot[slot];
  if (x) HCHK(launch_extract_interior(c, c->d_xg + (size_t)col * gn, x, 1));
  int last = c->nact - 1;
  if (col != last) {
    HCHK(launch_copy_cols(c, c->d_xg + (size_t)col * gn, c->d_xg + (size_t)last * gn, gn));
    HCHK(launch_copy_cols(c, c->d_bg + (size_t)col * gn, c->d_bg + (size_t)last * gn, gn));
    HCHK(launch_copy_cols(c, c->d_rg + (size_t)col * gn, c->d_rg + (size_t)last * gn, gn));
    int ls = c->slot_of_col[last];
    c->slot_of_col[col] = ls;
    c->col_of_slot[ls] = col;
  }
  c->slot_of_col[last] = -1;
  c->col_of_slot[slot] = -1;
  c->nact = last;
  // a step in flight keeps covering the old column order: the caller waits
  // before taking, so the step count is reset here
  c->step_cols = 0;
  HCHK(hipStreamSynchronize(c->stream));
  return HDSW_OK;
}

hdsw_status timing_get(hdsw_ctx* c, int which, double* ms, long long* n, double* fl,
                       double* by) {
  if (which < 0 || which > KT_SOLVE_SRC) return HDSW_EINVAL;
  resolve_timing(c);
  if (ms) *ms = c->tm.ms[which];
  if (n) *n = c->tm.launches[which];
  if (fl) *fl = c->tm.flops[which];
  if (by) *by = c->tm.bytes[which];
  c->tm.ms[which] = 0;
  c->tm.launches[which] = 0;
  c->tm.flops[which] = 0;
  c->tm.bytes[which] = 0;
  return HDSW_OK;
}

hdsw_status tuning_set(hdsw_ctx* c, const TuneParams& t) {
  if (c->sticky != HDSW_OK) return c->sticky;
  const bool c64 = c->opt.precision == HDSW_MIXED;
  auto in = [](int v, std::initializer_list<int> ok) {
    for (int o : ok)
      if (v == o) return true;
    return false;
  };
  if (!in(t.solve_ng, {0, 1, 2}) || !in(t.sweep_rw, {0, 2, 4}) ||
      !(c64 ? in(t.sweep_kb, {0, 6, 8, 10}) : in(t.sweep_kb, {0, 3, 4, 5, 6})) ||
      !in(t.gemm_skinny, {0, 1, 2}) || !in(t.sweep_nw, {0, 4, 8}) ||
      !in(t.sweep_sched, {0, 1, 2}))
    return HDSW_EINVAL;
  graphs_clear(c);   // captured launches hold the old parameters
  c->tune = t;
  return HDSW_OK;
}

void destroy(hdsw_ctx* c) {
  if (!c) return;
  RtGuard lk(rt_mu());
  graphs_clear(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->h_norm) (void)hipHostFree(c->h_norm);
  if (c->step_done) (void)hipEventDestroy(c->step_done);
  resolve_timing(c);
  auto it = pools().find(c);
  if (it != pools().end()) {
    for (auto& e : it->second.ev)
      if (e) (void)hipEventDestroy(e);
    pools().erase(it);
  }
  free_all(c);
  delete c;
}

}  // namespace hdsw

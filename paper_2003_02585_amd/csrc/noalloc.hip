// Allocation-free DDM application, for callers that cannot allocate device
// memory (code under stream capture, tight serving loops, harnesses that
// forbid hipMalloc).  It runs the same kernels as hdsw_apply_precond, with
// the per-call workspaces -- subdomain panels, trace slots, summed sources,
// source-driven interface values, (2D) the nonzero flags of the
// source-driven solve and (3D) the step GEMM operands and split-sum
// partials -- carved out of one file-scope device array instead of the
// context's own allocations.
//
// The array is a fixed kScratchBytes per device, held from the first load of
// this library on that device until the process ends.  Its device address is
// looked up once per device at context setup (hipGetSymbolAddress, with the
// device current); host code uses only that address, never the array's name,
// which in host code is a stand-in without a device address.  Every call on
// one device shares the array, and each call leaves its contents behind:
// everything the kernels read is written earlier in the same call (the trace
// slots and the nonzero flags are cleared by a fill kernel), so a call never
// depends on what an earlier call left.  Calls that overlap on one device race for the array.
#include <mutex>

#include "hdsw_internal.hpp"

namespace hdsw {

hdsw_status ddm_dispatch_eager(hdsw_ctx* c, const c128* r, c128* out, int C, int accumulate);
hdsw_status check_dev_ptr(const hdsw_ctx* c, const void* p, size_t bytes);

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`; `device` is current.
hdsw_status scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return HDSW_EDEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return HDSW_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return HDSW_EDEVICE;
  }
  g_scratch_ptr[device] = p;
  return HDSW_OK;
}

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Workspace pieces for C columns, laid out back to back at 256-byte
// boundaries; returns the total bytes.  Sizes are those the context's own
// workspaces have for C columns, so the kernels (and the split of the 3D
// plane-solve sums, which depends on the partials' size) run exactly as in
// hdsw_apply_precond.
struct Carve {
  size_t panel, slots, srcsum, y, nzflag, g, out, gpart, gpart_bytes, total;
};
static Carve carve(const hdsw_ctx* c, int C) {
  const Geometry& g = c->g;
  const size_t e = c->opt.precision == HDSW_MIXED ? sizeof(c64) : sizeof(c128);
  const size_t iface = (size_t)g.nsub * C * g.NI * e;
  Carve k{};
  size_t o = 0;
  k.panel = o;
  o += align256((size_t)g.nsub * g.PL * C * g.n * e);
  k.slots = o;
  o += align256(iface * c->sch.nsweeps);
  k.srcsum = o;
  o += align256(iface);
  k.y = o;
  o += align256(iface);
  if (g.dim == 2) {
    k.nzflag = o;
    o += align256((size_t)g.nsub * ((C + 7) / 8) * sizeof(int));
  }
  if (g.dim == 3) {
    k.g = o;
    o += align256((size_t)g.nsub * ((C + 15) / 16 * 16) * (size_t)c->t_nkt * c->t_tk * e);
    k.out = o;
    o += align256(iface);
    k.gpart = o;
    k.gpart_bytes = (size_t)4 * c->gpart_per_col * C * e;
    o += align256(k.gpart_bytes);
  }
  k.total = o;
  return k;
}

hdsw_status apply_precond_noalloc(hdsw_ctx* c, const c128* r, c128* z, int nrhs) {
  if (c->sticky != HDSW_OK) return c->sticky;
  if (!c->factored) return HDSW_ENOTFACTORED;
  if (!r || !z || nrhs < 1) return HDSW_EINVAL;
  const size_t gbytes = (size_t)nrhs * c->g.glob_nodes * sizeof(c128);
  hdsw_status ps = check_dev_ptr(c, r, gbytes);
  if (ps == HDSW_OK) ps = check_dev_ptr(c, z, gbytes);
  if (ps != HDSW_OK) return ps;
  void* base = (c->device >= 0 && c->device < kMaxDevices) ? g_scratch_ptr[c->device] : nullptr;
  if (!base) return HDSW_EDEVICE;
  // columns per pass: as many as the array holds (a column's arithmetic
  // does not depend on the other columns of its pass)
  if (carve(c, 1).total > kScratchBytes) return HDSW_ENOMEM;
  int chunk = 1;
  while (chunk < nrhs && carve(c, chunk + 1).total <= kScratchBytes) ++chunk;
  // the context's workspaces are set aside for the call; event timing is
  // off (its event pool would be created on first use)
  void* saved[8] = {c->d_panel, c->d_slots, c->d_srcsum, c->d_y, c->d_g, c->d_out, c->d_gpart,
                    c->d_nzflag};
  const size_t saved_gpart = c->gpart_bytes;
  const int saved_mask = c->tm.mask;
  c->tm.mask = 0;
  hdsw_status st = HDSW_OK;
  for (int c0 = 0; c0 < nrhs && st == HDSW_OK; c0 += chunk) {
    const int C = std::min(chunk, nrhs - c0);
    const Carve k = carve(c, C);
    unsigned char* b = (unsigned char*)base;
    c->d_panel = b + k.panel;
    c->d_slots = b + k.slots;
    c->d_srcsum = b + k.srcsum;
    c->d_y = b + k.y;
    c->d_nzflag = c->g.dim == 2 ? (int*)(b + k.nzflag) : nullptr;
    c->d_g = c->g.dim == 3 ? b + k.g : nullptr;
    c->d_out = c->g.dim == 3 ? b + k.out : nullptr;
    c->d_gpart = c->g.dim == 3 ? b + k.gpart : nullptr;
    c->gpart_bytes = k.gpart_bytes;
    st = ddm_dispatch_eager(c, r + (size_t)c0 * c->g.glob_nodes,
                            z + (size_t)c0 * c->g.glob_nodes, C, 0);
  }
  c->d_panel = saved[0];
  c->d_slots = saved[1];
  c->d_srcsum = saved[2];
  c->d_y = saved[3];
  c->d_g = saved[4];
  c->d_out = saved[5];
  c->d_gpart = saved[6];
  c->d_nzflag = (int*)saved[7];
  c->gpart_bytes = saved_gpart;
  c->tm.mask = saved_mask;
  if (st != HDSW_OK) return st;
  if (hipStreamSynchronize(c->stream) != hipSuccess) {
    c->sticky = HDSW_EDEVICE;
    return HDSW_EDEVICE;
  }
  return HDSW_OK;
}

}  // namespace hdsw

// extern "C" entry points of libhdsw (declared in include/hdsw.h).  Argument
// marshalling and error mapping only; the work is in driver.cpp / krylov.cpp
// and the kernels.
#include <new>

#include "hdsw_internal.hpp"

namespace hdsw {
hdsw_status setup_impl(const hdsw_grid*, const double*, const hdsw_partition*, int,
                       const hdsw_options*, void*, hdsw_ctx**);
hdsw_status factor(hdsw_ctx*);
hdsw_status solve(hdsw_ctx*, const c128*, c128*, int, hdsw_solve_info*);
hdsw_status apply_precond(hdsw_ctx*, const c128*, c128*, int);
hdsw_status apply_precond_noalloc(hdsw_ctx*, const c128*, c128*, int);
hdsw_status residual(hdsw_ctx*, const c128*, const c128*, c128*, int, double*);
hdsw_status timing_get(hdsw_ctx*, int, double*, long long*, double*, double*);
hdsw_status batch_reserve(hdsw_ctx*, int);
hdsw_status batch_add(hdsw_ctx*, const c128*, int, int*);
hdsw_status batch_step(hdsw_ctx*);
hdsw_status batch_wait(hdsw_ctx*, double*);
hdsw_status batch_ready(hdsw_ctx*);
hdsw_status batch_take(hdsw_ctx*, int, c128*);
hdsw_status tuning_set(hdsw_ctx*, const TuneParams&);
void destroy(hdsw_ctx*);
}  // namespace hdsw

extern "C" {

void hdsw_default_options(hdsw_options* o) {
  if (!o) return;
  o->precision = HDSW_MIXED;
  o->rounds = 1;
  o->pml_R = 1e-16;
  o->tol = 1e-10;
  o->max_iter = 30;
  o->gmres_m = 0;
  o->dedup = 1;
  o->graphs = 1;
  o->hbm_budget = 0;
  o->dev_alloc = nullptr;
  o->dev_free = nullptr;
  o->alloc_ctx = nullptr;
}

hdsw_status hdsw_setup(const hdsw_grid* grid, const double* kappa_host,
                       const hdsw_partition* part, int pml_width, const hdsw_options* opt,
                       void* stream, hdsw_ctx** out) {
  try {
    return hdsw::setup_impl(grid, kappa_host, part, pml_width, opt, stream, out);
  } catch (const std::bad_alloc&) {
    return HDSW_ENOMEM;
  } catch (...) {
    return HDSW_EDEVICE;
  }
}

// An exception other than bad_alloc out of a context call leaves the
// context in an unknown state: the error is made sticky.
static hdsw_status fail_ctx(hdsw_ctx* ctx) {
  ctx->sticky = HDSW_EDEVICE;
  return HDSW_EDEVICE;
}

hdsw_status hdsw_factor(hdsw_ctx* ctx) {
  if (!ctx) return HDSW_EINVAL;
  try {
    return hdsw::factor(ctx);
  } catch (const std::bad_alloc&) {
    return HDSW_ENOMEM;
  } catch (...) {
    return fail_ctx(ctx);
  }
}

hdsw_status hdsw_solve(hdsw_ctx* ctx, const hdsw_c128* f, hdsw_c128* x, int nrhs,
                       hdsw_solve_info* info) {
  if (!ctx) return HDSW_EINVAL;
  try {
    return hdsw::solve(ctx, reinterpret_cast<const hdsw::c128*>(f),
                       reinterpret_cast<hdsw::c128*>(x), nrhs, info);
  } catch (const std::bad_alloc&) {
    return HDSW_ENOMEM;
  } catch (...) {
    return fail_ctx(ctx);
  }
}

hdsw_status hdsw_apply_precond(hdsw_ctx* ctx, const hdsw_c128* r, hdsw_c128* z, int nrhs) {
  if (!ctx) return HDSW_EINVAL;
  try {
    return hdsw::apply_precond(ctx, reinterpret_cast<const hdsw::c128*>(r),
                               reinterpret_cast<hdsw::c128*>(z), nrhs);
  } catch (const std::bad_alloc&) {
    return HDSW_ENOMEM;
  } catch (...) {
    return fail_ctx(ctx);
  }
}

hdsw_status hdsw_apply_precond_noalloc(hdsw_ctx* ctx, const hdsw_c128* r, hdsw_c128* z,
                                       int nrhs) {
  if (!ctx) return HDSW_EINVAL;
  try {
    return hdsw::apply_precond_noalloc(ctx, reinterpret_cast<const hdsw::c128*>(r),
                                       reinterpret_cast<hdsw::c128*>(z), nrhs);
  } catch (...) {
    return fail_ctx(ctx);
  }
}

hdsw_status hdsw_residual(hdsw_ctx* ctx, const hdsw_c128* b, const hdsw_c128* x,
                          hdsw_c128* r, int nrhs, double* rnorm) {
  if (!ctx) return HDSW_EINVAL;
  try {
    return hdsw::residual(ctx, reinterpret_cast<const hdsw::c128*>(b),
                          reinterpret_cast<const hdsw::c128*>(x),
                          reinterpret_cast<hdsw::c128*>(r), nrhs, rnorm);
  } catch (...) {
    return fail_ctx(ctx);
  }
}

hdsw_status hdsw_query(const hdsw_ctx* ctx, size_t* factor_bytes, int* n_distinct_ops,
                       size_t* workspace_bytes) {
  if (!ctx) return HDSW_EINVAL;
  if (factor_bytes) *factor_bytes = ctx->factor_bytes;
  if (n_distinct_ops) *n_distinct_ops = ctx->nops;
  if (workspace_bytes)
    *workspace_bytes = ctx->alloc_bytes > ctx->factor_bytes ? ctx->alloc_bytes - ctx->factor_bytes : 0;
  return HDSW_OK;
}

hdsw_status hdsw_timing_enable(hdsw_ctx* ctx, int enable) {
  if (!ctx) return HDSW_EINVAL;
  ctx->tm.mask = enable & 31;
  return HDSW_OK;
}

hdsw_status hdsw_timing_get(hdsw_ctx* ctx, int which, double* total_ms, long long* launches,
                            double* flops, double* bytes) {
  if (!ctx) return HDSW_EINVAL;
  return hdsw::timing_get(ctx, which, total_ms, launches, flops, bytes);
}

hdsw_status hdsw_batch_reserve(hdsw_ctx* ctx, int capacity) {
  if (!ctx) return HDSW_EINVAL;
  try {
    return hdsw::batch_reserve(ctx, capacity);
  } catch (const std::bad_alloc&) {
    return HDSW_ENOMEM;
  } catch (...) {
    return fail_ctx(ctx);
  }
}

hdsw_status hdsw_batch_add(hdsw_ctx* ctx, const hdsw_c128* f, int nrhs, int* slots) {
  if (!ctx) return HDSW_EINVAL;
  try {
    return hdsw::batch_add(ctx, reinterpret_cast<const hdsw::c128*>(f), nrhs, slots);
  } catch (...) {
    return fail_ctx(ctx);
  }
}

hdsw_status hdsw_batch_step(hdsw_ctx* ctx) {
  if (!ctx) return HDSW_EINVAL;
  try {
    return hdsw::batch_step(ctx);
  } catch (...) {
    return fail_ctx(ctx);
  }
}

hdsw_status hdsw_batch_wait(hdsw_ctx* ctx, double* rel_residual) {
  if (!ctx) return HDSW_EINVAL;
  try {
    return hdsw::batch_wait(ctx, rel_residual);
  } catch (...) {
    return fail_ctx(ctx);
  }
}

hdsw_status hdsw_batch_ready(hdsw_ctx* ctx) {
  if (!ctx) return HDSW_EINVAL;
  try {
    return hdsw::batch_ready(ctx);
  } catch (...) {
    return fail_ctx(ctx);
  }
}

hdsw_status hdsw_batch_take(hdsw_ctx* ctx, int slot, hdsw_c128* x) {
  if (!ctx) return HDSW_EINVAL;
  try {
    return hdsw::batch_take(ctx, slot, reinterpret_cast<hdsw::c128*>(x));
  } catch (...) {
    return fail_ctx(ctx);
  }
}

hdsw_status hdsw_tuning_set(hdsw_ctx* ctx, const hdsw_tuning* t) {
  if (!ctx || !t) return HDSW_EINVAL;
  hdsw::TuneParams p;
  p.solve_ng = t->solve_ng;
  p.sweep_rw = t->sweep_rw;
  p.sweep_kb = t->sweep_kb;
  p.gemm_skinny = t->gemm_skinny;
  p.sweep_nw = t->sweep_nw;
  p.sweep_sched = t->sweep_sched;
  try {
    return hdsw::tuning_set(ctx, p);
  } catch (...) {
    return fail_ctx(ctx);
  }
}

hdsw_status hdsw_tuning_get(const hdsw_ctx* ctx, hdsw_tuning* t) {
  if (!ctx || !t) return HDSW_EINVAL;
  t->solve_ng = ctx->tune.solve_ng;
  t->sweep_rw = ctx->tune.sweep_rw;
  t->sweep_kb = ctx->tune.sweep_kb;
  t->gemm_skinny = ctx->tune.gemm_skinny;
  t->sweep_nw = ctx->tune.sweep_nw;
  t->sweep_sched = ctx->tune.sweep_sched;
  return HDSW_OK;
}

void hdsw_destroy(hdsw_ctx* ctx) { hdsw::destroy(ctx); }

const char* hdsw_status_str(hdsw_status s) {
  switch (s) {
    case HDSW_OK: return "HDSW_OK";
    case HDSW_EINVAL: return "HDSW_EINVAL: invalid argument";
    case HDSW_ENOMEM: return "HDSW_ENOMEM: device memory or HBM budget exhausted";
    case HDSW_EDEVICE: return "HDSW_EDEVICE: HIP runtime error (context unusable)";
    case HDSW_ENOTFACTORED: return "HDSW_ENOTFACTORED: call hdsw_factor first";
    case HDSW_ENOCONV: return "HDSW_ENOCONV: iteration limit reached";
    case HDSW_EBUSY: return "HDSW_EBUSY: context in use";
  }
  return "HDSW: unknown status";
}

}  // extern "C"

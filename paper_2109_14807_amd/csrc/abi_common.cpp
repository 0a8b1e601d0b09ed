// Status strings, per-thread error detail and descriptor validation.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include "common.h"

namespace {
thread_local char g_last_error[512] = "";
}

glint_status glint_fail(glint_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return code;
}

glint_status glint_check_desc(const glint_ndf_desc* d) {
  GLINT_REQUIRE(d != nullptr, "desc is NULL");
  GLINT_REQUIRE(d->nu >= 1 && d->nv >= 1, "map size %d x %d must be positive", d->nu, d->nv);
  GLINT_REQUIRE(d->nlevels >= 1 && d->nlevels <= 16, "nlevels %d outside 1..16", d->nlevels);
  const int64_t kmax = int64_t(1) << (d->nlevels - 1);
  GLINT_REQUIRE(kmax <= d->nu && kmax <= d->nv,
                "coarsest footprint %lld exceeds the map size", static_cast<long long>(kmax));
  GLINT_REQUIRE(glint_pow2(d->nbins) && d->nbins >= 4 && d->nbins <= 256,
                "nbins %d must be a power of two in 4..256", d->nbins);
  GLINT_REQUIRE(d->sigma > 0.0 && isfinite(d->sigma), "sigma must be positive and finite");
  return GLINT_OK;
}

int32_t glint_window_k(const glint_ndf_desc* d) {
  const double w = 2.0 / d->nbins;
  const double k = ceil(8.0 * d->sigma / w) + 1.0;
  return k >= d->nbins ? d->nbins : static_cast<int32_t>(k);
}

extern "C" {

const char* glint_status_string(glint_status s) {
  switch (s) {
    case GLINT_OK: return "ok";
    case GLINT_E_INVALID: return "invalid argument";
    case GLINT_E_UNSUPPORTED: return "unsupported";
    case GLINT_E_HIP: return "HIP runtime error";
    case GLINT_E_WORKSPACE: return "workspace too small";
  }
  return "unknown status";
}

const char* glint_last_error(void) { return g_last_error; }

int32_t glint_version(void) { return 1; }

int32_t glint_window_radius(const glint_ndf_desc* desc) {
  if (glint_check_desc(desc) != GLINT_OK) return -1;
  return glint_window_k(desc);
}

}  // extern "C"

// Host-side helpers shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>

#include "../../include/mont.h"
#include "mont_kernels.hpp"

namespace mont {

mont_status_t fail(mont_status_t code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
mont_status_t hip_fail(hipError_t e, const char *what);
KCtx to_kctx(const mont_ctx_t &c);
int width_class(uint32_t w);
mont_status_t setup_ctx(uint64_t N, uint32_t w, mont_ctx_t *ctx);
mont_status_t check_ctx(const mont_ctx_t *ctx);
mont_status_t check_variant(const mont_ctx_t *ctx, int variant);
Launch get_launch(int op, int wc, int variant);
void set_launch(int op, int wc, int variant, const Launch &l);

// Tuned shapes, persisted as JSON lines in $MONT_TUNE_CACHE (mont_tunecache.cpp).
using TuneRecord = std::map<std::string, double>;
std::string tune_key_prefix();  // "<gfx arch>:v<mont_version()>:"
bool tune_lookup(const std::string &key, TuneRecord &out);
void tune_store(const std::string &key, const TuneRecord &r);

}  // namespace mont

// Host-side helpers shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>

#include "../../include/mont.h"
#include "mont_kernels.hpp"
#include "mont_tuneline.hpp"

namespace mont {

mont_status_t fail(mont_status_t code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

// Diagnostics on stderr, by the level in $MONT_LOG (read at each use): unset
// or 0 silent; 1 every error a call returns, with its message; 2 also tuning
// decisions, graph rebuilds and serving events (deadline expiries, retired
// slots, cancellations); 3 also one line per batch launch.
int log_level();
void log_msg(int level, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
// $MONT_TUNE: -1 unset (the MONT_BATCH_TUNE flag decides), 0 never tune (the
// flag and mont_tune_mul's sweep are ignored), 1 tune every batch whose shape
// was not set explicitly.
int tune_override();
mont_status_t hip_fail(hipError_t e, const char *what);
KCtx to_kctx(const mont_ctx_t &c);
int width_class(uint32_t w);
mont_status_t setup_ctx(uint64_t N, uint32_t w, mont_ctx_t *ctx);
mont_status_t check_ctx(const mont_ctx_t *ctx);
mont_status_t check_variant(const mont_ctx_t *ctx, int variant);
Launch get_launch(int op, int wc, int variant);
void set_launch(int op, int wc, int variant, const Launch &l);

// Tuned shapes, persisted as JSON lines in $MONT_TUNE_CACHE (mont_tunecache.cpp;
// line format in mont_tuneline.hpp).
std::string tune_key_prefix();  // "<gfx arch>:v<mont_version()>:"
bool tune_lookup(const std::string &key, TuneRecord &out);
void tune_store(const std::string &key, const TuneRecord &r);

}  // namespace mont

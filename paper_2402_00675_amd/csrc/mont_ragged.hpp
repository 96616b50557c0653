// Descriptors of the persistent ragged-batch kernel, shared by the batch API
// and the serving loop.
#pragma once

#include "../../include/mont.h"
#include "mont_kernels.hpp"

namespace mont {

struct DSeg {
    uint64_t off;    // element offset of in0 / out in the pools of its width
    uint64_t off1;   // element offset of in1 (b as w-bit elements; exponents as uint64)
    uint32_t op;
    uint32_t variant;
    uint32_t wc;     // width class 0/1/2 = 16/32/64 bits
    uint32_t ctx;    // index of the segment's constants in the launch's KCtx table
};
static_assert(sizeof(DSeg) == 32, "segment descriptor layout");

struct DTile {
    uint32_t seg;
    uint32_t cnt;
    uint64_t start;  // element index inside the segment
};

struct DPools {
    const void *in0[3];
    const void *in1[3];
    void *out[3];
};

// One persistent launch over `ntiles` tiles; segment i reduces with the
// constants ctab[segs[i].ctx] (ctr: two zeroed uint32 that the kernel leaves
// zeroed again when dyn = 1).  nt selects non-temporal loads and stores.
hipError_t launch_ragged(const KCtx *ctab, const DSeg *segs, const DTile *tiles, uint32_t ntiles, const DPools &P,
                         uint32_t *ctr, uint32_t dyn, uint32_t grid, bool nt, hipStream_t s);
void *ragged_kernel_ptr(bool nt);

// Validates segment i of a batch (context index, op, variant, sizes, operand
// alignment) and fills its device descriptor; the error text names the segment.
mont_status_t make_dseg(const mont_ctx_t *ctxs, uint32_t nctx, const mont_seg_t &sg, uint32_t i, DSeg &d);
// Elements per tile of a segment of width class wc and operation op.
uint32_t seg_tile_elems(uint32_t tile_base, uint32_t pow_tile, uint32_t wc, uint32_t op);

}  // namespace mont

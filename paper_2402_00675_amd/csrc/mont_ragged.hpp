// Descriptors of the persistent ragged-batch kernel, shared by the batch API,
// the allocation-free batch and the serving loop.
#pragma once

#include "../../include/mont.h"
#include "mont_kernels.hpp"

namespace mont {

// One segment as the host validates it (make_dseg); the kernel never reads it.
struct DSeg {
    uint64_t off;    // element offset of in0 / out in the pools of its width
    uint64_t off1;   // element offset of in1 (b as w-bit elements; exponents as uint64)
    uint32_t op;
    uint32_t variant;
    uint32_t wc;     // width class 0/1/2 = 16/32/64 bits
    uint32_t ctx;    // index of the segment's constants in the launch's KCtx table
};

// One tile of work as the kernel reads it (32 bytes, one scalar load): its
// element range in the pools and everything needed to process it, so the only
// other load before the data is the tile's constants, ctab[ctx].
struct DTile {
    uint64_t g0;   // first element in in0 and out (a 2w-bit T index for MONT_OP_REDC)
    uint64_t g1;   // the same element's index in in1 (w-bit b, or uint64 exponent)
    uint32_t cnt;  // elements
    uint32_t ctx;  // constants: ctab[ctx]
    uint32_t op;   // MONT_OP_*
    uint32_t vw;   // variant | width class << 8
};
static_assert(sizeof(DTile) == 32, "tile record layout");

inline DTile make_tile(const DSeg &d, uint64_t start, uint32_t cnt)
{
    DTile t;
    t.g0 = d.off + start;
    t.g1 = d.off1 + start;
    t.cnt = cnt;
    t.ctx = d.ctx;
    t.op = d.op;
    t.vw = d.variant | (d.wc << 8);
    return t;
}

struct DPools {
    const void *in0[3];
    const void *in1[3];
    void *out[3];
};

// Counters of the dynamic schedule: 8 claim counters (one per XCD) and a done
// counter, each uint32 on its own 128-byte line.
constexpr uint32_t CTR_STRIDE = 32;                      // uint32 between counters
constexpr size_t CTR_BYTES = 9 * CTR_STRIDE * sizeof(uint32_t);

// One launch over `ntiles` tiles, tile i reducing with the constants
// ctab[tiles[i].ctx]: grid = ntiles for one pass, fewer for a persistent grid
// (static round-robin, or tiles claimed from the counters in ctr when dyn = 1;
// ctr: CTR_BYTES of zeroes that the kernel leaves zeroed again).  nt selects
// non-temporal loads and stores; block is the workgroup size (64 or 256).
hipError_t launch_ragged(const KCtx *ctab, const DTile *tiles, uint32_t ntiles, const DPools &P, uint32_t *ctr,
                         uint32_t dyn, uint32_t grid, bool nt, hipStream_t s, uint32_t block = BLOCK);
void *ragged_kernel_ptr(bool nt, uint32_t block);

// Validates segment i of a batch (context index, op, variant, sizes, operand
// alignment) and fills its host descriptor; the error text names the segment.
mont_status_t make_dseg(const mont_ctx_t *ctxs, uint32_t nctx, const mont_seg_t &sg, uint32_t i, DSeg &d);
// Elements per tile of a segment of width class wc and operation op.
uint32_t seg_tile_elems(uint32_t tile_base, uint32_t pow_tile, uint32_t wc, uint32_t op);

}  // namespace mont

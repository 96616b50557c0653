// Serving loop: the scheduler core (mont_sched.hpp) driven by a service
// thread, with a GPU backend that runs each batch as one persistent ragged
// launch on its own HIP stream.
//
// Device layout per word-size class c (32-bit, 64-bit residues), for an
// arena of cap element slots:
//   in0[c]  cap * es bytes   first operand a / base x
//   in1[c]  cap * 8 bytes    second operand b (es bytes at slot*8) or the
//                            exponent (8 bytes at slot*8)
//   out[c]  cap * es bytes   result
// so one slot index addresses all three, and a job's slots never alias
// another job's.  Each stream slot owns pinned host staging for its tables,
// device copies of them, a self-resetting tile counter and a completion
// event; a slot is reused only after its event fired.
//
// Per-modulus constants are resident: one device table of KCtx entries that
// the segment descriptors index.  A modulus's entry is computed and
// installed (by a small kernel, from the batch's staging upload) the first
// time a batch needs it; entries used by launched batches are pinned by
// reference counts, unpinned ones stay cached and the least recently used is
// reused when the table is full.  Installs happen on the installing batch's
// stream ahead of its other work and are followed by an event that every
// later batch's stream waits for, so no kernel reads an entry before it is
// written; a pinned entry is never rewritten.
//
// Staging.  A job whose host buffers lie in a region the caller declared as
// pinned, device-mapped host memory (mont_serve_host_region, verified with
// hipPointerGetAttributes) is copied into the arena and back by two copy
// kernels per batch that read and write host memory through its device
// mapping: one launch for all of a batch's inputs and one for all its
// results, instead of three DMA copies per job.  Other buffers take
// hipMemcpyAsync.  Per batch the stream runs: one table upload, a wait for
// the latest constant install, this batch's installs, DMA inputs, gather
// kernel, ragged kernel, scatter kernel, DMA results, event.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mont_common.hpp"
#ifdef MONT_DEBUG
#include "mont_debug.hpp"
#endif
#include "mont_ragged.hpp"
#include "mont_sched.hpp"

namespace mont {

static double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// One host-to-device or device-to-host copy of `words` 32-bit words, run by k_xfer.
struct XDesc {
    const uint32_t *src;
    uint32_t *dst;
    uint64_t words;
    uint64_t pad;
};

struct XTile {
    uint32_t desc;
    uint32_t words;
    uint64_t start;
};

constexpr uint32_t XTILE_WORDS = 8192;  // 32 KiB per workgroup
constexpr int XFER_U = 8;               // words in flight per lane

// Copies tiles of descriptors; src or dst may be device-mapped host memory.
__global__ void __launch_bounds__(BLOCK) k_xfer(const XDesc *__restrict__ d, const XTile *__restrict__ t,
                                                uint32_t ntiles)
{
    const uint32_t ti = blockIdx.x;
    if (ti >= ntiles)
        return;
    const XTile tl = t[ti];
    const XDesc ds = d[tl.desc];
    const uint32_t *src = ds.src + tl.start;
    uint32_t *dst = ds.dst + tl.start;
    for (uint32_t base = threadIdx.x; base < tl.words; base += BLOCK * XFER_U) {
        uint32_t v[XFER_U];
#pragma unroll
        for (int u = 0; u < XFER_U; ++u) {
            const uint32_t i = base + u * BLOCK;
            if (i < tl.words)
                v[u] = src[i];
        }
#pragma unroll
        for (int u = 0; u < XFER_U; ++u) {
            const uint32_t i = base + u * BLOCK;
            if (i < tl.words)
                dst[i] = v[u];
        }
    }
}

// Writes new resident constant entries: tab[idx[i]] = src[i].
__global__ void __launch_bounds__(BLOCK) k_install(KCtx *__restrict__ tab, const KCtx *__restrict__ src,
                                                   const uint32_t *__restrict__ idx, uint32_t n)
{
    const uint32_t i = blockIdx.x * BLOCK + threadIdx.x;
    if (i < n)
        tab[idx[i]] = src[i];
}

struct ServeSlot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    std::vector<uint32_t> pinned;     // resident constant entries its batch uses
    unsigned char *hstage = nullptr;  // pinned: [segs][tiles][xin desc][xin tiles][xout desc][xout tiles]
    unsigned char *dstage = nullptr;  // device copy
    size_t stage_cap = 0;
    uint32_t *dctr = nullptr;
};

struct HostRegion {
    uintptr_t lo, hi, dev;
};

class GpuBackend : public mont_sched::Backend {
  public:
    int dev = 0;
    uint64_t cap[2] = {0, 0};
    void *in0[2] = {nullptr, nullptr}, *in1[2] = {nullptr, nullptr}, *out[2] = {nullptr, nullptr};
    std::vector<ServeSlot> slot;
    uint32_t tile_base = 8192, pow_tile = 1024, grid_max = 0;
    // resident constants
    KCtx *dctab = nullptr;
    struct CEnt {
        uint64_t N = 0;
        uint32_t cls = 0, refs = 0;
        uint64_t tick = 0;
        bool used = false;
    };
    std::vector<CEnt> cent;
    std::unordered_map<uint64_t, uint32_t> cidx[2];  // N -> entry, per word-size class
    std::vector<uint32_t> cfree;
    std::set<std::pair<uint64_t, uint32_t>> clru;  // (last use, entry) of unpinned entries
    uint64_t ctick = 0;
    hipEvent_t tab_ev = nullptr;  // recorded after the latest install
    bool tab_ev_valid = false;
    std::vector<KCtx> newc;
    std::vector<uint32_t> newi;
    std::atomic<uint64_t> ctx_uploads{0}, ctx_hits{0};
    // scratch for building a batch's tables
    std::vector<DTile> tiles;
    std::vector<XDesc> xin, xout;
    std::vector<XTile> xtin, xtout;
    struct Dma {
        void *dst;
        const void *src;
        size_t bytes;
    };
    std::vector<Dma> dma_in, dma_out;
    std::mutex reg_mu;
    std::vector<HostRegion> regions;  // sorted by lo, disjoint

    // Device address of [p, p + bytes) when it lies in one declared region.
    uintptr_t alias(const void *p, size_t bytes)
    {
        const uintptr_t a = (uintptr_t)p;
        if (a & 3u)
            return 0;
        auto it = std::upper_bound(regions.begin(), regions.end(), a,
                                   [](uintptr_t v, const HostRegion &r) { return v < r.lo; });
        if (it == regions.begin())
            return 0;
        --it;
        if (a + bytes > it->hi)
            return 0;
        return it->dev + (a - it->lo);
    }

    mont_status_t add_region(void *p, size_t bytes)
    {
        if (!p || bytes == 0 || ((uintptr_t)p & 3u) || (bytes & 3u))
            return fail(MONT_E_INVAL, "host region must be non-empty, 4-byte aligned and sized");
        hipPointerAttribute_t a0{}, a1{};
        const void *last = (const char *)p + bytes - 1;
        if (hipPointerGetAttributes(&a0, p) != hipSuccess || hipPointerGetAttributes(&a1, last) != hipSuccess) {
            (void)hipGetLastError();
            return fail(MONT_E_INVAL, "host region is not pinned host memory");
        }
        if (a0.type != hipMemoryTypeHost || a1.type != hipMemoryTypeHost || !a0.devicePointer || !a1.devicePointer ||
            (uintptr_t)a1.devicePointer - (uintptr_t)a0.devicePointer != bytes - 1)
            return fail(MONT_E_INVAL, "host region is not device-mapped pinned host memory");
        HostRegion r{(uintptr_t)p, (uintptr_t)p + bytes, (uintptr_t)a0.devicePointer};
        std::lock_guard<std::mutex> g(reg_mu);
        for (const HostRegion &q : regions)
            if (r.lo < q.hi && q.lo < r.hi) {
                if (r.lo >= q.lo && r.hi <= q.hi)
                    return MONT_OK;  // already covered
                return fail(MONT_E_INVAL, "host region overlaps a declared region");
            }
        regions.insert(std::upper_bound(regions.begin(), regions.end(), r,
                                        [](const HostRegion &x, const HostRegion &y) { return x.lo < y.lo; }),
                       r);
        return MONT_OK;
    }

    mont_status_t init(const mont_server_cfg_t &c, uint32_t nslots, uint64_t budget)
    {
        (void)hipGetDevice(&dev);
        // bytes per slot: 32-bit class 4 + 8 + 4, 64-bit class 8 + 8 + 8
        cap[0] = (budget / 2) / 16 / mont_sched::ALIGN * mont_sched::ALIGN;
        cap[1] = (budget / 2) / 24 / mont_sched::ALIGN * mont_sched::ALIGN;
        const size_t es[2] = {4, 8};
        for (int k = 0; k < 2; ++k) {
            if (hipMalloc(&in0[k], cap[k] * es[k]) != hipSuccess || hipMalloc(&in1[k], cap[k] * 8) != hipSuccess ||
                hipMalloc(&out[k], cap[k] * es[k]) != hipSuccess)
                return fail(MONT_E_NOMEM, "serving arena of %llu bytes", (unsigned long long)budget);
        }
        if (c.tile_elems)
            tile_base = c.tile_elems;
        grid_max = (uint32_t)device_cus() * 8;
        // every in-flight job pins at most one entry; batches abandoned at their
        // deadline keep theirs until they end, hence the margin; 2^18 more entries
        // (16 MiB) keep that many moduli cached
        const uint32_t ncent = 2 * c.max_jobs_in_flight + (1u << 18);
        if (hipMalloc(&dctab, (size_t)ncent * sizeof(KCtx)) != hipSuccess)
            return fail(MONT_E_NOMEM, "resident constant table");
        cent.resize(ncent);
        cfree.reserve(ncent);
        for (uint32_t i = ncent; i-- > 0;)
            cfree.push_back(i);
        if (hipEventCreateWithFlags(&tab_ev, hipEventDisableTiming) != hipSuccess)
            return fail(MONT_E_DEVICE, "table event");
        slot.resize(nslots);
        const size_t max_jobs = c.max_batch_jobs;
        for (ServeSlot &s : slot)
            if (mont_status_t rc = make_slot(s, max_jobs * (sizeof(KCtx) + 4 + 64 * sizeof(DTile) +
                                                            96 * sizeof(XDesc))))
                return rc;
        return MONT_OK;
    }

    // A stream, completion event, tile counter and staging tables for one slot.
    mont_status_t make_slot(ServeSlot &s, size_t stage_bytes)
    {
        hipError_t e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipMalloc(&s.dctr, CTR_BYTES);
        if (e == hipSuccess)
            e = hipMemsetAsync(s.dctr, 0, CTR_BYTES, s.stream);
        if (e != hipSuccess)
            return hip_fail(e, "serving slot");
        return reserve(s, stage_bytes);
    }

    // Releases a slot's resources; waits for its stream first.
    static void free_slot(ServeSlot &s)
    {
        if (s.stream)
            (void)hipStreamSynchronize(s.stream);
        if (s.done)
            (void)hipEventDestroy(s.done);
        if (s.stream)
            (void)hipStreamDestroy(s.stream);
        if (s.hstage)
            (void)hipHostFree(s.hstage);
        if (s.dstage)
            (void)hipFree(s.dstage);
        if (s.dctr)
            (void)hipFree(s.dctr);
        s = ServeSlot{};
    }

    // Slots whose batch missed its deadline, kept until that batch ends.
    std::map<int, ServeSlot> retired;
    int next_ticket = 0;

    int retire(int si) override
    {
        ServeSlot fresh;
        if (make_slot(fresh, slot[si].stage_cap) != MONT_OK) {
            free_slot(fresh);
            log_msg(2, "serve: slot %d missed its deadline and could not be renewed; it stays out of use", si);
            return -1;
        }
        const int t = next_ticket++;
        retired[t] = slot[si];
        slot[si] = fresh;
        log_msg(2, "serve: slot %d missed its deadline; its batch is retired as ticket %d, the slot renewed", si, t);
        return t;
    }

    int poll_retired(int t) override
    {
        auto it = retired.find(t);
        if (it == retired.end())
            return 1;
        const hipError_t e = hipEventQuery(it->second.done);
        if (e == hipErrorNotReady)
            return 0;
        unpin(it->second.pinned);
        free_slot(it->second);
        retired.erase(it);
        log_msg(2, "serve: retired batch %d ended (%s)", t, e == hipSuccess ? "ok" : hipGetErrorString(e));
        return e == hipSuccess ? 1 : -1;
    }

    // Grows the slot's staging buffers (only while the slot is idle).
    mont_status_t reserve(ServeSlot &s, size_t bytes)
    {
        if (bytes <= s.stage_cap)
            return MONT_OK;
        bytes = std::max(bytes, 2 * s.stage_cap);
        if (s.hstage)
            (void)hipHostFree(s.hstage);
        if (s.dstage)
            (void)hipFree(s.dstage);
        s.hstage = nullptr;
        s.dstage = nullptr;
        s.stage_cap = 0;
        if (hipHostMalloc((void **)&s.hstage, bytes, hipHostMallocDefault) != hipSuccess ||
            hipMalloc(&s.dstage, bytes) != hipSuccess)
            return fail(MONT_E_NOMEM, "batch staging tables");
        s.stage_cap = bytes;
        return MONT_OK;
    }

    ~GpuBackend() override
    {
        for (ServeSlot &s : slot)
            free_slot(s);
        for (auto &r : retired)
            free_slot(r.second);
        if (tab_ev)
            (void)hipEventDestroy(tab_ev);
        if (dctab)
            (void)hipFree(dctab);
        for (int k = 0; k < 2; ++k) {
            if (in0[k])
                (void)hipFree(in0[k]);
            if (in1[k])
                (void)hipFree(in1[k]);
            if (out[k])
                (void)hipFree(out[k]);
        }
    }

    int slots() const override { return (int)slot.size(); }
    double now() override { return now_s(); }

    // The resident entry of (N, w), pinned for the caller; a new entry's
    // constants are queued in newc/newi for this batch's install.  -1 when
    // every entry is pinned or the modulus is invalid.
    int64_t acquire(uint64_t N, uint32_t w)
    {
        const uint32_t k = w == 64 ? 1 : 0;
        auto it = cidx[k].find(N);
        if (it != cidx[k].end()) {
            CEnt &e = cent[it->second];
            if (e.refs++ == 0)
                clru.erase({e.tick, it->second});
            ++ctx_hits;
            return it->second;
        }
        mont_ctx_t c;
        if (setup_ctx(N, w, &c) != MONT_OK)
            return -1;
        uint32_t i;
        if (!cfree.empty()) {
            i = cfree.back();
            cfree.pop_back();
        } else if (!clru.empty()) {
            i = clru.begin()->second;
            clru.erase(clru.begin());
            cidx[cent[i].cls].erase(cent[i].N);
        } else {
            return -1;
        }
        cent[i] = CEnt{N, k, 1, 0, true};
        cidx[k][N] = i;
        newc.push_back(to_kctx(c));
        newi.push_back(i);
        ++ctx_uploads;
        return i;
    }

    void unpin(std::vector<uint32_t> &v)
    {
        for (uint32_t i : v) {
            CEnt &e = cent[i];
            if (--e.refs == 0) {
                e.tick = ++ctick;
                clru.insert({e.tick, i});
            }
        }
        v.clear();
    }

    std::atomic<uint64_t> enqueue_ns{0};

    int launch(int si, const std::vector<mont_sched::Job *> &jobs) override
    {
        const double t0 = now_s();
        const int rc = enqueue(si, jobs);
        enqueue_ns += (uint64_t)((now_s() - t0) * 1e9);
        return rc;
    }

    static size_t up16(size_t x) { return (x + 15) / 16 * 16; }

    static void split(std::vector<XTile> &t, uint32_t desc, uint64_t words)
    {
        for (uint64_t st = 0; st < words; st += XTILE_WORDS)
            t.push_back({desc, (uint32_t)std::min<uint64_t>(XTILE_WORDS, words - st), st});
    }

    int enqueue(int si, const std::vector<mont_sched::Job *> &jobs)
    {
        ServeSlot &s = slot[si];
        newc.clear();
        newi.clear();
        s.pinned.clear();
        for (const mont_sched::Job *jp : jobs) {
            const int64_t ci = acquire(jp->N, jp->w);
            if (ci < 0) {
                unpin(s.pinned);
                fail(MONT_E_NOMEM, "resident constant table full");
                return -1;
            }
            s.pinned.push_back((uint32_t)ci);
        }
        const int rc = enqueue_pinned(si, jobs);
        if (rc)
            unpin(s.pinned);
        return rc;
    }

    int enqueue_pinned(int si, const std::vector<mont_sched::Job *> &jobs)
    {
        ServeSlot &s = slot[si];
        tiles.clear();
        xin.clear();
        xout.clear();
        xtin.clear();
        xtout.clear();
        dma_in.clear();
        dma_out.clear();
        const size_t es[2] = {4, 8};
        for (uint32_t i = 0; i < jobs.size(); ++i) {
            const mont_sched::Job &j = *jobs[i];
            DSeg d;
            d.ctx = s.pinned[i];
            d.off = j.off;
            // in1 slot = 8 bytes: exponents index uint64 at off, products index w-bit b at off * 8 / es
            d.off1 = j.op == mont_sched::OP_POW ? j.off : j.off * (8 / es[j.cls]);
            d.op = j.op == mont_sched::OP_POW ? MONT_OP_POW : MONT_OP_MUL;
            d.variant = CLASSIC;
            d.wc = j.cls == 0 ? 1 : 2;
            const uint64_t te = j.op == mont_sched::OP_POW ? pow_tile : (j.cls == 0 ? tile_base : tile_base / 2);
            for (uint64_t st = 0; st < j.n; st += te)
                tiles.push_back(make_tile(d, st, (uint32_t)std::min<uint64_t>(te, j.n - st)));
        }
        {
            std::lock_guard<std::mutex> g(reg_mu);
            for (const mont_sched::Job *jp : jobs) {
                const mont_sched::Job &j = *jp;
                const size_t b = es[j.cls];
                char *d0 = (char *)in0[j.cls] + j.off * b;
                char *d1 = (char *)in1[j.cls] + j.off * 8;
                char *dout = (char *)out[j.cls] + j.off * b;
                const size_t n0 = b * j.n, n1 = (j.op == mont_sched::OP_POW ? 8 : b) * j.n;
                const uintptr_t a0 = alias(j.in0, n0), a1 = alias(j.in1, n1), ao = alias(j.out, n0);
                if (a0)
                    xin.push_back({(const uint32_t *)a0, (uint32_t *)d0, n0 / 4, 0});
                else
                    dma_in.push_back({d0, j.in0, n0});
                if (a1)
                    xin.push_back({(const uint32_t *)a1, (uint32_t *)d1, n1 / 4, 0});
                else
                    dma_in.push_back({d1, j.in1, n1});
                if (ao)
                    xout.push_back({(const uint32_t *)dout, (uint32_t *)ao, n0 / 4, 0});
                else
                    dma_out.push_back({j.out, dout, n0});
            }
        }
        for (uint32_t d = 0; d < xin.size(); ++d)
            split(xtin, d, xin[d].words);
        for (uint32_t d = 0; d < xout.size(); ++d)
            split(xtout, d, xout[d].words);
        // one packed table upload per batch
        const size_t o_newc = 0;
        const size_t o_newi = up16(o_newc + newc.size() * sizeof(KCtx));
        const size_t o_tile = up16(o_newi + newi.size() * sizeof(uint32_t));
        const size_t o_xin = up16(o_tile + tiles.size() * sizeof(DTile));
        const size_t o_xtin = up16(o_xin + xin.size() * sizeof(XDesc));
        const size_t o_xout = up16(o_xtin + xtin.size() * sizeof(XTile));
        const size_t o_xtout = up16(o_xout + xout.size() * sizeof(XDesc));
        const size_t total = up16(o_xtout + xtout.size() * sizeof(XTile));
        if (reserve(s, total))
            return -1;
        std::memcpy(s.hstage + o_newc, newc.data(), newc.size() * sizeof(KCtx));
        std::memcpy(s.hstage + o_newi, newi.data(), newi.size() * sizeof(uint32_t));
        std::memcpy(s.hstage + o_tile, tiles.data(), tiles.size() * sizeof(DTile));
        std::memcpy(s.hstage + o_xin, xin.data(), xin.size() * sizeof(XDesc));
        std::memcpy(s.hstage + o_xtin, xtin.data(), xtin.size() * sizeof(XTile));
        std::memcpy(s.hstage + o_xout, xout.data(), xout.size() * sizeof(XDesc));
        std::memcpy(s.hstage + o_xtout, xtout.data(), xtout.size() * sizeof(XTile));

        // tables first, then the constants this batch installs (after every earlier
        // install: the entries it reuses may have been installed by another stream)
        hipError_t e = hipMemcpyAsync(s.dstage, s.hstage, total, hipMemcpyHostToDevice, s.stream);
        if (e == hipSuccess && tab_ev_valid)
            e = hipStreamWaitEvent(s.stream, tab_ev, 0);
        if (e == hipSuccess && !newc.empty()) {
            hipLaunchKernelGGL(k_install, dim3((unsigned)((newc.size() + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0,
                               s.stream, dctab, (const KCtx *)(s.dstage + o_newc),
                               (const uint32_t *)(s.dstage + o_newi), (uint32_t)newc.size());
            e = hipGetLastError();
            if (e == hipSuccess)
                e = hipEventRecord(tab_ev, s.stream);
            if (e == hipSuccess)
                tab_ev_valid = true;
        }
        for (const Dma &m : dma_in)
            if (e == hipSuccess)
                e = hipMemcpyAsync(m.dst, m.src, m.bytes, hipMemcpyHostToDevice, s.stream);
        if (e == hipSuccess && !xtin.empty()) {
            hipLaunchKernelGGL(k_xfer, dim3((unsigned)xtin.size()), dim3(BLOCK), 0, s.stream,
                               (const XDesc *)(s.dstage + o_xin), (const XTile *)(s.dstage + o_xtin),
                               (uint32_t)xtin.size());
            e = hipGetLastError();
        }
        if (e == hipSuccess && !tiles.empty()) {
            DPools P{};
            P.in0[1] = in0[0];
            P.in1[1] = in1[0];
            P.out[1] = out[0];
            P.in0[2] = in0[1];
            P.in1[2] = in1[1];
            P.out[2] = out[1];
            const uint32_t grid = (uint32_t)std::max<size_t>(1, std::min<size_t>(tiles.size(), grid_max));
            e = launch_ragged(dctab, (const DTile *)(s.dstage + o_tile), (uint32_t)tiles.size(), P, s.dctr, 8u, grid,
                              true, s.stream);
        }
        if (e == hipSuccess && !xtout.empty()) {
            hipLaunchKernelGGL(k_xfer, dim3((unsigned)xtout.size()), dim3(BLOCK), 0, s.stream,
                               (const XDesc *)(s.dstage + o_xout), (const XTile *)(s.dstage + o_xtout),
                               (uint32_t)xtout.size());
            e = hipGetLastError();
        }
        for (const Dma &m : dma_out)
            if (e == hipSuccess)
                e = hipMemcpyAsync(m.dst, m.src, m.bytes, hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess)
            e = hipEventRecord(s.done, s.stream);
        if (e != hipSuccess) {
            hip_fail(e, "serving batch");
            return -1;
        }
        return 0;
    }

    int poll(int si) override
    {
        const hipError_t e = hipEventQuery(slot[si].done);
        if (e == hipErrorNotReady)
            return 0;
        unpin(slot[si].pinned);
        return e == hipSuccess ? 1 : -1;
    }
};

}  // namespace mont

using namespace mont;

// A cancellation request handed to the service thread (which owns the scheduler).
struct CancelReq {
    uint64_t id;
    mont_status_t result;
    bool pending;
};

struct mont_server {
    GpuBackend *be = nullptr;
    mont_sched::Scheduler *sched = nullptr;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::vector<mont_sched::Job> inbox;
    std::vector<CancelReq *> cancels;
    std::deque<mont_sched::Completion> outbox;
    bool stop = false;
    uint64_t accepted = 0, finished = 0, rejected = 0, canceled_inbox = 0;
    mont_sched::Stats last{};
    uint64_t cap[2] = {0, 0};
    int dev = 0;
};

static void service(mont_server *S)
{
    (void)hipSetDevice(S->dev);
    std::vector<mont_sched::Job> local;
    std::vector<CancelReq *> creq;
    std::vector<mont_sched::Completion> comp(1024);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->inbox.empty() && S->cancels.empty() && S->sched->idle() &&
                S->sched->pending_completions() == 0) {
                if (S->stop)
                    break;
                auto ready = [S] { return S->stop || !S->inbox.empty() || !S->cancels.empty(); };
                if (S->sched->device_busy())  // retired batches still running: keep polling them
                    S->cv_work.wait_for(lk, std::chrono::milliseconds(1), ready);
                else
                    S->cv_work.wait(lk, ready);
            }
            local.swap(S->inbox);
            creq.swap(S->cancels);
        }
        for (auto &j : local)
            S->sched->submit(j);
        local.clear();
        for (CancelReq *r : creq)
            r->result = S->sched->cancel(r->id);
        const bool did = S->sched->step();
        size_t k;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            while ((k = S->sched->take(comp.data(), comp.size())) > 0) {
                S->outbox.insert(S->outbox.end(), comp.begin(), comp.begin() + k);
                S->finished += k;
            }
            for (CancelReq *r : creq)
                r->pending = false;
            S->last = S->sched->stats();
        }
        creq.clear();
        S->cv_done.notify_all();
        if (!did && S->sched->device_busy())
            std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

static bool job_ok(const mont_server *S, const mont_job_t *j, mont_status_t *rc)
{
    if (!j || (j->w != 32 && j->w != 64) || (j->op != MONT_OP_MUL && j->op != MONT_OP_POW) || j->N < 3 ||
        !(j->N & 1u) || (j->w == 32 && (j->N >> 32)) || (j->n && (!j->in0 || !j->in1 || !j->out))) {
        *rc = fail(MONT_E_INVAL, "malformed job");
        return false;
    }
    if (mont_sched::Arena::span(j->n) > S->cap[j->w == 64 ? 1 : 0]) {
        *rc = fail(MONT_E_DOMAIN, "job of %llu elements exceeds the device budget", (unsigned long long)j->n);
        return false;
    }
    return true;
}

static mont_sched::Job to_job(const mont_job_t *j, double t)
{
    mont_sched::Job x;
    x.id = j->id;
    x.N = j->N;
    x.w = j->w;
    x.op = j->op == MONT_OP_POW ? mont_sched::OP_POW : mont_sched::OP_MUL;
    x.n = j->n;
    x.in0 = j->in0;
    x.in1 = j->in1;
    x.out = j->out;
    x.t_submit = t;
    return x;
}

extern "C" {

double mont_serve_now(void) { return now_s(); }

mont_status_t mont_serve_create(const mont_server_cfg_t *cfg, mont_server_t **out)
{
    if (!out)
        return fail(MONT_E_INVAL, "null handle");
    *out = nullptr;
    mont_server_cfg_t c{};
    if (cfg)
        c = *cfg;
    if (!c.hbm_budget_bytes)
        c.hbm_budget_bytes = 8ull << 30;
    if (!c.max_jobs_in_flight)
        c.max_jobs_in_flight = 4096;
    if (!c.streams)
        c.streams = 3;
    if (!c.max_batch_jobs)
        c.max_batch_jobs = 512;
    if (c.streams > 16 || c.tile_elems % 256 || c.tile_elems > (1u << 20))
        return fail(MONT_E_INVAL, "streams <= 16 and tile_elems a multiple of 256 up to 2^20");
    mont_server *S = new (std::nothrow) mont_server;
    if (!S)
        return fail(MONT_E_NOMEM, "server");
    S->be = new (std::nothrow) GpuBackend;
    mont_status_t rc = S->be ? S->be->init(c, c.streams, c.hbm_budget_bytes) : MONT_E_NOMEM;
    if (rc) {
        delete S->be;
        delete S;
        return rc;
    }
    S->dev = S->be->dev;
    S->cap[0] = S->be->cap[0];
    S->cap[1] = S->be->cap[1];
    mont_sched::Config sc;
    sc.cap[0] = S->cap[0];
    sc.cap[1] = S->cap[1];
    sc.max_in_flight = c.max_jobs_in_flight;
    sc.max_batch_jobs = c.max_batch_jobs;
    sc.deadline_s = (c.deadline_us ? c.deadline_us : 30000000u) * 1e-6;
    S->sched = new mont_sched::Scheduler(sc, S->be);
    S->th = std::thread(service, S);
    *out = S;
    return MONT_OK;
}

mont_status_t mont_serve_submit(mont_server_t *S, const mont_job_t *job)
{
    if (!S)
        return fail(MONT_E_INVAL, "null server");
    mont_status_t rc;
    if (!job_ok(S, job, &rc)) {
        std::lock_guard<std::mutex> lk(S->mu);
        ++S->rejected;
        return rc;
    }
#ifdef MONT_DEBUG
    {
        // operands are in host memory: products must meet classic REDC's range, bases lie below N
        uint64_t bad = 0;
        for (uint64_t i = 0; i < job->n; ++i) {
            const uint64_t x = job->w == 32 ? ((const uint32_t *)job->in0)[i] : ((const uint64_t *)job->in0)[i];
            if (job->op == MONT_OP_POW) {
                bad += x >= job->N;
            } else {
                const uint64_t y = job->w == 32 ? ((const uint32_t *)job->in1)[i] : ((const uint64_t *)job->in1)[i];
                bool neg;
                dbg_u128 mag;
                dbg_product(CLASSIC, job->w, x, y, &neg, &mag);
                bad += !dbg_t_in_range(CLASSIC, job->w, job->N, 0, neg, mag);
            }
        }
        debug_count_host(bad);
    }
#endif
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->inbox.push_back(to_job(job, now_s()));
        ++S->accepted;
    }
    S->cv_work.notify_one();
    return MONT_OK;
}

mont_status_t mont_serve_host_region(mont_server_t *S, void *ptr, size_t bytes)
{
    if (!S)
        return fail(MONT_E_INVAL, "null server");
    return S->be->add_region(ptr, bytes);
}

int64_t mont_serve_submit_timed(mont_server_t *S, const mont_job_t *jobs, const double *arrival_s, uint64_t n)
{
    if (!S || (n && (!jobs || !arrival_s)))
        return fail(MONT_E_INVAL, "null argument");
    const double t0 = now_s();
    int64_t ok = 0;
    for (uint64_t i = 0; i < n; ++i) {
        const double due = t0 + arrival_s[i];
        for (;;) {
            const double left = due - now_s();
            if (left <= 0)
                break;
            if (left > 200e-6)
                std::this_thread::sleep_for(std::chrono::duration<double>(left - 150e-6));
            else
                std::this_thread::yield();
        }
        if (mont_serve_submit(S, &jobs[i]) == MONT_OK)
            ++ok;
    }
    return ok;
}

int64_t mont_serve_poll(mont_server_t *S, mont_completion_t *out, uint32_t max, int32_t wait_ms)
{
    if (!S || (max && !out))
        return fail(MONT_E_INVAL, "null argument");
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->outbox.empty() && wait_ms > 0)
        S->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [S] { return !S->outbox.empty(); });
    uint32_t k = 0;
    while (k < max && !S->outbox.empty()) {
        const mont_sched::Completion &c = S->outbox.front();
        out[k].id = c.id;
        out[k].status = c.status;
        out[k].reserved = 0;
        out[k].t_submit = c.t_submit;
        out[k].t_admit = c.t_admit;
        out[k].t_launch = c.t_launch;
        out[k].t_done = c.t_done;
        S->outbox.pop_front();
        ++k;
    }
    return k;
}

mont_status_t mont_serve_drain(mont_server_t *S, int32_t timeout_ms)
{
    if (!S)
        return fail(MONT_E_INVAL, "null server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto done = [S] { return S->finished >= S->accepted; };
    if (timeout_ms < 0) {
        S->cv_done.wait(lk, done);
        return MONT_OK;
    }
    return S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done)
               ? MONT_OK
               : fail(MONT_E_BUSY, "jobs still in flight");
}

mont_status_t mont_serve_stats(const mont_server_t *S, mont_server_stats_t *st)
{
    if (!S || !st)
        return fail(MONT_E_INVAL, "null argument");
    mont_server *M = const_cast<mont_server *>(S);
    std::lock_guard<std::mutex> lk(M->mu);
    const mont_sched::Stats &x = M->last;
    st->submitted = M->accepted + M->rejected;
    st->completed = x.completed;
    st->rejected = M->rejected;
    st->launches = x.launches;
    st->jobs_launched = x.jobs_launched;
    st->queued = x.queued + M->inbox.size();
    st->staged = x.staged;
    st->in_flight = x.in_flight;
    st->bytes_in_use = x.used_slots[0] * 16 + x.used_slots[1] * 24;
    st->peak_bytes_in_use = x.peak_slots[0] * 16 + x.peak_slots[1] * 24;
    st->enqueue_ns = M->be->enqueue_ns.load();
    st->canceled = x.canceled + M->canceled_inbox;
    st->timed_out = x.timed_out;
    st->quarantined_bytes = x.quarantined_slots[0] * 16 + x.quarantined_slots[1] * 24;
    st->dead_streams = x.dead_slots;
    st->ctx_uploads = M->be->ctx_uploads.load();
    st->ctx_hits = M->be->ctx_hits.load();
    return MONT_OK;
}

mont_status_t mont_serve_cancel(mont_server_t *S, uint64_t id)
{
    if (!S)
        return fail(MONT_E_INVAL, "null server");
    std::unique_lock<std::mutex> lk(S->mu);
    // not yet seen by the service thread: complete it here
    for (auto it = S->inbox.begin(); it != S->inbox.end(); ++it)
        if (it->id == id) {
            const double t = now_s();
            S->outbox.push_back({it->id, MONT_E_CANCELED, it->t_submit, 0.0, 0.0, t});
            S->inbox.erase(it);
            ++S->finished;
            ++S->canceled_inbox;
            lk.unlock();
            S->cv_done.notify_all();
            return MONT_OK;
        }
    log_msg(2, "serve: cancel request for job %llu", (unsigned long long)id);
    CancelReq r{id, MONT_OK, true};
    S->cancels.push_back(&r);
    S->cv_work.notify_one();
    S->cv_done.wait(lk, [&r] { return !r.pending; });
    if (r.result == mont_sched::E_BUSY)
        return fail(MONT_E_BUSY, "job %llu is in a launched batch", (unsigned long long)id);
    if (r.result != MONT_OK)
        return fail(MONT_E_INVAL, "no job %llu is waiting", (unsigned long long)id);
    return MONT_OK;
}

void mont_serve_destroy(mont_server_t *S)
{
    if (!S)
        return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->th.joinable())
        S->th.join();
    delete S->sched;
    delete S->be;
    delete S;
}

}  // extern "C"

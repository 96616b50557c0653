// Scheduler core of the serving loop (host only, no HIP): admission of jobs
// by device-memory budget, continuous batching into launch slots, and
// completion bookkeeping.  A Backend performs the copies and launches; the
// GPU backend lives in mont_serve.cpp, and the tests drive the same core with
// a backend that only records what it was asked to do.
//
// Memory model: each word-size class (32-bit, 64-bit residues) owns an arena
// of element slots.  A job of n elements takes one interval of n slots
// (rounded up to ALIGN) in its class; the device pools are laid out so that
// one slot index addresses the job's first operand, second operand
// (8 bytes per slot: room for a uint64 exponent) and result.
//
// Policy: strict FIFO admission (a job that does not fit blocks the ones
// behind it, so large jobs cannot starve); admitted jobs are fused into one
// batch as soon as a launch slot is free; up to `slots` batches are in flight
// at once, so jobs arriving while the device is busy join the next batch.
//
// Robustness: a batch not finished `deadline_s` after its launch is given up:
// its jobs complete with E_DEVICE at once, the backend retires the slot's
// stream (fresh resources take its place) and the batch's device memory stays
// reserved ("quarantined") until the retired work is seen to finish, so no
// later job is placed where a late kernel could still write.  A slot that
// cannot be renewed leaves service; with no slot left every waiting job fails.
// Jobs that are queued or admitted but not yet launched can be cancelled
// (E_CANCELED); a launched job cannot (E_BUSY).
#pragma once

#include <algorithm>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <vector>

namespace mont_sched {

constexpr uint64_t ALIGN = 64;  // element slots; keeps every pool address 16-byte aligned

enum { OK = 0, E_INVAL = -1, E_DOMAIN = -2, E_DEVICE = -5, E_BUSY = -6, E_CANCELED = -7 };
enum { OP_MUL = 0, OP_POW = 2 };

class Arena {
  public:
    void reset(uint64_t cap)
    {
        cap_ = cap / ALIGN * ALIGN;
        free_.clear();
        if (cap_)
            free_[0] = cap_;
        used_ = 0;
    }
    static uint64_t span(uint64_t n) { return (std::max<uint64_t>(n, 1) + ALIGN - 1) / ALIGN * ALIGN; }
    bool alloc(uint64_t n, uint64_t *off)
    {
        const uint64_t need = span(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need)
                continue;
            *off = it->first;
            const uint64_t rest = it->second - need, noff = it->first + need;
            free_.erase(it);
            if (rest)
                free_[noff] = rest;
            used_ += need;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t n)
    {
        const uint64_t len = span(n);
        used_ -= len;
        auto it = free_.emplace(off, len).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t cap() const { return cap_; }
    uint64_t used() const { return used_; }
    size_t fragments() const { return free_.size(); }

  private:
    uint64_t cap_ = 0, used_ = 0;
    std::map<uint64_t, uint64_t> free_;  // offset -> length
};

struct Job {
    uint64_t id = 0;
    uint64_t N = 0;
    uint32_t w = 0;   // 32 or 64
    uint32_t op = 0;  // OP_MUL or OP_POW
    uint64_t n = 0;
    const void *in0 = nullptr;
    const void *in1 = nullptr;
    void *out = nullptr;
    uint32_t cls = 0;  // 0: 32-bit, 1: 64-bit
    uint64_t off = 0;  // arena slot
    double t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
    int32_t status = OK;
};

struct Completion {
    uint64_t id;
    int32_t status;
    double t_submit, t_admit, t_launch, t_done;
};

class Backend {
  public:
    virtual ~Backend() = default;
    virtual int slots() const = 0;
    // Enqueue copies in, the batch kernel and copies out; 0 on success.
    virtual int launch(int slot, const std::vector<Job *> &jobs) = 0;
    // 1: the slot's batch finished, 0: still running, < 0: failed.
    virtual int poll(int slot) = 0;
    virtual double now() = 0;
    // The slot's batch missed its deadline: give the slot fresh resources and
    // keep the old ones until that batch ends.  Returns a ticket (>= 0) for
    // poll_retired, or < 0 when the slot cannot be renewed.
    virtual int retire(int slot) = 0;
    // 0 while the retired batch still runs; otherwise it has ended (1) or
    // failed (< 0) and its resources are released.
    virtual int poll_retired(int ticket) = 0;
};

struct Config {
    uint64_t cap[2] = {0, 0};  // element slots per class
    uint32_t max_in_flight = 4096;
    uint32_t max_batch_jobs = 512;
    double deadline_s = 0;     // per-batch completion deadline (0: none)
};

struct Stats {
    uint64_t submitted = 0, completed = 0, rejected = 0, launches = 0, jobs_launched = 0;
    uint64_t used_slots[2] = {0, 0}, peak_slots[2] = {0, 0};
    uint64_t queued = 0, staged = 0, in_flight = 0;
    uint64_t canceled = 0, timed_out = 0, quarantined_slots[2] = {0, 0}, dead_slots = 0;
};

class Scheduler {
  public:
    Scheduler(const Config &c, Backend *b) : cfg_(c), be_(b)
    {
        arena_[0].reset(c.cap[0]);
        arena_[1].reset(c.cap[1]);
        slot_jobs_.resize(b->slots());
        slot_t_.assign(b->slots(), 0.0);
        slot_dead_.assign(b->slots(), false);
    }

    // Validates and queues a job (n == 0 completes at once).
    int submit(Job j)
    {
        ++st_.submitted;
        int rc = OK;
        if ((j.w != 32 && j.w != 64) || (j.op != OP_MUL && j.op != OP_POW) || j.N < 3 || !(j.N & 1u) ||
            (j.w == 32 && (j.N >> 32)))
            rc = E_INVAL;
        else if (j.n && (!j.in0 || !j.in1 || !j.out))
            rc = E_INVAL;
        j.cls = j.w == 64 ? 1 : 0;
        if (!rc && Arena::span(j.n) > arena_[j.cls].cap())
            rc = E_DOMAIN;  // can never be admitted
        if (rc) {
            ++st_.rejected;
            finish(j, rc, be_->now());
            return rc;
        }
        if (j.n == 0) {
            ++st_.completed;
            finish(j, OK, be_->now());
            return OK;
        }
        if (live_slots() == 0) {
            ++st_.completed;
            finish(j, E_DEVICE, be_->now());
            return OK;
        }
        queue_.push_back(j);
        return OK;
    }

    // Cancels job `id` if it has not been launched: OK (it completes with
    // E_CANCELED), E_BUSY (it is in a launched batch) or E_INVAL (no such job
    // is waiting).
    int cancel(uint64_t id)
    {
        for (auto it = queue_.begin(); it != queue_.end(); ++it)
            if (it->id == id) {
                Job j = *it;
                queue_.erase(it);
                ++st_.completed;
                ++st_.canceled;
                finish(j, E_CANCELED, be_->now());
                return OK;
            }
        for (auto it = staged_.begin(); it != staged_.end(); ++it)
            if (it->id == id) {
                Job j = *it;
                staged_.erase(it);
                arena_[j.cls].release(j.off, j.n);
                --in_flight_;
                ++st_.completed;
                ++st_.canceled;
                finish(j, E_CANCELED, be_->now());
                return OK;
            }
        for (const auto &sj : slot_jobs_)
            for (const Job &j : sj)
                if (j.id == id)
                    return E_BUSY;
        return E_INVAL;
    }

    // One pass: collect finished batches, admit waiting jobs, launch a batch.
    bool step()
    {
        bool did = false;
        for (size_t q = 0; q < quarantine_.size();) {
            if (quarantine_[q].ticket < 0 || be_->poll_retired(quarantine_[q].ticket) == 0) {
                ++q;
                continue;
            }
            for (const Span &sp : quarantine_[q].spans) {
                arena_[sp.cls].release(sp.off, sp.n);
                quarantined_[sp.cls] -= Arena::span(sp.n);
            }
            quarantine_.erase(quarantine_.begin() + q);
            did = true;
        }
        for (size_t s = 0; s < slot_jobs_.size(); ++s) {
            if (slot_jobs_[s].empty())
                continue;
            const int r = be_->poll((int)s);
            if (r == 0) {
                if (cfg_.deadline_s > 0 && be_->now() - slot_t_[s] > cfg_.deadline_s) {
                    expire((int)s);
                    did = true;
                }
                continue;
            }
            const double t = be_->now();
            for (Job &j : slot_jobs_[s]) {
                arena_[j.cls].release(j.off, j.n);
                --in_flight_;
                ++st_.completed;
                finish(j, r > 0 ? OK : E_DEVICE, t);
            }
            slot_jobs_[s].clear();
            did = true;
        }
        while (!queue_.empty() && in_flight_ < cfg_.max_in_flight) {
            Job &j = queue_.front();
            uint64_t off;
            if (!arena_[j.cls].alloc(j.n, &off))
                break;  // FIFO: wait for memory
            j.off = off;
            j.t_admit = be_->now();
            staged_.push_back(j);
            queue_.pop_front();
            ++in_flight_;
            did = true;
        }
        for (int k = 0; k < 2; ++k)
            st_.peak_slots[k] = std::max(st_.peak_slots[k], arena_[k].used());
        if (live_slots() == 0 && (!queue_.empty() || !staged_.empty())) {
            // no launch slot left: nothing waiting can run
            const double t = be_->now();
            for (Job &j : staged_) {
                arena_[j.cls].release(j.off, j.n);
                --in_flight_;
                ++st_.completed;
                finish(j, E_DEVICE, t);
            }
            staged_.clear();
            for (Job &j : queue_) {
                ++st_.completed;
                finish(j, E_DEVICE, t);
            }
            queue_.clear();
            did = true;
        }
        if (!staged_.empty()) {
            int slot = -1;
            for (size_t s = 0; s < slot_jobs_.size(); ++s)
                if (slot_jobs_[s].empty() && !slot_dead_[s]) {
                    slot = (int)s;
                    break;
                }
            if (slot >= 0) {
                const size_t take = std::min<size_t>(staged_.size(), cfg_.max_batch_jobs);
                std::vector<Job> &sj = slot_jobs_[slot];
                sj.assign(staged_.begin(), staged_.begin() + take);
                staged_.erase(staged_.begin(), staged_.begin() + take);
                std::vector<Job *> ptrs;
                ptrs.reserve(sj.size());
                const double t = be_->now();
                slot_t_[slot] = t;
                for (Job &j : sj) {
                    j.t_launch = t;
                    ptrs.push_back(&j);
                }
                if (be_->launch(slot, ptrs) != 0) {
                    for (Job &j : sj) {
                        arena_[j.cls].release(j.off, j.n);
                        --in_flight_;
                        ++st_.completed;
                        finish(j, E_DEVICE, be_->now());
                    }
                    sj.clear();
                } else {
                    ++st_.launches;
                    st_.jobs_launched += sj.size();
                }
                did = true;
            }
        }
        return did;
    }

    size_t take(Completion *out, size_t max)
    {
        size_t k = 0;
        while (k < max && !done_.empty()) {
            out[k++] = done_.front();
            done_.pop_front();
        }
        return k;
    }
    size_t pending_completions() const { return done_.size(); }

    // No job waits or runs (memory of retired batches may still be quarantined).
    bool idle() const
    {
        if (!queue_.empty() || !staged_.empty())
            return false;
        for (const auto &s : slot_jobs_)
            if (!s.empty())
                return false;
        return true;
    }
    // Work on the device to poll: launched batches or retired ones still running.
    bool device_busy() const
    {
        for (const Quarantine &q : quarantine_)
            if (q.ticket >= 0)
                return true;
        for (const auto &s : slot_jobs_)
            if (!s.empty())
                return true;
        return false;
    }

    Stats stats() const
    {
        Stats s = st_;
        s.used_slots[0] = arena_[0].used();
        s.used_slots[1] = arena_[1].used();
        s.queued = queue_.size();
        s.staged = staged_.size();
        s.in_flight = in_flight_;
        s.quarantined_slots[0] = quarantined_[0];
        s.quarantined_slots[1] = quarantined_[1];
        s.dead_slots = (uint64_t)std::count(slot_dead_.begin(), slot_dead_.end(), true);
        return s;
    }
    const Arena &arena(int k) const { return arena_[k]; }

  private:
    struct Span {
        uint32_t cls;
        uint64_t off, n;
    };
    struct Quarantine {
        int ticket;
        std::vector<Span> spans;
    };

    int live_slots() const { return (int)std::count(slot_dead_.begin(), slot_dead_.end(), false); }

    // Slot s's batch missed its deadline: its jobs fail now, its memory waits
    // for the retired work to end (forever if the slot cannot be renewed).
    void expire(int s)
    {
        const double t = be_->now();
        Quarantine q;
        for (Job &j : slot_jobs_[s]) {
            q.spans.push_back({j.cls, j.off, j.n});
            quarantined_[j.cls] += Arena::span(j.n);
            --in_flight_;
            ++st_.completed;
            ++st_.timed_out;
            finish(j, E_DEVICE, t);
        }
        slot_jobs_[s].clear();
        q.ticket = be_->retire(s);
        if (q.ticket < 0)
            slot_dead_[s] = true;
        quarantine_.push_back(std::move(q));
    }

    void finish(Job &j, int status, double t)
    {
        j.status = status;
        j.t_done = t;
        done_.push_back({j.id, status, j.t_submit, j.t_admit, j.t_launch, t});
    }

    Config cfg_;
    Backend *be_;
    Arena arena_[2];
    std::deque<Job> queue_;
    std::vector<Job> staged_;
    std::vector<std::vector<Job>> slot_jobs_;
    std::vector<double> slot_t_;  // launch time of the slot's batch
    std::vector<bool> slot_dead_;
    std::vector<Quarantine> quarantine_;
    uint64_t quarantined_[2] = {0, 0};
    std::deque<Completion> done_;
    uint64_t in_flight_ = 0;
    Stats st_;
};

}  // namespace mont_sched

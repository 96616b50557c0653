// Test harness: the serving scheduler core driven by a backend that only
// records launches.  The test decides when each launch slot finishes, so
// admission, batching and memory accounting can be checked deterministically
// on a machine without a GPU.
#include <cstdint>
#include <map>
#include <vector>

#include "../../paper_2402_00675_amd/csrc/mont_sched.hpp"

namespace {

struct FakeBackend : mont_sched::Backend {
    std::vector<int> state;                       // 0 running, 1 done, -1 failed
    std::vector<std::vector<uint64_t>> launched;  // job ids of the slot's current launch
    std::vector<std::vector<uint64_t>> offsets;
    int fail_next = 0, fail_retire = 0, next_ticket = 0;
    std::map<int, int> retired;                   // ticket -> 0 running, 1 done, -1 failed
    std::vector<int> retire_count;
    double clock = 0;
    explicit FakeBackend(int n) : state(n, 0), launched(n), offsets(n), retire_count(n, 0) {}
    int slots() const override { return (int)state.size(); }
    int launch(int s, const std::vector<mont_sched::Job *> &jobs) override
    {
        if (fail_next) {
            fail_next = 0;
            return -1;
        }
        launched[s].clear();
        offsets[s].clear();
        for (auto *j : jobs) {
            launched[s].push_back(j->id);
            offsets[s].push_back(j->off);
        }
        state[s] = 0;
        return 0;
    }
    int poll(int s) override { return state[s]; }
    double now() override { return clock; }  // advanced by the test
    int retire(int s) override
    {
        if (fail_retire) {
            fail_retire = 0;
            return -1;
        }
        ++retire_count[s];
        state[s] = 0;
        retired[next_ticket] = 0;
        return next_ticket++;
    }
    int poll_retired(int t) override
    {
        const int r = retired.at(t);
        if (r != 0)
            retired.erase(t);
        return r;
    }
};

struct Sim {
    FakeBackend be;
    mont_sched::Scheduler sched;
    char dummy[8];
    Sim(const mont_sched::Config &c, int slots) : be(slots), sched(c, &be) {}
};

}  // namespace

extern "C" {

void *sim_create(uint64_t cap32, uint64_t cap64, uint32_t max_in_flight, uint32_t max_batch, int slots,
                 double deadline_s)
{
    mont_sched::Config c;
    c.cap[0] = cap32;
    c.cap[1] = cap64;
    c.max_in_flight = max_in_flight;
    c.max_batch_jobs = max_batch;
    c.deadline_s = deadline_s;
    return new Sim(c, slots);
}

void sim_advance(void *p, double dt) { ((Sim *)p)->be.clock += dt; }

int sim_cancel(void *p, uint64_t id) { return ((Sim *)p)->sched.cancel(id); }

void sim_fail_next_retire(void *p) { ((Sim *)p)->be.fail_retire = 1; }

// Ends retired batch `ticket` with `status` (1 done, -1 failed); -1 if unknown.
int sim_finish_retired(void *p, int ticket, int status)
{
    Sim *s = (Sim *)p;
    auto it = s->be.retired.find(ticket);
    if (it == s->be.retired.end())
        return -1;
    it->second = status;
    return 0;
}

int sim_retire_count(void *p, int slot) { return ((Sim *)p)->be.retire_count[slot]; }

int sim_idle(void *p) { return ((Sim *)p)->sched.idle() ? 1 : 0; }

int sim_submit(void *p, uint64_t id, uint64_t N, uint32_t w, uint32_t op, uint64_t n)
{
    Sim *s = (Sim *)p;
    mont_sched::Job j;
    j.id = id;
    j.N = N;
    j.w = w;
    j.op = op;
    j.n = n;
    j.in0 = j.in1 = s->dummy;
    j.out = s->dummy;
    return s->sched.submit(j);
}

int sim_step(void *p) { return ((Sim *)p)->sched.step() ? 1 : 0; }

void sim_finish_slot(void *p, int slot, int status) { ((Sim *)p)->be.state[slot] = status; }

void sim_fail_next_launch(void *p) { ((Sim *)p)->be.fail_next = 1; }

int64_t sim_take(void *p, uint64_t *ids, int32_t *status, uint64_t max)
{
    std::vector<mont_sched::Completion> c(max);
    const size_t k = ((Sim *)p)->sched.take(c.data(), max);
    for (size_t i = 0; i < k; ++i) {
        ids[i] = c[i].id;
        status[i] = c[i].status;
    }
    return (int64_t)k;
}

int64_t sim_slot_jobs(void *p, int slot, uint64_t *ids, uint64_t *offs, uint64_t max)
{
    Sim *s = (Sim *)p;
    const auto &v = s->be.launched[slot];
    size_t k = 0;
    for (; k < v.size() && k < max; ++k) {
        ids[k] = v[k];
        offs[k] = s->be.offsets[slot][k];
    }
    return (int64_t)k;
}

void sim_stats(void *p, uint64_t *o)
{
    const mont_sched::Stats st = ((Sim *)p)->sched.stats();
    uint64_t v[] = {st.submitted,     st.completed,     st.rejected,  st.launches,
                    st.jobs_launched, st.used_slots[0], st.used_slots[1], st.peak_slots[0],
                    st.peak_slots[1], st.queued,        st.staged,      st.in_flight,
                    st.canceled,      st.timed_out,     st.quarantined_slots[0], st.quarantined_slots[1],
                    st.dead_slots};
    for (size_t i = 0; i < sizeof v / sizeof v[0]; ++i)
        o[i] = v[i];
}

void sim_destroy(void *p) { delete (Sim *)p; }

}  // extern "C"

// Serving loop: concurrent depth-first searches admitted first come first
// served by slots and device memory, each step call advancing every admitted
// search (or, under a per-call cap on children, the searches that waited
// longest) with one shared set of launches.
#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <vector>

#include "search.h"

using namespace fspbb;

namespace {

struct Job {
    int64_t id = 0;
    fsp_instance_s *inst = nullptr;
    int32_t ub0 = 0;
    int64_t pool_cap = 0, node_budget = 0;
    size_t est = 0;
    std::unique_ptr<Search> S;
};

struct Done {
    fsp_status status = FSP_OK;
    fsp_solve_result res{};
    std::vector<int32_t> perm;
};

// Device bytes a search holds right after Search::start.
size_t initial_bytes(int n, int64_t pool_cap, bool rows)
{
    Search S;
    S.n = n;
    S.pool_cap = pool_cap;
    S.cap_stack = initial_stack_rows(pool_cap);
    S.B.Kcap = pool_cap;
    S.B.Ccap = pool_cap;
    S.B.n = n;
    S.B.rows = rows;
    return S.device_bytes();
}

}  // namespace

struct fsp_server_s {
    int device = 0;
    fsp_server_config cfg{};
    TickContext ctx;
    int64_t next_id = 1;
    std::deque<std::unique_ptr<Job>> pending;
    std::deque<std::unique_ptr<Job>> active;  // front = waited longest for a step
    std::map<int64_t, Done> done;
    fsp_server_stats st{};

    // Device bytes of the admitted searches, without and with the shared
    // step scratch.
    size_t search_bytes() const
    {
        size_t b = 0;
        for (const auto &j : active)
            if (j->S) b += j->S->device_bytes();
        return b;
    }
    size_t mem_used() const { return search_bytes() + ctx.device_bytes(); }

    void finish(Job &j, fsp_status status)
    {
        Done d;
        d.status = status;
        if (j.S && (status == FSP_OK || status == FSP_BUDGET)) {
            d.perm.resize(j.S->n);
            j.S->result(&d.res, d.perm.data());
        }
        if (j.S) j.S->release(ctx.s);
        done[j.id] = std::move(d);
    }
};

extern "C" {

fsp_status fsp_server_create(const fsp_server_config *cfg, void *stream, fsp_server *out)
{
    if (!out) return FSP_E_INVAL;
    *out = nullptr;
    if (!cfg || cfg->mem_budget_bytes <= 0 || cfg->max_active < 1 || cfg->tick_children < 0) return FSP_E_INVAL;
    fsp_server_s *v = new (std::nothrow) fsp_server_s();
    if (!v) return FSP_E_NOMEM;
    if (hipGetDevice(&v->device) != hipSuccess) { delete v; return FSP_E_DEVICE; }
    v->cfg = *cfg;
    v->ctx.s = (hipStream_t)stream;
    *out = v;
    return FSP_OK;
}

fsp_status fsp_server_submit(fsp_server srv, fsp_instance inst, int32_t ub0, int64_t pool_cap,
                             int64_t node_budget, int64_t *id_out)
{
    if (!srv || !inst || !id_out || pool_cap < 1 || node_budget < 1 || (ub0 < 0 && ub0 != FSP_UB_NEH))
        return FSP_E_INVAL;
    if (inst->device != srv->device) return FSP_E_INVAL;
    auto j = std::make_unique<Job>();
    j->inst = inst;
    j->ub0 = ub0;
    j->pool_cap = pool_cap;
    j->node_budget = node_budget;
    j->est = initial_bytes(inst->n, pool_cap, !kids16_eligible(inst));
    if ((int64_t)j->est > srv->cfg.mem_budget_bytes) return FSP_E_NOMEM;
    j->id = srv->next_id++;
    *id_out = j->id;
    srv->pending.push_back(std::move(j));
    return FSP_OK;
}

fsp_status fsp_server_step(fsp_server srv, int64_t *done_ids, int32_t done_cap, int32_t *n_done,
                           fsp_server_stats *stats)
{
    if (!srv || done_cap < 0 || (done_cap > 0 && !done_ids)) return FSP_E_INVAL;
    DeviceGuard g(srv->device);
    if (!g.ok) return FSP_E_DEVICE;
    int32_t nd = 0;
    auto report = [&](int64_t id) {
        if (nd < done_cap) done_ids[nd] = id;
        ++nd;
    };

    // admission, first come first served; the admitted searches' roots are
    // bounded together.  With nothing admitted, the shared step scratch is
    // handed back if it alone would keep the next search out.
    const size_t budget = (size_t)srv->cfg.mem_budget_bytes;
    if (srv->active.empty() && !srv->pending.empty() &&
        srv->ctx.device_bytes() + srv->pending.front()->est > budget)
        srv->ctx.release();
    size_t used = srv->search_bytes();
    std::vector<std::unique_ptr<Job>> admit;
    std::vector<StartArgs> args;
    while (!srv->pending.empty() && srv->active.size() + admit.size() < (size_t)srv->cfg.max_active) {
        Job &j = *srv->pending.front();
        const bool first = srv->active.empty() && admit.empty();
        args.push_back(StartArgs{j.inst, j.ub0, j.pool_cap, j.node_budget});
        if (used + j.est + start_scratch_after(args, srv->ctx) > budget && !first) {
            args.pop_back();
            break;
        }
        used += j.est;
        admit.push_back(std::move(srv->pending.front()));
        srv->pending.pop_front();
    }
    if (!admit.empty()) {
        std::vector<Search *> ss;
        for (auto &jp : admit) {
            jp->S = std::make_unique<Search>();
            ss.push_back(jp->S.get());
        }
        hipError_t e = start_many(ss, args, srv->ctx);
        for (auto &jp : admit) {
            if (e != hipSuccess || jp->S->done) {
                srv->finish(*jp, e != hipSuccess ? fail_status(e) : jp->S->status);
                if (e == hipSuccess) srv->st.nodes_bounded += jp->S->nodes;
                report(jp->id);
                continue;
            }
            srv->st.nodes_bounded += jp->S->nodes;
            srv->active.push_back(std::move(jp));
        }
    }

    // the searches of this step: all, or those that waited longest up to the
    // children cap.  A search whose step would take the searches' memory and
    // the shared step scratch past the budget (its stack doubling, larger
    // step buffers, or bringing a moved-out stack back) is held back; it
    // keeps its place at the front.  When every search is held back, the
    // others' stacks go to host memory, largest first, until the search that
    // waited longest fits with a fresh step scratch; only a search that does
    // not fit even alone ends with FSP_E_NOMEM.
    std::vector<Search *> sel;
    std::vector<StepSel> qs;
    std::vector<char> picked(srv->active.size(), 0);
    int64_t children = 0;
    size_t grown = srv->search_bytes();
    for (size_t i = 0; i < srv->active.size(); ++i) {
        Search &S = *srv->active[i]->S;
        const StepSel q = select_step(S);
        if (srv->cfg.tick_children > 0 && !sel.empty() && children + q.nch > srv->cfg.tick_children) break;
        const size_t after = grown - S.device_bytes() + bytes_after_step(S, q);
        sel.push_back(&S);
        qs.push_back(q);
        if (after + tick_scratch_after(sel, qs, srv->ctx) > budget) {
            sel.pop_back();
            qs.pop_back();
            continue;
        }
        grown = after;
        picked[i] = 1;
        children += q.nch;
    }
    fsp_status ret = FSP_OK;
    if (sel.empty() && !srv->active.empty()) {
        Search &F = *srv->active[0]->S;
        const StepSel q0 = select_step(F);
        TickContext fresh;
        std::vector<Search *> one{&F};
        std::vector<StepSel> oq{q0};
        const size_t need = bytes_after_step(F, q0) + tick_scratch_after(one, oq, fresh);
        size_t others = srv->search_bytes() - F.device_bytes();
        std::vector<size_t> order;
        for (size_t i = 1; i < srv->active.size(); ++i) order.push_back(i);
        std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
            return srv->active[a]->S->device_bytes() > srv->active[b]->S->device_bytes();
        });
        for (size_t i : order) {
            if (need + others <= budget) break;
            Search &O = *srv->active[i]->S;
            if (O.swapped) continue;
            const size_t b0 = O.device_bytes();
            hipError_t e = O.swap_out(srv->ctx.s);
            if (e != hipSuccess) {
                ret = fail_status(e);
                break;
            }
            others = others - b0 + O.device_bytes();
            ++srv->st.swap_outs;
        }
        if (ret == FSP_OK && need + others <= budget) {
            srv->ctx.release();
            sel.push_back(&F);
            qs.push_back(q0);
            picked[0] = 1;
            children = q0.nch;
        } else if (ret == FSP_OK) {
            std::unique_ptr<Job> jp = std::move(srv->active[0]);
            srv->active.erase(srv->active.begin());
            srv->finish(*jp, FSP_E_NOMEM);
            report(jp->id);
            picked.erase(picked.begin());
        }
    }
    // moved-out stacks of the stepped searches come back first
    for (size_t i = 0; ret == FSP_OK && i < sel.size(); ++i) {
        if (!sel[i]->swapped) continue;
        hipError_t e = sel[i]->swap_in(srv->ctx.s);
        if (e != hipSuccess) ret = fail_status(e);
        else ++srv->st.swap_ins;
    }
    if (ret != FSP_OK) {
        for (auto &jp : srv->active) {
            srv->finish(*jp, ret);
            report(jp->id);
        }
        srv->active.clear();
        sel.clear();
    }
    if (!sel.empty()) {
        std::vector<int64_t> before(sel.size());
        for (size_t i = 0; i < sel.size(); ++i) before[i] = sel[i]->nodes;
        hipError_t e = tick(sel, srv->ctx);
        if (e != hipSuccess) {
            ret = fail_status(e);
            for (auto &jp : srv->active) {
                srv->finish(*jp, ret);
                report(jp->id);
            }
            srv->active.clear();
        } else {
            for (size_t i = 0; i < sel.size(); ++i) srv->st.nodes_bounded += sel[i]->nodes - before[i];
            ++srv->st.ticks;
            // stepped searches go to the back in their order; finished ones leave
            std::deque<std::unique_ptr<Job>> rest;
            for (size_t i = 0; i < srv->active.size(); ++i)
                if (!picked[i]) rest.push_back(std::move(srv->active[i]));
            for (size_t i = 0; i < srv->active.size(); ++i) {
                if (!picked[i]) continue;
                std::unique_ptr<Job> &jp = srv->active[i];
                if (jp->S->done) {
                    srv->finish(*jp, jp->S->status);
                    report(jp->id);
                } else {
                    rest.push_back(std::move(jp));
                }
            }
            srv->active.swap(rest);
        }
    }
    srv->st.active = (int32_t)srv->active.size();
    srv->st.pending = (int32_t)srv->pending.size();
    srv->st.mem_used = (int64_t)srv->mem_used();
    srv->st.last_children = ret == FSP_OK ? children : 0;
    srv->st.last_searches = ret == FSP_OK ? (int32_t)sel.size() : 0;
    if (n_done) *n_done = nd;
    if (stats) *stats = srv->st;
    return ret;
}

fsp_status fsp_server_poll(fsp_server srv, int64_t id, fsp_solve_result *res, int32_t *perm_out)
{
    if (!srv || !res) return FSP_E_INVAL;
    auto it = srv->done.find(id);
    if (it == srv->done.end()) {
        for (const auto &j : srv->active)
            if (j->id == id) return FSP_PENDING;
        for (const auto &j : srv->pending)
            if (j->id == id) return FSP_PENDING;
        return FSP_E_INVAL;
    }
    const Done &d = it->second;
    *res = d.res;
    if (perm_out && !d.perm.empty()) std::copy(d.perm.begin(), d.perm.end(), perm_out);
    const fsp_status st = d.status;
    srv->done.erase(it);
    return st;
}

fsp_status fsp_server_destroy(fsp_server srv)
{
    if (!srv) return FSP_OK;
    {
        DeviceGuard g(srv->device);
        hipStreamSynchronize(srv->ctx.s);
        for (auto &jp : srv->active)
            if (jp->S) jp->S->release(srv->ctx.s);
        srv->ctx.release();
    }
    delete srv;
    return FSP_OK;
}

}  // extern "C"

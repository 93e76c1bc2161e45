// Serving loop: many per-projection solves in flight at once, of different
// volume sizes, their work batched into shared launches.
//
// The caller hands the server one device arena.  A request is admitted when
// its workspace (ray table, warped volume, projection, reduction scratch)
// fits in the arena's free space and a slot is free; the volumes and modes
// of the registered models stay resident in the caller's memory.  Every
// step() runs one operation of every admitted request's solve state machine
// (an evaluation, a residual or a gradient; or the admission work; or the
// tumour localisation at the end), with each kind of operation for all
// requests in one launch per (dtype, K) or (dtype, slab axis) group, then
// reads back all their scalars in one transfer and advances the machines.
// Requests that arrive while others run are admitted at the next step as
// memory and slots free up.  A batched block runs exactly what the same
// block of the request's own launch runs, so every request's result is bit
// for bit the one solve_projection gives for it alone.
#include <algorithm>
#include <deque>
#include <map>
#include <vector>

#include "host.h"
#include "internal.h"
#include "solver.h"

using namespace pcas;
using namespace pcas::host;

namespace {

// scalars read back per request and step (the fused evaluation's sums are
// the most: eval_sums(K))
constexpr int GATHER = 72;
static_assert(eval_sums(PCAS_MAX_K) <= GATHER, "gather width");

struct Model {
    pcas_dtype dt;
    pcas_vol vol;
    VolDims vd;
    int K;
    const void *f0, *mean, *U;
};

enum Phase { PH_PREPARE, PH_RUN, PH_LOCATE, PH_DONE };

struct Request {
    int64_t id = 0;
    int model = 0;
    pcas_proj proj{};
    Frame fr{};
    ForwardPlan plan{};
    const void *y = nullptr;
    pcas_opts opts{};
    double w0[PCAS_MAX_K] = {0};
    SolveWs L{};
    size_t off = 0;
    char *ws = nullptr;
    int64_t M = 0;
    double sy = 0.0, syy = 0.0;
    SolveMachine m;
    Phase phase = PH_PREPARE;
    int status = PCAS_OK;
    double w[PCAS_MAX_K] = {0};
    pcas_report rep{};
    double cost = 0.0;   // relative GPU work of one of its operations (see op_cost)
    // reference fit of the next refitted FP32 evaluation's moments, and the
    // slot and reference of the moments in scal()[0..2] (as in a solve alone)
    double ref_a = 1.0, ref_b = 0.0;
    int mom_slot = -1;
    double mom_a0 = 0.0, mom_b0 = 0.0;
    FitArgs eval_fit{};   // the pending FP32 evaluation's fit and reference
    // a speculative gradient launched behind this pass's evaluation (as in a
    // solve alone): its point and slot, and how many were taken
    bool spec = false;
    int spec_slot = 0;
    double spec_w[PCAS_MAX_K] = {0};
    int spec_grads = 0;
    // grad_mode 2 (the fused evaluation): the projection plan of the K + 1
    // volumes and, per line-search slot, the point and sums of its last
    // evaluation, from which its gradient follows on the host
    ForwardPlan plan_e{};
    struct Fused {
        bool valid = false;
        double w[PCAS_MAX_K] = {0};
        double a0 = 0.0, b0 = 0.0;
        double m[eval_sums(PCAS_MAX_K)] = {0};
    } fused[2];
    bool fused_eval() const { return opts.grad_mode == 2; }

    double *scal() const { return (double *)(ws + L.scalars); }
    uint32_t *counters() const { return (uint32_t *)(ws + L.counters); }
    double *partials() const { return (double *)(ws + L.partials); }
    char *proj_slot(int slot) const { return ws + (slot ? L.p2 : L.p); }
};

// First-fit allocation over [0, size) in 256-byte units, coalescing on free.
class Arena {
public:
    void init(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += bytes;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align256(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
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
    size_t used() const { return used_; }

private:
    std::map<size_t, size_t> free_;
    size_t used_ = 0;
};

}  // namespace

struct pcas_server {
    hipStream_t s = nullptr;
    char *arena = nullptr;
    size_t arena_bytes = 0;
    int max_active = 0;
    Arena pool;                       // the arena beyond the reserved tables
    size_t pool_base = 0;
    // reserved at the start of the arena: job tables, gather pointers, gather output
    char *tables_dev = nullptr;
    size_t tables_bytes = 0;
    char *tables_host = nullptr;      // pinned staging of the tables
    double *gather_host = nullptr;    // pinned
    std::vector<Model> models;
    std::deque<Request *> pending;
    std::vector<Request *> active;
    std::map<int64_t, Request *> finished;
    int64_t next_id = 1;
    double substep_share = 0.25;      // extra passes for cheap requests (see step)
};

namespace {

size_t table_bytes(int max_active) {
    const size_t per = sizeof(WarpJob) + sizeof(FwdJob) + sizeof(ResJob) + sizeof(AdjJob) +
                       sizeof(SpecJob) + sizeof(double *) + sizeof(SumJob) +
                       GATHER * sizeof(double);
    return align256(per * (size_t)max_active + 4096);
}

// A request's workspace: the fused evaluation (grad_mode 2) also holds the
// warped image with its K Jacobian volumes and the wider reduction scratch.
SolveWs request_layout(const Model &md, const pcas_proj *proj, int grad_mode) {
    return solve_layout(md.dt, &md.vol, proj, md.K, grad_mode == 2);
}
size_t request_bytes(const Model &md, const pcas_proj *proj, int grad_mode) {
    return request_layout(md, proj, grad_mode).total;
}

void finish_request(pcas_server *S, Request *r, int status) {
    r->status = status;
    r->rep.spec_grads = r->spec_grads;
    r->phase = PH_DONE;
    S->pool.release(r->off, r->L.total);
    r->ws = nullptr;
    S->finished[r->id] = r;
}

// Work of a newly admitted request: counters, ray table, sums of y.
int admit(pcas_server *S, Request *r) {
    const Model &md = S->models[r->model];
    r->ws = S->arena + S->pool_base + r->off;
    HIPCHK(launch_fill_u32(r->counters(), 64, 0u, S->s));
    HIPCHK(launch_ray_table(md.dt, md.vd, r->fr, r->ws + r->L.rays, S->s));
    HIPCHK(launch_brick_live(md.vd, r->fr, (uint8_t *)(r->ws + r->L.live), S->s));
    HIPCHK(launch_pair_sums(md.dt, r->M, r->y, r->y, r->partials(), &r->counters()[2],
                            r->scal() + 16, S->s));
    r->phase = PH_PREPARE;
    return PCAS_OK;
}

// Appends jobs to a table in groups with a common launch key, assigning
// block0 within each group; returns (key, first job, count, blocks) per group.
template <class Job, class Key>
struct Groups {
    struct G {
        Key key;
        int first, count, blocks;
    };
    std::vector<std::pair<Key, Job>> items;
    std::vector<G> groups;
    void add(const Key &k, const Job &j) { items.push_back({k, j}); }
    // Writes the jobs to dst, grouped and in submission order within a group.
    size_t emit(Job *dst) {
        std::stable_sort(items.begin(), items.end(),
                         [](const auto &a, const auto &b) { return a.first < b.first; });
        groups.clear();
        int n = 0;
        for (size_t i = 0; i < items.size(); ++i) {
            if (i == 0 || !(items[i].first == items[i - 1].first))
                groups.push_back({items[i].first, n, 0, 0});
            G &g = groups.back();
            Job j = items[i].second;
            j.block0 = g.blocks;
            g.blocks += j.nblocks;
            g.count += 1;
            dst[n++] = j;
        }
        return (size_t)n;
    }
};

// The objective's fit at a request, as a solve alone takes it: (a, b) fixed
// if given, else Eq. A.1's refit if the request fits intensities, else (1, 0).
FitArgs fit_of(const Request &r, const double *ab_fixed) {
    FitArgs fa{FIT_FIXED, 1.0, 0.0, r.sy, r.syy, (double)r.M};
    if (ab_fixed) {
        fa.a = ab_fixed[0];
        fa.b = ab_fixed[1];
    } else if (r.opts.fit_intensity) {
        fa.mode = FIT_REFIT;
    }
    return fa;
}

ResJob res_job(const Request &r, int slot, const FitArgs &fa) {
    ResJob rj;
    rj.M = r.M;
    rj.p = r.proj_slot(slot);
    rj.y = r.y;
    rj.fa = fa;
    rj.src = r.scal();
    rj.partials = r.partials();
    rj.counter = &r.counters()[3];
    rj.out = r.scal() + 3;
    rj.block0 = 0;
    rj.nblocks = sums_blocks(r.M);
    return rj;
}

// Advances one request with the scalars its operation produced (jab: J, a,
// b of an evaluation formed on the host, else sc[3..5]).
void advance(pcas_server *S, Request *r, const double *sc, int32_t *n_done,
             const double *jab = nullptr, const double *H = nullptr) {
    const Model &md = S->models[r->model];
    bool done = false;
    int status = PCAS_OK;
    if (r->phase == PH_PREPARE) {
        r->sy = sc[16];
        r->syy = sc[18];
        if (!isfinite(r->sy) || !isfinite(r->syy)) {
            status = PCAS_ENONFINITE;
            done = true;
        } else if (r->opts.fit_intensity) {
            const double m = (double)r->M, det = r->syy * m - r->sy * r->sy;
            if (!(fabs(det) > 1e-12 * r->syy * m)) {
                status = PCAS_ESINGULAR;
                done = true;
            }
        }
        if (!done) {
            r->m.start(r->opts, md.K, noise_model(md.dt, r->opts, r->M, r->sy, r->syy), r->w0);
            r->phase = PH_RUN;
        }
    } else if (r->phase == PH_RUN) {
        const SolveOp &op = r->m.op();
        if (op.kind == OP_EVAL || op.kind == OP_RESID) {
            const double J = jab ? jab[0] : sc[3], a = jab ? jab[1] : sc[4], b = jab ? jab[2] : sc[5];
            if (!isfinite(a) || !isfinite(b)) {
                status = PCAS_ESINGULAR;
                done = true;
            } else if (!isfinite(J)) {
                status = PCAS_ENONFINITE;
                done = true;
            } else {
                r->ref_a = a;
                r->ref_b = b;
                r->m.eval_result(J, a, b);
            }
        } else if (op.kind == OP_GRAD) {
            for (int k = 0; k < md.K; ++k)
                if (!isfinite(sc[8 + k])) {
                    status = PCAS_ENONFINITE;
                    done = true;
                }
            if (!done) r->m.grad_result(sc + 8, H);
        }
        if (!done && r->m.done()) {
            r->rep = r->m.report();
            for (int k = 0; k < md.K; ++k) r->w[k] = r->m.w()[k];
            if (r->opts.locate)
                r->phase = PH_LOCATE;
            else
                done = true;
        }
        if (done && status != PCAS_OK) r->rep = r->m.report();
    } else if (r->phase == PH_LOCATE) {
        for (int c = 0; c < 3; ++c) r->rep.tumour_mm[c] = sc[24 + c];
        r->rep.locate_iters = (int32_t)sc[27];
        done = true;
    }
    if (done) {
        finish_request(S, r, status);   // phase becomes PH_DONE
        ++*n_done;
    }
}

// Queues the gradient at an evaluation's point behind it, gated by the
// request's gate (a, b, go) at scal()[SCAL_GATE]: the same job a gradient pass
// would run, and its sum in the gather (skipped when the gate is shut).
template <class Groups_>
void speculate(const Model &md, Request *r, const SolveOp &op, Groups_ &adjs, SumJob &sj) {
    AdjJob aj = make_adj_job(md.vd, r->fr, md.K, r->ws + r->L.rays, r->proj_slot(op.slot), r->y, 0.0,
                             0.0, md.f0, md.mean, md.U, op.w, r->partials(), nullptr, r->scal() + 8);
    aj.gate = r->scal() + SCAL_GATE;
    adjs.add({md.dt, md.K}, aj);
    sj = SumJob{};
    sj.partials = r->partials();
    sj.out = r->scal() + 8;
    sj.scale = 2.0;
    sj.nblocks = aj.nblocks;
    sj.width = ADJ_THREADS;
    sj.ns = md.K;
    sj.offset = 8;
    sj.gate = r->scal() + SCAL_GATE;
    r->spec = true;
    r->spec_slot = op.slot;
    for (int k = 0; k < md.K; ++k) r->spec_w[k] = op.w[k];
}

// After an evaluation's result: when the gate opened and the machine asks
// for the gradient at exactly that point, fit and slot, feed it the one
// that came back with the evaluation.
void take_speculative_gradient(pcas_server *S, Request *r, const double *sc, int32_t *n_done) {
    if (!r->spec) return;
    r->spec = false;
    if (r->phase != PH_RUN || sc[SCAL_GATE + 2] == 0.0) return;
    const SolveOp &op = r->m.op();
    const int K = S->models[r->model].K;
    if (op.kind != OP_GRAD || op.slot != r->spec_slot ||
        memcmp(op.w, r->spec_w, K * sizeof(double)) || memcmp(&op.ab[0], &sc[SCAL_GATE], sizeof(double)) ||
        memcmp(&op.ab[1], &sc[SCAL_GATE + 1], sizeof(double)))
        return;
    ++r->spec_grads;
    advance(S, r, sc, n_done);   // OP_GRAD: the gradient at sc[8..]
}

// grad_mode 2: while the machine asks for the gradient at the point whose
// sums a slot holds, the gradient follows from them on the host (as
// solve_projection forms it) and the machine advances without a launch.
void feed_fused_gradients(pcas_server *S, Request *r, int32_t *n_done) {
    const int K = S->models[r->model].K;
    while (r->fused_eval() && r->phase == PH_RUN) {
        const SolveOp &op = r->m.op();
        if (op.kind != OP_GRAD) return;
        const Request::Fused &F = r->fused[op.slot];
        if (!F.valid || memcmp(F.w, op.w, K * sizeof(double))) return;
        double sc[GATHER] = {0}, H[PCAS_MAX_K * PCAS_MAX_K];
        gradient_from_moments(F.m, K, op.ab[0], op.ab[1], F.a0, F.b0, sc + 8);
        gn_matrix_from_moments(F.m, K, r->opts.fit_intensity != 0, r->sy, r->syy, (double)r->M, H);
        advance(S, r, sc, n_done, nullptr, H);   // OP_GRAD: the gradient at sc[8..]
    }
}

// One pass: the next operation of every request in `set`, batched by kind
// (one launch per kind, dtype and K or slab axis), one read-back, and every
// machine advanced.  Finished requests leave with phase PH_DONE.
int run_pass(pcas_server *S, const std::vector<Request *> &set, int32_t *n_done) {
    if (set.empty()) return PCAS_OK;

    // this pass's operations, batched
    typedef std::pair<int, int> DK;   // (dtype, K) or (dtype, axis)
    Groups<WarpJob, DK> warps, warpjacs;
    Groups<FwdJob, DK> fwds, fwd_evals;   // fwd_evals: (16 dtype + K, axis + 2 tile shape)
    Groups<ResJob, int> ress;
    Groups<AdjJob, DK> adjs;
    std::vector<SpecJob> specs;
    std::vector<Request *> locates, refused;
    // FP32 projections and all gradients leave block partials only; the
    // gather finishes each request's sum (same order as a solve alone)
    std::vector<SumJob> sums(set.size());
    for (size_t ri = 0; ri < set.size(); ++ri) {
        Request *r = set[ri];
        const Model &md = S->models[r->model];
        if (r->phase == PH_LOCATE) {
            locates.push_back(r);
            continue;
        }
        if (r->phase != PH_RUN) continue;
        const SolveOp &op = r->m.op();
        if (op.kind == OP_EVAL && r->fused_eval()) {
            // the warp with the Jacobian volumes, then one projection of all
            // K + 1 that leaves the objective's moments and the gradient's
            // sums (FP32: finished by the gather; FP64: by the projection's
            // last block, then the two-pass residual below writes J, a, b
            // in front of the gradient's sums)
            r->fused[op.slot].valid = false;
            WarpJob wj;
            wj.vd = md.vd;
            wj.f0 = md.f0;
            wj.mean = md.mean;
            wj.U = md.U;
            wj.w = WVec{};
            for (int k = 0; k < md.K; ++k) wj.w.w[k] = op.w[k];
            wj.f = r->ws + r->L.vol2;
            wj.block0 = 0;
            wj.nblocks = warp_jac_blocks(nvox_of(&md.vol));
            wj.live = (const uint8_t *)(r->ws + r->L.live);
            warpjacs.add({md.dt, md.K}, wj);
            FitArgs ff = fit_of(*r, op.fixed_ab ? op.ab : nullptr);
            if (md.dt == PCAS_F32) {
                ff.a0 = ff.mode == FIT_FIXED ? ff.a : r->ref_a;
                ff.b0 = ff.mode == FIT_FIXED ? ff.b : r->ref_b;
            }
            const bool defer = md.dt == PCAS_F32;
            const FwdJob fj = make_fwd_job(md.vd, r->fr, r->plan_e, r->ws + r->L.rays,
                                           r->ws + r->L.vol2, r->proj_slot(op.slot), r->y, ff,
                                           r->partials(), defer ? nullptr : &r->counters()[0],
                                           r->scal());
            fwd_evals.add({16 * (int)md.dt + md.K, r->plan_e.axis + 2 * r->plan_e.tile}, fj);
            if (defer) {
                SumJob &sj = sums[ri];
                sj.partials = r->partials();
                sj.out = r->scal();
                sj.scale = 1.0;
                sj.nblocks = fj.nblocks;
                sj.width = EVAL_SUM_WIDTH;
                sj.ns = eval_sums(md.K);
                sj.offset = 0;
            }
            r->mom_slot = op.slot;
            r->mom_a0 = ff.a0;
            r->mom_b0 = ff.b0;
            r->eval_fit = ff;
            r->spec = false;
        } else if (op.kind == OP_EVAL) {
            WarpJob wj;
            wj.vd = md.vd;
            wj.f0 = md.f0;
            wj.mean = md.mean;
            wj.U = md.U;
            wj.w = WVec{};
            for (int k = 0; k < md.K; ++k) wj.w.w[k] = op.w[k];
            wj.f = r->ws + r->L.f;
            wj.block0 = 0;
            wj.nblocks = warp_blocks(nvox_of(&md.vol));
            wj.live = (const uint8_t *)(r->ws + r->L.live);
            warps.add({md.dt, md.K}, wj);
            // the objective as a solve alone forms it: FP32 from moments about
            // the reference fit in the projection's last block, FP64 by the
            // two-pass residual below
            FitArgs ff = fit_of(*r, op.fixed_ab ? op.ab : nullptr);
            if (md.dt == PCAS_F32) {
                ff.a0 = ff.mode == FIT_FIXED ? ff.a : r->ref_a;
                ff.b0 = ff.mode == FIT_FIXED ? ff.b : r->ref_b;
            } else {
                ff.mode = FIT_NONE;
            }
            const bool defer = md.dt == PCAS_F32;   // FP64's residual reads the sums on the GPU
            const FwdJob fj = make_fwd_job(md.vd, r->fr, r->plan, r->ws + r->L.rays, r->ws + r->L.f,
                                           r->proj_slot(op.slot), r->y, ff, r->partials(),
                                           defer ? nullptr : &r->counters()[0], r->scal());
            fwds.add({md.dt, r->plan.axis}, fj);
            if (defer) {
                SumJob &sj = sums[ri];
                sj.partials = r->partials();
                sj.out = r->scal();
                sj.scale = 1.0;
                sj.nblocks = fj.nblocks;
                sj.width = FWD_THREADS;
                sj.ns = 3;
                sj.offset = 0;
            }
            r->mom_slot = op.slot;
            r->mom_a0 = ff.a0;
            r->mom_b0 = ff.b0;
            r->eval_fit = ff;
            r->spec = false;
            if (defer && r->opts.speculate && r->opts.grad_mode == 1 &&
                op.next_grad.mode != GRAD_NEVER) {
                SpecJob sp;
                sp.partials = r->partials();
                sp.nblocks = fj.nblocks;
                sp.fit = ff;
                sp.rule = op.next_grad;
                sp.mo = r->scal();
                sp.gate = r->scal() + SCAL_GATE;
                specs.push_back(sp);
                speculate(md, r, op, adjs, sums[ri]);
            }
        }
        if ((op.kind == OP_EVAL && md.dt != PCAS_F32) || op.kind == OP_RESID) {
            FitArgs fa = fit_of(*r, op.fixed_ab ? op.ab : nullptr);
            if (fa.mode == FIT_REFIT) {   // the refit reads the moments of this slot's projection
                if (op.slot != r->mom_slot) {
                    refused.push_back(r);
                    continue;
                }
                fa.a0 = r->mom_a0;
                fa.b0 = r->mom_b0;
            }
            ress.add(md.dt, res_job(*r, op.slot, fa));
            if (op.kind == OP_EVAL && r->opts.speculate && r->opts.grad_mode == 1 &&
                op.next_grad.mode != GRAD_NEVER) {
                SpecJob sp;   // FP64: the gate reads the two-pass residual's (J, a, b)
                sp.jab = r->scal() + 3;
                sp.rule = op.next_grad;
                sp.gate = r->scal() + SCAL_GATE;
                specs.push_back(sp);
                speculate(md, r, op, adjs, sums[ri]);
            }
        } else if (op.kind == OP_GRAD) {
            const AdjJob aj = make_adj_job(md.vd, r->fr, md.K, r->ws + r->L.rays, r->proj_slot(op.slot),
                                           r->y, op.ab[0], op.ab[1], md.f0, md.mean, md.U, op.w,
                                           r->partials(), nullptr, r->scal() + 8);
            adjs.add({md.dt, md.K}, aj);
            SumJob &sj = sums[ri];
            sj.partials = r->partials();
            sj.out = r->scal() + 8;
            sj.scale = 2.0;
            sj.nblocks = aj.nblocks;
            sj.width = ADJ_THREADS;
            sj.ns = md.K;
            sj.offset = 8;
        }
    }
    // tables: [warp jobs][fwd jobs][res jobs][adj jobs][gather pointers][gather out]
    const int na = (int)set.size();
    char *h = S->tables_host;
    size_t o = 0;
    auto carve = [&](size_t bytes) {
        const size_t at = o;
        o = (o + bytes + 255) & ~(size_t)255;
        return at;
    };
    const size_t o_w = carve(warps.items.size() * sizeof(WarpJob));
    warps.emit((WarpJob *)(h + o_w));
    const size_t o_wj = carve(warpjacs.items.size() * sizeof(WarpJob));
    warpjacs.emit((WarpJob *)(h + o_wj));
    const size_t o_f = carve(fwds.items.size() * sizeof(FwdJob));
    fwds.emit((FwdJob *)(h + o_f));
    const size_t o_fe = carve(fwd_evals.items.size() * sizeof(FwdJob));
    fwd_evals.emit((FwdJob *)(h + o_fe));
    const size_t o_r = carve(ress.items.size() * sizeof(ResJob));
    ress.emit((ResJob *)(h + o_r));
    const size_t o_a = carve(adjs.items.size() * sizeof(AdjJob));
    adjs.emit((AdjJob *)(h + o_a));
    const size_t o_sp = carve(specs.size() * sizeof(SpecJob));
    for (size_t i = 0; i < specs.size(); ++i) ((SpecJob *)(h + o_sp))[i] = specs[i];
    const size_t o_p = carve(na * sizeof(double *));
    for (int i = 0; i < na; ++i) ((const double **)(h + o_p))[i] = set[i]->scal();
    const size_t o_s = carve(na * sizeof(SumJob));
    for (int i = 0; i < na; ++i) ((SumJob *)(h + o_s))[i] = sums[i];
    const size_t o_g = carve(na * GATHER * sizeof(double));
    if (o > S->tables_bytes) return hip_fail(hipErrorInvalidValue, "serving tables overflow");
    HIPCHK(hipMemcpyAsync(S->tables_dev, h, o_g, hipMemcpyHostToDevice, S->s));
    char *d = S->tables_dev;
    for (auto &g : warps.groups)
        HIPCHK(launch_warp_pca_batch((pcas_dtype)g.key.first, g.key.second,
                                     (const WarpJob *)(d + o_w) + g.first, g.count, g.blocks, S->s));
    for (auto &g : warpjacs.groups)
        HIPCHK(launch_warp_jac_batch((pcas_dtype)g.key.first, g.key.second,
                                     (const WarpJob *)(d + o_wj) + g.first, g.count, g.blocks, S->s));
    for (auto &g : fwds.groups)
        HIPCHK(launch_drr_forward_sums_batch((pcas_dtype)g.key.first, g.key.second,
                                             (const FwdJob *)(d + o_f) + g.first, g.count, g.blocks,
                                             S->s));
    for (auto &g : fwd_evals.groups)
        HIPCHK(launch_drr_forward_eval_batch((pcas_dtype)(g.key.first / 16), g.key.first % 16,
                                             g.key.second & 1, g.key.second >> 1,
                                             (const FwdJob *)(d + o_fe) + g.first, g.count,
                                             g.blocks, S->s));
    for (auto &g : ress.groups)
        HIPCHK(launch_residual_batch((pcas_dtype)g.key, (const ResJob *)(d + o_r) + g.first,
                                     g.count, g.blocks, S->s));
    // the gates of the speculative gradients, after the evaluations they read
    HIPCHK(launch_spec_decide_batch((const SpecJob *)(d + o_sp), (int)specs.size(), S->s));
    for (auto &g : adjs.groups)
        HIPCHK(launch_drr_adjoint_chain_batch((pcas_dtype)g.key.first, g.key.second,
                                              (const AdjJob *)(d + o_a) + g.first, g.count,
                                              g.blocks, S->s));
    for (Request *r : locates) {
        const Model &md = S->models[r->model];
        HIPCHK(launch_locate(md.dt, md.vd, md.K, md.mean, md.U, r->w, r->opts.c0_mm,
                             r->opts.locate_tol, r->opts.locate_max_iter, r->scal() + 24, S->s));
    }
    HIPCHK(launch_gather_scalars((const double *const *)(d + o_p), (double *)(d + o_g), na, GATHER,
                                 (const SumJob *)(d + o_s), S->s));
    HIPCHK(hipMemcpyAsync(S->gather_host, d + o_g, na * GATHER * sizeof(double),
                          hipMemcpyDeviceToHost, S->s));
    HIPCHK(hipStreamSynchronize(S->s));

    // advance every request of the pass with its results; FP32 evaluations
    // whose moment sum for J would cancel wait for the two-pass residual
    std::vector<Request *> redo;
    for (int i = 0; i < na; ++i) {
        Request *r = set[i];
        const double *sc = S->gather_host + i * GATHER;
        if (std::find(refused.begin(), refused.end(), r) != refused.end()) {
            host::g_last_error = "serving: refit without moments";
            finish_request(S, r, PCAS_EHIP);
            ++*n_done;
            continue;
        }
        if (r->phase == PH_RUN && r->m.op().kind == OP_EVAL && r->fused_eval()) {
            // keep the sums the evaluation left in its slot (the gradient's
            // part: sc[6..]; FP64's J, a, b are at sc[3..5])
            const SolveOp &op = r->m.op();
            const int K = S->models[r->model].K;
            Request::Fused &F = r->fused[op.slot];
            for (int j = 0; j < eval_sums(K); ++j) F.m[j] = sc[j];
            for (int k = 0; k < K; ++k) F.w[k] = op.w[k];
            F.a0 = r->eval_fit.a0;
            F.b0 = r->eval_fit.b0;
            F.valid = true;
        }
        if (r->phase == PH_RUN && r->m.op().kind == OP_EVAL && S->models[r->model].dt == PCAS_F32) {
            // the objective from the projection's moments, as a solve alone forms it
            double jab[3], kappa;
            objective_from_moments(sc, r->eval_fit, &jab[0], &jab[1], &jab[2], &kappa);
            if (isfinite(jab[1]) && isfinite(jab[2]) && !(kappa <= MOMENT_KAPPA_MAX)) {
                r->eval_fit.a = jab[1];   // the fit found, for the two-pass sum
                r->eval_fit.b = jab[2];
                r->spec = false;          // its gate stayed shut (kappa)
                redo.push_back(r);
                continue;
            }
            advance(S, r, sc, n_done, jab);
            take_speculative_gradient(S, r, sc, n_done);
            feed_fused_gradients(S, r, n_done);
            continue;
        }
        advance(S, r, sc, n_done);
        take_speculative_gradient(S, r, sc, n_done);
        feed_fused_gradients(S, r, n_done);
    }
    if (redo.empty()) return PCAS_OK;

    // the two-pass residual at the fits found, for those evaluations
    std::vector<ResJob> rj;
    for (Request *r : redo) {
        FitArgs fa = fit_of(*r, nullptr);
        fa.mode = FIT_FIXED;
        fa.a = r->eval_fit.a;
        fa.b = r->eval_fit.b;
        ResJob j = res_job(*r, r->m.op().slot, fa);
        j.block0 = 0;
        rj.push_back(j);
    }
    const int nr = (int)redo.size();
    o = 0;
    const size_t o_r2 = carve(nr * sizeof(ResJob));
    int blocks = 0;
    for (int i = 0; i < nr; ++i) {   // one dtype (FP32): a single launch
        rj[i].block0 = blocks;
        blocks += rj[i].nblocks;
        ((ResJob *)(h + o_r2))[i] = rj[i];
    }
    const size_t o_p2 = carve(nr * sizeof(double *));
    for (int i = 0; i < nr; ++i) ((const double **)(h + o_p2))[i] = redo[i]->scal();
    const size_t o_g2 = carve(nr * GATHER * sizeof(double));
    if (o > S->tables_bytes) return hip_fail(hipErrorInvalidValue, "serving tables overflow");
    HIPCHK(hipMemcpyAsync(S->tables_dev, h, o_g2, hipMemcpyHostToDevice, S->s));
    HIPCHK(launch_residual_batch(PCAS_F32, (const ResJob *)(d + o_r2), nr, blocks, S->s));
    HIPCHK(launch_gather_scalars((const double *const *)(d + o_p2), (double *)(d + o_g2), nr,
                                 GATHER, nullptr, S->s));
    HIPCHK(hipMemcpyAsync(S->gather_host, d + o_g2, nr * GATHER * sizeof(double),
                          hipMemcpyDeviceToHost, S->s));
    HIPCHK(hipStreamSynchronize(S->s));
    for (int i = 0; i < nr; ++i) {
        advance(S, redo[i], S->gather_host + i * GATHER, n_done);
        feed_fused_gradients(S, redo[i], n_done);
    }
    return PCAS_OK;
}

// Relative work of one operation of a request: its warp streams the volume
// (N voxels) and its projection marches about M * diagonal / step samples.
double op_cost(const Model &md, const Request &r) {
    double diag = 0.0;
    for (int c = 0; c < 3; ++c) {
        const double e = (md.vol.n[c] - 1) * md.vol.spacing[c];
        diag += e * e;
    }
    return (double)nvox_of(&md.vol) + (double)r.M * sqrt(diag) / r.proj.step;
}

int step(pcas_server *S, int32_t *n_done) {
    *n_done = 0;
    // 1. admission: every pending request that fits, in arrival order
    for (auto it = S->pending.begin(); it != S->pending.end() && (int)S->active.size() < S->max_active;) {
        Request *r = *it;
        if (!S->pool.alloc(r->L.total, &r->off)) {
            ++it;
            continue;
        }
        int st = admit(S, r);
        if (st) return st;
        r->cost = op_cost(S->models[r->model], *r);
        S->active.push_back(r);
        it = S->pending.erase(it);
    }

    if (S->active.empty()) return PCAS_OK;

    // main pass: every admitted request
    int st = run_pass(S, S->active, n_done);
    if (st) return st;
    // extra passes for the cheap requests (operation cost at most a quarter of
    // the most expensive one's) while their summed cost stays within
    // substep_share of the main pass's: small requests then advance several
    // operations while large ones advance one, instead of waiting out every
    // large step.
    if (S->substep_share > 0.0) {
        double main_cost = 0.0, max_cost = 0.0;
        for (Request *r : S->active) {
            main_cost += r->cost;
            max_cost = fmax(max_cost, r->cost);
        }
        double spent = 0.0;
        for (int pass = 0; pass < 64; ++pass) {
            std::vector<Request *> small;
            double c = 0.0;
            for (Request *r : S->active)
                if ((r->phase == PH_RUN || r->phase == PH_LOCATE) && r->cost <= 0.25 * max_cost) {
                    small.push_back(r);
                    c += r->cost;
                }
            if (small.empty() || spent + c > S->substep_share * main_cost) break;
            if ((st = run_pass(S, small, n_done))) return st;
            spent += c;
        }
    }
    std::vector<Request *> still;
    for (Request *r : S->active)
        if (r->phase != PH_DONE) still.push_back(r);
    S->active.swap(still);
    return PCAS_OK;
}
}  // namespace

extern "C" {

size_t pcas_server_reserved_bytes(int32_t max_active) {
    return max_active < 1 ? 0 : table_bytes(max_active);
}

int pcas_server_create(void *arena, size_t arena_bytes, int32_t max_active, void *stream,
                       pcas_server **out) {
    if (!out || !arena || !aligned(arena, 256) || max_active < 1 || max_active > 4096)
        return PCAS_EINVAL;
    const size_t tb = table_bytes(max_active);
    if (arena_bytes < tb + 256) return PCAS_EWORKSPACE;
    pcas_server *S = new pcas_server();
    S->s = (hipStream_t)stream;
    S->arena = (char *)arena;
    S->arena_bytes = arena_bytes;
    S->max_active = max_active;
    S->tables_dev = S->arena;
    S->tables_bytes = tb;
    S->pool_base = tb;
    S->pool.init((arena_bytes - tb) & ~(size_t)255);
    hipError_t e = hipHostMalloc((void **)&S->tables_host, tb, hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&S->gather_host, (size_t)max_active * GATHER * sizeof(double),
                          hipHostMallocDefault);
    if (e != hipSuccess) {
        if (S->tables_host) (void)hipHostFree(S->tables_host);
        delete S;
        return hip_fail(e, "hipHostMalloc(serving tables)");
    }
    *out = S;
    return PCAS_OK;
}

int pcas_server_destroy(pcas_server *S) {
    if (!S) return PCAS_EINVAL;
    for (Request *r : S->pending) delete r;
    for (Request *r : S->active) delete r;
    for (auto &kv : S->finished) delete kv.second;
    if (S->tables_host) (void)hipHostFree(S->tables_host);
    if (S->gather_host) (void)hipHostFree(S->gather_host);
    delete S;
    return PCAS_OK;
}

int pcas_server_add_model(pcas_server *S, pcas_dtype dtype, const pcas_vol *vol, int32_t K,
                          const void *f0, const void *mean, const void *U, int32_t *model_id) {
    if (!S || !dtype_ok(dtype) || K < 1 || K > PCAS_MAX_K || !f0 || !U || !model_id)
        return PCAS_EINVAL;
    int st = check_vol(vol);
    if (st) return st;
    if ((st = check_vol_bytes(vol, dtype))) return st;
    Model md{dtype, *vol, make_dims(vol), K, f0, mean, U};
    S->models.push_back(md);
    *model_id = (int32_t)S->models.size() - 1;
    return PCAS_OK;
}

size_t pcas_server_request_bytes(pcas_server *S, int32_t model_id, const pcas_proj *proj,
                                 const pcas_opts *opts) {
    if (!S || model_id < 0 || model_id >= (int)S->models.size()) return 0;
    const Model &md = S->models[model_id];
    if (check_proj(proj, &md.vol) != PCAS_OK) return 0;
    pcas_opts o;
    if (!opts) pcas_default_opts(&o);
    return request_bytes(md, proj, opts ? opts->grad_mode : o.grad_mode);
}

int pcas_server_submit(pcas_server *S, int32_t model_id, const pcas_proj *proj, const void *y,
                       const double *w0, const pcas_opts *opts, int64_t *request_id) {
    if (!S || model_id < 0 || model_id >= (int)S->models.size() || !y || !w0 || !request_id)
        return PCAS_EINVAL;
    const Model &md = S->models[model_id];
    int st = check_proj(proj, &md.vol);
    if (st) return st;
    if ((st = check_opts(opts))) return st;
    if (opts->grad_mode == 0) return PCAS_EINVAL;   // routes 1 and 2 are served
    if (!finite_vec(w0, md.K)) return PCAS_ENONFINITE;
    const size_t need = request_bytes(md, proj, opts->grad_mode);
    if (need > S->arena_bytes - S->pool_base) return PCAS_EWORKSPACE;   // could never be admitted
    Request *r = new Request();
    r->id = S->next_id++;
    r->model = model_id;
    r->proj = *proj;
    r->fr = make_frame(proj);
    r->plan = plan_drr_forward(md.dt, md.vd, r->fr, 1);
    if (opts->grad_mode == 2) r->plan_e = plan_drr_forward(md.dt, md.vd, r->fr, md.K + 1);
    r->y = y;
    r->opts = *opts;
    for (int k = 0; k < md.K; ++k) r->w0[k] = w0[k];
    r->L = request_layout(md, proj, opts->grad_mode);
    r->M = npix_of(proj);
    S->pending.push_back(r);
    *request_id = r->id;
    return PCAS_OK;
}

int pcas_server_step(pcas_server *S, int32_t *n_completed) {
    if (!S || !n_completed) return PCAS_EINVAL;
    return step(S, n_completed);
}

int pcas_server_poll(pcas_server *S, int64_t request_id, double *w_out, pcas_report *report,
                     int32_t *done) {
    if (!S || !done) return PCAS_EINVAL;
    auto it = S->finished.find(request_id);
    if (it == S->finished.end()) {
        *done = 0;
        return PCAS_OK;
    }
    Request *r = it->second;
    const int K = S->models[r->model].K;
    if (w_out)
        for (int k = 0; k < K; ++k) w_out[k] = r->w[k];
    if (report) *report = r->rep;
    const int status = r->status;
    S->finished.erase(it);
    delete r;
    *done = 1;
    return status;
}

int pcas_server_set_substep_share(pcas_server *S, double share) {
    if (!S || !(share >= 0.0 && share <= 16.0)) return PCAS_EINVAL;
    S->substep_share = share;
    return PCAS_OK;
}

int pcas_server_stats(pcas_server *S, int32_t *n_pending, int32_t *n_active, size_t *arena_used) {
    if (!S) return PCAS_EINVAL;
    if (n_pending) *n_pending = (int32_t)S->pending.size();
    if (n_active) *n_active = (int32_t)S->active.size();
    if (arena_used) *arena_used = S->pool.used() + S->pool_base;
    return PCAS_OK;
}

}  // extern "C"

// chi0_batch.cpp -- the batched entry point: many independent chi0 problems run as one fused
// launch sequence over a flat table of (instance, q, frequency-chunk) items.
//
// Schedule (computed on the host, identical for chi0_batch_workspace_size and create):
//   * an item is one instance, one q and up to 512 frequencies; (instance, q) groups share the
//     matrix elements W of that q;
//   * each item gets K_B workgroups in proportion to its estimated cost (64-unit rounds times
//     64-frequency slots), 1..1024 and at most one per round;
//   * groups are cut into stages whose W fits the stage budget; every stage is one K_A launch
//     over its groups' k-tiles, one K_B launch over its items' workgroups, one K_R launch;
//   * inside a stage the K_B workgroups are ordered by decreasing cost per workgroup, so the
//     hardware dispatcher hands out the longest work first (longest-job-first without a
//     device queue, and deterministic: every workgroup owns a fixed slice of partial sums);
//   * before its K_B launch a stage takes the band ranges of its groups (e(k) and e(k+q) of each
//     window band), from which K_B skips the band pairs with no carved region, as the single-plan
//     calls do.
// Workspace: [item table | K_A, K_B, K_R block->item tables and group->item tables |
//             W arena | partial-sum arena | band ranges of every group].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "chi0_host.h"
#include "chi0_internal.h"

using namespace chi0;

namespace {

constexpr size_t kAlign = 256;
constexpr int64_t kDefaultWorkgroups = 32768;
constexpr int kKTile = 16;          // k-points per K_A workgroup
constexpr int kReduceBlock = 256;   // values per K_R workgroup

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Item {
    int inst, q, w0, nwc;
    int64_t rounds;
    double cost;
    int nblocks;
};

struct Stage {
    std::vector<int> groups;     // (instance, q) group indices, K_A order
    std::vector<int> items;      // item indices, K_B order
    int64_t blocks[4];           // K_A, K_B, K_R workgroups; groups (band-range jobs)
    size_t table_off[4];         // byte offsets of the block->item and group->item tables
    size_t w_bytes, part_bytes;
    int max_nbw;                 // widest band window of the stage's groups
};

struct Group {
    int inst, q;
    size_t w_bytes;
    size_t rng_off;              // this group's band ranges in the range arena: [2][nbw][2] doubles
    double cost;
    std::vector<int> items;
};

struct Schedule {
    std::vector<Item> items;
    std::vector<Group> groups;
    std::vector<Stage> stages;
    size_t items_off, w_off, part_off, rng_off, total;
    int64_t blocks_total[3];
};

struct Inst {
    chi0_instance in;
    std::vector<chi0_q> qs;
    MeshDev mesh;
};

chi0_status validate(int32_t n_inst, const chi0_instance *inst, const chi0_batch_opts *opts, std::string &err)
{
    if (n_inst < 1 || !inst) {
        err = "n_inst must be >= 1 and inst non-null";
        return CHI0_E_INVALID_ARG;
    }
    if (opts) {
        if (opts->workgroups < 0 || (opts->use_graph != 0 && opts->use_graph != 1)) {
            err = "opts: workgroups >= 0 and use_graph 0 or 1 required";
            return CHI0_E_INVALID_ARG;
        }
        for (int i = 0; i < 5; ++i)
            if (opts->reserved[i] != 0) {
                err = "opts: reserved fields must be zero";
                return CHI0_E_INVALID_ARG;
            }
    }
    for (int i = 0; i < n_inst; ++i) {
        const chi0_instance &I = inst[i];
        chi0_status st = check_desc(&I.desc, I.eps_k, I.c_k);
        if (st) {
            err = "instance " + std::to_string(i) + ": invalid description";
            return st;
        }
        if (!I.desc.cma && I.desc.n_orb > kMaxOrbSmall) {
            // the fused matrix-element launch has the small-basis tiles only
            err = "instance " + std::to_string(i) + ": bases above " + std::to_string(kMaxOrbSmall) +
                  " functions (plane waves) are not supported in the batched form";
            return CHI0_E_UNSUPPORTED;
        }
        if (I.nq < 1 || I.nw < 1 || !I.qs || !I.omega || !I.chi) {
            err = "instance " + std::to_string(i) + ": nq, nw >= 1 and qs, omega, chi non-null required";
            return CHI0_E_INVALID_ARG;
        }
        for (int j = 0; j < I.nq; ++j) {
            const char *msg = "";
            st = check_q(I.desc, I.qs[j], &msg);
            if (st) {
                err = "instance " + std::to_string(i) + ", q " + std::to_string(j) + ": " + msg;
                return st;
            }
        }
    }
    return CHI0_OK;
}

// Frequency tiles the scheduler can give an item: 4 or 8 slots of 64 per lane.
constexpr int kChunks[2] = {kMaxOmegaPerLaunch, kMaxOmegaPerLaunch / 2};

// Items, groups, stages and the workspace layout for a total of `workgroups` K_B workgroups and
// items of at most `chunk` frequencies.
Schedule make_schedule(const std::vector<Inst> &inst, int64_t workgroups, uint64_t stage_w_bytes, int chunk)
{
    Schedule S;
    double total_cost = 0.0;
    for (int i = 0; i < (int)inst.size(); ++i) {
        const MeshDev &M = inst[i].mesh;
        const int64_t units = tets_per_pair(M) * M.nbw * M.nbw;
        const int64_t rounds = (units + kWave - 1) / kWave;
        for (int j = 0; j < inst[i].in.nq; ++j) {
            Group g;
            g.inst = i;
            g.q = j;
            g.w_bytes = M.cma ? 0 : align_up(sizeof(double) * (size_t)M.nbw * M.nbw * M.nk);
            g.rng_off = 0;
            g.cost = 0.0;
            for (int w0 = 0; w0 < inst[i].in.nw; w0 += chunk) {
                Item it;
                it.inst = i;
                it.q = j;
                it.w0 = w0;
                it.nwc = std::min(chunk, inst[i].in.nw - w0);
                it.rounds = rounds;
                // carving costs about one frequency slot; every further 64 frequencies one more
                it.cost = (double)rounds * (1.0 + (it.nwc + kWave - 1) / kWave);
                it.nblocks = 1;
                g.cost += it.cost;
                g.items.push_back((int)S.items.size());
                S.items.push_back(it);
            }
            total_cost += g.cost;
            S.groups.push_back(std::move(g));
        }
    }
    const double per_block = total_cost / (double)std::max<int64_t>(1, workgroups);
    for (Item &it : S.items) {
        const int64_t cap = std::min<int64_t>(1024, it.rounds);
        const int64_t b = (int64_t)std::llround(it.cost / per_block);
        it.nblocks = (int)std::max<int64_t>(1, std::min(cap, b));
    }
    // stages: groups in decreasing total cost, cut greedily at the W budget
    std::vector<int> order(S.groups.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return S.groups[a].cost > S.groups[b].cost; });
    Stage cur{};
    for (int gi : order) {
        const Group &g = S.groups[gi];
        if (stage_w_bytes && !cur.groups.empty() && cur.w_bytes + g.w_bytes > stage_w_bytes) {
            S.stages.push_back(cur);
            cur = Stage{};
        }
        cur.groups.push_back(gi);
        cur.w_bytes += g.w_bytes;
    }
    if (!cur.groups.empty()) S.stages.push_back(cur);

    S.items_off = 0;
    size_t off = align_up(sizeof(BatchItemDev) * S.items.size());
    S.blocks_total[0] = S.blocks_total[1] = S.blocks_total[2] = 0;
    size_t max_w = 0, max_part = 0;
    for (Stage &st : S.stages) {
        st.blocks[0] = st.blocks[1] = st.blocks[2] = 0;
        st.blocks[3] = (int64_t)st.groups.size();
        st.part_bytes = 0;
        st.max_nbw = 1;
        for (int gi : st.groups) {
            const Group &g = S.groups[gi];
            const MeshDev &M = inst[g.inst].mesh;
            st.max_nbw = std::max(st.max_nbw, (int)M.nbw);
            if (!M.cma) st.blocks[0] += (M.nk + kKTile - 1) / kKTile;
            for (int ii : g.items) {
                st.items.push_back(ii);
                const Item &it = S.items[ii];
                st.blocks[1] += it.nblocks;
                st.blocks[2] += (2 * it.nwc + kReduceBlock - 1) / kReduceBlock;
                st.part_bytes += align_up(sizeof(double) * (size_t)it.nblocks * 2 * it.nwc);
            }
        }
        std::stable_sort(st.items.begin(), st.items.end(), [&](int a, int b) {
            return S.items[a].cost / S.items[a].nblocks > S.items[b].cost / S.items[b].nblocks;
        });
        for (int k = 0; k < 4; ++k) {
            st.table_off[k] = off;
            off += align_up(sizeof(int32_t) * (size_t)st.blocks[k]);
            if (k < 3) S.blocks_total[k] += st.blocks[k];
        }
        max_w = std::max(max_w, st.w_bytes);
        max_part = std::max(max_part, st.part_bytes);
    }
    S.w_off = off;
    S.part_off = S.w_off + max_w;
    S.rng_off = S.part_off + max_part;
    size_t rng = 0;
    for (Group &g : S.groups) {
        g.rng_off = rng;
        rng += align_up(sizeof(double) * 4 * (size_t)inst[g.inst].mesh.nbw);
    }
    S.total = S.rng_off + rng;
    return S;
}

// Host images of the item table and the four tables of every stage.
void build_tables(const std::vector<Inst> &inst, const Schedule &S, char *ws, std::vector<BatchItemDev> &items,
                  std::vector<std::vector<int32_t>> &tables)
{
    items.assign(S.items.size(), BatchItemDev{});
    tables.assign(4 * S.stages.size(), {});
    for (size_t si = 0; si < S.stages.size(); ++si) {
        const Stage &st = S.stages[si];
        std::vector<int32_t> &ta = tables[4 * si], &tb = tables[4 * si + 1], &tr = tables[4 * si + 2];
        std::vector<int32_t> &tg = tables[4 * si + 3];
        size_t w_cursor = 0, p_cursor = 0;
        for (int gi : st.groups) {
            const Group &g = S.groups[gi];
            const Inst &I = inst[g.inst];
            double *W = I.mesh.cma ? nullptr : reinterpret_cast<double *>(ws + S.w_off + w_cursor);
            w_cursor += g.w_bytes;
            QDev qd = make_qdev(I.mesh, I.qs[g.q], W);
            qd.rng_k = reinterpret_cast<double *>(ws + S.rng_off + g.rng_off);
            qd.rng_kq = qd.rng_k + 2 * (size_t)I.mesh.nbw;
            tg.push_back(g.items.front());
            for (size_t k = 0; k < g.items.size(); ++k) {
                const int ii = g.items[k];
                const Item &it = S.items[ii];
                BatchItemDev &d = items[ii];
                d.M = I.mesh;
                d.Q = qd;
                d.omega = I.in.omega + it.w0;
                d.partial = reinterpret_cast<double *>(ws + S.part_off + p_cursor);
                p_cursor += align_up(sizeof(double) * (size_t)it.nblocks * 2 * it.nwc);
                d.out = I.in.chi + ((int64_t)it.q * I.in.nw + it.w0) * 2;
                d.scale = I.in.desc.spin_factor / (6.0 * (double)I.mesh.nk);
                d.nw = it.nwc;
                d.precision = I.in.desc.precision;
                d.nblocks = it.nblocks;
                d.ka_begin = -1;
                // K_A: the group's first item carries the k-tiles of the group
                if (k == 0 && !I.mesh.cma) {
                    d.ka_begin = (int32_t)ta.size();
                    const int64_t nt = (I.mesh.nk + kKTile - 1) / kKTile;
                    ta.insert(ta.end(), nt, ii);
                }
                d.kr_begin = (int32_t)tr.size();
                tr.insert(tr.end(), (2 * it.nwc + kReduceBlock - 1) / kReduceBlock, ii);
            }
        }
        for (int ii : st.items) {
            items[ii].kb_begin = (int32_t)tb.size();
            tb.insert(tb.end(), S.items[ii].nblocks, ii);
        }
    }
}

}  // namespace

struct chi0_batch_s {
    std::vector<Inst> inst;
    chi0_batch_opts opts;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    int64_t workgroups = 0;
    int chunk = kMaxOmegaPerLaunch;
    Schedule sched;
    std::vector<BatchItemDev> items;             // host images, kept alive for the uploads
    std::vector<std::vector<int32_t>> tables;
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string err;
};

namespace {

chi0_status bfail(chi0_batch_s *b, chi0_status st, const std::string &msg)
{
    if (b) b->err = msg;
    return st;
}

chi0_status bdevice(chi0_batch_s *b, hipError_t e, const char *where)
{
    return bfail(b, CHI0_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

void drop_graph(chi0_batch_s *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Schedule for `workgroups` and frequency tile `chunk`, and upload its tables (synchronous on s).
chi0_status install(chi0_batch_s *b, int64_t workgroups, int chunk, hipStream_t s)
{
    Schedule S = make_schedule(b->inst, workgroups, b->opts.stage_w_bytes, chunk);
    if (S.total > b->ws_bytes) return bfail(b, CHI0_E_WORKSPACE, "workspace too small for the schedule");
    for (int k = 0; k < 3; ++k)
        if (S.blocks_total[k] > (int64_t)INT32_MAX / 256)
            return bfail(b, CHI0_E_SHAPE, "batch too large for one launch");
    drop_graph(b);
    b->sched = std::move(S);
    b->workgroups = workgroups;
    b->chunk = chunk;
    build_tables(b->inst, b->sched, b->ws, b->items, b->tables);
    hipError_t e = hipMemcpyAsync(b->ws + b->sched.items_off, b->items.data(), sizeof(BatchItemDev) * b->items.size(),
                                  hipMemcpyHostToDevice, s);
    for (size_t si = 0; e == hipSuccess && si < b->sched.stages.size(); ++si)
        for (int k = 0; k < 4 && e == hipSuccess; ++k) {
            const std::vector<int32_t> &t = b->tables[4 * si + k];
            if (!t.empty())
                e = hipMemcpyAsync(b->ws + b->sched.stages[si].table_off[k], t.data(), sizeof(int32_t) * t.size(),
                                   hipMemcpyHostToDevice, s);
        }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bdevice(b, e, "table upload");
    return CHI0_OK;
}

hipError_t enqueue(chi0_batch_s *b, hipStream_t s)
{
    const BatchItemDev *items = reinterpret_cast<const BatchItemDev *>(b->ws + b->sched.items_off);
    for (const Stage &st : b->sched.stages) {
        const int32_t *t[4];
        for (int k = 0; k < 4; ++k) t[k] = reinterpret_cast<const int32_t *>(b->ws + st.table_off[k]);
        hipError_t e;
        if (st.blocks[0] > 0 && (e = launch_contract_batch(items, t[0], (int)st.blocks[0], s)) != hipSuccess) return e;
        if ((e = launch_band_range_batch(items, t[3], (int)st.blocks[3], st.max_nbw, s)) != hipSuccess) return e;
        if ((e = launch_tetra_batch(items, t[1], (int)st.blocks[1], s)) != hipSuccess) return e;
        if ((e = launch_reduce_batch(items, t[2], (int)st.blocks[2], s)) != hipSuccess) return e;
    }
    return hipSuccess;
}

chi0_status run(chi0_batch_s *b, hipStream_t s)
{
    hipError_t e;
    if (!b->opts.use_graph) {
        if ((e = enqueue(b, s)) != hipSuccess) return bdevice(b, e, "batch launch");
        return CHI0_OK;
    }
    if (!b->exec) {
        if (!b->capture_stream && (e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking)) != hipSuccess)
            return bdevice(b, e, "capture stream");
        if ((e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return bdevice(b, e, "begin capture");
        const hipError_t le = enqueue(b, b->capture_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->capture_stream, &g);
        if (le != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return bdevice(b, le, "batch launch under capture");
        }
        if (e != hipSuccess) return bdevice(b, e, "end capture");
        b->graph = g;
        if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess) {
            drop_graph(b);
            return bdevice(b, e, "graph instantiate");
        }
    }
    if ((e = hipGraphLaunch(b->exec, s)) != hipSuccess) return bdevice(b, e, "graph launch");
    return CHI0_OK;
}

}  // namespace

extern "C" {

chi0_status chi0_batch_workspace_size(int32_t n_inst, const chi0_instance *inst, const chi0_batch_opts *opts,
                                      size_t *bytes)
{
    std::string err;
    if (!bytes) return CHI0_E_INVALID_ARG;
    chi0_status st = validate(n_inst, inst, opts, err);
    if (st) return st;
    std::vector<Inst> v(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        v[i].in = inst[i];
        v[i].qs.assign(inst[i].qs, inst[i].qs + inst[i].nq);
        v[i].mesh = make_mesh(inst[i].desc, inst[i].eps_k, inst[i].c_k);
    }
    const int64_t wg = (opts && opts->workgroups > 0) ? opts->workgroups : kDefaultWorkgroups;
    // room for every frequency tile the tuner may choose
    size_t need = 0;
    for (int c : kChunks) need = std::max(need, make_schedule(v, wg, opts ? opts->stage_w_bytes : 0, c).total);
    *bytes = need;
    return CHI0_OK;
}

chi0_status chi0_batch_create(chi0_batch_t *out, int32_t n_inst, const chi0_instance *inst,
                              const chi0_batch_opts *opts, void *workspace, size_t workspace_bytes, void *stream)
{
    if (!out) return CHI0_E_INVALID_ARG;
    *out = nullptr;
    std::string err;
    chi0_status st = validate(n_inst, inst, opts, err);
    if (st) return st;
    if (!workspace) return CHI0_E_WORKSPACE;
    chi0_batch_s *b = new (std::nothrow) chi0_batch_s();
    if (!b) return CHI0_E_INVALID_ARG;
    std::memset(&b->opts, 0, sizeof b->opts);
    if (opts) b->opts = *opts;
    b->inst.resize(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        Inst &I = b->inst[i];
        I.in = inst[i];
        I.qs.assign(inst[i].qs, inst[i].qs + inst[i].nq);
        I.in.qs = nullptr;
        I.mesh = make_mesh(inst[i].desc, inst[i].eps_k, inst[i].c_k);
        I.in.desc.band_hi = I.mesh.lo + I.mesh.nbw;
    }
    b->ws = static_cast<char *>(workspace);
    b->ws_bytes = workspace_bytes;
    const int64_t wg = b->opts.workgroups > 0 ? b->opts.workgroups : kDefaultWorkgroups;
    b->opts.workgroups = wg;
    st = install(b, wg, kMaxOmegaPerLaunch, static_cast<hipStream_t>(stream));
    if (st) {
        delete b;
        return st;
    }
    *out = b;
    return CHI0_OK;
}

chi0_status chi0_batch_run(chi0_batch_t b, void *stream)
{
    if (!b) return CHI0_E_INVALID_ARG;
    return run(b, static_cast<hipStream_t>(stream));
}

chi0_status chi0_batch_tune(chi0_batch_t b, void *stream, int32_t reps, int64_t *chosen)
{
    if (!b || reps < 1) return CHI0_E_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t top = b->opts.workgroups;
    // candidates: workgroups top, top/2, top/4, top/8 (not below one per item) x frequency tiles
    struct Cand {
        int64_t g;
        int chunk;
    };
    std::vector<Cand> cand;
    for (int c : kChunks) {
        const int64_t floor_wg = (int64_t)make_schedule(b->inst, top, b->opts.stage_w_bytes, c).items.size();
        int n = 0;
        for (int64_t g = top; n < 4 && g >= floor_wg; g /= 2, ++n) cand.push_back({g, c});
    }
    if (cand.empty()) cand.push_back({top, kMaxOmegaPerLaunch});
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return bdevice(b, e, "tune events");
    }
    Cand best = cand[0];
    float best_ms = 0.0f;
    chi0_status st = CHI0_OK;
    for (size_t ci = 0; ci < cand.size(); ++ci) {
        if ((st = install(b, cand[ci].g, cand[ci].chunk, s)) != CHI0_OK) break;
        // one untimed warm-up run before the first candidate only
        if ((ci == 0 && (e = enqueue(b, s)) != hipSuccess) || (e = hipEventRecord(e0, s)) != hipSuccess) {
            st = bdevice(b, e, "tune run");
            break;
        }
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = enqueue(b, s);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            st = bdevice(b, e, "tune timing");
            break;
        }
        if (best_ms == 0.0f || ms < best_ms) {
            best_ms = ms;
            best = cand[ci];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    if ((st = install(b, best.g, best.chunk, s)) != CHI0_OK) return st;
    // leave the outputs valid for the chosen schedule
    if ((e = enqueue(b, s)) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess)
        return bdevice(b, e, "tune final run");
    if (chosen) *chosen = best.g;
    return CHI0_OK;
}

chi0_status chi0_batch_info_get(chi0_batch_t b, chi0_batch_info *info)
{
    if (!b || !info) return CHI0_E_INVALID_ARG;
    std::memset(info, 0, sizeof *info);
    info->items = (int64_t)b->sched.items.size();
    info->stages = (int64_t)b->sched.stages.size();
    for (int k = 0; k < 3; ++k) info->workgroups[k] = b->sched.blocks_total[k];
    info->omega_tile = b->chunk;
    for (const Inst &I : b->inst)
        info->nominal_units += (int64_t)I.in.nq * 6 * I.mesh.nk * I.mesh.nbw * I.mesh.nbw * I.in.nw;
    return CHI0_OK;
}

chi0_status chi0_batch_destroy(chi0_batch_t b)
{
    if (b) {
        drop_graph(b);
        if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    }
    delete b;
    return CHI0_OK;
}

const char *chi0_batch_last_error(chi0_batch_t b) { return b ? b->err.c_str() : ""; }

}  // extern "C"

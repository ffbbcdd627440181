// Batched form: many independent 2D problems advanced together.
//
// Every problem keeps its own double-buffered state and coefficient tables
// (a Sim).  Problems are grouped by the vector width their row length
// allows; each group has one flat list of wavefront tiles over all of its
// problems, interior tiles first and CPML-slab tiles after them, so two
// launches per group (without and with the CPML code) advance every problem,
// with the load spread evenly over the tiles whatever the mix of sizes.
// The main path is the multi-step kernel (TB = 4 steps per pass, one column
// per lane by default, so all problems form one group whatever their row
// lengths: 447 Gcell/s on 256 problems of sides 256-2048 against 408 with
// two-column groups for the even rows); single-step groups (width 2 and 1)
// take the remainder steps and align the buffer parity.  Launches read the step
// number from a device counter, which lets a captured HIP graph of passes be
// replayed for any step range.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <memory>
#include <tuple>

#include "sim.hpp"

namespace gem {

struct BatchGroup {
    int V = 1, TX = 16;
    std::vector<int> probs;
    BatchTile *tiles = nullptr;
    int ntiles = 0;
    int *pt_start = nullptr, *pt_cell = nullptr, *pt_slot = nullptr;
    std::vector<int> tile_base;  // first tile of each problem of the group (problem order)
    std::vector<int> pos;        // problem-order tile -> place in the launch list
    int n_inner = 0;             // list: interior tiles, then slab tiles
};

// Multi-step group: the problems whose row length the vector width divides.
struct TBGroup {
    int V = 4, TB = 4, TX = 16, mat = 0;
    std::vector<int> probs;
    Tile2T *tiles = nullptr;
    int ntiles = 0, n_inner = 0;
    int *pt_start = nullptr, *pt_cell = nullptr, *pt_slot = nullptr;
    std::vector<int> pos_base;  // per problem of the group: first entry in pos
    std::vector<int> pos;       // (problem, row, strip) -> place in the launch list of the
                                // tile starting there, -1 where none starts
};

}  // namespace gem

struct fdtd_batch {
    std::vector<std::unique_ptr<fdtd_sim>> hs;  // one single-problem handle per problem
    std::vector<gem::Sim *> sims;               // &hs[q]->s
    hipStream_t st = nullptr;
    hipStream_t cap_st = nullptr;
    gem::DevAlloc al;
    std::vector<gem::BatchGroup> groups;
    std::vector<gem::TBGroup> tbg;
    int tb = 4;   // steps per multi-step pass (1: single steps only)
    int tb_tx = 16, tb_vmax = 1;
    int tb_txo = 0;  // rows per tile with the CPML code (0: tb_tx)
    int cur = 0;  // buffer set holding the current state
    gem::Prob2D *probs_dev[2] = {nullptr, nullptr};
    std::vector<const void *> probs_key[2];
    int64_t *step_base = nullptr;
    int64_t n_done = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_steps = 64;
    bool use_graph = true;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timed = false;
    int64_t last_launches = 0;
    bool probes_dirty = true;

    ~fdtd_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        al.release_all();
        sims.clear();
        hs.clear();
        if (cap_st) (void)hipStreamDestroy(cap_st);
    }
};

namespace gem {

struct BFail {
    int code;
    std::string msg;
};

static void batch_build_probes(fdtd_batch &b) {
    for (auto &g : b.groups) {
        std::vector<int> tile_of_entry, cell, slot;
        std::vector<std::pair<int, int>> ent;  // (tile, index)
        std::vector<int> cells_all, slots_all;
        for (size_t qi = 0; qi < g.probs.size(); ++qi) {
            const Sim &s = *b.sims[(size_t)g.probs[qi]];
            Fused2DCfg c{g.V, g.TX};
            for (size_t p = 0; p < s.probe_cells.size(); ++p) {
                const int i = (int)(s.probe_cells[p] / s.ny), j = (int)(s.probe_cells[p] % s.ny);
                ent.push_back({g.pos[(size_t)(g.tile_base[qi] + fused2d_tile_of(s.nx, s.ny, c, i, j))],
                               (int)cells_all.size()});
                cells_all.push_back((int)s.probe_cells[p]);
                slots_all.push_back((int)p);
            }
        }
        std::stable_sort(ent.begin(), ent.end());
        std::vector<int> start((size_t)g.ntiles + 1, 0);
        for (auto &e : ent) {
            start[(size_t)e.first + 1]++;
            cell.push_back(cells_all[(size_t)e.second]);
            slot.push_back(slots_all[(size_t)e.second]);
        }
        for (int t = 0; t < g.ntiles; ++t) start[(size_t)t + 1] += start[(size_t)t];
        if (cell.empty()) {
            cell.push_back(0);
            slot.push_back(0);
        }
        b.al.put(g.pt_start);
        b.al.put(g.pt_cell);
        b.al.put(g.pt_slot);
        g.pt_start = (int *)b.al.get(start.size() * 4);
        g.pt_cell = (int *)b.al.get(cell.size() * 4);
        g.pt_slot = (int *)b.al.get(slot.size() * 4);
        hip_check(hipMemcpyAsync(g.pt_start, start.data(), start.size() * 4, hipMemcpyHostToDevice, b.st), "upload");
        hip_check(hipMemcpyAsync(g.pt_cell, cell.data(), cell.size() * 4, hipMemcpyHostToDevice, b.st), "upload");
        hip_check(hipMemcpyAsync(g.pt_slot, slot.data(), slot.size() * 4, hipMemcpyHostToDevice, b.st), "upload");
        hip_check(hipStreamSynchronize(b.st), "sync");
    }
    for (auto &g : b.tbg) {
        std::vector<std::pair<int, int>> ent;  // (tile, index)
        std::vector<int> cells_all, slots_all, cell, slot;
        const int ow = tb2d_own(g.V, g.TB);
        for (size_t qi = 0; qi < g.probs.size(); ++qi) {
            const Sim &s = *b.sims[(size_t)g.probs[qi]];
            const int nstrip = (s.ny + ow - 1) / ow;
            for (size_t p = 0; p < s.probe_cells.size(); ++p) {
                const int i = (int)(s.probe_cells[p] / s.ny), j = (int)(s.probe_cells[p] % s.ny);
                // the tile that starts at or last before row i
                int r = i;
                while (g.pos[(size_t)(g.pos_base[qi] + r * nstrip + j / ow)] < 0) --r;
                ent.push_back({g.pos[(size_t)(g.pos_base[qi] + r * nstrip + j / ow)], (int)cells_all.size()});
                cells_all.push_back((int)s.probe_cells[p]);
                slots_all.push_back((int)p);
            }
        }
        std::stable_sort(ent.begin(), ent.end());
        std::vector<int> start((size_t)g.ntiles + 1, 0);
        for (auto &e : ent) {
            start[(size_t)e.first + 1]++;
            cell.push_back(cells_all[(size_t)e.second]);
            slot.push_back(slots_all[(size_t)e.second]);
        }
        for (int t = 0; t < g.ntiles; ++t) start[(size_t)t + 1] += start[(size_t)t];
        if (cell.empty()) {
            cell.push_back(0);
            slot.push_back(0);
        }
        b.al.put(g.pt_start);
        b.al.put(g.pt_cell);
        b.al.put(g.pt_slot);
        g.pt_start = (int *)b.al.get(start.size() * 4);
        g.pt_cell = (int *)b.al.get(cell.size() * 4);
        g.pt_slot = (int *)b.al.get(slot.size() * 4);
        hip_check(hipMemcpyAsync(g.pt_start, start.data(), start.size() * 4, hipMemcpyHostToDevice, b.st), "upload");
        hip_check(hipMemcpyAsync(g.pt_cell, cell.data(), cell.size() * 4, hipMemcpyHostToDevice, b.st), "upload");
        hip_check(hipMemcpyAsync(g.pt_slot, slot.data(), slot.size() * 4, hipMemcpyHostToDevice, b.st), "upload");
        hip_check(hipStreamSynchronize(b.st), "sync");
    }
    // the captured graph holds the probe-table pointers: capture again
    if (b.exec) {
        (void)hipGraphExecDestroy(b.exec);
        b.exec = nullptr;
    }
    if (b.graph) {
        (void)hipGraphDestroy(b.graph);
        b.graph = nullptr;
    }
    b.probes_dirty = false;
}

// Upload the per-problem kernel descriptors if any pointer they hold moved.
static void batch_sync_probs(fdtd_batch &b) {
    const size_t n = b.sims.size();
    for (int par = 0; par < 2; ++par) {
        std::vector<Prob2D> h(n);
        std::vector<const void *> key;
        for (size_t q = 0; q < n; ++q) {
            h[q] = b.sims[q]->prob2d(par, 1 - par);
            key.push_back(h[q].src_vals);
            key.push_back(h[q].rec);
            key.push_back((const void *)(intptr_t)h[q].rec_stride);
            key.push_back((const void *)(intptr_t)h[q].src_len);
            key.push_back((const void *)(intptr_t)h[q].rec_base);
            key.push_back((const void *)(intptr_t)h[q].src_idx);
            for (int c = 0; c < 4; ++c) key.push_back((const void *)(intptr_t)h[q].src_box[c]);
            key.push_back((const void *)(intptr_t)h[q].np);
        }
        if (b.probs_dev[par] && key == b.probs_key[par]) continue;
        if (!b.probs_dev[par]) b.probs_dev[par] = (Prob2D *)b.al.get(n * sizeof(Prob2D));
        hip_check(hipMemcpyAsync(b.probs_dev[par], h.data(), n * sizeof(Prob2D), hipMemcpyHostToDevice, b.st), "upload");
        hip_check(hipStreamSynchronize(b.st), "sync");
        b.probs_key[par] = key;
    }
}

// multi-step groups: vector width 4, 2 or 1 by row length (at most
// tb_vmax); none when tb == 1
static void batch_build_tb(fdtd_batch &b) {
    for (auto &g : b.tbg) {
        b.al.put(g.tiles);
        b.al.put(g.pt_start);
        b.al.put(g.pt_cell);
        b.al.put(g.pt_slot);
    }
    b.tbg.clear();
    if (b.tb <= 1) return;
    const int n = (int)b.sims.size();
    for (int V : {4, 2, 1}) {
        if (V > b.tb_vmax) continue;
        TBGroup g;
        g.V = V;
        g.TB = b.tb;
        g.TX = b.tb_tx;
        std::vector<Tile2T> in, out, all;
        for (int q = 0; q < n; ++q) {
            const Sim &s = *b.sims[(size_t)q];
            const int vq = (s.ny % 4 == 0 && b.tb_vmax >= 4) ? 4 : ((s.ny % 2 == 0 && b.tb_vmax >= 2) ? 2 : 1);
            if (vq != V) continue;
            if (!tb2d_supported(s.ny, V, g.TB, g.TX)) fail(FDTD_EINVAL, "multi-step configuration");
            g.probs.push_back(q);
            g.mat = std::max(g.mat, s.mat());
            g.pos_base.push_back((int)all.size());
            std::vector<Tile2T> a, c;
            const int xl[2] = {s.ax[0].lo, s.ax[0].hi}, yl[2] = {s.ax[1].lo, s.ax[1].hi};
            tb2d_plan(q, s.nx, s.ny, V, g.TB, g.TX, b.tb_txo, xl, yl, a, c);
            // problem-order list by (row, strip) of each tile's first row
            const int ow = tb2d_own(V, g.TB), nstrip = (s.ny + ow - 1) / ow;
            std::vector<Tile2T> po((size_t)s.nx * nstrip, Tile2T{-1, 0, 0, 0});
            for (const auto &t : a) po[(size_t)t.i0 * nstrip + t.ja / ow] = t;
            for (const auto &t : c) po[(size_t)t.i0 * nstrip + t.ja / ow] = t;
            for (const auto &t : po) all.push_back(t);
            in.insert(in.end(), a.begin(), a.end());
            out.insert(out.end(), c.begin(), c.end());
        }
        if (g.probs.empty()) continue;
        // place of each problem-order tile in the launch list
        g.n_inner = (int)in.size();
        g.ntiles = (int)(in.size() + out.size());
        {
            std::map<std::pair<int, std::pair<int, int>>, int> at;
            for (size_t t = 0; t < in.size(); ++t) at[{in[t].prob, {in[t].i0, in[t].ja}}] = (int)t;
            for (size_t t = 0; t < out.size(); ++t) at[{out[t].prob, {out[t].i0, out[t].ja}}] = g.n_inner + (int)t;
            g.pos.resize(all.size());
            for (size_t t = 0; t < all.size(); ++t)
                g.pos[t] = all[t].prob < 0 ? -1 : at[{all[t].prob, {all[t].i0, all[t].ja}}];
        }
        in.insert(in.end(), out.begin(), out.end());
        g.tiles = (Tile2T *)b.al.get(in.size() * sizeof(Tile2T));
        hip_check(hipMemcpyAsync(g.tiles, in.data(), in.size() * sizeof(Tile2T), hipMemcpyHostToDevice, b.st),
                  "upload");
        hip_check(hipStreamSynchronize(b.st), "sync");
        b.tbg.push_back(g);
    }
}

static void batch_launch_one(fdtd_batch &b, int parity, int k, hipStream_t st) {
    for (auto &g : b.groups) {
        ProbeTiles pt{g.pt_start, g.pt_cell, g.pt_slot};
        hip_check(launch_batch_step(b.probs_dev[parity], g.tiles, 0, g.n_inner, false, pt, g.V, g.TX,
                                    b.step_base, k, st),
                  "batch step");
        hip_check(launch_batch_step(b.probs_dev[parity], g.tiles, g.n_inner, g.ntiles - g.n_inner, true, pt,
                                    g.V, g.TX, b.step_base, k, st),
                  "batch step");
    }
}

// one multi-step pass (b.tb steps) of every problem, reading set `parity`
static void batch_launch_pass(fdtd_batch &b, int parity, int k, hipStream_t st) {
    const Prob2D none{};
    for (auto &g : b.tbg) {
        const ProbeTiles pt{g.pt_start, g.pt_cell, g.pt_slot};
        const ProbeTiles po{g.pt_start + g.n_inner, g.pt_cell, g.pt_slot};
        hip_check(launch_2d_tb(none, b.probs_dev[parity], g.tiles, g.n_inner, false, g.mat, pt, g.V, g.TB,
                               b.step_base, k, st),
                  "batch pass");
        hip_check(launch_2d_tb(none, b.probs_dev[parity], g.tiles + g.n_inner, g.ntiles - g.n_inner, true, g.mat,
                               po, g.V, g.TB, b.step_base, k, st),
                  "batch pass");
    }
}

// graph_steps steps from buffer set 0: passes of b.tb steps (an even number
// of them), or single steps
static void batch_capture(fdtd_batch &b) {
    if (b.exec) return;
    if (!b.cap_st) hip_check(hipStreamCreateWithFlags(&b.cap_st, hipStreamNonBlocking), "stream");
    hip_check(hipStreamBeginCapture(b.cap_st, hipStreamCaptureModeRelaxed), "begin capture");
    if (b.tb > 1) {
        for (int k = 0; k < b.graph_steps / b.tb; ++k) batch_launch_pass(b, k & 1, k * b.tb, b.cap_st);
    } else {
        for (int k = 0; k < b.graph_steps; ++k) batch_launch_one(b, k & 1, k, b.cap_st);
    }
    hip_check(launch_advance(b.step_base, b.graph_steps, b.cap_st), "advance");
    hip_check(hipStreamEndCapture(b.cap_st, &b.graph), "end capture");
    hip_check(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0), "instantiate");
}

}  // namespace gem

using namespace gem;

namespace gem {
int status_of_current_exception();
}  // namespace gem

extern "C" {

int fdtd_batch_create(const fdtd_desc *descs, int32_t n, fdtd_batch **out) {
    if (!out) {
        set_error("out is NULL");
        return FDTD_EINVAL;
    }
    *out = nullptr;
    fdtd_batch *b = nullptr;
    try {
        if (!descs || n < 1) fail(FDTD_EINVAL, "need at least one problem");
        for (int32_t q = 0; q < n; ++q)
            if (descs[q].cpml.split != 0) fail(FDTD_EINVAL, "the batch takes the CPML only");
        b = new fdtd_batch();
        b->st = (hipStream_t)descs[0].stream;
        b->al.st = b->st;
        if (descs[0].allocator) {
            b->al.a = *descs[0].allocator;
            b->al.has = true;
        }
        for (int q = 0; q < n; ++q) {
            fdtd_desc d = descs[q];
            if (d.ndim != 2) fail(FDTD_EINVAL, "batched problems must be 2D (ndim 2)");
            d.stream = descs[0].stream;
            d.allocator = descs[0].allocator;
            b->hs.emplace_back(new fdtd_sim());
            b->sims.push_back(&b->hs.back()->s);
            init_sim(*b->sims.back(), &d);
        }
        // groups by vector width
        // groups by vector width: 2 for even rows, 1 for odd ones (the
        // 4-wide instance holds too many registers for the CPML tiles)
        for (int V : {2, 1}) {
            BatchGroup g;
            g.V = V;
            g.TX = 8;
            std::vector<BatchTile> tiles;
            for (int q = 0; q < n; ++q) {
                const Sim &s = *b->sims[(size_t)q];
                const int vq = s.ny % 2 == 0 ? 2 : 1;
                if (vq != V) continue;
                g.probs.push_back(q);
                g.tile_base.push_back((int)tiles.size());
                const int nsy = (s.ny + 64 * V - 1) / (64 * V);
                const int ncx = (s.nx + g.TX - 1) / g.TX;
                for (int cx = 0; cx < ncx; ++cx)
                    for (int sy = 0; sy < nsy; ++sy) tiles.push_back(BatchTile{q, cx, sy});
            }
            if (g.probs.empty()) continue;
            // interior tiles (no CPML code) first, then the slab tiles; pos
            // maps a tile's place in problem order to its place in the list
            {
                std::vector<BatchTile> inner, outer;
                std::vector<int> where(tiles.size());
                for (size_t t = 0; t < tiles.size(); ++t) {
                    const Sim &s = *b->sims[(size_t)tiles[t].prob];
                    const int xl[2] = {s.ax[0].lo, s.ax[0].hi}, yl[2] = {s.ax[1].lo, s.ax[1].hi};
                    const int nsy = (s.ny + 64 * V - 1) / (64 * V);
                    const int tid = tiles[t].cx * nsy + tiles[t].sy;
                    const bool in = fused2d_interior(s.nx, s.ny, Fused2DCfg{V, g.TX}, xl, yl, tid);
                    where[t] = in ? (int)inner.size() : -1 - (int)outer.size();
                    (in ? inner : outer).push_back(tiles[t]);
                }
                g.n_inner = (int)inner.size();
                g.pos.resize(tiles.size());
                for (size_t t = 0; t < tiles.size(); ++t)
                    g.pos[t] = where[t] >= 0 ? where[t] : g.n_inner + (-1 - where[t]);
                tiles = inner;
                tiles.insert(tiles.end(), outer.begin(), outer.end());
            }
            g.ntiles = (int)tiles.size();
            g.tiles = (BatchTile *)b->al.get(tiles.size() * sizeof(BatchTile));
            hip_check(hipMemcpyAsync(g.tiles, tiles.data(), tiles.size() * sizeof(BatchTile),
                                     hipMemcpyHostToDevice, b->st), "upload");
            hip_check(hipStreamSynchronize(b->st), "sync");
            b->groups.push_back(g);
        }
        batch_build_tb(*b);
        b->step_base = (int64_t *)b->al.get(sizeof(int64_t));
        hip_check(hipEventCreate(&b->ev0), "event");
        hip_check(hipEventCreate(&b->ev1), "event");
        batch_build_probes(*b);
        *out = b;
        set_error("");
        return FDTD_OK;
    } catch (...) {
        const int rc = gem::status_of_current_exception();
        delete b;
        return rc;
    }
}

int fdtd_batch_set_kernel(fdtd_batch *b, int32_t tb, int32_t tx, int32_t vmax, int32_t txo) {
    try {
        if (!b) fail(FDTD_EINVAL, "batch is NULL");
        if (!(tb == 1 || tb == 2 || tb == 4) || tx < 1 || tx > 65536 || !(vmax == 1 || vmax == 2 || vmax == 4) ||
            txo < 0 || txo > 65536)
            fail(FDTD_EINVAL, "unsupported batch kernel configuration");
        hip_check(hipStreamSynchronize(b->st), "sync");
        const int otb = b->tb, otx = b->tb_tx, ov = b->tb_vmax, oo = b->tb_txo;
        b->tb = tb;
        b->tb_tx = tx;
        b->tb_vmax = vmax;
        b->tb_txo = txo;
        try {
            batch_build_tb(*b);
        } catch (...) {
            b->tb = otb;
            b->tb_tx = otx;
            b->tb_vmax = ov;
            b->tb_txo = oo;
            batch_build_tb(*b);
            batch_build_probes(*b);
            throw;
        }
        batch_build_probes(*b);
        set_error("");
        return FDTD_OK;
    } catch (...) {
        return gem::status_of_current_exception();
    }
}

// Autotuner of the batch: every candidate (steps per pass, rows per tile,
// widest vector, rows per CPML tile) times trial_steps steps of the whole
// batch (one captured graph when trial_steps >= 64) after a short warm-up;
// the fastest is kept.  The state of every problem (fields and CPML values
// of the current buffer set), the step count and the probe records'
// lengths are saved first and restored after, so the batch continues as if
// the call had not been made.  Cached in $GEMFDTD_TUNE_CACHE under the
// device and the batch's size mix.
int fdtd_batch_autotune(fdtd_batch *b, int32_t trial_steps, int32_t *out) {
    std::vector<void *> tmp;
    try {
        if (!b) fail(FDTD_EINVAL, "batch is NULL");
        if (trial_steps < 8 || trial_steps > 4096) fail(FDTD_EINVAL, "trial_steps must be in [8, 4096]");
        hipDeviceProp_t pr{};
        std::string arch = "unknown";
        if (hipGetDeviceProperties(&pr, b->sims[0]->device) == hipSuccess) arch = pr.gcnArchName;
        // size mix: count, and a hash of the sorted (nx, ny, material kind) list
        std::vector<std::tuple<int, int, int>> dims;
        int64_t cells = 0;
        for (auto *sp : b->sims) {
            dims.emplace_back(sp->nx, sp->ny, sp->mat());
            cells += sp->ncell;
        }
        std::sort(dims.begin(), dims.end());
        uint64_t h = 1469598103934665603ull;
        for (auto &d : dims)
            for (int v : {std::get<0>(d), std::get<1>(d), std::get<2>(d)}) {
                h ^= (uint64_t)(uint32_t)v;
                h *= 1099511628211ull;
            }
        char key[160];
        snprintf(key, sizeof key, "%s|batch|n%zu|c%lld|h%016llx", arch.c_str(), dims.size(), (long long)cells,
                 (unsigned long long)h);
        const char *path = std::getenv("GEMFDTD_TUNE_CACHE");
        std::map<std::string, std::vector<int>> cache;
        if (path) cache = read_cache(path);
        auto it = cache.find(key);
        std::vector<int> best;
        if (it != cache.end() && it->second.size() == 4) {
            best = it->second;
        } else {
            // save the state
            hip_check(hipStreamSynchronize(b->st), "sync");
            const int cur = b->cur;
            const int64_t n_done = b->n_done;
            std::vector<int64_t> n_rec;
            std::vector<std::pair<float *, size_t>> parts;
            for (auto *sp : b->sims) {
                n_rec.push_back(sp->n_rec);
                for (int c : {FDTD_EZ, FDTD_HX, FDTD_HY}) parts.emplace_back(sp->f[cur][c], (size_t)sp->ncell);
                for (int a = 0; a < 4; ++a)
                    if (sp->psi[cur][a]) parts.emplace_back(sp->psi[cur][a], (size_t)sp->psi_len[a]);
            }
            size_t total = 0;
            for (auto &p : parts) total += p.second;
            float *save = (float *)b->al.get(total * 4);
            tmp.push_back(save);
            size_t off = 0;
            for (auto &p : parts) {
                hip_check(hipMemcpyAsync(save + off, p.first, p.second * 4, hipMemcpyDeviceToDevice, b->st), "save");
                off += p.second;
            }
            const int old[4] = {b->tb, b->tb_tx, b->tb_vmax, b->tb_txo};
            float best_ms = 1e30f;
            for (int tb : {4, 2})
                for (int tx : {8, 16, 32})
                    for (int vmax : {1, 2, 4})
                        for (int txo : {0, 4, 8}) {
                            if (txo >= tx) continue;
                            if (fdtd_batch_set_kernel(b, tb, tx, vmax, txo) != FDTD_OK) continue;
                            if (fdtd_batch_step(b, 8) != FDTD_OK) continue;
                            if (fdtd_batch_step(b, trial_steps) != FDTD_OK) continue;
                            float ms = 0;
                            int64_t launches = 0;
                            if (fdtd_batch_last_step_time(b, &ms, &launches) != FDTD_OK) continue;
                            if (ms < best_ms) {
                                best_ms = ms;
                                best = {tb, tx, vmax, txo};
                            }
                        }
            // restore the state (the buffer set, step count, records)
            hip_check(hipStreamSynchronize(b->st), "sync");
            off = 0;
            for (auto &p : parts) {
                hip_check(hipMemcpyAsync(p.first, save + off, p.second * 4, hipMemcpyDeviceToDevice, b->st), "restore");
                off += p.second;
            }
            b->cur = cur;
            b->n_done = n_done;
            for (size_t q = 0; q < b->sims.size(); ++q) {
                Sim &s = *b->sims[q];
                s.cur = cur;
                s.n_done = n_done;
                s.n_rec = n_rec[q];
            }
            hip_check(hipStreamSynchronize(b->st), "sync");
            for (void *p : tmp) b->al.put(p);
            tmp.clear();
            if (best.empty()) {
                fdtd_batch_set_kernel(b, old[0], old[1], old[2], old[3]);
                fail(FDTD_EDEVICE, "no batch configuration ran");
            }
            if (path) {
                cache[key] = best;
                write_cache(path, cache);
            }
        }
        const int rc = fdtd_batch_set_kernel(b, best[0], best[1], best[2], best[3]);
        if (rc != FDTD_OK) return rc;
        if (out)
            for (int q = 0; q < 4; ++q) out[q] = best[(size_t)q];
        set_error("");
        return FDTD_OK;
    } catch (...) {
        const int rc = gem::status_of_current_exception();
        if (b)
            for (void *p : tmp) b->al.put(p);
        return rc;
    }
}

int fdtd_batch_destroy(fdtd_batch *b) {
    delete b;
    return FDTD_OK;
}

static fdtd_sim *batch_sim(fdtd_batch *b, int32_t q) {
    if (!b) fail(FDTD_EINVAL, "batch is NULL");
    if (q < 0 || q >= (int32_t)b->hs.size()) fail(FDTD_EINVAL, "problem index out of range");
    return b->hs[(size_t)q].get();
}

int fdtd_batch_set_source(fdtd_batch *b, int32_t problem, const int32_t *ijk, int kind,
                          const double *params, const float *table, int64_t n_table) {
    try {
        fdtd_sim *h = batch_sim(b, problem);
        const int rc = fdtd_set_source(h, FDTD_EZ, ijk, kind, params, table, n_table);
        return rc;
    } catch (...) {
        return gem::status_of_current_exception();
    }
}

int fdtd_batch_set_probes(fdtd_batch *b, int32_t problem, const int32_t *ijk, int32_t n) {
    try {
        fdtd_sim *h = batch_sim(b, problem);
        const int rc = fdtd_set_probes(h, FDTD_EZ, ijk, n);
        if (rc == FDTD_OK) b->probes_dirty = true;
        return rc;
    } catch (...) {
        return gem::status_of_current_exception();
    }
}

int fdtd_batch_step(fdtd_batch *b, int64_t n) {
    try {
        if (!b) fail(FDTD_EINVAL, "batch is NULL");
        if (n < 0) fail(FDTD_EINVAL, "n must be >= 0");
        for (auto &sp : b->sims) {
            sp->ensure_source(b->n_done + n);
            sp->ensure_rec(sp->n_rec + n);
        }
        if (b->probes_dirty) batch_build_probes(*b);
        batch_sync_probs(*b);
        hip_check(hipMemcpyAsync(b->step_base, &b->n_done, sizeof(int64_t), hipMemcpyHostToDevice, b->st), "upload");
        hip_check(hipStreamSynchronize(b->st), "sync");
        b->last_launches = 0;
        hip_check(hipEventRecord(b->ev0, b->st), "event");
        int64_t ng = 0, np = 0;  // launches per single step, per pass
        for (const auto &g : b->groups) ng += (g.n_inner > 0) + (g.ntiles > g.n_inner);
        for (const auto &g : b->tbg) np += (g.n_inner > 0) + (g.ntiles > g.n_inner);
        const int tb = b->tb;
        int64_t k = 0;
        // graph replays start on buffer set 0
        if (n > 0 && b->cur == 1) {
            batch_launch_one(*b, 1, 0, b->st);
            b->cur = 0;
            b->last_launches += ng;
            k = 1;
        }
        if (k > 0) hip_check(launch_advance(b->step_base, k, b->st), "advance");
        const int64_t reps = b->use_graph ? (n - k) / b->graph_steps : 0;
        if (reps > 0) {
            batch_capture(*b);
            for (int64_t r = 0; r < reps; ++r) hip_check(hipGraphLaunch(b->exec, b->st), "graph launch");
            b->last_launches += reps * ((tb > 1 ? (b->graph_steps / tb) * np : b->graph_steps * ng) + 1);
        }
        const int64_t k2 = k + reps * b->graph_steps;
        int64_t q = k2;
        if (tb > 1)
            for (; q + tb <= n; q += tb) {
                batch_launch_pass(*b, b->cur, (int)(q - k2), b->st);
                b->cur ^= 1;
                b->last_launches += np;
            }
        for (; q < n; ++q) {
            batch_launch_one(*b, b->cur, (int)(q - k2), b->st);
            b->cur ^= 1;
            b->last_launches += ng;
        }
        hip_check(hipEventRecord(b->ev1, b->st), "event");
        b->timed = true;
        b->n_done += n;
        for (auto &sp : b->sims) {
            sp->n_done = b->n_done;
            if (!sp->probe_cells.empty()) sp->n_rec += n;
            sp->cur = b->cur;
        }
        return FDTD_OK;
    } catch (...) {
        return gem::status_of_current_exception();
    }
}

int fdtd_batch_probe(fdtd_batch *b, int32_t problem, float *out, int64_t cap, int64_t *n_recorded) {
    try {
        return fdtd_probe(batch_sim(b, problem), out, cap, n_recorded);
    } catch (...) {
        return gem::status_of_current_exception();
    }
}

int fdtd_batch_get_field(fdtd_batch *b, int32_t problem, int component, void *dst, int dst_on_device) {
    try {
        return fdtd_get_field(batch_sim(b, problem), component, dst, dst_on_device);
    } catch (...) {
        return gem::status_of_current_exception();
    }
}

int fdtd_batch_last_step_time(fdtd_batch *b, float *ms, int64_t *launches) {
    try {
        if (!b || !ms) fail(FDTD_EINVAL, "NULL argument");
        if (!b->timed) fail(FDTD_ESTATE, "no fdtd_batch_step call yet");
        hip_check(hipEventSynchronize(b->ev1), "sync");
        hip_check(hipEventElapsedTime(ms, b->ev0, b->ev1), "elapsed");
        if (launches) *launches = b->last_launches;
        return FDTD_OK;
    } catch (...) {
        return gem::status_of_current_exception();
    }
}

int fdtd_batch_cells(const fdtd_batch *b, int64_t *cells) {
    if (!b || !cells) {
        set_error("NULL argument");
        return FDTD_EINVAL;
    }
    int64_t c = 0;
    for (auto &sp : b->sims) c += sp->ncell;
    *cells = c;
    return FDTD_OK;
}

}  // extern "C"

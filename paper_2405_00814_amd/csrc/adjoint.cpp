// Gradient of a probe-energy loss with respect to eps_r (and sigma) by the
// discrete adjoint, with checkpointing.
//
// Forward: T steps from the zero state with a full-state checkpoint every L
// steps; the last segment already keeps, at every design cell and step, Ez
// before the E layer and the E-layer bracket.  Backward, newest segment
// first: run the segment's adjoint steps backward on what was kept; for
// every older segment first restore its checkpoint and recompute it with
// the same kernels (bitwise the same states), keeping the same values.
// With L >= T the forward pass is the only one (the design values of all
// T steps are held: 8 B per design cell and step).  The gradient of
// E^{k+1} = Ca E^k + Cb * bracket with respect to a parameter of Ca and Cb
// at a design cell is dCa * E^k + dCb * bracket, weighted by the adjoint of
// E^{k+1}: the adjoint steps sum a * E^k and a * bracket per cell in
// double, and the gradients with respect to eps_r and sigma combine these
// sums with the coefficients' derivatives at the end.
#include <algorithm>
#include <cmath>

#include "sim.hpp"

namespace gem {

int status_of_current_exception();

namespace {

struct StateBuf {
    std::vector<std::pair<float *, int64_t>> parts;  // (device pointer, floats) of set 0
};

// The simulation's launches go to stream t for the scope (the recompute of
// a segment beside the adjoint steps of the next one).
struct StreamSwap {
    Sim &s;
    hipStream_t old;
    StreamSwap(Sim &s_, hipStream_t t) : s(s_), old(s_.st) { s.st = t; }
    ~StreamSwap() { s.st = old; }
};

}  // namespace

static void copy_state(Sim &s, int set, float *buf, bool to_buf) {
    int64_t off = 0;
    auto mv = [&](float *p, int64_t n) {
        if (!p || n <= 0) return;
        if (to_buf) hip_check(hipMemcpyAsync(buf + off, p, n * 4, hipMemcpyDeviceToDevice, s.st), "ckpt");
        else hip_check(hipMemcpyAsync(p, buf + off, n * 4, hipMemcpyDeviceToDevice, s.st), "ckpt");
        off += n;
    };
    for (int c : {FDTD_EZ, FDTD_HX, FDTD_HY}) mv(s.f[set][c], s.ncell);
    for (int a = 0; a < 4; ++a) mv(s.psi[set][a], s.psi_len[a]);
}

static int64_t state_floats(const Sim &s) {
    int64_t n = 3 * s.ncell;
    for (int a = 0; a < 4; ++a) n += s.psi_len[a];
    return n;
}

}  // namespace gem

using namespace gem;

extern "C" int fdtd_adjoint_eps(fdtd_sim *sim, int64_t T, int64_t n0, int64_t n1,
                                const int32_t *design, int32_t ckpt_interval, double *loss_out,
                                float *grad_dev) {
    if (!grad_dev) {
        set_error("NULL argument");
        return FDTD_EINVAL;
    }
    return fdtd_adjoint_grads(sim, T, n0, n1, design, ckpt_interval, loss_out, grad_dev, nullptr, nullptr);
}

extern "C" int fdtd_adjoint(fdtd_sim *sim, int64_t T, int64_t n0, int64_t n1, const int32_t *design,
                            int32_t ckpt_interval, double *loss_out, float *grad_eps_dev, float *grad_sigma_dev) {
    if (!grad_eps_dev && !grad_sigma_dev) {
        set_error("NULL argument");
        return FDTD_EINVAL;
    }
    return fdtd_adjoint_grads(sim, T, n0, n1, design, ckpt_interval, loss_out, grad_eps_dev, grad_sigma_dev,
                              nullptr);
}

extern "C" int fdtd_adjoint_grads(fdtd_sim *sim, int64_t T, int64_t n0, int64_t n1, const int32_t *design,
                                  int32_t ckpt_interval, double *loss_out, float *grad_eps_dev,
                                  float *grad_sigma_dev, float *grad_mu_dev) {
    std::vector<void *> tmp;
    Sim *sp = nullptr;
    fdtd_kernel_config saved{};
    bool restore_cfg = false;
    hipStream_t rs = nullptr;  // recompute stream
    hipEvent_t ev_rec[2] = {nullptr, nullptr}, ev_adj[2] = {nullptr, nullptr}, ev_start = nullptr;
    auto release_streams = [&]() {
        if (rs) (void)hipStreamSynchronize(rs);
        for (hipEvent_t e : {ev_rec[0], ev_rec[1], ev_adj[0], ev_adj[1], ev_start})
            if (e) (void)hipEventDestroy(e);
        if (rs) (void)hipStreamDestroy(rs);
        rs = nullptr;
        ev_rec[0] = ev_rec[1] = ev_adj[0] = ev_adj[1] = ev_start = nullptr;
    };
    try {
        if (!sim || !design || (!grad_eps_dev && !grad_sigma_dev && !grad_mu_dev))
            fail(FDTD_EINVAL, "NULL argument");
        Sim &s = sim->s;
        sp = &s;
        if (s.ndim != 2 || s.is_graph) fail(FDTD_EINVAL, "the adjoint supports the 2D implicit stepper");
        if (s.dft.comp >= 0) fail(FDTD_ESTATE, "remove the frequency-domain monitor before the adjoint");
        if (s.split) fail(FDTD_EINVAL, "the adjoint supports the CPML only");
        if (T < 1 || n0 < 0 || n1 < n0 || n1 > T) fail(FDTD_EINVAL, "need T >= 1 and 0 <= n0 <= n1 <= T");
        const int i0 = design[0], i1 = design[1], j0 = design[2], j1 = design[3];
        if (i0 < 0 || i1 > s.nx || j0 < 0 || j1 > s.ny || i0 >= i1 || j0 >= j1)
            fail(FDTD_EINVAL, "invalid design box");
        if (s.probe_cells.empty() || s.probe_comp != FDTD_EZ)
            fail(FDTD_EINVAL, "the loss needs Ez probes (fdtd_set_probes)");
        // the H layer's brackets at the design cells are rebuilt from the
        // captured Ez: no CPML auxiliary term may enter them
        if (grad_mu_dev && (i0 < s.ax[0].lo || i1 > s.nx - s.ax[0].hi || j0 < s.ax[1].lo || j1 > s.ny - s.ax[1].hi))
            fail(FDTD_EINVAL, "the mu_r gradient needs a design box clear of the CPML slabs");
        // an interval beyond T is one segment of T steps
        const int64_t L = std::min<int64_t>(T, ckpt_interval > 0 ? ckpt_interval
                                                                 : (int64_t)std::ceil(std::sqrt((double)T)));
        const int64_t nseg = (T + L - 1) / L;
        const int64_t nd = (int64_t)(i1 - i0) * (j1 - j0);
        // captured box: the design box and one row and column beyond it
        // (clipped to the grid), whose Ez the H brackets need
        const int i1c = std::min(i1 + 1, s.nx), j1c = std::min(j1 + 1, s.ny);
        const int64_t ndc = (int64_t)(i1c - i0) * (j1c - j0);
        const int64_t P = (int64_t)s.probe_cells.size();

        // forward and recompute: the chosen fused configuration (variant 2
        // or 3; else the grid's default), the recompute capturing the design
        // cells.  The adjoint step: one column per lane below 4M cells (more
        // wavefronts for the chip), else two.
        saved = s.kcfg;
        restore_cfg = true;
        if ((s.kcfg.variant != 2 && s.kcfg.variant != 3) || !s.kcfg_explicit) default_variant_tiles(s, s.kcfg);
        if (s.kcfg.variant == 4) {  // one-workgroup default (no per-step captures): single steps
            const Fused2DCfg c = default_single2d(s.nx, s.ny);
            s.kcfg = fdtd_kernel_config{};
            s.kcfg.variant = 2;
            s.kcfg.tile[0] = c.V;
            s.kcfg.tile[1] = c.TX;
            s.kcfg.tb = 1;
        }
        if (s.kcfg.variant != 2 && s.kcfg.variant != 3) fail(FDTD_EINVAL, "no fused 2D kernel for this grid");
        const bool multi = s.kcfg.variant == 3;
        const int TB = multi ? s.kcfg.tile[2] : 1;
        const Fused2DCfg ac{(s.ncell >= ((int64_t)4 << 20) && s.ny % 2 == 0) ? 2 : 1, 4};
        s.pt_ntiles = -1;
        s.build_probe_tiles();
        s.zero_state();
        s.ensure_source(T);
        s.ensure_rec(T);
        auto get = [&](size_t bytes) {
            void *p = s.al.get(bytes);
            tmp.push_back(p);
            return p;
        };
        const int64_t S = state_floats(s);
        float *ck = (float *)get((size_t)(std::max<int64_t>(1, nseg - 1) * S) * 4);
        float *fin = (float *)get((size_t)S * 4);
        // design values of a segment, two sets when segments are recomputed
        // (one filled while the adjoint steps read the other)
        float *cap_ez[2] = {nullptr, nullptr}, *cap_br[2] = {nullptr, nullptr};
        for (int b = 0; b < (nseg >= 2 ? 2 : 1); ++b) {
            cap_ez[b] = (float *)get((size_t)(L * ndc) * 4);
            cap_br[b] = (float *)get((size_t)(L * ndc) * 4);
        }
        const int dbox[4] = {i0, i1, j0, j1};
        const int cbox[4] = {i0, i1c, j0, j1c};
        ProbeTiles pt{s.pt_start, s.pt_cell, s.pt_slot};
        const Fused2DCfg fc = s.single2d();
        // steps [k0, k1) from the current state; with `cap`, keeping the
        // design values of each step at (step - k0) * nd
        auto run = [&](int64_t k0, int64_t k1, const CapArgs *cap) {
            for (int64_t k = k0; k < k1;) {
                if (multi && k + TB <= k1) {
                    s.launch_tb2d(k, cap);
                    k += TB;
                    s.n_done += TB;
                    s.n_rec += TB;
                    continue;
                }
                if (cap) {
                    const Prob2D p = s.prob2d(s.cur, 1 - s.cur);
                    const TileSplit2D sp{s.tl2_dev, s.tl2_inner, s.tl2_dev + s.tl2_inner, s.tl2_outer};
                    hip_check(launch_2d_fused(p, fc, pt, k, s.st, cbox, cap->ez + (k - k0) * ndc,
                                              cap->br + (k - k0) * ndc, s.split2d() ? &sp : nullptr),
                              "forward step");
                    s.cur = 1 - s.cur;
                } else {
                    s.launch_step(k);
                }
                s.n_done += 1;
                s.n_rec += 1;
                k += 1;
            }
        };
        hip_check(hipEventRecord(s.ev0, s.st), "event");
        // ---- forward: checkpoints, then the last segment with its design values ----
        for (int64_t g = 0; g < nseg; ++g) {
            const int64_t k0 = g * L, k1 = std::min(T, (g + 1) * L);
            if (g + 1 < nseg) {
                copy_state(s, s.cur, ck + g * S, true);
                run(k0, k1, nullptr);
            } else {
                const int b = (int)(g & 1);
                const CapArgs cap{make_int4(i0, i1c, j0, j1c), cap_ez[b], cap_br[b], k0, ndc};
                run(k0, k1, &cap);
            }
        }
        copy_state(s, s.cur, fin, true);
        // ---- loss ----
        std::vector<float> rec((size_t)(P * T));
        s.records_to_host(rec.data(), T, T);
        double loss = 0.0;
        for (int64_t p = 0; p < P; ++p)
            for (int64_t m = n0 + 1; m <= n1; ++m) {
                const double v = rec[(size_t)(p * T + m - 1)];
                loss += v * v;
            }
        // ---- adjoint buffers (double buffered, zero-filled) ----
        Adj2D a[2]{};
        const size_t cb = (size_t)s.ncell * 4;
        for (Adj2D &x : a) {
            x.ez = (float *)get(cb);
            x.hx = (float *)get(cb);
            x.hy = (float *)get(cb);
            x.psi_hx = (float *)get((size_t)std::max<int64_t>(1, s.psi_len[0]) * 4);
            x.psi_hy = (float *)get((size_t)std::max<int64_t>(1, s.psi_len[1]) * 4);
            x.psi_ezx = (float *)get((size_t)std::max<int64_t>(1, s.psi_len[2]) * 4);
            x.psi_ezy = (float *)get((size_t)std::max<int64_t>(1, s.psi_len[3]) * 4);
        }
        int acur = 0;
        double *sez = (double *)get((size_t)nd * 8);  // zero-filled
        double *sbr = (double *)get((size_t)nd * 8);
        double *shx = grad_mu_dev ? (double *)get((size_t)nd * 8) : nullptr;
        double *shy = grad_mu_dev ? (double *)get((size_t)nd * 8) : nullptr;
        // derivatives of Ca = (e - h)/(e + h) and Cb = dt/(e + h), e = eps0
        // eps_r, h = sigma dt / 2, at the design cells (FP64):
        //   d/d eps_r: dCa = 2 eps0 h / (e + h)^2,  dCb = -eps0 dt / (e + h)^2
        //   d/d sigma: dCa = -dt e / (e + h)^2,     dCb = -dt^2 / (2 (e + h)^2)
        //   d/d mu_r (Hx -= Db bx, Hy += Db by, Db = dt / (mu0 mu_r)):
        //     dL/d mu_r = (Db / mu_r) (sum aHx bx - sum aHy by)
        std::vector<double> hd((size_t)(6 * nd));
        for (int i = i0; i < i1; ++i)
            for (int j = j0; j < j1; ++j) {
                const int64_t c = (int64_t)i * s.ny + j;
                const int64_t q = (int64_t)(i - i0) * (j1 - j0) + (j - j0);
                const double er = s.eps_r.empty() ? 1.0 : s.eps_r[(size_t)c];
                const double sg = s.sigma.empty() ? 0.0 : s.sigma[(size_t)c];
                const double e = kEps0 * er, h = 0.5 * sg * s.dt;
                const double den = (e + h) * (e + h);
                hd[(size_t)q] = kEps0 * 2.0 * h / den;
                hd[(size_t)(nd + q)] = -kEps0 * s.dt / den;
                hd[(size_t)(2 * nd + q)] = -s.dt * e / den;
                hd[(size_t)(3 * nd + q)] = -0.5 * s.dt * s.dt / den;
                const double mr = s.mu_r.empty() ? 1.0 : s.mu_r[(size_t)c];
                const double dbm = s.dt / (kMu0 * mr) / mr;
                hd[(size_t)(4 * nd + q)] = dbm;
                hd[(size_t)(5 * nd + q)] = -dbm;
            }
        double *dcoef = (double *)get((size_t)(6 * nd) * 8);
        hip_check(hipMemcpyAsync(dcoef, hd.data(), (size_t)(6 * nd) * 8, hipMemcpyHostToDevice, s.st), "upload");
        // probed cells (sorted) and their probe entries, for the loss seed
        std::vector<int> ust, pcell, pslot;
        {
            std::vector<std::pair<int64_t, int>> e;
            for (int64_t p = 0; p < P; ++p) e.push_back({s.probe_cells[(size_t)p], (int)p});
            std::sort(e.begin(), e.end());
            for (size_t q = 0; q < e.size(); ++q) {
                if (q == 0 || e[q].first != e[q - 1].first) ust.push_back((int)q);
                pcell.push_back((int)e[q].first);
                pslot.push_back(e[q].second);
            }
            ust.push_back((int)e.size());
        }
        const int nu = (int)ust.size() - 1;
        int *d_ust = (int *)get(ust.size() * 4);
        int *d_pcell = (int *)get(pcell.size() * 4);
        int *d_pslot = (int *)get(pslot.size() * 4);
        hip_check(hipMemcpyAsync(d_ust, ust.data(), ust.size() * 4, hipMemcpyHostToDevice, s.st), "upload");
        hip_check(hipMemcpyAsync(d_pcell, pcell.data(), pcell.size() * 4, hipMemcpyHostToDevice, s.st), "upload");
        hip_check(hipMemcpyAsync(d_pslot, pslot.data(), pslot.size() * 4, hipMemcpyHostToDevice, s.st), "upload");
        // the same entries grouped by tile of the adjoint kernel
        const int nsy = (s.ny + 62 * ac.V - 1) / (62 * ac.V), ncx = (s.nx + ac.TX - 1) / ac.TX;
        std::vector<int> tst((size_t)nsy * ncx + 1, 0), tcell, tslot;
        {
            std::vector<std::pair<int, int>> e;  // (tile, entry)
            for (size_t q = 0; q < pcell.size(); ++q) {
                const int i = pcell[q] / s.ny, j = pcell[q] % s.ny;
                e.push_back({(i / ac.TX) * nsy + j / (62 * ac.V), (int)q});
            }
            std::stable_sort(e.begin(), e.end(), [](const std::pair<int, int> &u, const std::pair<int, int> &v) {
                return u.first < v.first;
            });
            for (auto &x : e) {
                tst[(size_t)x.first + 1]++;
                tcell.push_back(pcell[(size_t)x.second]);
                tslot.push_back(pslot[(size_t)x.second]);
            }
            for (size_t t = 0; t + 1 < tst.size(); ++t) tst[t + 1] += tst[t];
        }
        int *d_tst = (int *)get(tst.size() * 4);
        int *d_tcell = (int *)get(std::max<size_t>(1, tcell.size()) * 4);
        int *d_tslot = (int *)get(std::max<size_t>(1, tslot.size()) * 4);
        hip_check(hipMemcpyAsync(d_tst, tst.data(), tst.size() * 4, hipMemcpyHostToDevice, s.st), "upload");
        hip_check(hipMemcpyAsync(d_tcell, tcell.data(), tcell.size() * 4, hipMemcpyHostToDevice, s.st), "upload");
        hip_check(hipMemcpyAsync(d_tslot, tslot.data(), tslot.size() * 4, hipMemcpyHostToDevice, s.st), "upload");
        const ProbeTiles apt{d_tst, d_tcell, d_tslot};
        hip_check(hipStreamSynchronize(s.st), "sync");
        // ---- backward over segments, newest first (the last one kept by
        //      the forward).  Segment g's adjoint steps run on the
        //      simulation's stream while segment g-1 is recomputed on a
        //      second stream: two sets of design values, events ordering
        //      each set's reuse.  The adjoint steps read the probe records
        //      from a copy taken after the forward, as a recompute rewrites
        //      its segment's records (multi-step passes grouped from another
        //      start step can differ in the last bits). ----
        float *rec_snap = (float *)get((size_t)std::max<int64_t>(1, P * s.rec_cap) * 4);
        hip_check(hipMemcpyAsync(rec_snap, s.rec_dev, (size_t)(P * s.rec_cap) * 4, hipMemcpyDeviceToDevice, s.st),
                  "records");
        const hipStream_t st0 = s.st;
        if (nseg >= 2) {
            hip_check(hipStreamCreateWithFlags(&rs, hipStreamNonBlocking), "stream");
            for (hipEvent_t *e : {&ev_rec[0], &ev_rec[1], &ev_adj[0], &ev_adj[1], &ev_start})
                hip_check(hipEventCreateWithFlags(e, hipEventDisableTiming), "event");
            hip_check(hipEventRecord(ev_start, st0), "event");  // checkpoints written
            hip_check(hipStreamWaitEvent(rs, ev_start, 0), "stream wait");
        }
        auto recompute = [&](int64_t g) {
            const int64_t k0 = g * L, k1 = std::min(T, (g + 1) * L);
            const int b = (int)(g & 1);
            // set b was last read by the adjoint steps of segment g + 2 (the
            // last segment's values come from the forward, in set b too)
            if (g + 2 < nseg) hip_check(hipStreamWaitEvent(rs, ev_adj[b], 0), "stream wait");
            StreamSwap sw(s, rs);
            copy_state(s, 0, ck + g * S, false);
            s.cur = 0;
            s.n_done = k0;
            s.n_rec = k0;
            const CapArgs cap{make_int4(i0, i1c, j0, j1c), cap_ez[b], cap_br[b], k0, ndc};
            run(k0, k1, &cap);
            hip_check(hipEventRecord(ev_rec[b], rs), "event");
        };
        for (int64_t g = nseg - 1; g >= 0; --g) {
            const int64_t k0 = g * L, k1 = std::min(T, (g + 1) * L);
            const int b = (int)(g & 1);
            if (g >= 1) recompute(g - 1);
            if (g + 1 < nseg) hip_check(hipStreamWaitEvent(st0, ev_rec[b], 0), "stream wait");
            const Prob2D p = s.prob2d(0, 0);
            for (int64_t k = k1 - 1; k >= k0; --k) {
                // the first step's input is seeded here, every later one by
                // the step that writes it
                if (k == T - 1 && T > n0 && T <= n1)
                    hip_check(launch_adj2d_seed(a[acur].ez, d_ust, d_pcell, d_pslot, nu, rec_snap, s.rec_cap, T - 1,
                                                st0),
                              "adjoint seed");
                const int seed_out = (k > n0 && k <= n1) ? 1 : 0;
                hip_check(launch_adj2d_fused(p, a[acur], a[1 - acur], dbox, cbox, cap_ez[b] + (k - k0) * ndc,
                                             cap_br[b] + (k - k0) * ndc, sez, sbr, shx, shy, seed_out, apt,
                                             rec_snap, s.rec_cap, k - 1, ac.V, ac.TX, st0),
                          "adjoint step");
                acur = 1 - acur;
            }
            if (rs) hip_check(hipEventRecord(ev_adj[b], st0), "event");
        }
        if (grad_eps_dev)
            hip_check(launch_grad_combine(sez, sbr, dcoef, dcoef + nd, grad_eps_dev, nd, s.st), "gradient");
        if (grad_sigma_dev)
            hip_check(launch_grad_combine(sez, sbr, dcoef + 2 * nd, dcoef + 3 * nd, grad_sigma_dev, nd, s.st),
                      "gradient");
        if (grad_mu_dev)
            hip_check(launch_grad_combine(shx, shy, dcoef + 4 * nd, dcoef + 5 * nd, grad_mu_dev, nd, s.st),
                      "gradient");
        // leave the forward state after T steps
        copy_state(s, 0, fin, false);
        s.cur = 0;
        s.n_done = T;
        s.n_rec = T;
        hip_check(hipEventRecord(s.ev1, s.st), "event");
        s.timed = true;
        s.last_launches = T * 3 + 1;
        hip_check(hipStreamSynchronize(s.st), "sync");
        release_streams();
        for (void *p : tmp) s.al.put(p);
        tmp.clear();
        s.kcfg = saved;
        s.pt_ntiles = -1;
        s.build_probe_tiles();
        if (loss_out) *loss_out = loss;
        return FDTD_OK;
    } catch (...) {
        const int rc = status_of_current_exception();
        if (sp) {
            (void)hipStreamSynchronize(sp->st);
            release_streams();
            for (void *p : tmp) sp->al.put(p);
            if (restore_cfg) {
                sp->kcfg = saved;
                sp->pt_ntiles = -1;
            }
        }
        return rc;
    }
}

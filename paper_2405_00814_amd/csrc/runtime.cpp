// Host runtime behind the C ABI: validation, edge-weight folding (Prop. 1
// weights as per-cell and per-axis tables), device state, stepping, I/O.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>

#include "sim.hpp"

namespace gem {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

struct Fail {
    int code;
    std::string msg;
};

void fail(int code, const std::string &msg) { throw Fail{code, msg}; }

// Status for the exception being handled (call from a catch block only).
int status_of_current_exception() {
    try {
        throw;
    } catch (const Fail &f) {
        set_error(f.msg);
        return f.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return FDTD_ENOMEM;
    } catch (...) {
        set_error("unexpected internal error");
        return FDTD_EDEVICE;
    }
}

void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) {
        if (e == hipErrorOutOfMemory) fail(FDTD_ENOMEM, std::string(what) + ": out of device memory");
        fail(FDTD_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    }
}

// ---------------------------------------------------------------------------
// Device memory
// ---------------------------------------------------------------------------
void *DevAlloc::get(size_t bytes) {
    if (bytes == 0) bytes = 4;
    bytes = (bytes + 255) & ~size_t(255);
    void *p = nullptr;
    if (has) {
        p = a.alloc(a.ctx, bytes, (void *)st);
        if (!p) fail(FDTD_ENOMEM, "allocator returned NULL");
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail(FDTD_ENOMEM, "hipMalloc failed");
        }
    }
    blocks.push_back(p);
    hip_check(hipMemsetAsync(p, 0, bytes, st), "hipMemsetAsync");
    return p;
}

void DevAlloc::put(void *p) {
    if (!p) return;
    auto it = std::find(blocks.begin(), blocks.end(), p);
    if (it == blocks.end()) return;
    blocks.erase(it);
    if (has) a.free(a.ctx, p, (void *)st);
    else {
        (void)hipStreamSynchronize(st);
        (void)hipFree(p);
    }
}

void DevAlloc::release_all() {
    if (blocks.empty()) return;
    (void)hipStreamSynchronize(st);
    for (void *p : blocks) {
        if (has) a.free(a.ctx, p, (void *)st);
        else (void)hipFree(p);
    }
    blocks.clear();
}

template <class T>
static T *dev_upload(DevAlloc &al, const T *h, size_t n, hipStream_t st) {
    T *d = (T *)al.get(n * sizeof(T));
    // an empty host list (nullptr) padded to one element uploads zeros
    if (n && h) hip_check(hipMemcpyAsync(d, h, n * sizeof(T), hipMemcpyHostToDevice, st), "upload");
    else if (n) hip_check(hipMemsetAsync(d, 0, n * sizeof(T), st), "upload");
    // callers pass short-lived host vectors: finish the copy before returning
    hip_check(hipStreamSynchronize(st), "upload sync");
    return d;
}

// ---------------------------------------------------------------------------
// CPML axis tables.  rho is the normalised depth into the layer (1 at the
// PEC wall), sampled at x = i (E-type) and x = i + 1/2 (H-type).
// ---------------------------------------------------------------------------
AxisHost build_axis(int n, int lo, int hi, double d, double dt, const fdtd_cpml &cp) {
    AxisHost A;
    A.n = n;
    A.lo = lo;
    A.hi = hi;
    const double eta0 = std::sqrt(kMu0 / kEps0);
    const double m = cp.m;
    const double smax = cp.sigma_max > 0 ? cp.sigma_max : 0.8 * (m + 1.0) / (eta0 * d);
    for (int half = 0; half < 2; ++half) {
        std::vector<float> &K = half ? A.kH : A.kE;
        std::vector<float> &B = half ? A.bH : A.bE;
        std::vector<float> &Cc = half ? A.cH : A.cE;
        K.resize(n);
        B.resize(n);
        Cc.resize(n);
        for (int i = 0; i < n; ++i) {
            const double x = i + (half ? 0.5 : 0.0);
            double rho = 0.0;
            if (lo > 0 && x < lo) rho = (lo - x) / lo;
            if (hi > 0 && x > n - hi) rho = std::max(rho, (x - (n - hi)) / hi);
            double kap = 1.0, b = 1.0, c = 0.0;
            if (rho > 0.0) {
                const double g = std::pow(rho, m);
                const double sg = smax * g;
                kap = 1.0 + (cp.kappa_max - 1.0) * g;
                const double al = cp.alpha_max * std::pow(1.0 - rho, cp.m_alpha);
                b = std::exp(-(sg / kap + al) * dt / kEps0);
                c = (sg > 0.0) ? sg * (b - 1.0) / (kap * (sg + kap * al)) : 0.0;
            }
            K[i] = (float)(1.0 / (kap * d));
            B[i] = (float)b;
            Cc[i] = (float)(c / d);
        }
    }
    return A;
}

// Tables of the split-field PML (same grading and positions as the CPML):
// k = 1/d, b = (1 - s)/(1 + s), c = 1/(1 + s), s = sigma dt / (2 eps0) (the
// magnetic layer at the H positions matched, sigma*/mu0 = sigma/eps0).
AxisHost build_axis_split(int n, int lo, int hi, double d, double dt, const fdtd_cpml &cp) {
    AxisHost A;
    A.n = n;
    A.lo = lo;
    A.hi = hi;
    const double eta0 = std::sqrt(kMu0 / kEps0);
    const double m = cp.m;
    const double smax = cp.sigma_max > 0 ? cp.sigma_max : 0.8 * (m + 1.0) / (eta0 * d);
    for (int half = 0; half < 2; ++half) {
        std::vector<float> &K = half ? A.kH : A.kE;
        std::vector<float> &B = half ? A.bH : A.bE;
        std::vector<float> &Cc = half ? A.cH : A.cE;
        K.assign(n, (float)(1.0 / d));
        B.resize(n);
        Cc.resize(n);
        for (int i = 0; i < n; ++i) {
            const double x = i + (half ? 0.5 : 0.0);
            double rho = 0.0;
            if (lo > 0 && x < lo) rho = (lo - x) / lo;
            if (hi > 0 && x > n - hi) rho = std::max(rho, (x - (n - hi)) / hi);
            const double s = smax * std::pow(rho, m) * dt / (2.0 * kEps0);
            B[i] = (float)((1.0 - s) / (1.0 + s));
            Cc[i] = (float)(1.0 / (1.0 + s));
        }
    }
    return A;
}

AxisDev upload_axis(DevAlloc &al, const AxisHost &h, hipStream_t st) {
    AxisDev a{};
    a.n = h.n;
    a.lo = h.lo;
    a.hi = h.hi;
    a.kE = dev_upload(al, h.kE.data(), h.n, st);
    a.bE = dev_upload(al, h.bE.data(), h.n, st);
    a.cE = dev_upload(al, h.cE.data(), h.n, st);
    a.kH = dev_upload(al, h.kH.data(), h.n, st);
    a.bH = dev_upload(al, h.bH.data(), h.n, st);
    a.cH = dev_upload(al, h.cH.data(), h.n, st);
    return a;
}

int src_nparams(int kind) { return kind == FDTD_SRC_MODGAUSS ? 4 : (kind == FDTD_SRC_TABLE ? 0 : 3); }

double source_sample(int kind, const double *par, double dt, int64_t n) {
    const double t = (double)(n + 1) * dt;
    if (kind == FDTD_SRC_GAUSSIAN) {
        const double u = (t - par[1]) / par[2];
        return par[0] * std::exp(-u * u);
    }
    if (kind == FDTD_SRC_RICKER) {
        double a = kPi * par[2] * (t - par[1]);
        a *= a;
        return par[0] * (1.0 - 2.0 * a) * std::exp(-a);
    }
    if (kind == FDTD_SRC_SINE) {
        double r = 1.0;
        if (t < par[2]) {
            const double q = std::sin(0.5 * kPi * t / par[2]);
            r = q * q;
        }
        return par[0] * r * std::sin(2.0 * kPi * par[1] * t);
    }
    if (kind == FDTD_SRC_MODGAUSS) {
        const double u = (t - par[1]) / par[2];
        return par[0] * std::exp(-u * u) * std::sin(2.0 * kPi * par[3] * (t - par[1]));
    }
    return 0.0;
}

// ---------------------------------------------------------------------------
// Sim
// ---------------------------------------------------------------------------
Sim::~Sim() {
    graph_reset();
    if (gr.cap_st) (void)hipStreamDestroy(gr.cap_st);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (evf) (void)hipEventDestroy(evf);
    if (evj) (void)hipEventDestroy(evj);
    if (side) (void)hipStreamDestroy(side);
    al.release_all();
}

Prob2D Sim::prob2d(int si, int so) const {
    Prob2D p{};
    p.nx = nx;
    p.ny = ny;
    p.ca = lossy ? ca : nullptr;
    p.cb = cb;
    p.db = mumap ? db : nullptr;
    p.db0 = db0;
    p.x = ax[0];
    p.y = ax[1];
    p.s0 = State2D{f[si][FDTD_EZ], f[si][FDTD_HX], f[si][FDTD_HY], psi[si][0], psi[si][1], psi[si][2], psi[si][3]};
    p.ezy = split ? ezy : nullptr;
    p.s1 = State2D{f[so][FDTD_EZ], f[so][FDTD_HX], f[so][FDTD_HY], psi[so][0], psi[so][1], psi[so][2], psi[so][3]};
    p.src_idx = src_idx;
    for (int q = 0; q < 6; ++q) p.src_box[q] = src_box[q];
    p.src_vals = src_dev;
    p.src_len = src_len;
    p.np = (int)probe_cells.size();
    p.probe_idx = probe_dev;
    p.probe_comp = probe_comp;
    p.rec = rec_dev;
    p.rec_stride = rec_cap;
    p.rec_base = n_done - n_rec;
    return p;
}

Prob3D Sim::prob3d(int si, int so) const {
    Prob3D p{};
    p.nx = nx;
    p.ny = ny;
    p.nz = nz;
    p.ca = lossy ? ca : nullptr;
    p.cb = cb;
    p.db = mumap ? db : nullptr;
    p.db0 = db0;
    p.x = ax[0];
    p.y = ax[1];
    p.z = ax[2];
    for (int c = 0; c < 6; ++c) {
        p.s0.f[c] = f[si][c];
        p.s1.f[c] = f[so][c];
    }
    for (int a = 0; a < NPSI3; ++a) {
        p.s0.psi[a] = psi[si][a];
        p.s1.psi[a] = psi[so][a];
    }
    p.src_idx = src_idx;
    for (int q = 0; q < 6; ++q) p.src_box[q] = src_box[q];
    p.src_comp = src_comp;
    p.src_vals = src_dev;
    p.src_len = src_len;
    p.np = (int)probe_cells.size();
    p.probe_comp = probe_comp;
    p.probe_idx = probe_dev64;
    p.rec = rec_dev;
    p.rec_stride = rec_cap;
    p.rec_base = n_done - n_rec;
    return p;
}

void Sim::ensure_source(int64_t upto) {
    if (src_idx < 0 || src_kind == FDTD_SRC_TABLE) return;
    if (upto <= src_cap) return;
    int64_t cap = std::max<int64_t>({upto, 2 * src_cap, 4096});
    std::vector<float> h((size_t)cap);
    for (int64_t n = 0; n < cap; ++n) h[(size_t)n] = (float)source_sample(src_kind, src_par, dt, n);
    float *d = dev_upload(al, h.data(), (size_t)cap, st);
    al.put(src_dev);
    src_dev = d;
    src_cap = cap;
    src_len = cap;
}

void Sim::ensure_rec(int64_t upto) {
    const int64_t P = (int64_t)probe_cells.size();
    if (P == 0 || upto <= rec_cap) return;
    const int64_t cap = std::max<int64_t>({upto, 2 * rec_cap, 1024});
    float *d = (float *)al.get((size_t)(P * cap) * sizeof(float));
    if (rec_dev && n_rec > 0)
        hip_check(hipMemcpy2DAsync(d, cap * sizeof(float), rec_dev, rec_cap * sizeof(float),
                                   n_rec * sizeof(float), P, hipMemcpyDeviceToDevice, st),
                  "record copy");
    al.put(rec_dev);
    rec_dev = d;
    rec_cap = cap;
}

// The first m records of every probe to host memory, row p at out + p * ld
// (synchronous).  A 2D device-to-host copy into pageable memory has read
// back zeros under a profiler's kernel tracing (rocprofv3), so the rows are
// gathered on the device into one block first and leave by 1D copies.
void Sim::records_to_host(float *out, int64_t ld, int64_t m) {
    const int64_t P = (int64_t)probe_cells.size();
    if (P > 0 && m > 0) {
        float *tmp = (float *)al.get((size_t)(P * m) * sizeof(float));
        hip_check(hipMemcpy2DAsync(tmp, m * sizeof(float), rec_dev, rec_cap * sizeof(float), m * sizeof(float), P,
                                   hipMemcpyDeviceToDevice, st),
                  "record gather");
        if (ld == m) {
            hip_check(hipMemcpyAsync(out, tmp, (size_t)(P * m) * sizeof(float), hipMemcpyDeviceToHost, st),
                      "record copy");
        } else {
            for (int64_t q = 0; q < P; ++q)
                hip_check(hipMemcpyAsync(out + q * ld, tmp + q * m, (size_t)m * sizeof(float), hipMemcpyDeviceToHost,
                                         st),
                          "record copy");
        }
        hip_check(hipStreamSynchronize(st), "sync");
        al.put(tmp);
    }
    hip_check(hipStreamSynchronize(st), "sync");
}

void Sim::build_probe_tiles() {
    if (kcfg.variant < 2 || is_graph) return;
    const int a = kcfg.tile[0], b = kcfg.tile[1], c3 = kcfg.tile[2];
    const int mat = this->mat();
    const int vm = kcfg.variant * 4 + mat;
    if (pt_ntiles >= 0 && pt_cfg[0] == a && pt_cfg[1] == b && pt_cfg[2] == (int)probe_cells.size() &&
        pt_cfg[3] == c3 && pt_cfg[4] == vm && pt_cfg[5] == kcfg.tile[3] && pt_start)
        return;
    // invalid until the rebuild completes: a failure below (out of memory)
    // leaves the cache empty, and every stepping call rebuilds before it
    // launches; each list is uploaded before its predecessor is released
    pt_ntiles = -1;
    auto swap_in = [&](auto *&slot, auto *fresh) {
        al.put(slot);
        slot = fresh;
    };
    if (ndim == 2) {
        const Fused2DCfg c = single2d();
        const int xl[2] = {ax[0].lo, ax[0].hi}, yl[2] = {ax[1].lo, ax[1].hi};
        const int nt = fused2d_ntiles(nx, ny, c);
        std::vector<int> ids, outer;
        for (int t = 0; t < nt; ++t) (fused2d_interior(nx, ny, c, xl, yl, t) ? ids : outer).push_back(t);
        tl2_inner = (int)ids.size();
        tl2_outer = (int)outer.size();
        ids.insert(ids.end(), outer.begin(), outer.end());
        swap_in(tl2_dev, dev_upload(al, ids.data(), std::max<size_t>(ids.size(), 1), st));
    }
    if (ndim == 3) {
        const int xl[2] = {ax[0].lo, ax[0].hi}, yl[2] = {ax[1].lo, ax[1].hi}, zl[2] = {ax[2].lo, ax[2].hi};
        wave3d_plan(nx, ny, nz, Fused3DCfg{a, c3}, xl, yl, zl, plan3);
        swap_in(tl_dev, dev_upload(al, plan3.tiles.data(), plan3.tiles.size(), st));
        if (kcfg.variant == 3) {
            two3d_plan(nx, ny, nz, Fused3DCfg{a, c3}, mat, b == 0, kcfg.tile[3], cus, xl, yl, zl, plan2);
            plan2_mat = mat;
            swap_in(tb_dev, plan2.tb.empty() ? nullptr : dev_upload(al, plan2.tb.data(), plan2.tb.size(), st));
            swap_in(tbo_dev, plan2.tbo.empty() ? nullptr : dev_upload(al, plan2.tbo.data(), plan2.tbo.size(), st));
            swap_in(p1_dev, plan2.pass1.tiles.empty()
                                ? nullptr
                                : dev_upload(al, plan2.pass1.tiles.data(), plan2.pass1.tiles.size(), st));
            swap_in(p2_dev, plan2.pass2.tiles.empty()
                                ? nullptr
                                : dev_upload(al, plan2.pass2.tiles.data(), plan2.pass2.tiles.size(), st));
            alloc_set(2);
        }
    }
    int ntiles;
    std::vector<int> tile(probe_cells.size());
    if (ndim == 2) {
        const Fused2DCfg c = single2d();
        ntiles = fused2d_ntiles(nx, ny, c);
        for (size_t q = 0; q < probe_cells.size(); ++q) {
            const int i = (int)(probe_cells[q] / ny), j = (int)(probe_cells[q] % ny);
            tile[q] = fused2d_tile_of(nx, ny, c, i, j);
        }
    } else {
        ntiles = wave3d_ngroups(nx, ny);
        for (size_t q = 0; q < probe_cells.size(); ++q) {
            const int64_t cell = probe_cells[q];
            const int i = (int)(cell / ((int64_t)ny * nz));
            const int j = (int)((cell / nz) % ny);
            tile[q] = wave3d_group_of(ny, i, j);
        }
    }
    std::vector<int> order(probe_cells.size());
    for (size_t q = 0; q < order.size(); ++q) order[q] = (int)q;
    std::stable_sort(order.begin(), order.end(), [&](int u, int v) { return tile[u] < tile[v]; });
    std::vector<int> start((size_t)ntiles + 1, 0), cell(order.size()), slot(order.size());
    for (size_t q = 0; q < order.size(); ++q) {
        cell[q] = (int)probe_cells[order[q]];
        slot[q] = order[q];
        start[(size_t)tile[order[q]] + 1]++;
    }
    for (int t = 0; t < ntiles; ++t) start[(size_t)t + 1] += start[(size_t)t];
    swap_in(pt_start, dev_upload(al, start.data(), start.size(), st));
    swap_in(pt_cell, dev_upload(al, cell.data(), std::max<size_t>(cell.size(), 1), st));
    swap_in(pt_slot, dev_upload(al, slot.data(), std::max<size_t>(slot.size(), 1), st));
    if (ndim == 3 && kcfg.variant == 3) {
        // which slab tiles record probes (a probe cell in their own planes
        // and rows), so that the others skip the group look-ups
        auto tile_of = [&](const std::vector<TileTB> &tl, int i, int j) {
            for (size_t t = 0; t < tl.size(); ++t)
                if (i >= tl[t].i0 && i < tl[t].i1 && j >= tl[t].j0 && j < tl[t].j0 + tl[t].nrows) return (int)t;
            return -1;
        };
        std::vector<int> fo(std::max<size_t>(plan2.tbo.size(), 1), 0);
        // probes of the interior tiles: the instance of the interior launch
        // has no probe read-out (with it, its plane loop ran 4 % slower
        // at 512^3, although no tile but the few probed ones executed it)
        std::vector<int> gc, gs;
        std::vector<Tile3> tw;
        const int V = 4, seg = 64 * V;
        for (size_t q = 0; q < probe_cells.size(); ++q) {
            const int64_t c = probe_cells[q];
            const int i = (int)(c / ((int64_t)ny * nz)), j = (int)((c / nz) % ny), k = (int)(c % nz);
            const int to = tile_of(plan2.tbo, i, j);
            if (to >= 0 || !plan2.slab_tb) {
                if (to >= 0) fo[(size_t)to] = 1;
                continue;
            }
            gc.push_back((int)c);
            gs.push_back((int)q);
            const int k0 = k / seg * seg;
            const Tile3 t{i, i + 1, j, k0, std::min(k0 + seg, nz), k0, 1, 1};
            bool dup = false;
            for (const Tile3 &u : tw) dup = dup || (u.i0 == t.i0 && u.j0 == t.j0 && u.k0 == t.k0);
            if (!dup) tw.push_back(t);
        }
        swap_in(tbo_any, dev_upload(al, fo.data(), fo.size(), st));
        pw.l.clear();
        pw.tiles = tw;
        if (!tw.empty()) {
            while (pw.tiles.size() % 8) pw.tiles.push_back(Tile3{0, 0, 0, 0, 0, 0, 0, 0});
            Wave3DLaunch l{};
            l.V = V;
            l.wpb = 8;
            l.pxy = false;
            l.pz = ax[2].lo + ax[2].hi > 0;
            l.off = 0;
            l.n = (int)pw.tiles.size();
            l.cells = (int64_t)tw.size() * seg;
            pw.l.push_back(l);
        }
        swap_in(pw_dev, tw.empty() ? nullptr : dev_upload(al, pw.tiles.data(), pw.tiles.size(), st));
        swap_in(pg_cell, gc.empty() ? nullptr : dev_upload(al, gc.data(), gc.size(), st));
        swap_in(pg_slot, gs.empty() ? nullptr : dev_upload(al, gs.data(), gs.size(), st));
        n_pg = (int)gc.size();
    }
    pt_cfg[0] = a;
    pt_cfg[1] = b;
    pt_cfg[2] = (int)probe_cells.size();
    pt_cfg[3] = c3;
    pt_cfg[4] = vm;
    pt_cfg[5] = kcfg.tile[3];
    if (ndim == 2 && kcfg.variant == 3) {
        const int V = kcfg.tile[0], TX = kcfg.tile[1], TB = kcfg.tile[2];
        const int xl[2] = {ax[0].lo, ax[0].hi}, yl[2] = {ax[1].lo, ax[1].hi};
        std::vector<Tile2T> in, out;
        tb2d_plan(0, nx, ny, V, TB, TX, kcfg.tile[3], xl, yl, in, out);
        tb2_inner = (int)in.size();
        tb2_outer = (int)out.size();
        in.insert(in.end(), out.begin(), out.end());
        swap_in(tb2_dev, dev_upload(al, in.data(), std::max<size_t>(in.size(), 1), st));
        // probe groups by position in the list: the tile starting at or
        // last before the probe's row in its strip
        const int ow = tb2d_own(V, TB), nstrip = (ny + ow - 1) / ow;
        std::vector<int> pos((size_t)nx * nstrip, -1);
        for (size_t q = 0; q < in.size(); ++q) pos[(size_t)in[q].i0 * nstrip + in[q].ja / ow] = (int)q;
        std::vector<int> tl(probe_cells.size());
        for (size_t q = 0; q < probe_cells.size(); ++q) {
            int i = (int)(probe_cells[q] / ny);
            const int j = (int)(probe_cells[q] % ny);
            while (pos[(size_t)i * nstrip + j / ow] < 0) --i;
            tl[q] = pos[(size_t)i * nstrip + j / ow];
        }
        std::vector<int> ord(probe_cells.size());
        for (size_t q = 0; q < ord.size(); ++q) ord[q] = (int)q;
        std::stable_sort(ord.begin(), ord.end(), [&](int u, int v) { return tl[u] < tl[v]; });
        std::vector<int> st2(in.size() + 1, 0), ce(ord.size()), sl(ord.size());
        for (size_t q = 0; q < ord.size(); ++q) {
            ce[q] = (int)probe_cells[ord[q]];
            sl[q] = ord[q];
            st2[(size_t)tl[ord[q]] + 1]++;
        }
        for (size_t t = 0; t < in.size(); ++t) st2[t + 1] += st2[t];
        swap_in(pt2_start, dev_upload(al, st2.data(), st2.size(), st));
        swap_in(pt2_cell, dev_upload(al, ce.data(), std::max<size_t>(ce.size(), 1), st));
        swap_in(pt2_slot, dev_upload(al, sl.data(), std::max<size_t>(sl.size(), 1), st));
    }
    pt_ntiles = ntiles;
}

Fused2DCfg Sim::single2d() const {
    if (kcfg.variant == 2) return Fused2DCfg{kcfg.tile[0], kcfg.tile[1]};
    return default_single2d(nx, ny);
}

// TB steps of the 2D grid in one pass: interior tiles without the CPML code
// on `st` and, at the same time, the tiles near a slab with it on the second
// stream.  The two sets read state n and write state n+TB of disjoint cells
// (own columns and rows; probe slots and design-cell captures of their own
// tiles), so they run concurrently: the few CPML tiles, long dependent chains
// of row loads, fill the CUs beside the interior tiles instead of running
// after them on an almost empty device.  `st` waits for both.
void Sim::launch_tb2d(int64_t step, const CapArgs *cap) {
    const int V = kcfg.tile[0], TB = kcfg.tile[2];
    const Prob2D p = prob2d(cur, 1 - cur);
    const ProbeTiles pt{pt2_start, pt2_cell, pt2_slot};
    const ProbeTiles po{pt2_start + tb2_inner, pt2_cell, pt2_slot};
    const bool fork = tb2_inner > 0 && tb2_outer > 0;
    if (fork) {
        hip_check(hipEventRecord(evf, st), "event");
        hip_check(hipStreamWaitEvent(side, evf, 0), "stream wait");
    }
    hip_check(launch_2d_tb(p, nullptr, tb2_dev + tb2_inner, tb2_outer, true, mat(), po, V, TB, nullptr, step,
                           fork ? side : st, cap),
              "2d multi-step (cpml)");
    if (fork) hip_check(hipEventRecord(evj, side), "event");
    hip_check(launch_2d_tb(p, nullptr, tb2_dev, tb2_inner, false, mat(), pt, V, TB, nullptr, step, st, cap),
              "2d multi-step");
    if (fork) hip_check(hipStreamWaitEvent(st, evj, 0), "stream wait");
    cur = 1 - cur;
    last_launches += (tb2_inner > 0) + (tb2_outer > 0);
}


// After step `step` (state step+1): the monitor's sums gain the field
// sample times exp(-2 pi i f t) dt, t = (step+1) dt for E and (step+1/2) dt
// for H (the sample's time on the leapfrog grid).
// The sample goes to the next row of the ring with its phase factors; a
// full ring is summed.
void Sim::dft_accumulate(int64_t step) {
    const int r = dft.nbuf;
    const double t = ((double)step + (dft.comp >= FDTD_HX ? 0.5 : 1.0)) * dt;
    for (int q = 0; q < dft.nf; ++q) {
        const double a = 2.0 * kPi * dft.f[q] * t;
        dft.pend.re[r][q] = std::cos(a) * dt;
        dft.pend.im[r][q] = -std::sin(a) * dt;
    }
    const float *fld = is_graph ? g.x : f[cur][dft.comp];
    const DftBox box{dft.box[0], dft.box[2], dft.box[4], dft.box[3] - dft.box[2], dft.box[5] - dft.box[4], ny, nz};
    hip_check(launch_dft_gather(fld, dft.idx, box, dft.npts, dft.ring + (int64_t)r * dft.npts, st), "dft");
    dft.nbuf = r + 1;
    dft.nacc += 1;
    last_launches += 1;
    if (dft.nbuf == kDftBatch) {
        dft_flush();
        last_launches += 1;
    }
}

// Sum the buffered samples into the monitor's FP64 sums.
void Sim::dft_flush() {
    if (dft.comp < 0 || dft.nbuf == 0) return;
    hip_check(launch_dft_flush(dft.ring, dft.npts, dft.nbuf, dft.nf, dft.pend, dft.acc, st), "dft sums");
    dft.nbuf = 0;
}

void Sim::launch_step(int64_t step) {
    if (is_graph) {
        graph_step(*this, step);
        return;
    }
    if (kcfg.variant == 1) {
        if (ndim == 2) hip_check(launch_2d_ref(prob2d(cur, cur), step, st), "2d reference step");
        else hip_check(launch_3d_ref(prob3d(cur, cur), step, st), "3d reference step");
        last_launches += 2 + (probe_cells.empty() ? 0 : 1);
        return;
    }
    ProbeTiles pt{pt_start, pt_cell, pt_slot};
    if (ndim == 2) {
        const Fused2DCfg c = single2d();
        const TileSplit2D sp{tl2_dev, tl2_inner, tl2_dev + tl2_inner, tl2_outer};
        hip_check(launch_2d_fused(prob2d(cur, 1 - cur), c, pt, step, st, nullptr, nullptr, nullptr,
                                  split2d() ? &sp : nullptr),
                  "2d fused step");
    } else {
        hip_check(launch_3d_wave(prob3d(cur, 1 - cur), plan3, tl_dev, pt, step, st, lev), "3d fused step");
    }
    cur = 1 - cur;
    if (ndim == 3) {
        last_launches += (int64_t)plan3.l.size();
    } else {
        const bool pml = ax[0].lo + ax[0].hi + ax[1].lo + ax[1].hi > 0;
        last_launches += (pml && split2d()) ? (tl2_inner > 0) + (tl2_outer > 0) : 1;
    }
}

void Sim::alloc_set(int set) {
    if (f[set][FDTD_EZ]) return;
    const size_t n = (size_t)ncell;
    // all or nothing: a set is used only when every array of it exists
    float *nf[6] = {}, *np[NPSI3] = {};
    try {
        if (ndim == 2) {
            for (int c : {FDTD_EZ, FDTD_HX, FDTD_HY}) nf[c] = (float *)al.get(n * 4);
        } else {
            for (int c = 0; c < 6; ++c) nf[c] = (float *)al.get(n * 4);
        }
        for (int a = 0; a < NPSI3; ++a)
            if (psi_len[a] > 0) np[a] = (float *)al.get((size_t)psi_len[a] * 4);
    } catch (...) {
        for (float *p : nf) al.put(p);
        for (float *p : np) al.put(p);
        throw;
    }
    for (int c = 0; c < 6; ++c) f[set][c] = nf[c];
    for (int a = 0; a < NPSI3; ++a) psi[set][a] = np[a];
}

// Two steps n -> n+2 from set cur into set 1-cur.  Slab tiles in the
// two-step kernel: the tiles near the x/y slabs (their step-1 psi kept in
// set 2), then the interior tiles, both reading set cur only.  Else the
// x/y-slab cells S and their rim M take a single step into set 2 (pass1),
// the interior tiles two steps at once, then S its second single step from
// set 2 (pass2).  The writes to set 1-cur are disjoint in their target
// cells; pass2 reads set 2 only where pass1 wrote it.  ev (optional):
// pair_launches() + 1 events, one before every launch and one after the
// last.
size_t Sim::pair_launches() const {
    return plan2.slab_tb ? 2 : plan2.pass1.l.size() + 1 + plan2.pass2.l.size();
}

void Sim::launch_pair(int64_t step, hipEvent_t *ev) {
    const int A = cur, B = 1 - cur, C = 2;
    const ProbeTiles pt{pt_start, pt_cell, pt_slot};
    const size_t n1 = plan2.pass1.l.size();
    const Prob3D pab = prob3d(A, B);
    if ((pab.db ? 2 : (pab.ca ? 1 : 0)) != plan2_mat) fail(FDTD_ESTATE, "two-step plan out of date");
    if (plan2.slab_tb) {
        const State3D mid = prob3d(C, C).s1;
        // the slab tiles in two groups: those near both slab kinds, and
        // those near one kind (a code path per kind, without the other
        // kind's psi code)
        const int nb = plan2.tbo_n[0], n1 = plan2.tbo_n[1];
        auto slab_pt = [&](int off) {
            ProbeTiles q = pt;
            q.tile_any = tbo_any + off;
            return q;
        };
        // second stream: the probes of the interior tiles at step n+1 (a
        // single step of their rows from set cur into the fields of set 2,
        // whose psi arrays the slab tiles use: the rows are clear of the x/y
        // slabs, so it writes none of those), and the few tiles near both
        // slab kinds, beside the others (all only read set cur)
        const bool fork = n_pg > 0 || nb > 0;
        if (fork) {
            hip_check(hipEventRecord(evf, st), "event");
            hip_check(hipStreamWaitEvent(side, evf, 0), "stream wait");
            if (n_pg > 0) hip_check(launch_3d_wave(prob3d(A, C), pw, pw_dev, pt, step, side), "3d probe rows");
            if (nb > 0)
                hip_check(launch_3d_two(pab, tbo_dev, nb, slab_pt(0), step, side, &mid, 3), "3d two-step (slab corners)");
            hip_check(hipEventRecord(evj, side), "event");
        }
        if (ev) hip_check(hipEventRecord(ev[0], st), "event");
        if (n1 > 0) hip_check(launch_3d_two(pab, tbo_dev + nb, n1, slab_pt(nb), step, st, &mid, 4), "3d two-step (slabs)");
        if (ev) hip_check(hipEventRecord(ev[1], st), "event");
        const ProbeTiles none{nullptr, nullptr, nullptr};
        hip_check(launch_3d_two(pab, tb_dev, (int)plan2.tb.size(), none, step, st), "3d two-step");
        if (ev) hip_check(hipEventRecord(ev[2], st), "event");
        if (fork) hip_check(hipStreamWaitEvent(st, evj, 0), "stream wait");
        if (n_pg > 0)  // and at step n+2, from the output set
            hip_check(launch_3d_probe_list(prob3d(B, A), pg_cell, pg_slot, n_pg, step + 1, st), "3d probes");
        cur = B;
        last_launches += (nb > 0) + (n1 > 0) + (plan2.tb.empty() ? 0 : 1) + (n_pg > 0 ? 2 : 0);
        return;
    }
    hip_check(launch_3d_wave(prob3d(A, C), plan2.pass1, p1_dev, pt, step, st, ev), "3d pass1");
    hip_check(launch_3d_two(pab, tb_dev, (int)plan2.tb.size(), pt, step, st), "3d two-step");
    hip_check(launch_3d_wave(prob3d(C, B), plan2.pass2, p2_dev, pt, step + 1, st, ev ? ev + n1 + 1 : nullptr),
              "3d pass2");
    cur = B;
    last_launches += (int64_t)(n1 + plan2.pass2.l.size()) + (plan2.tb.empty() ? 0 : 1);
}

void Sim::graph_reset() {
    if (gr.exec) (void)hipGraphExecDestroy(gr.exec);
    if (gr.graph) (void)hipGraphDestroy(gr.graph);
    gr.exec = nullptr;
    gr.graph = nullptr;
    gr.key.clear();
}

// Whole replays of the captured graph of kcfg.tb steps (multi-step passes
// of both tile lists, an even number of passes, then the counter advance)
// from buffer set 0: the state must start on set 0 (the caller aligns it).
// Returns the steps done.
int64_t Sim::graph_advance(int64_t n) {
    const int G = kcfg.tb, TB = kcfg.tile[2], V = kcfg.tile[0];
    const int64_t reps = n / G;
    if (reps == 0) return 0;
    if (!gr.probs) {
        gr.probs = (Prob2D *)al.get(2 * sizeof(Prob2D));
        gr.step_base = (int64_t *)al.get(sizeof(int64_t));
    }
    // the problem of each parity (its source table and record may have
    // moved): data, not part of the graph
    const Prob2D h[2] = {prob2d(0, 1), prob2d(1, 0)};
    hip_check(hipMemcpyAsync(gr.probs, h, sizeof h, hipMemcpyHostToDevice, st), "upload");
    hip_check(hipMemcpyAsync(gr.step_base, &n_done, sizeof(int64_t), hipMemcpyHostToDevice, st), "upload");
    const std::vector<const void *> key = {tb2_dev, pt2_start, pt2_cell, pt2_slot, gr.probs, gr.step_base,
                                           (const void *)(intptr_t)G, (const void *)(intptr_t)TB,
                                           (const void *)(intptr_t)V, (const void *)(intptr_t)tb2_inner,
                                           (const void *)(intptr_t)tb2_outer, (const void *)(intptr_t)mat()};
    if (!gr.exec || key != gr.key) {
        graph_reset();
        if (!gr.cap_st) hip_check(hipStreamCreateWithFlags(&gr.cap_st, hipStreamNonBlocking), "stream");
        hip_check(hipStreamBeginCapture(gr.cap_st, hipStreamCaptureModeRelaxed), "begin capture");
        const Prob2D none{};
        const ProbeTiles pt{pt2_start, pt2_cell, pt2_slot};
        const ProbeTiles po{pt2_start + tb2_inner, pt2_cell, pt2_slot};
        hipError_t e = hipSuccess;
        for (int k = 0; k < G / TB && e == hipSuccess; ++k) {
            e = launch_2d_tb(none, gr.probs + (k & 1), tb2_dev, tb2_inner, false, mat(), pt, V, TB, gr.step_base,
                             (int64_t)k * TB, gr.cap_st);
            if (e == hipSuccess)
                e = launch_2d_tb(none, gr.probs + (k & 1), tb2_dev + tb2_inner, tb2_outer, true, mat(), po, V, TB,
                                 gr.step_base, (int64_t)k * TB, gr.cap_st);
        }
        if (e == hipSuccess) e = launch_advance(gr.step_base, G, gr.cap_st);
        const hipError_t e2 = hipStreamEndCapture(gr.cap_st, &gr.graph);
        hip_check(e, "graph capture");
        hip_check(e2, "end capture");
        hip_check(hipGraphInstantiate(&gr.exec, gr.graph, nullptr, nullptr, 0), "instantiate");
        gr.key = key;
        gr.steps = G;
    }
    for (int64_t r = 0; r < reps; ++r) hip_check(hipGraphLaunch(gr.exec, st), "graph launch");
    const int per = G / TB;
    last_launches += reps * (per * ((tb2_inner > 0) + (tb2_outer > 0)) + 1);
    return reps * G;
}

// n steps: pairs through the two-step pass where it is selected, single
// steps otherwise
void Sim::advance(int64_t n) {
    // a frequency-domain monitor needs every step's field: single steps
    const bool mon = dft.comp >= 0;
    const bool two = kcfg.variant == 3 && ndim == 3 && !is_graph && !mon;
    const bool tb2 = kcfg.variant == 3 && ndim == 2 && !is_graph && !mon;
    const int64_t inc = probe_cells.empty() ? 0 : 1;
    int64_t q = 0;
    // whole grid in one workgroup: all n steps in one launch (single steps
    // where the probes no longer fit it)
    if (kcfg.variant == 4 && ndim == 2 && !is_graph && !mon && n > 0 && res2d_ok()) {
        hip_check(launch_2d_resident(prob2d(cur, 1 - cur), mat(), n_done, n, st), "2d resident steps");
        cur = 1 - cur;
        n_done += n;
        n_rec += n * inc;
        last_launches += (n + 65535) / 65536;
        return;
    }
    if (two)
        for (; q + 2 <= n; q += 2) {
            launch_pair(n_done);
            n_done += 2;
            n_rec += 2 * inc;
        }
    if (tb2) {
        const int TB = kcfg.tile[2];
        // graph replays start on buffer set 0: one eager pass aligns
        if (kcfg.tb > 1 && n - q >= kcfg.tb + (cur ? TB : 0)) {
            if (cur == 1) {
                launch_tb2d(n_done);
                n_done += TB;
                n_rec += TB * inc;
                q += TB;
            }
            const int64_t g = graph_advance(n - q);
            n_done += g;
            n_rec += g * inc;
            q += g;
        }
        for (; q + TB <= n; q += TB) {
            launch_tb2d(n_done);
            n_done += TB;
            n_rec += TB * inc;
        }
    }
    for (; q < n; ++q) {
        launch_step(n_done);
        if (mon) dft_accumulate(n_done);
        n_done += 1;
        n_rec += inc;
    }
}

// The split-field PML's layer cells must be vacuum (their tables assume
// eps0, mu0, no loss).
void Sim::split_check() const {
    const int xlo = ax[0].lo, xhi = ax[0].hi, ylo = ax[1].lo, yhi = ax[1].hi;
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            if (!(i < xlo || i >= nx - xhi || j < ylo || j >= ny - yhi)) continue;
            const size_t c = (size_t)i * ny + j;
            if ((!eps_r.empty() && eps_r[c] != 1.f) || (!mu_r.empty() && mu_r[c] != 1.f) ||
                (!sigma.empty() && sigma[c] != 0.f))
                fail(FDTD_EINVAL, "the split-field PML needs vacuum in its layer cells");
        }
}

void Sim::zero_state() {
    for (int s = 0; s < 3; ++s) {
        for (int c = 0; c < 6; ++c)
            if (f[s][c]) hip_check(hipMemsetAsync(f[s][c], 0, (size_t)ncell * 4, st), "memset");
        for (int a = 0; a < NPSI3; ++a)
            if (psi[s][a]) hip_check(hipMemsetAsync(psi[s][a], 0, (size_t)psi_len[a] * 4, st), "memset");
    }
    if (is_graph && g.x) hip_check(hipMemsetAsync(g.x, 0, (size_t)g.nnodes * 4, st), "memset");
    if (dft.acc) hip_check(hipMemsetAsync(dft.acc, 0, (size_t)(2 * dft.nf * dft.npts) * 8, st), "memset");
    dft.nacc = 0;
    dft.nbuf = 0;
    if (ezy) hip_check(hipMemsetAsync(ezy, 0, (size_t)ncell * 4, st), "memset");
    cur = 0;
    n_done = 0;
    n_rec = 0;
}

// Fold eps_r, sigma, mu_r into Ca, Cb, Db (double, rounded once) and upload.
void Sim::refold(int64_t c0, int64_t c1) {
    (void)c0;
    (void)c1;
    std::vector<float> hcb((size_t)ncell), hca, hdb;
    if (lossy) hca.resize((size_t)ncell);
    for (int64_t c = 0; c < ncell; ++c) {
        const double er = eps_r.empty() ? 1.0 : eps_r[(size_t)c];
        const double sg = sigma.empty() ? 0.0 : sigma[(size_t)c];
        const double eps = kEps0 * er;
        const double sh = sg * dt / (2.0 * eps);
        hcb[(size_t)c] = (float)((dt / eps) / (1.0 + sh));
        if (lossy) hca[(size_t)c] = (float)((1.0 - sh) / (1.0 + sh));
    }
    if (!cb) cb = (float *)al.get((size_t)ncell * 4);
    hip_check(hipMemcpyAsync(cb, hcb.data(), (size_t)ncell * 4, hipMemcpyHostToDevice, st), "cb");
    if (lossy) {
        if (!ca) ca = (float *)al.get((size_t)ncell * 4);
        hip_check(hipMemcpyAsync(ca, hca.data(), (size_t)ncell * 4, hipMemcpyHostToDevice, st), "ca");
    }
    db0 = (float)(dt / (kMu0 * (mu_r.empty() ? 1.0 : mu_r[0])));
    if (mumap) {
        hdb.resize((size_t)ncell);
        for (int64_t c = 0; c < ncell; ++c) hdb[(size_t)c] = (float)(dt / (kMu0 * mu_r[(size_t)c]));
        if (!db) db = (float *)al.get((size_t)ncell * 4);
        hip_check(hipMemcpyAsync(db, hdb.data(), (size_t)ncell * 4, hipMemcpyHostToDevice, st), "db");
    }
    // the host vectors must live until the copies finish
    hip_check(hipStreamSynchronize(st), "sync");
}

// 2D defaults (measured on MI355X over grids of 256^2 .. 6400^2): single
// steps below 1.5M cells (one column per lane below 8M cells, two above),
// four steps per pass from 1.5M cells on with one column per lane (two were
// 10-20 % slower at every size) and the row chunk from tb2d_default_tx.
constexpr int64_t kTB2MinCells = (int64_t)3 << 19;
constexpr int64_t kWide2DCells = (int64_t)8 << 20;
constexpr int kTB2DefaultTX = 4;
// smallest 3D grid (cells) on which the default takes two steps per pass
constexpr int64_t kTwoStepMinCells = (int64_t)1 << 23;

Fused2DCfg default_single2d(int nx, int ny) {
    const bool wide = (int64_t)nx * ny >= kWide2DCells && ny % 2 == 0;
    return wide ? Fused2DCfg{2, 4} : Fused2DCfg{1, 2};
}

int default_variant_tiles(const Sim &s, fdtd_kernel_config &k) {
    k = fdtd_kernel_config{};
    k.tb = 1;
    if (s.split) {  // the split-field PML runs in the reference kernels only
        k.variant = 1;
        return 0;
    }
    if (s.ndim == 2) {
        if (!s.is_graph && s.res2d_ok()) {  // small grid without CPML: one workgroup
            k.variant = 4;
            return 0;
        }
        const int vt = 1, tx = tb2d_default_tx(s.nx, s.ny, vt, s.cus);
        if (s.ncell >= kTB2MinCells && tb2d_supported(s.ny, vt, 4, tx)) {
            k.variant = 3;
            k.tile[0] = vt;
            k.tile[1] = tx;
            k.tile[2] = 4;
            k.tile[3] = tx >= 16 ? tx / 4 : 0;  // CPML tiles in quarters of long chunks
            return 0;
        }
        const Fused2DCfg c = default_single2d(s.nx, s.ny);
        if (fused2d_supported(s.nx, s.ny, c)) {
            k.variant = 2;
            k.tile[0] = c.V;
            k.tile[1] = c.TX;
            return 0;
        }
    } else {
        Fused3DCfg c{s.nz % 4 == 0 ? 4 : (s.nz % 2 == 0 ? 2 : 1), 0};
        if (wave3d_supported(s.nx, s.ny, s.nz, c)) {
            // two steps per pass on grids large enough for its interior
            // tiles to dominate; single steps otherwise
            const bool two = c.V == 4 && s.ncell >= kTwoStepMinCells &&
                             two3d_supported(s.nx, s.ny, s.nz, s.ax[2].lo, s.ax[2].hi);
            k.variant = two ? 3 : 2;
            k.tile[0] = c.V;
            return 0;
        }
    }
    k.variant = 1;
    return 0;
}

static bool config_ok(const Sim &s, const fdtd_kernel_config &k) {
    // tb: 0 or 1; for 2D multi-step passes also the steps per replayed graph
    // (an even number of passes, at most 1024 steps)
    const bool graph_tb = s.ndim == 2 && k.variant == 3 && k.tile[2] > 0 && k.tb >= 2 * k.tile[2] && k.tb <= 1024 &&
                          k.tb % (2 * k.tile[2]) == 0 && !s.is_graph;
    if (k.tb != 0 && k.tb != 1 && !graph_tb) return false;
    if (k.variant == 1) return true;
    if (s.split) return false;
    if (k.variant == 4)  // whole grid in one workgroup: checked again (probes) at every step call
        return s.ndim == 2 && !s.is_graph && k.tile[0] == 0 && k.tile[1] == 0 && k.tile[2] == 0 &&
               k.tile[3] == 0 && s.res2d_ok();
    if (k.variant != 2 && k.variant != 3) return false;
    if (s.ndim == 2) {
        if (k.variant == 2) return fused2d_supported(s.nx, s.ny, Fused2DCfg{k.tile[0], k.tile[1]});
        return k.tile[3] >= 0 && k.tile[3] <= 65536 && tb2d_supported(s.ny, k.tile[0], k.tile[2], k.tile[1]) &&
               fused2d_supported(s.nx, s.ny, default_single2d(s.nx, s.ny));
    }
    if (k.variant == 2 && (k.tile[1] != 0 || k.tile[3] != 0)) return false;
    if (k.variant == 3 && (k.tile[1] < 0 || k.tile[1] > 1 || k.tile[3] < 0 || k.tile[3] > 4096)) return false;
    if (!wave3d_supported(s.nx, s.ny, s.nz, Fused3DCfg{k.tile[0], k.tile[2]})) return false;
    return k.variant == 2 || (k.tile[0] == 4 && two3d_supported(s.nx, s.ny, s.nz, s.ax[2].lo, s.ax[2].hi));
}

// ---------------------------------------------------------------------------
// Creation
// ---------------------------------------------------------------------------
static bool finite_pos(double v) { return std::isfinite(v) && v > 0; }

static void check_map(const float *m, int64_t n, double lo, const char *name) {
    if (!m) return;
    for (int64_t c = 0; c < n; ++c)
        if (!std::isfinite(m[c]) || m[c] < lo) {
            std::ostringstream o;
            o << name << "[" << c << "] = " << m[c] << " is invalid (must be finite and >= " << lo << ")";
            fail(FDTD_EINVAL, o.str());
        }
}

void validate_desc(const fdtd_desc *d) {
    if (!d) fail(FDTD_EINVAL, "desc is NULL");
    if (d->ndim != 2 && d->ndim != 3) fail(FDTD_EINVAL, "ndim must be 2 or 3");
    if (d->nx < 3 || d->ny < 3) fail(FDTD_EINVAL, "nx and ny must be >= 3");
    if (d->ndim == 3 && d->nz < 3) fail(FDTD_EINVAL, "nz must be >= 3 for ndim 3");
    if (d->ndim == 2 && d->nz != 1) fail(FDTD_EINVAL, "nz must be 1 for ndim 2");
    const int64_t ncell = (int64_t)d->nx * d->ny * d->nz;
    if (ncell >= ((int64_t)1 << 31)) fail(FDTD_EINVAL, "grid too large (more than 2^31 cells)");
    if (!finite_pos(d->dx) || !finite_pos(d->dy) || (d->ndim == 3 && !finite_pos(d->dz)))
        fail(FDTD_EINVAL, "spatial steps must be finite and > 0");
    if (!finite_pos(d->dt)) fail(FDTD_EINVAL, "dt must be finite and > 0");
    double s = 1.0 / (d->dx * d->dx) + 1.0 / (d->dy * d->dy);
    if (d->ndim == 3) s += 1.0 / (d->dz * d->dz);
    if (kC0 * d->dt * std::sqrt(s) > 1.0 + 1e-12) {
        std::ostringstream o;
        o << "dt = " << d->dt << " exceeds the Courant limit " << 1.0 / (kC0 * std::sqrt(s));
        fail(FDTD_EUNSTABLE, o.str());
    }
    const int n[3] = {d->nx, d->ny, d->nz};
    for (int a = 0; a < 3; ++a) {
        const int lo = d->cpml.npml[2 * a], hi = d->cpml.npml[2 * a + 1];
        if (lo < 0 || hi < 0) fail(FDTD_EINVAL, "npml must be >= 0");
        if (a == 2 && d->ndim == 2 && (lo || hi)) fail(FDTD_EINVAL, "npml along z must be 0 for ndim 2");
        if (lo + hi > 0 && lo + hi >= n[a]) fail(FDTD_EINVAL, "CPML thicker than the grid");
    }
    const fdtd_cpml &c = d->cpml;
    if (!(c.m >= 0) || !std::isfinite(c.m) || !(c.kappa_max >= 1.0) || !std::isfinite(c.kappa_max) ||
        !(c.alpha_max >= 0) || !std::isfinite(c.alpha_max) || !(c.m_alpha >= 0) ||
        !std::isfinite(c.m_alpha) || !std::isfinite(c.sigma_max))
        fail(FDTD_EINVAL, "invalid CPML parameters");
    if (c.split != 0 && c.split != 1) fail(FDTD_EINVAL, "cpml.split must be 0 or 1");
    if (c.split == 1 && d->ndim != 2) fail(FDTD_EINVAL, "the split-field PML is 2D only");
    check_map(d->eps_r, ncell, 1.0, "eps_r");
    check_map(d->mu_r, ncell, 1.0, "mu_r");
    check_map(d->sigma, ncell, 0.0, "sigma");
}

void init_sim(Sim &s, const fdtd_desc *d) {
    validate_desc(d);
    s.ndim = d->ndim;
    s.nx = d->nx;
    s.ny = d->ny;
    s.nz = d->nz;
    s.ncell = (int64_t)s.nx * s.ny * s.nz;
    s.dx = d->dx;
    s.dy = d->dy;
    s.dz = d->ndim == 3 ? d->dz : 1.0;
    s.dt = d->dt;
    s.cpml = d->cpml;
    s.split = d->cpml.split == 1;
    s.st = (hipStream_t)d->stream;
    hip_check(hipGetDevice(&s.device), "hipGetDevice");
    hip_check(hipDeviceGetAttribute(&s.cus, hipDeviceAttributeMultiprocessorCount, s.device), "device attribute");
    s.al.st = s.st;
    if (d->allocator) {
        if (!d->allocator->alloc || !d->allocator->free) fail(FDTD_EINVAL, "allocator callbacks missing");
        s.al.a = *d->allocator;
        s.al.has = true;
    }
    const size_t n = (size_t)s.ncell;
    if (d->eps_r) s.eps_r.assign(d->eps_r, d->eps_r + n);
    if (d->sigma) {
        s.sigma.assign(d->sigma, d->sigma + n);
        s.lossy = std::any_of(s.sigma.begin(), s.sigma.end(), [](float v) { return v > 0.f; });
    }
    if (d->mu_r) {
        s.mu_r.assign(d->mu_r, d->mu_r + n);
        const float m0 = s.mu_r[0];
        s.mumap = std::any_of(s.mu_r.begin(), s.mu_r.end(), [m0](float v) { return v != m0; });
    }
    s.refold(0, s.ncell);
    const double dd[3] = {s.dx, s.dy, s.dz};
    const int nn[3] = {s.nx, s.ny, s.nz};
    for (int a = 0; a < 3; ++a) {
        if (a == 2 && s.ndim == 2) {
            s.axh[a] = build_axis(1, 0, 0, 1.0, s.dt, s.cpml);
        } else {
            s.axh[a] = s.split ? build_axis_split(nn[a], s.cpml.npml[2 * a], s.cpml.npml[2 * a + 1], dd[a], s.dt, s.cpml)
                               : build_axis(nn[a], s.cpml.npml[2 * a], s.cpml.npml[2 * a + 1], dd[a], s.dt, s.cpml);
        }
        s.ax[a] = upload_axis(s.al, s.axh[a], s.st);
    }
    const int sx = s.ax[0].lo + s.ax[0].hi, sy = s.ax[1].lo + s.ax[1].hi, sz = s.ax[2].lo + s.ax[2].hi;
    if (s.ndim == 2) {
        s.psi_len[0] = (int64_t)s.nx * sy;  // psi_hx
        s.psi_len[1] = (int64_t)sx * s.ny;  // psi_hy
        s.psi_len[2] = (int64_t)sx * s.ny;  // psi_ezx
        s.psi_len[3] = (int64_t)s.nx * sy;  // psi_ezy
    } else {
        const int64_t X = (int64_t)sx * s.ny * s.nz, Y = (int64_t)s.nx * sy * s.nz,
                      Z = (int64_t)s.nx * s.ny * sz;
        const int64_t len[NPSI3] = {Y, Z, Z, X, X, Y, Y, Z, Z, X, X, Y};
        for (int a = 0; a < NPSI3; ++a) s.psi_len[a] = len[a];
    }
    for (int set = 0; set < 2; ++set) s.alloc_set(set);
    if (s.split) {
        s.split_check();
        s.ezy = (float *)s.al.get(n * 4);
    }
    hip_check(hipEventCreate(&s.ev0), "event");
    hip_check(hipEventCreate(&s.ev1), "event");
    hip_check(hipStreamCreateWithFlags(&s.side, hipStreamNonBlocking), "stream");
    hip_check(hipEventCreateWithFlags(&s.evf, hipEventDisableTiming), "event");
    hip_check(hipEventCreateWithFlags(&s.evj, hipEventDisableTiming), "event");
    default_variant_tiles(s, s.kcfg);
    hip_check(hipStreamSynchronize(s.st), "sync");
}


// ---------------------------------------------------------------------------
// Autotune cache: a flat JSON object {"key": [variant, t0, t1, t2, t3, tb], ...}
// ---------------------------------------------------------------------------
static std::string tune_key(const Sim &s) {
    hipDeviceProp_t pr{};
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&pr, s.device) == hipSuccess) arch = pr.gcnArchName;
    std::ostringstream o;
    o << arch << "|" << s.ndim << "|" << s.nx << "x" << s.ny << "x" << s.nz << "|L" << s.lossy << "|M"
      << s.mumap << "|P" << (s.ax[0].lo + s.ax[0].hi + s.ax[1].lo + s.ax[1].hi + s.ax[2].lo + s.ax[2].hi > 0);
    return o.str();
}

std::map<std::string, std::vector<int>> read_cache(const char *path) {
    std::map<std::string, std::vector<int>> m;
    std::ifstream f(path);
    if (!f) return m;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string t = ss.str();
    size_t p = 0;
    while (true) {
        size_t a = t.find('"', p);
        if (a == std::string::npos) break;
        size_t b = t.find('"', a + 1);
        if (b == std::string::npos) break;
        const std::string key = t.substr(a + 1, b - a - 1);
        size_t l = t.find('[', b), r = t.find(']', b);
        if (l == std::string::npos || r == std::string::npos || r < l) break;
        std::vector<int> v;
        std::stringstream vs(t.substr(l + 1, r - l - 1));
        std::string tok;
        while (std::getline(vs, tok, ',')) v.push_back(std::atoi(tok.c_str()));
        m[key] = v;
        p = r + 1;
    }
    return m;
}

void write_cache(const char *path, const std::map<std::string, std::vector<int>> &m) {
    const std::string tmp = std::string(path) + ".tmp";
    std::ofstream f(tmp);
    if (!f) return;
    f << "{\n";
    size_t q = 0;
    for (auto &kv : m) {
        f << "  \"" << kv.first << "\": [";
        for (size_t i = 0; i < kv.second.size(); ++i) f << (i ? ", " : "") << kv.second[i];
        f << "]" << (++q < m.size() ? "," : "") << "\n";
    }
    f << "}\n";
    f.close();
    std::rename(tmp.c_str(), path);
}

}  // namespace gem

using namespace gem;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
#define GEM_TRY try {
#define GEM_CATCH                                   \
    }                                               \
    catch (const Fail &f) {                         \
        set_error(f.msg);                           \
        return f.code;                              \
    }                                               \
    catch (const std::bad_alloc &) {                \
        set_error("host allocation failed");        \
        return FDTD_ENOMEM;                         \
    }                                               \
    catch (...) {                                   \
        set_error("unexpected internal error");     \
        return FDTD_EDEVICE;                        \
    }

extern "C" {

const char *fdtd_last_error(void) { return g_err.c_str(); }

const char *fdtd_version(void) { return "gemfdtd 0.1 (gfx950)"; }

int fdtd_create(const fdtd_desc *desc, fdtd_sim **out) {
    if (!out) {
        set_error("out is NULL");
        return FDTD_EINVAL;
    }
    *out = nullptr;
    fdtd_sim *h = nullptr;
    GEM_TRY
    h = new fdtd_sim();
    init_sim(h->s, desc);
    *out = h;
    set_error("");
    return FDTD_OK;
    }
    catch (const Fail &f) {
        delete h;
        set_error(f.msg);
        return f.code;
    }
    catch (...) {
        delete h;
        set_error("unexpected internal error");
        return FDTD_EDEVICE;
    }
}

int fdtd_create_graph(const fdtd_desc *desc, fdtd_sim **out) {
    if (!out) {
        set_error("out is NULL");
        return FDTD_EINVAL;
    }
    *out = nullptr;
    fdtd_sim *h = nullptr;
    GEM_TRY
    if (desc && desc->ndim != 2) fail(FDTD_EINVAL, "the explicit graph form supports ndim 2 only");
    validate_desc(desc);
    {
        // size check before any device work: node and nonzero counts of the
        // graph fit its int32 indices
        const int sx = desc->cpml.npml[0] + desc->cpml.npml[1], sy = desc->cpml.npml[2] + desc->cpml.npml[3];
        const int64_t N = (int64_t)desc->nx * desc->ny;
        const bool split = desc->cpml.split == 1;
        const int64_t nodes = split ? 4 * N : 3 * N + 2LL * desc->nx * sy + 2LL * desc->ny * sx;
        if (nodes >= ((int64_t)1 << 31)) fail(FDTD_EINVAL, "graph too large for 32-bit node indices");
        if (graph_layer_nnz_max(desc->nx, desc->ny, sx, sy, split) >= (int64_t)INT32_MAX)
            fail(FDTD_EINVAL, "graph too large: a layer would hold 2^31 or more nonzeros (int32 row pointers)");
    }
    h = new fdtd_sim();
    init_sim(h->s, desc);
    h->s.is_graph = true;
    build_graph(h->s);
    *out = h;
    set_error("");
    return FDTD_OK;
    }
    catch (const Fail &f) {
        delete h;
        set_error(f.msg);
        return f.code;
    }
    catch (...) {
        delete h;
        set_error("unexpected internal error");
        return FDTD_EDEVICE;
    }
}

int fdtd_destroy(fdtd_sim *sim) {
    if (!sim) return FDTD_OK;
    delete sim;
    return FDTD_OK;
}

static bool on_wall(const Sim &s, int comp, const int *c) {
    // E components tangential to the low PEC planes are never updated
    const int i = c[0], j = c[1], k = s.ndim == 3 ? c[2] : 1;
    if (comp == FDTD_EX) return j < 1 || k < 1;
    if (comp == FDTD_EY) return i < 1 || k < 1;
    if (comp == FDTD_EZ) return i < 1 || j < 1;
    return false;
}

static int64_t lin_cell(const Sim &s, const int32_t *ijk) {
    const int i = ijk[0], j = ijk[1], k = s.ndim == 3 ? ijk[2] : 0;
    if (i < 0 || i >= s.nx || j < 0 || j >= s.ny || k < 0 || k >= s.nz) return -1;
    return ((int64_t)i * s.ny + j) * s.nz + k;
}

static bool comp_ok(const Sim &s, int comp) {
    if (s.ndim == 2) return comp == FDTD_EZ || comp == FDTD_HX || comp == FDTD_HY;
    return comp >= 0 && comp < 6;
}


int fdtd_set_source(fdtd_sim *sim, int component, const int32_t *ijk, int kind, const double *params,
                    const float *table, int64_t n_table) {
    if (kind < 0 || !ijk) return fdtd_set_source_box(sim, component, ijk, ijk, kind, params, table, n_table);
    int32_t hi[3] = {ijk[0] + 1, ijk[1] + 1, 1};
    if (sim && sim->s.ndim == 3) hi[2] = ijk[2] + 1;
    return fdtd_set_source_box(sim, component, ijk, hi, kind, params, table, n_table);
}

int fdtd_set_source_box(fdtd_sim *sim, int component, const int32_t *lo, const int32_t *hi, int kind,
                        const double *params, const float *table, int64_t n_table) {
    GEM_TRY
    if (!sim) fail(FDTD_EINVAL, "sim is NULL");
    Sim &s = sim->s;
    if (kind < 0) {
        s.src_idx = -1;
        s.src_kind = -1;
        if (s.is_graph) graph_set_source_probes(s);
        return FDTD_OK;
    }
    if (!lo || !hi) fail(FDTD_EINVAL, "lo or hi is NULL");
    if (component < FDTD_EX || component > FDTD_EZ || (s.ndim == 2 && component != FDTD_EZ))
        fail(FDTD_EINVAL, "source component must be an E component present in the grid");
    const int n3[3] = {s.nx, s.ny, s.ndim == 3 ? s.nz : 1};
    int box[6] = {0, 1, 0, 1, 0, 1};
    for (int a = 0; a < s.ndim; ++a) {
        if (lo[a] < 0 || hi[a] > n3[a] || lo[a] >= hi[a]) fail(FDTD_EINVAL, "source box empty or outside the grid");
        box[2 * a] = lo[a];
        box[2 * a + 1] = hi[a];
    }
    const int64_t c = lin_cell(s, lo);
    // the PEC walls of an E component are low planes: the box avoids them if
    // its low corner does
    int cc[3] = {lo[0], lo[1], s.ndim == 3 ? lo[2] : 1};
    if (on_wall(s, component, cc)) fail(FDTD_EINVAL, "source box touches a PEC wall of that component");
    if (kind == FDTD_SRC_TABLE) {
        if (!table || n_table < 0) fail(FDTD_EINVAL, "table source needs table and n_table >= 0");
        for (int64_t n = 0; n < n_table; ++n)
            if (!std::isfinite(table[n])) fail(FDTD_EINVAL, "non-finite source table value");
    } else if (kind == FDTD_SRC_GAUSSIAN || kind == FDTD_SRC_RICKER || kind == FDTD_SRC_SINE ||
               kind == FDTD_SRC_MODGAUSS) {
        if (!params) fail(FDTD_EINVAL, "params is NULL");
        for (int q = 0; q < src_nparams(kind); ++q)
            if (!std::isfinite(params[q])) fail(FDTD_EINVAL, "non-finite source parameter");
        if ((kind == FDTD_SRC_GAUSSIAN || kind == FDTD_SRC_MODGAUSS) && !(params[2] > 0))
            fail(FDTD_EINVAL, "Gaussian tau must be > 0");
        if (kind == FDTD_SRC_RICKER && !(params[2] > 0)) fail(FDTD_EINVAL, "Ricker frequency must be > 0");
        if (kind == FDTD_SRC_SINE && (!(params[1] > 0) || !(params[2] >= 0)))
            fail(FDTD_EINVAL, "sine needs f > 0 and t_ramp >= 0");
        if (kind == FDTD_SRC_MODGAUSS && !(params[3] >= 0)) fail(FDTD_EINVAL, "modulation frequency must be >= 0");
    } else {
        fail(FDTD_EINVAL, "unknown source kind");
    }
    s.al.put(s.src_dev);
    s.src_dev = nullptr;
    s.src_cap = s.src_len = 0;
    s.src_comp = component;
    s.src_idx = c;
    for (int q = 0; q < 6; ++q) s.src_box[q] = box[q];
    s.src_kind = kind;
    if (kind == FDTD_SRC_TABLE) {
        s.src_table.assign(table, table + n_table);
        s.src_dev = dev_upload(s.al, s.src_table.data(), std::max<size_t>(1, (size_t)n_table), s.st);
        s.src_cap = std::max<int64_t>(1, n_table);
        s.src_len = n_table;
        hip_check(hipStreamSynchronize(s.st), "sync");
    } else {
        for (int q = 0; q < 4; ++q) s.src_par[q] = q < src_nparams(kind) ? params[q] : 0.0;
        s.ensure_source(std::max<int64_t>(s.n_done + 1, 1));
        hip_check(hipStreamSynchronize(s.st), "sync");
    }
    if (s.is_graph) graph_set_source_probes(s);
    return FDTD_OK;
    GEM_CATCH
}

int fdtd_set_probes(fdtd_sim *sim, int component, const int32_t *ijk, int32_t n) {
    GEM_TRY
    if (!sim) fail(FDTD_EINVAL, "sim is NULL");
    Sim &s = sim->s;
    if (n < 0 || n > 4096) fail(FDTD_EINVAL, "probe count must be in [0, 4096]");
    if (n > 0 && !ijk) fail(FDTD_EINVAL, "ijk is NULL");
    if (!comp_ok(s, component)) fail(FDTD_EINVAL, "probe component not present in this grid");
    if (s.is_graph && component != FDTD_EZ) fail(FDTD_EINVAL, "graph form probes Ez only");
    std::vector<int64_t> cells((size_t)n);
    for (int q = 0; q < n; ++q) {
        cells[(size_t)q] = lin_cell(s, ijk + (size_t)q * s.ndim);
        if (cells[(size_t)q] < 0) fail(FDTD_EINVAL, "probe cell outside the grid");
    }
    hip_check(hipStreamSynchronize(s.st), "sync");
    s.probe_cells = cells;
    s.probe_comp = component;
    s.al.put(s.probe_dev);
    s.al.put(s.probe_dev64);
    s.al.put(s.rec_dev);
    s.probe_dev = nullptr;
    s.probe_dev64 = nullptr;
    s.rec_dev = nullptr;
    s.rec_cap = 0;
    s.n_rec = 0;
    if (n > 0) {
        std::vector<int> c32((size_t)n);
        for (int q = 0; q < n; ++q) c32[(size_t)q] = (int)cells[(size_t)q];
        s.probe_dev = dev_upload(s.al, c32.data(), (size_t)n, s.st);
        s.probe_dev64 = dev_upload(s.al, cells.data(), (size_t)n, s.st);
    }
    s.pt_ntiles = -1;
    s.build_probe_tiles();
    if (s.is_graph) graph_set_source_probes(s);
    hip_check(hipStreamSynchronize(s.st), "sync");
    return FDTD_OK;
    GEM_CATCH
}

int fdtd_step(fdtd_sim *sim, int64_t n) {
    GEM_TRY
    if (!sim) fail(FDTD_EINVAL, "sim is NULL");
    if (n < 0) fail(FDTD_EINVAL, "n must be >= 0");
    Sim &s = sim->s;
    s.ensure_source(s.n_done + n);
    s.ensure_rec(s.n_rec + n);
    s.build_probe_tiles();
    s.last_launches = 0;
    hip_check(hipEventRecord(s.ev0, s.st), "event");
    s.advance(n);
    hip_check(hipEventRecord(s.ev1, s.st), "event");
    s.timed = true;
    return FDTD_OK;
    GEM_CATCH
}

int fdtd_last_step_time(fdtd_sim *sim, float *ms, int64_t *launches) {
    GEM_TRY
    if (!sim || !ms) fail(FDTD_EINVAL, "NULL argument");
    Sim &s = sim->s;
    if (!s.timed) fail(FDTD_ESTATE, "no fdtd_step call yet");
    hip_check(hipEventSynchronize(s.ev1), "event sync");
    hip_check(hipEventElapsedTime(ms, s.ev0, s.ev1), "elapsed");
    if (launches) *launches = s.last_launches;
    return FDTD_OK;
    GEM_CATCH
}

int fdtd_step_profile(fdtd_sim *sim, int32_t steps, fdtd_launch_stat *out, int32_t max, int32_t *n) {
    GEM_TRY
    if (!sim || !n) fail(FDTD_EINVAL, "NULL argument");
    if (steps < 1 || steps > 100000) fail(FDTD_EINVAL, "steps must be in [1, 100000]");
    if (max < 0 || (max > 0 && !out)) fail(FDTD_EINVAL, "bad output array");
    Sim &s = sim->s;
    if (s.dft.comp >= 0) fail(FDTD_ESTATE, "remove the frequency-domain monitor before profiling");
    s.ensure_source(s.n_done + steps);
    s.ensure_rec(s.n_rec + steps);
    s.build_probe_tiles();
    const bool fused3 = s.ndim == 3 && !s.is_graph && s.kcfg.variant >= 2;
    const bool two = fused3 && s.kcfg.variant == 3 && steps >= 2;
    const bool tb2 = s.ndim == 2 && !s.is_graph && s.kcfg.variant == 3 && steps >= s.kcfg.tile[2];
    const bool res = s.ndim == 2 && !s.is_graph && s.kcfg.variant == 4 && s.res2d_ok();
    // one timed unit: a step, a pair of steps for the 3D two-step pass, the
    // TB steps of the 2D multi-step pass, or all steps (one workgroup)
    const int32_t per = two ? 2 : (tb2 ? s.kcfg.tile[2] : (res ? steps : 1));
    const int32_t units = steps / per;
    const size_t nl = two ? s.pair_launches() : (fused3 ? s.plan3.l.size() : 1);
    // all events of all units are recorded first; one synchronisation at the end
    std::vector<hipEvent_t> ev((nl + 1) * (size_t)units, nullptr);
    struct Guard {
        std::vector<hipEvent_t> &e;
        Sim &s;
        ~Guard() {
            s.lev = nullptr;
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } guard{ev, s};
    for (auto &e : ev) hip_check(hipEventCreate(&e), "event");
    const int64_t inc = s.probe_cells.empty() ? 0 : 1;
    int64_t launches = 0;
    for (int32_t q = 0; q < units; ++q) {
        hipEvent_t *e = ev.data() + (nl + 1) * (size_t)q;
        s.last_launches = 0;
        if (two) {
            s.launch_pair(s.n_done, e);
        } else if (tb2) {
            hip_check(hipEventRecord(e[0], s.st), "event");
            s.launch_tb2d(s.n_done);
            hip_check(hipEventRecord(e[1], s.st), "event");
        } else if (res) {
            hip_check(hipEventRecord(e[0], s.st), "event");
            hip_check(launch_2d_resident(s.prob2d(s.cur, 1 - s.cur), s.mat(), s.n_done, per, s.st), "2d resident steps");
            s.cur = 1 - s.cur;
            s.last_launches += (per + 65535) / 65536;
            hip_check(hipEventRecord(e[1], s.st), "event");
        } else {
            if (fused3) s.lev = e;
            else hip_check(hipEventRecord(e[0], s.st), "event");
            s.launch_step(s.n_done);
            s.lev = nullptr;
            if (!fused3) hip_check(hipEventRecord(e[1], s.st), "event");
        }
        s.n_done += per;
        s.n_rec += per * inc;
        launches = s.last_launches;
    }
    for (int32_t q = units * per; q < steps; ++q) s.advance(1);
    hip_check(hipEventSynchronize(ev.back()), "event sync");
    std::vector<double> acc(nl, 0.0);
    for (int32_t q = 0; q < units; ++q)
        for (size_t l = 0; l < nl; ++l) {
            float ms = 0;
            const size_t b = (nl + 1) * (size_t)q + l;
            hip_check(hipEventElapsedTime(&ms, ev[b], ev[b + 1]), "elapsed");
            acc[l] += ms;
        }
    *n = (int32_t)nl;
    auto slab = [&](fdtd_launch_stat &o, const Wave3DLaunch &w) {
        o.cells = w.cells;
        o.psi = w.psi;
        o.cpml = w.pxy ? 2 : (w.pz ? 1 : 0);
        o.launches = 1;
        o.steps = 1;
    };
    for (size_t l = 0; l < nl && (int32_t)l < max; ++l) {
        fdtd_launch_stat &o = out[l];
        o.ms = (float)(acc[l] / units);
        const size_t n1 = s.plan2.pass1.l.size();
        const bool zc = s.ax[2].lo + s.ax[2].hi > 0;
        if (two && s.plan2.slab_tb) {
            const bool o1 = l == 0;
            o.cells = o1 ? s.plan2.tbo_cells : s.plan2.tb_cells;
            o.psi = o1 ? s.plan2.tbo_psi : s.plan2.tb_psi;
            o.cpml = o1 ? 2 : (zc ? 1 : 0);
            o.launches = (o1 ? s.plan2.tbo.empty() : s.plan2.tb.empty()) ? 0 : 1;
            o.steps = 2;
        } else if (two) {
            if (l < n1) {
                slab(o, s.plan2.pass1.l[l]);
            } else if (l == n1) {
                o.cells = s.plan2.tb_cells;
                o.psi = s.plan2.tb_psi;
                o.cpml = zc ? 1 : 0;
                o.launches = s.plan2.tb.empty() ? 0 : 1;
                o.steps = 2;
            } else {
                slab(o, s.plan2.pass2.l[l - n1 - 1]);
            }
        } else if (fused3) {
            slab(o, s.plan3.l[l]);
        } else {
            o.cells = s.ncell;
            o.psi = 0;
            for (int a = 0; a < NPSI3; ++a) o.psi += s.psi_len[a];
            o.cpml = -1;
            o.launches = (int32_t)launches;
            o.steps = per;
        }
    }
    return FDTD_OK;
    GEM_CATCH
}

int fdtd_probe(fdtd_sim *sim, float *out, int64_t cap, int64_t *n_recorded) {
    GEM_TRY
    if (!sim) fail(FDTD_EINVAL, "sim is NULL");
    Sim &s = sim->s;
    if (n_recorded) *n_recorded = s.n_rec;
    if (!out || s.probe_cells.empty()) return FDTD_OK;
    if (cap < 0) fail(FDTD_EINVAL, "cap must be >= 0");
    s.records_to_host(out, cap, std::min(cap, s.n_rec));
    return FDTD_OK;
    GEM_CATCH
}


int fdtd_set_dft(fdtd_sim *sim, int component, const int32_t *lo, const int32_t *hi, int32_t nf,
                 const double *freqs) {
    GEM_TRY
    if (!sim) fail(FDTD_EINVAL, "sim is NULL");
    Sim &s = sim->s;
    if (nf < 0 || nf > kDftMaxFreq) fail(FDTD_EINVAL, "nf must be in [0, 16]");
    if (nf > 0) {
        if (!lo || !hi || !freqs) fail(FDTD_EINVAL, "NULL argument");
        if (!comp_ok(s, component)) fail(FDTD_EINVAL, "component not present in this grid");
        if (s.is_graph && s.split && component == FDTD_EZ)
            fail(FDTD_EINVAL, "the split-field graph holds Ez in two nodes: monitor Hx or Hy");
        const int n3[3] = {s.nx, s.ny, s.ndim == 3 ? s.nz : 1};
        for (int a = 0; a < s.ndim; ++a)
            if (lo[a] < 0 || hi[a] > n3[a] || lo[a] >= hi[a]) fail(FDTD_EINVAL, "monitor box empty or outside the grid");
        for (int q = 0; q < nf; ++q)
            if (!std::isfinite(freqs[q]) || freqs[q] < 0) fail(FDTD_EINVAL, "frequencies must be finite and >= 0");
    }
    hip_check(hipStreamSynchronize(s.st), "sync");
    s.al.put(s.dft.idx);
    s.al.put(s.dft.acc);
    s.al.put(s.dft.ring);
    s.dft = Sim::Dft{};
    if (nf == 0) return FDTD_OK;
    Sim::Dft &d = s.dft;
    d.comp = component;
    d.nf = nf;
    for (int q = 0; q < nf; ++q) d.f[q] = freqs[q];
    const int b[6] = {lo[0], hi[0], lo[1], hi[1], s.ndim == 3 ? lo[2] : 0, s.ndim == 3 ? hi[2] : 1};
    for (int q = 0; q < 6; ++q) d.box[q] = b[q];
    d.npts = (int64_t)(b[1] - b[0]) * (b[3] - b[2]) * (b[5] - b[4]);
    if (s.is_graph) {  // the graph's node order is not the box's: an index list
        std::vector<int64_t> idx;
        for (int i = b[0]; i < b[1]; ++i)
            for (int j = b[2]; j < b[3]; ++j) idx.push_back(graph_node(s, component, i, j));
        d.idx = dev_upload(s.al, idx.data(), idx.size(), s.st);
    }
    d.acc = (double *)s.al.get((size_t)(2 * nf * d.npts) * 8);  // zero-filled
    d.ring = (float *)s.al.get((size_t)(kDftBatch * d.npts) * 4);
    hip_check(hipStreamSynchronize(s.st), "sync");
    return FDTD_OK;
    GEM_CATCH
}

int fdtd_get_dft(fdtd_sim *sim, double *re, double *im, int64_t *nsteps) {
    GEM_TRY
    if (!sim) fail(FDTD_EINVAL, "sim is NULL");
    Sim &s = sim->s;
    const Sim::Dft &d = s.dft;
    if (d.comp < 0) fail(FDTD_ESTATE, "no frequency-domain monitor set");
    if (nsteps) *nsteps = d.nacc;
    if (!re && !im) return FDTD_OK;
    if (!re || !im) fail(FDTD_EINVAL, "re and im must both be given");
    s.dft_flush();
    std::vector<double> h((size_t)(2 * d.nf * d.npts));
    hip_check(hipMemcpyAsync(h.data(), d.acc, h.size() * 8, hipMemcpyDeviceToHost, s.st), "dft copy");
    hip_check(hipStreamSynchronize(s.st), "sync");
    for (int q = 0; q < d.nf; ++q) {
        std::memcpy(re + (size_t)q * d.npts, h.data() + (size_t)(2 * q) * d.npts, (size_t)d.npts * 8);
        std::memcpy(im + (size_t)q * d.npts, h.data() + (size_t)(2 * q + 1) * d.npts, (size_t)d.npts * 8);
    }
    return FDTD_OK;
    GEM_CATCH
}

int fdtd_dft_sar(fdtd_sim *sim, const float *rho, const double *norm, float *sar) {
    GEM_TRY
    if (!sim || !rho || !sar) fail(FDTD_EINVAL, "NULL argument");
    Sim &s = sim->s;
    const Sim::Dft &d = s.dft;
    if (d.comp < 0) fail(FDTD_ESTATE, "no frequency-domain monitor set");
    if (d.comp != FDTD_EX && d.comp != FDTD_EY && d.comp != FDTD_EZ)
        fail(FDTD_EINVAL, "the absorption rate needs a monitor on an E component");
    SarScale sc{};
    for (int q = 0; q < d.nf; ++q) {
        const double n = norm ? norm[q] : 1.0;
        if (!std::isfinite(n) || n <= 0) fail(FDTD_EINVAL, "norm must be finite and > 0");
        sc.inv2n2[q] = 0.5 / (n * n);
    }
    std::vector<float> sg((size_t)d.npts, 0.f);
    int64_t c = 0;
    for (int i = d.box[0]; i < d.box[1]; ++i)
        for (int j = d.box[2]; j < d.box[3]; ++j)
            for (int k = d.box[4]; k < d.box[5]; ++k, ++c) {
                if (!std::isfinite(rho[c]) || rho[c] <= 0) fail(FDTD_EINVAL, "rho must be finite and > 0");
                if (!s.sigma.empty()) sg[(size_t)c] = s.sigma[(size_t)(((int64_t)i * s.ny + j) * s.nz + k)];
            }
    s.dft_flush();
    const size_t nb = (size_t)d.npts * 4;
    float *dsg = (float *)s.al.get(nb), *drho = (float *)s.al.get(nb), *dout = (float *)s.al.get(nb * d.nf);
    struct Put {
        Sim &s;
        void *a, *b, *c;
        ~Put() {
            (void)hipStreamSynchronize(s.st);
            s.al.put(a);
            s.al.put(b);
            s.al.put(c);
        }
    } put{s, dsg, drho, dout};
    hip_check(hipMemcpyAsync(dsg, sg.data(), nb, hipMemcpyHostToDevice, s.st), "upload");
    hip_check(hipMemcpyAsync(drho, rho, nb, hipMemcpyHostToDevice, s.st), "upload");
    hip_check(launch_sar(d.acc, d.npts, d.nf, dsg, drho, sc, dout, s.st), "sar");
    hip_check(hipMemcpyAsync(sar, dout, nb * d.nf, hipMemcpyDeviceToHost, s.st), "copy");
    hip_check(hipStreamSynchronize(s.st), "sync");
    return FDTD_OK;
    GEM_CATCH
}

int fdtd_get_field(fdtd_sim *sim, int component, void *dst, int dst_on_device) {
    GEM_TRY
    if (!sim || !dst) fail(FDTD_EINVAL, "NULL argument");
    Sim &s = sim->s;
    if (!comp_ok(s, component)) fail(FDTD_EINVAL, "component not present in this grid");
    const size_t bytes = (size_t)s.ncell * 4;
    if (s.is_graph) {
        std::vector<float> h((size_t)s.ncell);
        graph_get_field(s, component, h.data());
        if (dst_on_device) {
            hip_check(hipMemcpyAsync(dst, h.data(), bytes, hipMemcpyHostToDevice, s.st), "copy");
            hip_check(hipStreamSynchronize(s.st), "sync");
        } else {
            std::memcpy(dst, h.data(), bytes);
        }
        return FDTD_OK;
    }
    hip_check(hipMemcpyAsync(dst, s.f[s.cur][component], bytes,
                             dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s.st),
              "copy");
    if (!dst_on_device) hip_check(hipStreamSynchronize(s.st), "sync");
    return FDTD_OK;
    GEM_CATCH
}

int fdtd_set_field(fdtd_sim *sim, int component, const void *src, int src_on_device) {
    GEM_TRY
    if (!sim || !src) fail(FDTD_EINVAL, "NULL argument");
    Sim &s = sim->s;
    if (!comp_ok(s, component)) fail(FDTD_EINVAL, "component not present in this grid");
    const size_t bytes = (size_t)s.ncell * 4;
    if (s.is_graph) {
        std::vector<float> h((size_t)s.ncell);
        if (src_on_device) {
            hip_check(hipMemcpyAsync(h.data(), src, bytes, hipMemcpyDeviceToHost, s.st), "copy");
            hip_check(hipStreamSynchronize(s.st), "sync");
        } else {
            std::memcpy(h.data(), src, bytes);
        }
        graph_set_field(s, component, h.data());
        return FDTD_OK;
    }
    hip_check(hipMemcpyAsync(s.f[s.cur][component], src, bytes,
                             src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s.st),
              "copy");
    // split-field PML: a set Ez is all Ezx
    if (s.split && component == FDTD_EZ) hip_check(hipMemsetAsync(s.ezy, 0, bytes, s.st), "memset");
    hip_check(hipStreamSynchronize(s.st), "sync");
    return FDTD_OK;
    GEM_CATCH
}

// ---------------------------------------------------------------------------
// Whole-state save / restore: a 64-byte header (magic, grid, layer widths,
// form, step count), then every field and CPML array of the current state
// set in a fixed order (implicit form), or the node vector (graph form).
// ---------------------------------------------------------------------------
}  // extern "C"

// state file helpers (C++ linkage)
namespace {
struct StateHeader {
    char magic[8];
    int32_t ndim, nx, ny, nz;
    int32_t npml[6];
    int32_t split, graph;
    int64_t n_done;
};
static_assert(sizeof(StateHeader) <= 64, "state header");
constexpr char kStateMagic[8] = {'G', 'E', 'M', 'S', 'T', 'A', 'T', '1'};

StateHeader state_header(const Sim &s) {
    StateHeader h{};
    std::memcpy(h.magic, kStateMagic, 8);
    h.ndim = s.ndim;
    h.nx = s.nx;
    h.ny = s.ny;
    h.nz = s.nz;
    for (int q = 0; q < 6; ++q) h.npml[q] = s.cpml.npml[q];
    h.split = s.split ? 1 : 0;
    h.graph = s.is_graph ? 1 : 0;
    h.n_done = s.n_done;
    return h;
}

// (device pointer, bytes) of every array of the state, in file order
std::vector<std::pair<float *, size_t>> state_arrays(Sim &s) {
    std::vector<std::pair<float *, size_t>> v;
    if (s.is_graph) {
        v.emplace_back(s.g.x, (size_t)s.g.nnodes * 4);
        return v;
    }
    for (int c = 0; c < 6; ++c)
        if (s.f[s.cur][c]) v.emplace_back(s.f[s.cur][c], (size_t)s.ncell * 4);
    for (int a = 0; a < NPSI3; ++a)
        if (s.psi[s.cur][a]) v.emplace_back(s.psi[s.cur][a], (size_t)s.psi_len[a] * 4);
    if (s.ezy) v.emplace_back(s.ezy, (size_t)s.ncell * 4);
    return v;
}

int64_t state_size(Sim &s) {
    int64_t n = 64;
    for (auto &a : state_arrays(s)) n += (int64_t)a.second;
    return n;
}
}  // namespace

extern "C" {

int fdtd_state_bytes(fdtd_sim *sim, int64_t *bytes) {
    GEM_TRY
    if (!sim || !bytes) fail(FDTD_EINVAL, "NULL argument");
    *bytes = state_size(sim->s);
    return FDTD_OK;
    GEM_CATCH
}

int fdtd_save_state(fdtd_sim *sim, void *dst, int dst_on_device) {
    GEM_TRY
    if (!sim || !dst) fail(FDTD_EINVAL, "NULL argument");
    Sim &s = sim->s;
    if (s.dft.comp >= 0) s.dft_flush();
    const StateHeader h = state_header(s);
    char hb[64] = {};
    std::memcpy(hb, &h, sizeof h);
    const hipMemcpyKind up = dst_on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost;
    const hipMemcpyKind down = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    hip_check(hipMemcpyAsync(dst, hb, 64, up, s.st), "state copy");
    size_t off = 64;
    for (auto &a : state_arrays(s)) {
        hip_check(hipMemcpyAsync((char *)dst + off, a.first, a.second, down, s.st), "state copy");
        off += a.second;
    }
    // the header leaves from host memory: wait for it in either case
    hip_check(hipStreamSynchronize(s.st), "sync");
    return FDTD_OK;
    GEM_CATCH
}

int fdtd_load_state(fdtd_sim *sim, const void *src, int src_on_device) {
    GEM_TRY
    if (!sim || !src) fail(FDTD_EINVAL, "NULL argument");
    Sim &s = sim->s;
    StateHeader h{};
    if (src_on_device) {
        hip_check(hipMemcpyAsync(&h, src, sizeof h, hipMemcpyDeviceToHost, s.st), "state copy");
        hip_check(hipStreamSynchronize(s.st), "sync");
    } else {
        std::memcpy(&h, src, sizeof h);
    }
    const StateHeader mine = state_header(s);
    if (std::memcmp(h.magic, kStateMagic, 8) != 0) fail(FDTD_EINVAL, "not a saved state");
    bool same = h.ndim == mine.ndim && h.nx == mine.nx && h.ny == mine.ny && h.nz == mine.nz &&
                h.split == mine.split && h.graph == mine.graph;
    for (int q = 0; q < 6; ++q) same = same && h.npml[q] == mine.npml[q];
    if (!same) fail(FDTD_EINVAL, "the saved state belongs to a different grid, absorbing layer or form");
    if (h.n_done < 0) fail(FDTD_EINVAL, "invalid step count in the saved state");
    const hipMemcpyKind kind = src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    size_t off = 64;
    for (auto &a : state_arrays(s)) {
        hip_check(hipMemcpyAsync(a.first, (const char *)src + off, a.second, kind, s.st), "state copy");
        off += a.second;
    }
    s.n_done = h.n_done;
    s.n_rec = 0;
    hip_check(hipStreamSynchronize(s.st), "sync");
    return FDTD_OK;
    GEM_CATCH
}

int fdtd_reset(fdtd_sim *sim) {
    GEM_TRY
    if (!sim) fail(FDTD_EINVAL, "sim is NULL");
    sim->s.zero_state();
    hip_check(hipStreamSynchronize(sim->s.st), "sync");
    return FDTD_OK;
    GEM_CATCH
}

int fdtd_steps_done(const fdtd_sim *sim, int64_t *n) {
    if (!sim || !n) {
        set_error("NULL argument");
        return FDTD_EINVAL;
    }
    *n = sim->s.n_done;
    return FDTD_OK;
}

int fdtd_check_finite(fdtd_sim *sim) {
    GEM_TRY
    if (!sim) fail(FDTD_EINVAL, "sim is NULL");
    Sim &s = sim->s;
    int *flag = (int *)s.al.get(4);
    if (s.is_graph) {
        hip_check(launch_nonfinite(s.g.x, s.g.nnodes, flag, s.st), "finite check");
    } else {
        for (int c = 0; c < 6; ++c)
            if (s.f[s.cur][c]) hip_check(launch_nonfinite(s.f[s.cur][c], s.ncell, flag, s.st), "finite check");
        for (int a = 0; a < NPSI3; ++a)
            if (s.psi[s.cur][a]) hip_check(launch_nonfinite(s.psi[s.cur][a], s.psi_len[a], flag, s.st), "finite check");
    }
    int h = 0;
    hip_check(hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, s.st), "copy");
    hip_check(hipStreamSynchronize(s.st), "sync");
    s.al.put(flag);
    if (h) {
        set_error("a field holds NaN or Inf");
        return FDTD_ENONFINITE;
    }
    return FDTD_OK;
    GEM_CATCH
}


int fdtd_set_material(fdtd_sim *sim, const int32_t *lo, const int32_t *hi, const float *eps_r,
                      const float *sigma) {
    GEM_TRY
    if (!sim || !lo || !hi || !eps_r) fail(FDTD_EINVAL, "NULL argument");
    Sim &s = sim->s;
    const int nd = s.ndim;
    const int n[3] = {s.nx, s.ny, s.nz};
    int l[3] = {0, 0, 0}, h[3] = {1, 1, 1};
    for (int a = 0; a < nd; ++a) {
        l[a] = lo[a];
        h[a] = hi[a];
        if (l[a] < 0 || h[a] > n[a] || l[a] >= h[a]) fail(FDTD_EINVAL, "invalid box");
    }
    const int64_t bn = (int64_t)(h[0] - l[0]) * (h[1] - l[1]) * (h[2] - l[2]);
    check_map(eps_r, bn, 1.0, "eps_r");
    if (sigma) check_map(sigma, bn, 0.0, "sigma");
    if (s.split) {  // the split-field PML's layer stays vacuum
        int64_t q2 = 0;
        for (int i = l[0]; i < h[0]; ++i)
            for (int j = l[1]; j < h[1]; ++j, ++q2) {
                const bool layer = i < s.ax[0].lo || i >= s.nx - s.ax[0].hi || j < s.ax[1].lo || j >= s.ny - s.ax[1].hi;
                if (layer && (eps_r[q2] != 1.f || (sigma && sigma[q2] != 0.f)))
                    fail(FDTD_EINVAL, "the split-field PML needs vacuum in its layer cells");
            }
    }
    hip_check(hipStreamSynchronize(s.st), "sync");
    if (s.eps_r.empty()) s.eps_r.assign((size_t)s.ncell, 1.0f);
    if (sigma && s.sigma.empty()) s.sigma.assign((size_t)s.ncell, 0.0f);
    int64_t q = 0;
    for (int i = l[0]; i < h[0]; ++i)
        for (int j = l[1]; j < h[1]; ++j)
            for (int k = l[2]; k < h[2]; ++k, ++q) {
                const int64_t c = ((int64_t)i * s.ny + j) * s.nz + k;
                s.eps_r[(size_t)c] = eps_r[q];
                if (sigma) s.sigma[(size_t)c] = sigma[q];
            }
    if (sigma && !s.lossy)
        s.lossy = std::any_of(s.sigma.begin(), s.sigma.end(), [](float v) { return v > 0.f; });
    s.refold(0, s.ncell);
    if (s.is_graph) graph_refold(s);
    return FDTD_OK;
    GEM_CATCH
}

int fdtd_set_kernel(fdtd_sim *sim, const fdtd_kernel_config *cfg) {
    GEM_TRY
    if (!sim || !cfg) fail(FDTD_EINVAL, "NULL argument");
    Sim &s = sim->s;
    if (s.is_graph) fail(FDTD_EINVAL, "kernel selection applies to the implicit-graph stepper");
    fdtd_kernel_config k = *cfg;
    if (k.tb == 0) k.tb = 1;
    if (k.variant == 0) {
        default_variant_tiles(s, k);
    } else if (s.ndim == 2 && k.variant == 3) {
        if (k.tile[0] == 0) k.tile[0] = 1;
        if (k.tile[1] == 0) k.tile[1] = kTB2DefaultTX;
        if (k.tile[2] == 0) k.tile[2] = 4;
    } else if (s.ndim == 2 && k.variant == 2) {
        const Fused2DCfg c = default_single2d(s.nx, s.ny);
        if (k.tile[0] == 0) k.tile[0] = c.V;
        if (k.tile[1] == 0) k.tile[1] = c.TX;
    } else if (k.variant == 2 || k.variant == 3) {
        fdtd_kernel_config d;
        default_variant_tiles(s, d);
        if (k.tile[0] == 0) k.tile[0] = d.tile[0];
    }
    if (!config_ok(s, k)) fail(FDTD_EINVAL, "unsupported kernel configuration for this grid");
    hip_check(hipStreamSynchronize(s.st), "sync");
    // the current state must live in set 0 or 1 consistently: both variants read s.cur
    s.kcfg = k;
    s.kcfg_explicit = true;
    s.pt_ntiles = -1;
    s.build_probe_tiles();
    return FDTD_OK;
    GEM_CATCH
}

int fdtd_get_kernel(const fdtd_sim *sim, fdtd_kernel_config *cfg) {
    if (!sim || !cfg) {
        set_error("NULL argument");
        return FDTD_EINVAL;
    }
    *cfg = sim->s.kcfg;
    return FDTD_OK;
}

int fdtd_autotune(fdtd_sim *sim, int32_t trial_steps, fdtd_kernel_config *out) {
    GEM_TRY
    if (!sim) fail(FDTD_EINVAL, "sim is NULL");
    Sim &s = sim->s;
    if (s.is_graph) fail(FDTD_EINVAL, "autotune applies to the implicit-graph stepper");
    if (s.dft.comp >= 0) fail(FDTD_ESTATE, "remove the frequency-domain monitor before autotuning");
    if (trial_steps < 2) trial_steps = 2;
    trial_steps = (trial_steps + 3) / 4 * 4;  // whole passes of the multi-step kernels
    const std::string key = tune_key(s);
    const char *path = std::getenv("GEMFDTD_TUNE_CACHE");
    std::map<std::string, std::vector<int>> cache;
    if (path) cache = read_cache(path);
    auto it = cache.find(key);
    if (it != cache.end() && it->second.size() == 6) {
        fdtd_kernel_config k{};
        k.variant = it->second[0];
        for (int q = 0; q < 4; ++q) k.tile[q] = it->second[1 + q];
        k.tb = it->second[5];
        if (config_ok(s, k)) {
            s.kcfg = k;
            s.pt_ntiles = -1;
            s.build_probe_tiles();
            if (out) *out = k;
            return FDTD_OK;
        }
    }
    // candidates
    std::vector<fdtd_kernel_config> cand;
    if (s.ndim == 2) {
        {
            fdtd_kernel_config k{};
            k.variant = 4;
            k.tb = 1;
            if (config_ok(s, k)) cand.push_back(k);
        }
        for (int V : {1, 2, 4})
            for (int TX : {4, 8, 16, 32}) {
                fdtd_kernel_config k{};
                k.variant = 2;
                k.tile[0] = V;
                k.tile[1] = TX;
                k.tb = 1;
                if (config_ok(s, k)) cand.push_back(k);
            }
        for (int V : {1, 2, 4})
            for (int TB : {2, 4})
                for (int TX : {4, 8, 16, 32})
                    for (int TXo : {0, TX / 4}) {  // CPML tiles: whole chunks or quarters
                        if (TXo == TX / 4 && TX < 16) continue;
                        fdtd_kernel_config k{};
                        k.variant = 3;
                        k.tile[0] = V;
                        k.tile[1] = TX;
                        k.tile[2] = TB;
                        k.tile[3] = TXo;
                        k.tb = 1;
                        if (config_ok(s, k)) cand.push_back(k);
                    }
    } else {
        for (int TX : {8, 16, 32})
            for (int V : {1, 2, 4}) {
                fdtd_kernel_config k{};
                k.variant = 2;
                k.tile[0] = V;
                k.tile[2] = TX;
                k.tb = 1;
                if (config_ok(s, k)) cand.push_back(k);
            }
        for (int sp : {0, 1})
            for (int TX : {0, 16, 32, 64}) {
                fdtd_kernel_config k{};
                k.variant = 3;
                k.tile[0] = 4;
                k.tile[1] = sp;
                k.tile[2] = TX;
                k.tb = 1;
                if (config_ok(s, k)) cand.push_back(k);
            }
    }
    {
        fdtd_kernel_config k{};
        k.variant = 1;
        k.tb = 1;
        cand.push_back(k);
    }
    // snapshot the current state
    hip_check(hipStreamSynchronize(s.st), "sync");
    const int ncomp = s.ndim == 2 ? 3 : 6;
    std::vector<float *> bak;
    const int comps2[3] = {FDTD_EZ, FDTD_HX, FDTD_HY};
    auto comp_at = [&](int q) { return s.ndim == 2 ? comps2[q] : q; };
    for (int q = 0; q < ncomp; ++q) {
        float *b = (float *)s.al.get((size_t)s.ncell * 4);
        hip_check(hipMemcpyAsync(b, s.f[s.cur][comp_at(q)], (size_t)s.ncell * 4, hipMemcpyDeviceToDevice, s.st), "copy");
        bak.push_back(b);
    }
    std::vector<float *> bakp(NPSI3, nullptr);
    for (int a = 0; a < NPSI3; ++a)
        if (s.psi[s.cur][a]) {
            bakp[a] = (float *)s.al.get((size_t)s.psi_len[a] * 4);
            hip_check(hipMemcpyAsync(bakp[a], s.psi[s.cur][a], (size_t)s.psi_len[a] * 4, hipMemcpyDeviceToDevice, s.st), "copy");
        }
    const int64_t n_done0 = s.n_done, n_rec0 = s.n_rec;
    const int cur0 = s.cur;
    const fdtd_kernel_config k0 = s.kcfg;
    float best = 1e30f;
    fdtd_kernel_config bestk = k0;
    s.ensure_source(s.n_done + trial_steps + 4);
    s.ensure_rec(s.n_rec + trial_steps + 4);
    for (auto &k : cand) {
        s.kcfg = k;
        s.pt_ntiles = -1;
        s.build_probe_tiles();
        s.n_done = n_done0;
        s.n_rec = n_rec0;
        s.advance(4);  // warm-up
        hip_check(hipEventRecord(s.ev0, s.st), "event");
        s.advance(trial_steps);
        hip_check(hipEventRecord(s.ev1, s.st), "event");
        hip_check(hipEventSynchronize(s.ev1), "sync");
        float ms = 0;
        hip_check(hipEventElapsedTime(&ms, s.ev0, s.ev1), "elapsed");
        if (ms < best) {
            best = ms;
            bestk = k;
        }
        s.cur = cur0;
    }
    // restore
    for (int q = 0; q < ncomp; ++q)
        hip_check(hipMemcpyAsync(s.f[cur0][comp_at(q)], bak[q], (size_t)s.ncell * 4, hipMemcpyDeviceToDevice, s.st), "copy");
    for (int a = 0; a < NPSI3; ++a)
        if (bakp[a])
            hip_check(hipMemcpyAsync(s.psi[cur0][a], bakp[a], (size_t)s.psi_len[a] * 4, hipMemcpyDeviceToDevice, s.st), "copy");
    hip_check(hipStreamSynchronize(s.st), "sync");
    for (float *b : bak) s.al.put(b);
    for (float *b : bakp) s.al.put(b);
    s.n_done = n_done0;
    s.n_rec = n_rec0;
    s.cur = cur0;
    s.kcfg = bestk;
    s.pt_ntiles = -1;
    s.build_probe_tiles();
    if (path) {
        cache[key] = {bestk.variant, bestk.tile[0], bestk.tile[1], bestk.tile[2], bestk.tile[3], bestk.tb};
        write_cache(path, cache);
    }
    if (out) *out = bestk;
    return FDTD_OK;
    GEM_CATCH
}

}  // extern "C"

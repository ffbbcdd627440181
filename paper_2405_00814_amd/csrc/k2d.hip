// 2D TMz kernels: the two message-passing layers of one leapfrog step.
//
// H layer (Eq. 8-9 in TMz form, Prop. 2 first step): every cell gathers the
// Ez values at (i,j), (i,j+1), (i+1,j) into its Hx and Hy nodes.
// E layer (Eq. 7, Prop. 2 second step): every cell with i >= 1 and j >= 1
// gathers Hx(i,j), Hx(i,j-1), Hy(i,j), Hy(i-1,j) into its Ez node, with
// self weight Ca = A-/A+ and curl weight Cb = dt/(A+ eps).  CPML auxiliary
// values ride along in the boundary slabs.  The soft source is added after
// the E layer; probes sample Ez afterwards.
#include <algorithm>

#include "common.hpp"
#include "devutil.hpp"

namespace gem {

// ---------------------------------------------------------------------------
// Two-pass reference kernels (one thread per cell, in place on s0)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k2d_ref_h(Prob2D p) {
    const int64_t n = (int64_t)p.nx * p.ny;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int ny = p.ny;
    const int i = (int)(c / ny), j = (int)(c - (int64_t)i * ny);
    const float e0 = p.s0.ez[c];
    const float ey1 = (j + 1 < ny) ? p.s0.ez[c + 1] : 0.f;
    const float ex1 = (i + 1 < p.nx) ? p.s0.ez[c + ny] : 0.f;
    const float db = p.db ? p.db[c] : p.db0;
    if (p.ezy) {  // split-field PML: sigma* along the difference's axis
        p.s0.hx[c] = p.y.bH[j] * p.s0.hx[c] - db * p.y.cH[j] * p.y.kH[j] * (ey1 - e0);
        p.s0.hy[c] = p.x.bH[i] * p.s0.hy[c] + db * p.x.cH[i] * p.x.kH[i] * (ex1 - e0);
        return;
    }
    const float dEy = ey1 - e0;
    float ty = dEy * p.y.kH[j];
    const int jj = slab_index(p.y, j);
    if (jj >= 0) {
        const int sy = p.y.lo + p.y.hi;
        float *q = p.s0.psi_hx + (int64_t)i * sy + jj;
        const float ps = p.y.bH[j] * (*q) + p.y.cH[j] * dEy;
        *q = ps;
        ty += ps;
    }
    p.s0.hx[c] -= db * ty;
    const float dEx = ex1 - e0;
    float tx = dEx * p.x.kH[i];
    const int ii = slab_index(p.x, i);
    if (ii >= 0) {
        float *q = p.s0.psi_hy + (int64_t)ii * ny + j;
        const float ps = p.x.bH[i] * (*q) + p.x.cH[i] * dEx;
        *q = ps;
        tx += ps;
    }
    p.s0.hy[c] += db * tx;
}

__global__ __launch_bounds__(256) void k2d_ref_e(Prob2D p, int64_t step) {
    const int64_t n = (int64_t)p.nx * p.ny;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int ny = p.ny;
    const int i = (int)(c / ny), j = (int)(c - (int64_t)i * ny);
    float e = p.s0.ez[c];
    if (i >= 1 && j >= 1) {
        const float dHy = p.s0.hy[c] - p.s0.hy[c - ny];
        const float dHx = p.s0.hx[c] - p.s0.hx[c - 1];
        if (p.ezy && (slab_index(p.x, i) >= 0 || slab_index(p.y, j) >= 0)) {
            // split-field PML cell (vacuum): Ezx = Ez - Ezy and Ezy decay
            // with sigma_x and sigma_y
            const float zy = p.ezy[c];
            const float nx_ = p.x.bE[i] * (e - zy) + p.cb[c] * p.x.cE[i] * p.x.kE[i] * dHy;
            const float ny_ = p.y.bE[j] * zy - p.cb[c] * p.y.cE[j] * p.y.kE[j] * dHx;
            p.ezy[c] = ny_;
            e = nx_ + ny_;
            if (p.src_idx >= 0 && in_src(p.src_box, i, j, 0) && step < p.src_len) e += p.src_vals[step];
            p.s0.ez[c] = e;
            return;
        }
        float tx = dHy * p.x.kE[i];
        float ty = dHx * p.y.kE[j];
        const int ii = slab_index(p.x, i);
        if (ii >= 0) {
            float *q = p.s0.psi_ezx + (int64_t)ii * ny + j;
            const float ps = p.x.bE[i] * (*q) + p.x.cE[i] * dHy;
            *q = ps;
            tx += ps;
        }
        const int jj = slab_index(p.y, j);
        if (jj >= 0) {
            const int sy = p.y.lo + p.y.hi;
            float *q = p.s0.psi_ezy + (int64_t)i * sy + jj;
            const float ps = p.y.bE[j] * (*q) + p.y.cE[j] * dHx;
            *q = ps;
            ty += ps;
        }
        const float ca = p.ca ? p.ca[c] : 1.f;
        e = ca * e + p.cb[c] * (tx - ty);
    }
    if (p.src_idx >= 0 && in_src(p.src_box, i, j, 0) && step < p.src_len) e += p.src_vals[step];
    p.s0.ez[c] = e;
}

__global__ void k_probe_2d(Prob2D p, int64_t step) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < p.np) {
        const float *f = p.probe_comp == FDTD_HX ? p.s0.hx : (p.probe_comp == FDTD_HY ? p.s0.hy : p.s0.ez);
        p.rec[(int64_t)q * p.rec_stride + (step - p.rec_base)] = f[p.probe_idx[q]];
    }
}

hipError_t launch_2d_ref(const Prob2D &p, int64_t step, hipStream_t st) {
    const int64_t n = (int64_t)p.nx * p.ny;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k2d_ref_h, dim3(nb), dim3(256), 0, st, p);
    hipLaunchKernelGGL(k2d_ref_e, dim3(nb), dim3(256), 0, st, p, step);
    if (p.np > 0)
        hipLaunchKernelGGL(k_probe_2d, dim3((p.np + 63) / 64), dim3(64), 0, st, p, step);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused single-pass kernel.
//
// Each wavefront owns a strip of 64*V consecutive y cells (lane l holds
// columns y0 + l*V .. y0 + l*V + V - 1) and TX consecutive x rows, and
// marches along x with the previous row's H and the next row's Ez in
// registers.  y neighbours come from lane shuffles; the strip's edge columns
// are read directly (Ez at y0 + 64V for the H layer, and Hx at y0 - 1 is
// recomputed for the E layer).  The H row x0 - 1 is recomputed at the start.
// The state is double buffered: everything is read from s0 and written to
// s1, so neighbouring strips never see half-updated values.
// ---------------------------------------------------------------------------
// One wavefront tile: x rows [cx*TX, cx*TX + TX) of the strip sy.  Probe
// entries [pbeg, pend) of pt belong to this tile.
template <int V, bool PML, bool CAPTURE>
__device__ __forceinline__ void fused2d_tile(const Prob2D &p, int TX, int cx, int sy,
                                             const ProbeTiles &pt, int pbeg, int pend,
                                             int64_t step, int4 design, float *cap_ez,
                                             float *cap_br) {
    const int lane = threadIdx.x & 63;
    const int nx = p.nx, ny = p.ny;
    const int x0 = cx * TX, x1 = min(x0 + TX, nx);
    const int y0 = sy * 64 * V;
    const int jb = y0 + lane * V;
    const int jend = y0 + 64 * V;  // first column after the strip
    const bool valid = jb < ny;    // ny % V == 0: all V columns valid or none
    const int syw = p.y.lo + p.y.hi;
    const bool lossy = p.ca != nullptr;
    const bool mumap = p.db != nullptr;
    // the source box, read once (the batched tiles read p from memory): an
    // empty box without a source
    const bool hs = p.src_idx >= 0;
    const int si0 = hs ? p.src_box[0] : 0, si1 = hs ? p.src_box[1] : 0, sj0 = p.src_box[2], sj1 = p.src_box[3];

    float kHy[V], kEy[V], bHy[V], cHy[V], bEy[V], cEy[V];
    int jj[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int j = valid ? jb + v : 0;
        kHy[v] = p.y.kH[j];
        kEy[v] = p.y.kE[j];
        jj[v] = -1;
        bHy[v] = cHy[v] = bEy[v] = cEy[v] = 0.f;
        if (PML && valid) {
            jj[v] = slab_index(p.y, j);
            if (jj[v] >= 0) {
                bHy[v] = p.y.bH[j]; cHy[v] = p.y.cH[j];
                bEy[v] = p.y.bE[j]; cEy[v] = p.y.cE[j];
            }
        }
    }
    // profile of the column left of the strip (used by lane 0)
    const int jm = y0 - 1;
    float kHy_m = 0.f, bHy_m = 0.f, cHy_m = 0.f;
    int jj_m = -1;
    if (jm >= 0) {
        kHy_m = p.y.kH[jm];
        if (PML) {
            jj_m = slab_index(p.y, jm);
            if (jj_m >= 0) { bHy_m = p.y.bH[jm]; cHy_m = p.y.cH[jm]; }
        }
    }

    float ez_c[V], hy_p[V];
#pragma unroll
    for (int v = 0; v < V; ++v) { ez_c[v] = 0.f; hy_p[v] = 0.f; }
    if (valid) ldv<V>(ez_c, p.s0.ez + (int64_t)x0 * ny + jb);
    if (x0 > 0 && valid) {
        // H row x0 - 1 (Hy only; the E layer of row x0 needs Hy(x0-1, j))
        const int i = x0 - 1;
        const int64_t row = (int64_t)i * ny;
        float ez_m[V], hy_o[V], db[V];
        ldv<V>(ez_m, p.s0.ez + row + jb);
        ldv<V>(hy_o, p.s0.hy + row + jb);
        if (mumap) ldv<V>(db, p.db + row + jb);
        else {
#pragma unroll
            for (int v = 0; v < V; ++v) db[v] = p.db0;
        }
        const float kHx = p.x.kH[i];
        const int ii = PML ? slab_index(p.x, i) : -1;
        float ps_o[V];
        if (PML && ii >= 0) ldv<V>(ps_o, p.s0.psi_hy + (int64_t)ii * ny + jb);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const float dEx = ez_c[v] - ez_m[v];
            float tx = dEx * kHx;
            if (PML && ii >= 0) tx += p.x.bH[i] * ps_o[v] + p.x.cH[i] * dEx;
            hy_p[v] = hy_o[v] + db[v] * tx;
        }
    }

    const float sval = (p.src_idx >= 0 && step < p.src_len) ? p.src_vals[step] : 0.f;

    // The loads of a row are issued one iteration ahead (software pipelining):
    // stage holds Ez(ip+1), Hx(ip), Hy(ip) and the coefficients of row ip.
    float s_ezn[V], s_hx[V], s_hy[V], s_cb[V], s_ca[V], s_db[V];
    auto load_row = [&](int ip) {
        const int64_t rp = (int64_t)ip * ny;
#pragma unroll
        for (int v = 0; v < V; ++v) { s_ezn[v] = 0.f; s_hx[v] = s_hy[v] = s_cb[v] = 0.f; s_ca[v] = 1.f; s_db[v] = p.db0; }
        if (valid) {
            if (ip + 1 < nx) ldv<V>(s_ezn, p.s0.ez + rp + ny + jb);
            ldv<V>(s_hx, p.s0.hx + rp + jb);
            ldv<V>(s_hy, p.s0.hy + rp + jb);
            ldv<V>(s_cb, p.cb + rp + jb);
            if (lossy) ldv<V>(s_ca, p.ca + rp + jb);
            if (mumap) ldv<V>(s_db, p.db + rp + jb);
        }
    };
    load_row(x0);

    for (int i = x0; i < x1; ++i) {
        const int64_t row = (int64_t)i * ny;
        float ez_n[V], hx_o[V], hy_o[V], cb[V], ca[V], db[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            ez_n[v] = s_ezn[v]; hx_o[v] = s_hx[v]; hy_o[v] = s_hy[v];
            cb[v] = s_cb[v]; ca[v] = s_ca[v]; db[v] = s_db[v];
        }
        if (i + 1 < x1) load_row(i + 1);
        // Ez(i, j+1)
        float ez_r[V];
#pragma unroll
        for (int v = 0; v + 1 < V; ++v) ez_r[v] = ez_c[v + 1];
        float sh = lane_next(ez_c[0]);
        if (lane == 63) sh = (jend < ny) ? p.s0.ez[row + jend] : 0.f;
        ez_r[V - 1] = sh;

        const float kHx = p.x.kH[i], kEx = p.x.kE[i];
        const int ii = PML ? slab_index(p.x, i) : -1;
        // ---- H layer ----
        float hx_n[V], hy_n[V];
        float psx_o[V];
        if (PML && ii >= 0 && valid) ldv<V>(psx_o, p.s0.psi_hy + (int64_t)ii * ny + jb);
        float psx_n[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const float dEy = ez_r[v] - ez_c[v];
            float ty = dEy * kHy[v];
            if (PML && jj[v] >= 0) {
                const int64_t q = (int64_t)i * syw + jj[v];
                const float ps = bHy[v] * p.s0.psi_hx[q] + cHy[v] * dEy;
                p.s1.psi_hx[q] = ps;
                ty += ps;
            }
            hx_n[v] = hx_o[v] - db[v] * ty;
            const float dEx = ez_n[v] - ez_c[v];
            float tx = dEx * kHx;
            if (PML && ii >= 0) {
                psx_n[v] = p.x.bH[i] * psx_o[v] + p.x.cH[i] * dEx;
                tx += psx_n[v];
            }
            hy_n[v] = hy_o[v] + db[v] * tx;
        }
        if (PML && ii >= 0 && valid) stv<V>(p.s1.psi_hy + (int64_t)ii * ny + jb, psx_n);

        // Hx(i, j-1)
        float hx_l[V];
#pragma unroll
        for (int v = 1; v < V; ++v) hx_l[v] = hx_n[v - 1];
        float shl = lane_prev(hx_n[V - 1]);
        if (lane == 0) {
            shl = 0.f;
            if (jm >= 0) {
                const float ez_mm = p.s0.ez[row + jm];
                const float hxo = p.s0.hx[row + jm];
                const float dbm = mumap ? p.db[row + jm] : p.db0;
                const float dEy = ez_c[0] - ez_mm;
                float ty = dEy * kHy_m;
                if (PML && jj_m >= 0)
                    ty += bHy_m * p.s0.psi_hx[(int64_t)i * syw + jj_m] + cHy_m * dEy;
                shl = hxo - dbm * ty;
            }
        }
        hx_l[0] = shl;

        // ---- E layer ----
        float ez_w[V];
        float pex_o[V], pex_n[V];
        if (PML && ii >= 0 && valid) ldv<V>(pex_o, p.s0.psi_ezx + (int64_t)ii * ny + jb);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int j = jb + v;
            ez_w[v] = ez_c[v];
            if (PML && ii >= 0) pex_n[v] = (PML && ii >= 0) ? pex_o[v] : 0.f;
            if (i >= 1 && j >= 1) {
                const float dHy = hy_n[v] - hy_p[v];
                const float dHx = hx_n[v] - hx_l[v];
                float tx = dHy * kEx;
                float ty = dHx * kEy[v];
                if (PML && ii >= 0) {
                    pex_n[v] = p.x.bE[i] * pex_o[v] + p.x.cE[i] * dHy;
                    tx += pex_n[v];
                }
                if (PML && jj[v] >= 0) {
                    const int64_t q = (int64_t)i * syw + jj[v];
                    const float ps = bEy[v] * p.s0.psi_ezy[q] + cEy[v] * dHx;
                    if (valid) p.s1.psi_ezy[q] = ps;
                    ty += ps;
                }
                const float br = tx - ty;
                ez_w[v] = (lossy ? ca[v] * ez_c[v] : ez_c[v]) + cb[v] * br;
                if (CAPTURE && valid && i >= design.x && i < design.y && j >= design.z &&
                    j < design.w) {
                    const int64_t q = (int64_t)(i - design.x) * (design.w - design.z) + (j - design.z);
                    cap_ez[q] = ez_c[v];
                    cap_br[q] = br;
                }
            }
            if ((unsigned)(i - si0) < (unsigned)(si1 - si0) && (unsigned)(j - sj0) < (unsigned)(sj1 - sj0))
                ez_w[v] += sval;
        }
        if (valid) {
            stv<V>(p.s1.hx + row + jb, hx_n);
            stv<V>(p.s1.hy + row + jb, hy_n);
            stv<V>(p.s1.ez + row + jb, ez_w);
            if (PML && ii >= 0) stv<V>(p.s1.psi_ezx + (int64_t)ii * ny + jb, pex_n);
        }
        // probes owned by this tile
        for (int q = pbeg; q < pend; ++q) {
            const int cell = pt.cell[q];
            const int pi = cell / ny;
            if (pi == i) {
                const int pj = cell - pi * ny;
#pragma unroll
                for (int v = 0; v < V; ++v)
                    if (valid && pj == jb + v)
                        p.rec[(int64_t)pt.slot[q] * p.rec_stride + (step - p.rec_base)] =
                            p.probe_comp == FDTD_HX ? hx_n[v] : (p.probe_comp == FDTD_HY ? hy_n[v] : ez_w[v]);
            }
        }
#pragma unroll
        for (int v = 0; v < V; ++v) { ez_c[v] = ez_n[v]; hy_p[v] = hy_n[v]; }
    }
}

template <int V, bool PML, bool CAPTURE>
// list: tile ids of this launch (nullptr: tiles 0 .. ntiles-1)
__global__ __launch_bounds__(256) void k2d_fused(Prob2D p, int TX, int nsy, int ntiles,
                                                 const int *list, ProbeTiles pt, int64_t step,
                                                 int4 design, float *cap_ez, float *cap_br) {
    // (the tile index as a per-lane value: read as a scalar it made this
    // kernel 7 % slower on 1024^2 grids, whose steps are latency-bound)
    const int tw = xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (tw >= ntiles) return;  // whole wavefront leaves; no block barriers below
    const int t = list ? list[tw] : tw;
    const int cx = t / nsy, sy = t - cx * nsy;
    fused2d_tile<V, PML, CAPTURE>(p, TX, cx, sy, pt, pt.start[t], pt.start[t + 1], step, design,
                                  cap_ez, cap_br);
}

// Batched: the tile list spans many independent problems; the step index is
// read from device memory (base + k) so that a captured graph of launches can
// be replayed at any step.
// tiles [t0, t0 + ntiles) of a group's list; PML: the slab tiles
template <int V, bool PML>
__global__ __launch_bounds__(256) void k2d_batch(const Prob2D *__restrict__ probs,
                                                 const BatchTile *__restrict__ tiles, int t0, int ntiles,
                                                 ProbeTiles pt, int TX,
                                                 const int64_t *__restrict__ step_base, int k) {
    // the wavefront's tile, uniform across its lanes: read as a scalar, so
    // the problem's fields load into scalar registers (41 fewer VGPRs)
    const int tw = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * 4 + (int)(threadIdx.x >> 6));
    if (tw >= ntiles) return;
    const int t = t0 + tw;
    const BatchTile bt = tiles[t];
    const int64_t step = *step_base + k;
    fused2d_tile<V, PML, false>(probs[bt.prob], TX, bt.cx, bt.sy, pt, pt.start[t],
                                 pt.start[t + 1], step, make_int4(0, 0, 0, 0), nullptr, nullptr);
}

// Single-thread launch; the thread-indexed address keeps this an ordinary
// vector-memory read-modify-write.
__global__ void k_advance(int64_t *step_base, int64_t by) {
    const unsigned t = threadIdx.x;
    if (t == 0) step_base[t] += by;
}

hipError_t launch_batch_step(const Prob2D *probs_dev, const BatchTile *tiles, int t0, int ntiles,
                             bool pml, const ProbeTiles &pt, int V, int TX, const int64_t *step_base,
                             int k, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    const dim3 g((unsigned)((ntiles + 3) / 4)), b(256);
#define GEM_B(VV)                                                                                     \
    do {                                                                                              \
        if (pml) hipLaunchKernelGGL((k2d_batch<VV, true>), g, b, 0, st, probs_dev, tiles, t0, ntiles, pt, TX, step_base, k); \
        else hipLaunchKernelGGL((k2d_batch<VV, false>), g, b, 0, st, probs_dev, tiles, t0, ntiles, pt, TX, step_base, k); \
    } while (0)
    switch (V) {
        case 1: GEM_B(1); break;
        case 2: GEM_B(2); break;
        case 4: GEM_B(4); break;
        default: return hipErrorInvalidValue;
    }
#undef GEM_B
    return hipGetLastError();
}

hipError_t launch_advance(int64_t *step_base, int64_t by, hipStream_t st) {
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, st, step_base, by);
    return hipGetLastError();
}

int fused2d_ntiles(int nx, int ny, const Fused2DCfg &c) {
    const int nsy = (ny + 64 * c.V - 1) / (64 * c.V);
    const int ncx = (nx + c.TX - 1) / c.TX;
    return nsy * ncx;
}

int fused2d_tile_of(int nx, int ny, const Fused2DCfg &c, int i, int j) {
    (void)nx;
    const int nsy = (ny + 64 * c.V - 1) / (64 * c.V);
    return (i / c.TX) * nsy + j / (64 * c.V);
}

bool fused2d_supported(int nx, int ny, const Fused2DCfg &c) {
    (void)nx;
    return (c.V == 1 || c.V == 2 || c.V == 4) && ny % c.V == 0 && c.TX >= 1;
}

template <int V, bool PML, bool CAP>
static void go2d(const Prob2D &p, const Fused2DCfg &c, const int *list, int ntiles, const ProbeTiles &pt,
                 int64_t step, hipStream_t st, int4 d, float *ce, float *cbr) {
    if (ntiles <= 0) return;
    const int nsy = (p.ny + 64 * V - 1) / (64 * V);
    const unsigned nb = (unsigned)((ntiles + 3) / 4);
    hipLaunchKernelGGL((k2d_fused<V, PML, CAP>), dim3(nb), dim3(256), 0, st, p, c.TX, nsy, ntiles, list,
                       pt, step, d, ce, cbr);
}

hipError_t launch_2d_fused(const Prob2D &p, const Fused2DCfg &c, const ProbeTiles &pt,
                           int64_t step, hipStream_t st, const int *design, float *cap_ez,
                           float *cap_br, const TileSplit2D *split) {
    const bool pml = (p.x.lo + p.x.hi + p.y.lo + p.y.hi) > 0;
    const bool cap = design != nullptr;
    const int4 d = cap ? make_int4(design[0], design[1], design[2], design[3]) : make_int4(0, 0, 0, 0);
    // with CPML and a split: the interior tiles without the CPML code, then
    // the slab tiles with it
    const bool two = pml && split != nullptr;
    const int all = fused2d_ntiles(p.nx, p.ny, c);
#define GEM_GO(VV)                                                                                 \
    do {                                                                                           \
        if (two) {                                                                                 \
            if (cap) {                                                                             \
                go2d<VV, false, true>(p, c, split->inner, split->n_inner, pt, step, st, d, cap_ez, cap_br); \
                go2d<VV, true, true>(p, c, split->outer, split->n_outer, pt, step, st, d, cap_ez, cap_br);  \
            } else {                                                                               \
                go2d<VV, false, false>(p, c, split->inner, split->n_inner, pt, step, st, d, cap_ez, cap_br); \
                go2d<VV, true, false>(p, c, split->outer, split->n_outer, pt, step, st, d, cap_ez, cap_br);  \
            }                                                                                      \
        } else if (pml) {                                                                          \
            if (cap) go2d<VV, true, true>(p, c, nullptr, all, pt, step, st, d, cap_ez, cap_br);    \
            else go2d<VV, true, false>(p, c, nullptr, all, pt, step, st, d, cap_ez, cap_br);       \
        } else {                                                                                   \
            if (cap) go2d<VV, false, true>(p, c, nullptr, all, pt, step, st, d, cap_ez, cap_br);   \
            else go2d<VV, false, false>(p, c, nullptr, all, pt, step, st, d, cap_ez, cap_br);      \
        }                                                                                          \
    } while (0)
    switch (c.V) {
        case 1: GEM_GO(1); break;
        case 2: GEM_GO(2); break;
        case 4: GEM_GO(4); break;
        default: return hipErrorInvalidValue;
    }
#undef GEM_GO
    return hipGetLastError();
}

// Tiles clear of every CPML slab: rows [x0-1, x1) outside the x slabs and
// columns [y0-1, y0+64V) outside the y slabs (row x0-1 and column y0-1 are
// recomputed by the tile).
bool fused2d_interior(int nx, int ny, const Fused2DCfg &c, const int *xlohi, const int *ylohi, int t) {
    const int nsy = (ny + 64 * c.V - 1) / (64 * c.V);
    const int cx = t / nsy, sy = t - cx * nsy;
    const int x0 = cx * c.TX, x1 = std::min(x0 + c.TX, nx);
    const int y0 = sy * 64 * c.V, y1 = std::min(y0 + 64 * c.V, ny);
    auto clear = [](int n, int lo, int hi, int a, int b) {  // [a, b) outside both slabs
        return std::max(a, 0) >= lo && b <= n - hi;
    };
    return clear(nx, xlohi[0], xlohi[1], x0 - 1, x1) && clear(ny, ylohi[0], ylohi[1], y0 - 1, y1);
}

// ---------------------------------------------------------------------------
// Finite check: flag = 1 if any value is NaN or Inf.
// ---------------------------------------------------------------------------
__global__ void k_nonfinite(const float *a, int64_t n, int *flag) {
    int bad = 0;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(a[c]);
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

hipError_t launch_nonfinite(const float *a, int64_t n, int *flag, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_nonfinite, dim3((unsigned)nb), dim3(256), 0, st, a, n, flag);
    return hipGetLastError();
}

}  // namespace gem

// Builder of the explicit graph (Prop. 1) and its stepping.
//
// Node order: the paper's index maps, in the TMz relabelling of its TE form
// (paper z -> y, Hz -> Hy, Ey -> Ez):
//   Ez(i,j): t = 2i + 1 + nx(3j + 1)
//   Hx(i,j): u = i + 3 j nx
//   Hy(i,j): q = 2i + nx(3j + 1)
// followed by the CPML auxiliary values (psi_hx, psi_hy, psi_ezx, psi_ezy),
// each slab row by row with i fastest, the order of the field rows that
// read them.  Neighbourhoods: an Ez node gathers {itself, Hx(i,j),
// Hx(i,j-1), Hy(i,j), Hy(i-1,j)} (as printed in Prop. 1); Hx gathers
// {itself, Ez(i,j), Ez(i,j+1)} and Hy gathers {itself, Ez(i,j), Ez(i+1,j)}
// (forward offsets: with E owned at the lower cell corner this is the
// consistent staggering).  Each layer is one CSR sweep in place: the field
// rows, of which those with a psi edge first evaluate that auxiliary row
// (psi <- b psi + c D, read by no other row) and then use the new psi, as a
// sweep of the auxiliary rows followed by one of the field rows would.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "sim.hpp"

namespace gem {

namespace {

struct RowBuilder {
    std::vector<int> rowptr{0}, col, dst;
    std::vector<float> w;
    void edge(int64_t c, double v) {
        // row pointers are int32: a layer holds fewer than 2^31 nonzeros
        if (col.size() >= (size_t)INT32_MAX) fail(FDTD_EINVAL, "graph layer has 2^31 or more nonzeros");
        col.push_back((int)c);
        w.push_back((float)v);
    }
    void end_row(int64_t d) {
        dst.push_back((int)d);
        rowptr.push_back((int)col.size());
    }
};

template <class T>
T *up(DevAlloc &al, const std::vector<T> &h, hipStream_t st, int64_t &bytes) {
    T *d = (T *)al.get(std::max<size_t>(1, h.size()) * sizeof(T));
    if (!h.empty())
        hip_check(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st), "upload");
    bytes += (int64_t)h.size() * sizeof(T);
    return d;
}

}  // namespace

static void free_layer(Sim &s, Sim::Graph::Layer &L) {
    for (void *p : {(void *)L.rowptr, (void *)L.col, (void *)L.dst, (void *)L.w, (void *)L.chunk}) s.al.put(p);
    L = Sim::Graph::Layer{};
}

// Upload one layer: the field rows `m`, each edge to a node that a row of
// `aux` writes replaced by that row as a group of edges (a marker edge
// -1 - k with the edge's weight, then the auxiliary row's k edges, its own
// node first; every auxiliary row has exactly one such edge), and the
// chunk table of the field rows (per 64 rows: first destination and stride
// when the destinations step evenly, stride 0 otherwise; whether a row of
// the chunk holds a group).
static void put_layer(Sim &s, Sim::Graph::Layer &L, RowBuilder &m, RowBuilder *aux) {
    free_layer(s, L);
    if (aux && !aux->dst.empty()) {
        const auto mm = std::minmax_element(aux->dst.begin(), aux->dst.end());
        const int lo = *mm.first;
        std::vector<int> row_of((size_t)(*mm.second - lo) + 1, -1), readers(aux->dst.size(), 0);
        for (size_t a = 0; a < aux->dst.size(); ++a) {
            row_of[(size_t)(aux->dst[a] - lo)] = (int)a;
            if (aux->rowptr[a + 1] == aux->rowptr[a] || aux->col[(size_t)aux->rowptr[a]] != aux->dst[a])
                fail(FDTD_EINVAL, "graph builder: an auxiliary row must start with its own node");
        }
        RowBuilder g;
        for (size_t r = 0; r < m.dst.size(); ++r) {
            for (int q = m.rowptr[r]; q < m.rowptr[r + 1]; ++q) {
                const int c = m.col[(size_t)q];
                const int a = (c >= lo && c - lo < (int)row_of.size()) ? row_of[(size_t)(c - lo)] : -1;
                if (a < 0) {
                    g.col.push_back(c);
                    g.w.push_back(m.w[(size_t)q]);
                    continue;
                }
                readers[(size_t)a]++;
                const int k = aux->rowptr[(size_t)a + 1] - aux->rowptr[(size_t)a];
                g.col.push_back(-1 - k);
                g.w.push_back(m.w[(size_t)q]);
                for (int p = aux->rowptr[(size_t)a]; p < aux->rowptr[(size_t)a + 1]; ++p) {
                    g.col.push_back(aux->col[(size_t)p]);
                    g.w.push_back(aux->w[(size_t)p]);
                }
            }
            if (g.col.size() >= (size_t)INT32_MAX) fail(FDTD_EINVAL, "graph layer has 2^31 or more nonzeros");
            g.end_row(m.dst[r]);
        }
        for (int u : readers)
            if (u != 1) fail(FDTD_EINVAL, "graph builder: an auxiliary row without exactly one reader");
        L.naux = (int)aux->dst.size();
        m = std::move(g);
    }
    const int n = (int)m.dst.size();
    std::vector<int4> ch((size_t)(n + 63) / 64);
    for (int c = 0; c < (int)ch.size(); ++c) {
        const int r0 = 64 * c, r1 = std::min(n, r0 + 64);
        const int st = r1 - r0 > 1 ? m.dst[(size_t)r0 + 1] - m.dst[(size_t)r0] : 1;
        bool even = st != 0;
        for (int r = r0 + 1; r < r1 && even; ++r) even = m.dst[(size_t)r] - m.dst[(size_t)r - 1] == st;
        bool grp = false;
        for (int q = m.rowptr[(size_t)r0]; q < m.rowptr[(size_t)r1] && !grp; ++q) grp = m.col[(size_t)q] < 0;
        ch[(size_t)c] = make_int4(m.dst[(size_t)r0], even ? st : 0, grp ? 1 : 0, 0);
    }
    Sim::Graph &g = s.g;
    L.nrows = n;
    L.nnz = (int64_t)m.col.size();
    L.rowptr = up(s.al, m.rowptr, s.st, g.bytes);
    L.col = up(s.al, m.col, s.st, g.bytes);
    L.dst = up(s.al, m.dst, s.st, g.bytes);
    L.w = up(s.al, m.w, s.st, g.bytes);
    L.chunk = up(s.al, ch, s.st, g.bytes);
    hip_check(hipStreamSynchronize(s.st), "sync");
    m = RowBuilder{};
    if (aux) *aux = RowBuilder{};
}

// The graph of the split-field PML (Sec. IV, the 4 Nx Nz-node form, in the
// TMz relabelling): nodes Hx u = i + 4 j nx, Hy q = 3i + nx(4j + 1), Ezx
// tx = q + 1, Ezy tz = q + 2 for every cell, so the layer cells need no
// other layout.  H nodes gather both Ez parts of their two E neighbours,
// Ezx gathers Hy(i, j), Hy(i-1, j) and Ezy gathers Hx(i, j), Hx(i, j-1)
// (the k-offset of the printed neighbourhood of Eyz read as the j-offset,
// as the update equations require).  Weights: the per-axis split tables
// (self b, curl scale c, 1/d) times the cell's Ca (self) or Cb, Db (curl):
// in the interior b = c = 1, in the vacuum layer Ca = 1.
static void build_graph_split(Sim &s) {
    const int nx = s.nx, ny = s.ny;
    auto u = [&](int i, int j) -> int64_t { return (int64_t)i + 4LL * j * nx; };
    auto q = [&](int i, int j) -> int64_t { return 3LL * i + (int64_t)nx * (4LL * j + 1); };
    auto tx = [&](int i, int j) { return q(i, j) + 1; };
    auto tz = [&](int i, int j) { return q(i, j) + 2; };
    const int64_t nnodes = 4LL * nx * ny;
    if (nnodes >= ((int64_t)1 << 31)) fail(FDTD_EINVAL, "graph too large for 32-bit node indices");
    const AxisHost &X = s.axh[0], &Y = s.axh[1];
    auto cell = [&](int i, int j) { return (int64_t)i * ny + j; };
    auto eps = [&](int64_t c) { return kEps0 * (s.eps_r.empty() ? 1.0 : s.eps_r[(size_t)c]); };
    auto sh = [&](int64_t c) { return (s.sigma.empty() ? 0.0 : s.sigma[(size_t)c]) * s.dt / (2.0 * eps(c)); };
    auto cb_of = [&](int64_t c) { return (s.dt / eps(c)) / (1.0 + sh(c)); };
    auto ca_of = [&](int64_t c) { return (1.0 - sh(c)) / (1.0 + sh(c)); };
    auto db_of = [&](int64_t c) { return s.dt / (kMu0 * (s.mu_r.empty() ? 1.0 : s.mu_r[(size_t)c])); };
    RowBuilder hm, em;
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {  // Hx: -Db c_H,y (Ez(i, j+1) - Ez(i, j)) / dy
            const double w = db_of(cell(i, j)) * (double)Y.cH[j] * (double)Y.kH[j];
            hm.edge(u(i, j), Y.bH[j]);
            hm.edge(tx(i, j), w);
            hm.edge(tz(i, j), w);
            if (j + 1 < ny) {
                hm.edge(tx(i, j + 1), -w);
                hm.edge(tz(i, j + 1), -w);
            }
            hm.end_row(u(i, j));
        }
        for (int i = 0; i < nx; ++i) {  // Hy: +Db c_H,x (Ez(i+1, j) - Ez(i, j)) / dx
            const double w = db_of(cell(i, j)) * (double)X.cH[i] * (double)X.kH[i];
            hm.edge(q(i, j), X.bH[i]);
            hm.edge(tx(i, j), -w);
            hm.edge(tz(i, j), -w);
            if (i + 1 < nx) {
                hm.edge(tx(i + 1, j), w);
                hm.edge(tz(i + 1, j), w);
            }
            hm.end_row(q(i, j));
        }
    }
    for (int j = 1; j < ny; ++j)
        for (int i = 1; i < nx; ++i) {
            const int64_t c = cell(i, j);
            const double ca = ca_of(c), cb = cb_of(c);
            const double wx = cb * (double)X.cE[i] * (double)X.kE[i], wy = cb * (double)Y.cE[j] * (double)Y.kE[j];
            em.edge(tx(i, j), ca * (double)X.bE[i]);
            em.edge(q(i, j), wx);
            em.edge(q(i - 1, j), -wx);
            em.end_row(tx(i, j));
            em.edge(tz(i, j), ca * (double)Y.bE[j]);
            em.edge(u(i, j), -wy);
            em.edge(u(i, j - 1), wy);
            em.end_row(tz(i, j));
        }
    Sim::Graph &g = s.g;
    g.bytes = 0;
    put_layer(s, g.h, hm, nullptr);
    put_layer(s, g.e, em, nullptr);
    g.nmain = nnodes;
    g.nnodes = nnodes;
    if (!g.x) g.x = (float *)s.al.get((size_t)nnodes * 4);
    g.ez_node.resize((size_t)nx * ny);
    g.ez_node2.resize((size_t)nx * ny);
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) {
            g.ez_node[(size_t)cell(i, j)] = tx(i, j);
            g.ez_node2[(size_t)cell(i, j)] = tz(i, j);
        }
    for (int set = 0; set < 2; ++set) {
        for (int c = 0; c < 6; ++c) {
            s.al.put(s.f[set][c]);
            s.f[set][c] = nullptr;
        }
        for (int a = 0; a < NPSI3; ++a) {
            s.al.put(s.psi[set][a]);
            s.psi[set][a] = nullptr;
        }
    }
    s.al.put(s.ezy);
    s.ezy = nullptr;
    hip_check(hipStreamSynchronize(s.st), "sync");
}

// Nonzeros of the largest layer of the explicit graph of an nx x ny grid
// with sx / sy CPML cells across the x / y slabs (both faces together), an
// upper bound: non-split, Hx gathers itself, Ez(i,j), Ez(i,j+1) below the
// last row and, in a y slab, its psi as a group of 4 edges (marker, psi,
// two Ez), Hy likewise along x; Ez gathers itself and four H nodes and at
// most one group per slab direction; split, each H node gathers both Ez
// parts of its two E neighbours.
int64_t graph_layer_nnz_max(int nx, int ny, int sx, int sy, bool split) {
    const int64_t N = (int64_t)nx * ny, slab = (int64_t)nx * sy + (int64_t)ny * sx;
    const int64_t h = split ? 6 * N + 2LL * nx * (ny - 1) + 2LL * ny * (nx - 1)
                            : 4 * N + (int64_t)nx * (ny - 1) + (int64_t)ny * (nx - 1) + 4 * slab;
    const int64_t e = split ? 6 * N : 5 * N + 4 * slab;
    return std::max(h, e);
}

void build_graph(Sim &s) {
    if (s.split) {
        build_graph_split(s);
        return;
    }
    const int nx = s.nx, ny = s.ny;
    auto t = [&](int i, int j) -> int64_t { return 2LL * i + 1 + (int64_t)nx * (3LL * j + 1); };
    auto u = [&](int i, int j) -> int64_t { return (int64_t)i + 3LL * j * nx; };
    auto q = [&](int i, int j) -> int64_t { return 2LL * i + (int64_t)nx * (3LL * j + 1); };
    const int64_t N = (int64_t)nx * ny;
    const int64_t nmain = 3 * N;
    const AxisHost &X = s.axh[0], &Y = s.axh[1];
    const int sx = X.lo + X.hi, sy = Y.lo + Y.hi;
    const int64_t o_hx = nmain, o_hy = o_hx + (int64_t)nx * sy, o_ezx = o_hy + (int64_t)sx * ny,
                  o_ezy = o_ezx + (int64_t)sx * ny;
    const int64_t nnodes = o_ezy + (int64_t)nx * sy;
    if (nnodes >= ((int64_t)1 << 31)) fail(FDTD_EINVAL, "graph too large for 32-bit node indices");
    auto xs = [&](int i) { return i < X.lo ? i : (i >= nx - X.hi ? X.lo + i - (nx - X.hi) : -1); };
    auto ys = [&](int j) { return j < Y.lo ? j : (j >= ny - Y.hi ? Y.lo + j - (ny - Y.hi) : -1); };

    // coefficients per cell (same folding as the implicit stepper, in double)
    auto cb_of = [&](int64_t c) {
        const double er = s.eps_r.empty() ? 1.0 : s.eps_r[(size_t)c];
        const double sg = s.sigma.empty() ? 0.0 : s.sigma[(size_t)c];
        const double eps = kEps0 * er, sh = sg * s.dt / (2.0 * eps);
        return (s.dt / eps) / (1.0 + sh);
    };
    auto ca_of = [&](int64_t c) {
        const double er = s.eps_r.empty() ? 1.0 : s.eps_r[(size_t)c];
        const double sg = s.sigma.empty() ? 0.0 : s.sigma[(size_t)c];
        const double sh = sg * s.dt / (2.0 * kEps0 * er);
        return (1.0 - sh) / (1.0 + sh);
    };
    auto db_of = [&](int64_t c) { return s.dt / (kMu0 * (s.mu_r.empty() ? 1.0 : s.mu_r[(size_t)c])); };

    // psi nodes: y slabs (psi_hx, psi_ezy) by (slab row jj, i), x slabs
    // (psi_hy, psi_ezx) by (j, slab column ii)
    auto phx = [&](int i, int jj) { return o_hx + (int64_t)jj * nx + i; };
    auto phy = [&](int ii, int j) { return o_hy + (int64_t)j * sx + ii; };
    auto pezx = [&](int ii, int j) { return o_ezx + (int64_t)j * sx + ii; };
    auto pezy = [&](int i, int jj) { return o_ezy + (int64_t)jj * nx + i; };
    RowBuilder ha, hm, ea, em;
    // Field rows in increasing destination order within each layer; the
    // auxiliary rows in the order of the field rows that read them.
    // H layer, auxiliary rows
    for (int j = 0; j < ny; ++j) {
        const int jj = ys(j);
        if (jj >= 0)
            for (int i = 0; i < nx; ++i) {
                ha.edge(phx(i, jj), Y.bH[j]);
                ha.edge(t(i, j), -(double)Y.cH[j]);
                if (j + 1 < ny) ha.edge(t(i, j + 1), Y.cH[j]);
                ha.end_row(phx(i, jj));
            }
        for (int i = 0; i < nx; ++i) {
            const int ii = xs(i);
            if (ii < 0) continue;
            ha.edge(phy(ii, j), X.bH[i]);
            ha.edge(t(i, j), -(double)X.cH[i]);
            if (i + 1 < nx) ha.edge(t(i + 1, j), X.cH[i]);
            ha.end_row(phy(ii, j));
        }
    }
    // H layer, field rows (Hx then Hy of each Prop. 1 row k = j)
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            const int64_t c = (int64_t)i * ny + j;
            const double db = db_of(c);
            hm.edge(u(i, j), 1.0);
            hm.edge(t(i, j), db * Y.kH[j]);
            if (j + 1 < ny) hm.edge(t(i, j + 1), -db * Y.kH[j]);
            const int jj = ys(j);
            if (jj >= 0) hm.edge(phx(i, jj), -db);
            hm.end_row(u(i, j));
        }
        for (int i = 0; i < nx; ++i) {
            const int64_t c = (int64_t)i * ny + j;
            const double db = db_of(c);
            hm.edge(q(i, j), 1.0);
            hm.edge(t(i, j), -db * X.kH[i]);
            if (i + 1 < nx) hm.edge(t(i + 1, j), db * X.kH[i]);
            const int ii = xs(i);
            if (ii >= 0) hm.edge(phy(ii, j), db);
            hm.end_row(q(i, j));
        }
    }
    // E layer, auxiliary rows (cells the E layer updates: i >= 1, j >= 1),
    // in the field rows' order (j, then i)
    for (int j = 1; j < ny; ++j) {
        const int jj = ys(j);
        for (int i = 1; i < nx; ++i) {
            const int ii = xs(i);
            if (ii >= 0) {
                ea.edge(pezx(ii, j), X.bE[i]);
                ea.edge(q(i, j), X.cE[i]);
                ea.edge(q(i - 1, j), -(double)X.cE[i]);
                ea.end_row(pezx(ii, j));
            }
            if (jj >= 0) {
                ea.edge(pezy(i, jj), Y.bE[j]);
                ea.edge(u(i, j), Y.cE[j]);
                ea.edge(u(i, j - 1), -(double)Y.cE[j]);
                ea.end_row(pezy(i, jj));
            }
        }
    }
    // E layer, field rows
    for (int j = 1; j < ny; ++j)
        for (int i = 1; i < nx; ++i) {
            const int64_t c = (int64_t)i * ny + j;
            const double cbv = cb_of(c);
            em.edge(t(i, j), s.lossy ? ca_of(c) : 1.0);
            em.edge(u(i, j), -cbv * Y.kE[j]);
            em.edge(u(i, j - 1), cbv * Y.kE[j]);
            em.edge(q(i, j), cbv * X.kE[i]);
            em.edge(q(i - 1, j), -cbv * X.kE[i]);
            const int ii = xs(i), jj = ys(j);
            if (ii >= 0) em.edge(pezx(ii, j), cbv);
            if (jj >= 0) em.edge(pezy(i, jj), -cbv);
            em.end_row(t(i, j));
        }

    Sim::Graph &g = s.g;
    g.bytes = 0;
    put_layer(s, g.h, hm, &ha);
    put_layer(s, g.e, em, &ea);
    g.nmain = nmain;
    g.nnodes = nnodes;
    if (!g.x) g.x = (float *)s.al.get((size_t)nnodes * 4);
    g.ez_node.resize((size_t)N);
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j) g.ez_node[(size_t)i * ny + j] = t(i, j);
    // the implicit-stepper state buffers are not used by the graph form
    for (int set = 0; set < 2; ++set) {
        for (int c = 0; c < 6; ++c) {
            s.al.put(s.f[set][c]);
            s.f[set][c] = nullptr;
        }
        for (int a = 0; a < NPSI3; ++a) {
            s.al.put(s.psi[set][a]);
            s.psi[set][a] = nullptr;
        }
    }
    hip_check(hipStreamSynchronize(s.st), "sync");
}

void graph_refold(Sim &s) { build_graph(s); }

void graph_set_source_probes(Sim &s) {
    Sim::Graph &g = s.g;
    s.al.put(g.src_nodes);
    g.src_nodes = nullptr;
    g.nsrc = 0;
    if (s.src_idx >= 0) {
        std::vector<int> sn;
        for (int i = s.src_box[0]; i < s.src_box[1]; ++i)
            for (int j = s.src_box[2]; j < s.src_box[3]; ++j) sn.push_back((int)g.ez_node[(size_t)i * s.ny + j]);
        int64_t dummy = 0;
        g.src_nodes = up(s.al, sn, s.st, dummy);
        g.nsrc = (int)sn.size();
        hip_check(hipStreamSynchronize(s.st), "sync");
    }
    s.al.put(g.probe_node);
    s.al.put(g.probe_node2);
    g.probe_node = g.probe_node2 = nullptr;
    if (!s.probe_cells.empty()) {
        std::vector<int> pn(s.probe_cells.size()), pn2(s.probe_cells.size());
        for (size_t p = 0; p < pn.size(); ++p) pn[p] = (int)g.ez_node[(size_t)s.probe_cells[p]];
        int64_t dummy = 0;
        g.probe_node = up(s.al, pn, s.st, dummy);
        if (!g.ez_node2.empty()) {  // split field: Ez = Ezx + Ezy
            for (size_t p = 0; p < pn.size(); ++p) pn2[p] = (int)g.ez_node2[(size_t)s.probe_cells[p]];
            g.probe_node2 = up(s.al, pn2, s.st, dummy);
        }
        hip_check(hipStreamSynchronize(s.st), "sync");
    }
}

void graph_step(Sim &s, int64_t step) {
    Sim::Graph &g = s.g;
    for (auto *L : {&g.h, &g.e}) {
        const CsrLayerArgs a{L->rowptr, L->col, L->w, L->dst, L->chunk, L->nrows};
        hip_check(launch_csr_layer(a, g.x, s.st), "csr layer");
        s.last_launches += 1;
    }
    hip_check(launch_node_source_probe(g.x, g.src_nodes, g.nsrc, s.src_dev, s.src_len, step,
                                       (int)s.probe_cells.size(), g.probe_node, g.probe_node2, s.rec_dev, s.rec_cap,
                                       step - (s.n_done - s.n_rec), s.st),
              "source/probe");
    if (g.nsrc > 0 || !s.probe_cells.empty()) s.last_launches += 1;
}

static int64_t node_of(const Sim &s, int comp, int i, int j) {
    const int nx = s.nx;
    if (s.split) {  // Ez: its Ezx node (Ezy is the node after it)
        if (comp == FDTD_HX) return (int64_t)i + 4LL * j * nx;
        return 3LL * i + (int64_t)nx * (4LL * j + 1) + (comp == FDTD_EZ ? 1 : 0);
    }
    if (comp == FDTD_EZ) return 2LL * i + 1 + (int64_t)nx * (3LL * j + 1);
    if (comp == FDTD_HX) return (int64_t)i + 3LL * j * nx;
    return 2LL * i + (int64_t)nx * (3LL * j + 1);
}

int64_t graph_node(const Sim &s, int comp, int i, int j) { return node_of(s, comp, i, j); }

void graph_get_field(Sim &s, int comp, float *host) {
    std::vector<float> x((size_t)s.g.nnodes);
    hip_check(hipMemcpyAsync(x.data(), s.g.x, x.size() * 4, hipMemcpyDeviceToHost, s.st), "copy");
    hip_check(hipStreamSynchronize(s.st), "sync");
    const bool two = s.split && comp == FDTD_EZ;  // Ez = Ezx + Ezy
    for (int i = 0; i < s.nx; ++i)
        for (int j = 0; j < s.ny; ++j) {
            const size_t n0 = (size_t)node_of(s, comp, i, j);
            host[(size_t)i * s.ny + j] = two ? x[n0] + x[n0 + 1] : x[n0];
        }
}

void graph_set_field(Sim &s, int comp, const float *host) {
    std::vector<float> x((size_t)s.g.nnodes);
    hip_check(hipMemcpyAsync(x.data(), s.g.x, x.size() * 4, hipMemcpyDeviceToHost, s.st), "copy");
    hip_check(hipStreamSynchronize(s.st), "sync");
    const bool two = s.split && comp == FDTD_EZ;  // a set Ez is all Ezx
    for (int i = 0; i < s.nx; ++i)
        for (int j = 0; j < s.ny; ++j) {
            const size_t n0 = (size_t)node_of(s, comp, i, j);
            x[n0] = host[(size_t)i * s.ny + j];
            if (two) x[n0 + 1] = 0.f;
        }
    hip_check(hipMemcpyAsync(s.g.x, x.data(), x.size() * 4, hipMemcpyHostToDevice, s.st), "copy");
    hip_check(hipStreamSynchronize(s.st), "sync");
}

}  // namespace gem

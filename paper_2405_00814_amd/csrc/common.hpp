// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "gemfdtd.h"

namespace gem {

// ---------------------------------------------------------------------------
// Per-axis CPML tables (device, float32, length n), with 1/d folded in:
//   E-type difference along the axis at index i: D = F[i] - F[i-1]
//     psi <- bE[i] psi + cE[i] D;   term = kE[i] D + psi
//   H-type difference at index i:               D = F[i+1] - F[i]
//     psi <- bH[i] psi + cH[i] D;   term = kH[i] D + psi
// with kE = 1/(kappa_E d), cE = c_E / d (same for H).  Cells outside the two
// slabs have b = 1, c = 0 and carry no psi storage.
// slab index: i < lo -> i; i >= n - hi -> lo + i - (n - hi); else -1.
// ---------------------------------------------------------------------------
struct AxisDev {
    const float *kE, *bE, *cE, *kH, *bH, *cH;
    int n, lo, hi;
};

__host__ __device__ inline int slab_index(const AxisDev &a, int i) {
    if (i < a.lo) return i;
    if (i >= a.n - a.hi) return a.lo + i - (a.n - a.hi);
    return -1;
}

// 2D TMz state: three fields and four psi arrays.
//   psi_hx  [nx][sy]  (H-type, y)      psi_ezy [nx][sy]  (E-type, y)
//   psi_hy  [sx][ny]  (H-type, x)      psi_ezx [sx][ny]  (E-type, x)
// with sx = x.lo + x.hi, sy = y.lo + y.hi.
struct State2D {
    float *ez, *hx, *hy;
    float *psi_hx, *psi_hy, *psi_ezx, *psi_ezy;
};

// A 2D problem as the kernels see it.
struct Prob2D {
    int nx, ny;
    const float *ca;   // nullptr => 1
    const float *cb;
    const float *db;   // nullptr => db0
    float db0;
    AxisDev x, y;
    State2D s0;        // state read (n)
    State2D s1;        // state written (n+1); equal to s0 for in-place kernels
    // Split-field (Berenger) PML instead of the CPML (reference kernels
    // only): Ezy of every cell (Ez holds Ezx + Ezy), nullptr for the CPML.
    // The axis tables then hold k = 1/d, b = (1 - s)/(1 + s) and
    // c = 1/(1 + s), s = sigma dt / (2 eps0) at the E (i) and H (i + 1/2)
    // positions.
    float *ezy;
    int64_t src_idx;   // -1 => none; else the source box's first cell
    int src_box[6];    // source cells [b0, b1) x [b2, b3) (x [b4, b5) = [0, 1))
    const float *src_vals;  // device table, indexed by absolute step
    int64_t src_len;
    int np;
    const int *probe_idx;   // [np] linear cell index
    int probe_comp;         // FDTD_EZ, FDTD_HX or FDTD_HY
    float *rec;             // [np][rec_stride]
    int64_t rec_stride;
    int64_t rec_base;       // record index = step - rec_base
};

// 3D state: six fields and twelve psi arrays; psi_<F><a> lives in the slab
// of axis a: x-slab [sx][ny][nz], y-slab [nx][sy][nz], z-slab [nx][ny][sz].
enum { PSI_HXY, PSI_HXZ, PSI_HYZ, PSI_HYX, PSI_HZX, PSI_HZY,
       PSI_EXY, PSI_EXZ, PSI_EYZ, PSI_EYX, PSI_EZX, PSI_EZY, NPSI3 };

struct State3D {
    float *f[6];
    float *psi[NPSI3];
};

struct Prob3D {
    int nx, ny, nz;
    const float *ca, *cb, *db;
    float db0;
    AxisDev x, y, z;
    State3D s0, s1;
    int64_t src_idx;   // -1 => none; else the source box's first cell
    int src_box[6];    // source cells [b0, b1) x [b2, b3) x [b4, b5)
    int src_comp;
    const float *src_vals;
    int64_t src_len;
    int np;
    int probe_comp;
    const int64_t *probe_idx;
    float *rec;
    int64_t rec_stride;
    int64_t rec_base;
};

// Cell (i, j, k) lies in the source box b (2D: k = 0, b4 = 0, b5 = 1).
__host__ __device__ inline bool in_src(const int *b, int i, int j, int k) {
    return (unsigned)(i - b[0]) < (unsigned)(b[1] - b[0]) && (unsigned)(j - b[2]) < (unsigned)(b[3] - b[2]) &&
           (unsigned)(k - b[4]) < (unsigned)(b[5] - b[4]);
}

// Probes grouped by tile: tile t owns sorted entries [start[t], start[t+1]).
struct ProbeTiles {
    const int *start;   // [ntiles + 1]
    const int *cell;    // [np] per entry: packed (i, j[, k]) as linear index
    const int *slot;    // [np] original probe index
    // two-step 3D lists: per tile of the launch, nonzero when a probe cell
    // lies in its own planes and rows (nullptr: every tile looks its
    // groups up)
    const int *tile_any = nullptr;
};

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files).  All enqueue on `st`.
// ---------------------------------------------------------------------------
hipError_t launch_2d_ref(const Prob2D &p, int64_t step, hipStream_t st);
struct Fused2DCfg { int V; int TX; };
// Tile ids of the fused 2D kernel split into those clear of the CPML slabs
// and the rest (device arrays).
struct TileSplit2D {
    const int *inner;
    int n_inner;
    const int *outer;
    int n_outer;
};
// split (optional): launch the interior tiles without the CPML code and the
// slab tiles with it; nullptr: one launch over all tiles.
hipError_t launch_2d_fused(const Prob2D &p, const Fused2DCfg &c, const ProbeTiles &pt,
                           int64_t step, hipStream_t st, const int *design, float *cap_ez,
                           float *cap_br, const TileSplit2D *split = nullptr);
bool fused2d_interior(int nx, int ny, const Fused2DCfg &c, const int *xlohi, const int *ylohi, int t);

// 2D, TB steps per pass (temporal blocking).  A tile is one wavefront: rows
// [i0, i1) and columns [ja, ja + tb2d_own(V, TB)) (clipped to ny) of problem
// `prob`; the lanes at each side recompute the neighbouring columns.
struct Tile2T {
    int prob, i0, i1, ja;
};
constexpr int tb2d_halo(int V, int TB) { return (TB + V - 1) / V; }
constexpr int tb2d_own(int V, int TB) { return (64 - 2 * tb2d_halo(V, TB)) * V; }
bool tb2d_supported(int ny, int V, int TB, int TX);
// Tiles of one problem: rows in chunks of TX, strips of tb2d_own(V, TB)
// columns; `inner` takes the tiles whose dependency cone (rows i0-TB ..
// i1+TB-1, the strip's loaded columns) is clear of the CPML slabs, `outer`
// the others, cut into pieces of TXo rows (< 1: TX).  Ordered row chunk by
// row chunk.
void tb2d_plan(int prob, int nx, int ny, int V, int TB, int TX, int TXo, const int *xlohi, const int *ylohi,
               std::vector<Tile2T> &inner, std::vector<Tile2T> &outer);
// Default row chunk TX of the four-step pass at strip width V on `cus`
// compute units (see plan2d.cpp).
int tb2d_default_tx(int nx, int ny, int V, int cus);
// Capture of the design cells for the adjoint: for every step n of the
// pass, at cell (i, j) of the box design = [x, y) x [z, w), Ez before the E
// layer goes to ez[(n - k0) * nd + q] and the E layer's bracket to br[...],
// q = (i - x) * (w - z) + (j - z).
struct CapArgs {
    int4 design;
    float *ez, *br;
    int64_t k0, nd;
};
// probs_dev: nullptr for one problem p (tiles' prob ignored), else the
// device array the tiles index (step = *step_base + step).  mat: 0 Cb, 1
// Ca and Cb, 2 Ca, Cb and Db maps (null maps of a problem read as uniform).
// capture: one problem only (nullptr: none).
hipError_t launch_2d_tb(const Prob2D &p, const Prob2D *probs_dev, const Tile2T *tiles, int ntiles, bool pml,
                        int mat, const ProbeTiles &pt, int V, int TB, const int64_t *step_base, int64_t step,
                        hipStream_t st, const CapArgs *capture = nullptr);
int fused2d_ntiles(int nx, int ny, const Fused2DCfg &c);
int fused2d_tile_of(int nx, int ny, const Fused2DCfg &c, int i, int j);
bool fused2d_supported(int nx, int ny, const Fused2DCfg &c);

// Whole 2D grid in one workgroup (kernel variant 4): no CPML, no mu_r map
// (mat 0 or 1), at most 16
// rows per band of ny (rounded up to 64) columns in 1024 threads, at most
// 64 probes; the state in registers for all nsteps steps (s0 in, s1 out;
// several launches for more than 65536 steps).
bool res2d_supported(int nx, int ny, bool cpml, int np);
hipError_t launch_2d_resident(const Prob2D &p, int mat, int64_t step, int64_t nsteps, hipStream_t st);
hipError_t launch_3d_ref(const Prob3D &p, int64_t step, hipStream_t st);
// rec[slot[q]][step - rec_base] = p.s0 component probe_comp at cell[q], q < n
hipError_t launch_3d_probe_list(const Prob3D &p, const int *cell, const int *slot, int n, int64_t step,
                                hipStream_t st);
// Fused 3D.  V: z cells per thread; TX: x planes marched by one interior
// workgroup (0 = 16; workgroups with x/y CPML code march max(1, TX/4)).
struct Fused3DCfg { int V; int TX; };
// One workgroup's tile: planes [i0, i1), rows j0 .. j0+nrows-1 (one per
// wavefront, nrows <= wavefronts per workgroup, j0 + nrows <= ny), z cells
// [ks, k1) of the segment whose lanes start at the aligned base k0.
// i0 == i1 marks padding.
struct Tile3 {
    int i0, i1, j0, k0, k1, ks, nrows, rec;  // rec: 1 = record probes in this tile
};
// One launch of the fused 3D kernel over a list of tiles.
struct Wave3DLaunch {
    int V, wpb;    // z cells per thread; wavefronts (y rows) per workgroup
    bool pxy, pz;  // CPML code for x/y slabs, z slabs
    int off, n;    // tile list entries [off, off + n) (multiple of 8)
    int64_t cells; // cells the launch updates
    int64_t psi;   // CPML psi values it updates
};
struct Wave3DPlan {
    std::vector<Wave3DLaunch> l;
    std::vector<Tile3> tiles;  // host copy of the concatenated tile lists
};
void wave3d_plan(int nx, int ny, int nz, const Fused3DCfg &c, const int *xlohi, const int *ylohi,
                 const int *zlohi, Wave3DPlan &pl);
// ev (optional): pl.l.size() + 1 events, recorded on st before each launch
// and after the last one.
hipError_t launch_3d_wave(const Prob3D &p, const Wave3DPlan &pl, const Tile3 *tiles,
                          const ProbeTiles &pt, int64_t step, hipStream_t st,
                          hipEvent_t *ev = nullptr);
// Two steps per pass (temporal blocking).  A tile: planes [i0, i1), rows
// j0 .. j0+nrows-1, full z; i0 == i1 marks padding.
struct TileTB {
    int i0, i1, j0, nrows;
};
// z-slab cells (both ends together) the two-step kernel handles at most
constexpr int kTwoZMax = 64;
// Wavefronts per workgroup of the two-step kernel.  The instances with
// z-slab CPML or a Db map need more registers: 12 wavefronts (168 VGPRs)
// instead of 16 (128).
constexpr int two_waves(bool pz, int mat, bool pxy = false) { return (pz || mat == 2 || pxy) ? 12 : 16; }
// nz % 4 == 0, nz <= 512, zlo + zhi <= kTwoZMax, and no 4-cell group holds
// cells of both z slabs
bool two3d_supported(int nx, int ny, int nz, int zlo, int zhi);
// rows per band (the workgroup holds two halo rows more, RZ wavefronts per
// row)
int two3d_rows(int nz, bool pz, int mat, bool pxy);  // mat: 0 Cb, 1 Ca+Cb, 2 Ca+Cb+Db maps
// records probes at steps `step` and `step`+1 of cells it owns.  mid:
// nullptr for tiles whose cone is clear of the x/y slabs; else the state
// set whose x/y-slab psi arrays hold the step-1 psi (any tiles).  slab
// (with mid): 3 any tiles; 4 tiles whose cones touch x slabs only or y
// slabs only (the kernel holds a code path for each kind, without the
// other kind's psi code: a tile touching both would miss psi terms).
hipError_t launch_3d_two(const Prob3D &p, const TileTB *tiles, int n, const ProbeTiles &pt, int64_t step,
                         hipStream_t st, const State3D *mid = nullptr, int slab = 3);
// Plan of a two-step pass.  The interior tiles (cone clear of the x/y
// slabs) run the two-step kernel without x/y-slab code.  The rest, S:
//   slab_tb: tiles of the two-step kernel with x/y-slab code (tbo: x chunks
//     of txo planes, 0 = 16), which keep the step-1 psi in a third state
//     set; the interior list is ordered in 8 equal parts, one per XCD;
//   else two single steps: pass1 over S and its one-cell rim M (state n ->
//     the third state set, probes recorded in S only), pass2 over S (third
//     set -> state n+2).
struct TwoPlan {
    bool slab_tb = false;
    int rows = 0, rows_o = 0;  // rows per band: tb, tbo
    int tx = 0;                // x planes per interior tile
    std::vector<TileTB> tb, tbo;  // each padded to a multiple of 8
    // tbo in two groups, each a multiple of 8: the tiles whose cone touches
    // both the x and the y slabs, then those whose cone touches one kind
    int tbo_n[2] = {0, 0};
    int64_t tb_cells = 0, tb_psi = 0, tbo_cells = 0, tbo_psi = 0;
    Wave3DPlan pass1, pass2;
};
// c.TX = 0: slab_tb takes two3d_auto_tx's chunk for the interior tiles
// (cus: compute units of the device), the other mode 16.
void two3d_plan(int nx, int ny, int nz, const Fused3DCfg &c, int mat, bool slab_tb, int txo, int cus,
                const int *xlohi, const int *ylohi, const int *zlohi, TwoPlan &pl);
int two3d_auto_tx(int nxi, int nbands, int cus);
int wave3d_ngroups(int nx, int ny);
int wave3d_group_of(int ny, int i, int j);
bool wave3d_supported(int nx, int ny, int nz, const Fused3DCfg &c);

hipError_t launch_nonfinite(const float *a, int64_t n, int *flag, hipStream_t st);

// Frequency-domain monitor (dft.hip).  After each step launch_dft_gather
// copies the monitored cells' samples into one row of a ring of kDftBatch
// rows (cells of the box of a row-major grid, or through an index list);
// launch_dft_flush then adds, for the nk <= kDftBatch buffered steps,
// sum_k row_k[c] re[k][q] to acc[2q][c] and sum_k row_k[c] im[k][q] to
// acc[2q+1][c] (nf <= kDftMaxFreq frequencies, acc rows of npts doubles).
constexpr int kDftMaxFreq = 16;
constexpr int kDftBatch = 8;
struct DftPhases {
    double re[kDftBatch][kDftMaxFreq], im[kDftBatch][kDftMaxFreq];
};
struct DftBox {
    int i0, j0, k0;  // box origin
    int nj, nk;      // box extents along y and z
    int ny, nz;      // grid extents along y and z
};
hipError_t launch_dft_gather(const float *f, const int64_t *idx, const DftBox &box, int64_t npts, float *row,
                             hipStream_t st);
hipError_t launch_dft_flush(const float *ring, int64_t npts, int nk, int nf, const DftPhases &ph, double *acc,
                            hipStream_t st);
// Specific absorption rate from a monitor's sums: out[q][c] = sig[c] |X_qc|^2
// * inv2n2[q] / rho[c] (inv2n2 = 1 / (2 norm_q^2)), in FP64, stored FP32.
struct SarScale {
    double inv2n2[kDftMaxFreq];
};
hipError_t launch_sar(const double *acc, int64_t npts, int nf, const float *sig, const float *rho,
                      const SarScale &sc, float *out, hipStream_t st);

// One layer of the explicit graph, in place on the node vector x:
// x[dest(r)] = sum over the edges e of row r of w[e] * x[col[e]] for
// r < nrows, except that an edge with col[e] = -1 - k (k > 0) opens an
// auxiliary group: the next k edges of the row are an auxiliary row (its
// first edge its own node, read by no other row), whose sum is stored at
// that node and enters the row's sum times w[e].  dest(r): chunk[r / 64] =
// {d0, s, aux, 0} gives d0 + (r % 64) s when s != 0, else dst[r]; aux != 0
// when a row of the chunk has a group.
struct CsrLayerArgs {
    const int *rowptr, *col;
    const float *w;
    const int *dst;
    const int4 *chunk;
    int nrows;
};
hipError_t launch_csr_layer(const CsrLayerArgs &L, float *x, hipStream_t st);
// Soft source and probes on a node vector.
hipError_t launch_node_source_probe(float *x, const int *src_nodes, int nsrc, const float *src_vals,
                                    int64_t src_len, int64_t step, int np,
                                    const int *probe_node, const int *probe_node2, float *rec, int64_t rec_stride,
                                    int64_t rec_index, hipStream_t st);

// Batched 2D: one launch advances every problem by one step.
struct BatchTile { int prob; int cx; int sy; };
// tiles [t0, t0 + ntiles) of a group's list; pml: they touch a CPML slab
hipError_t launch_batch_step(const Prob2D *probs_dev, const BatchTile *tiles, int t0, int ntiles,
                             bool pml, const ProbeTiles &pt, int V, int TX, const int64_t *step_base,
                             int k, hipStream_t st);
hipError_t launch_advance(int64_t *step_base, int64_t by, hipStream_t st);

// Adjoint state of the 2D step (kadj.hip).
struct Adj2D {
    float *ez, *hx, *hy, *psi_hx, *psi_hy, *psi_ezx, *psi_ezy;
};
// out = dca sez + dcb sbr (the gradient with respect to the parameter whose
// Ca and Cb derivatives are dca, dcb), rounded to float
hipError_t launch_grad_combine(const double *sez, const double *sbr, const double *dca, const double *dcb, float *out,
                               int64_t n, hipStream_t st);
// One adjoint step in one pass: reads the adjoint state l0 (step k+1),
// writes l1 (step k), accumulates at the design cells sez += a Ez^k and
// sbr += a bracket (a: the adjoint Ez of step k+1).  When seed_out, the
// probe-loss seed of the next step is added to the written Ez:
// l1.ez[probe] += 2 * rec[slot][seed_k] (pt: probes grouped by tile in tile
// order, tile = (i / TX) * nsy + j / (62 V), entries of one cell
// consecutive).  Tiles of TX rows by 62*V columns; ny % V == 0.
// cbox: the captured box (design box plus one row and column, clipped) that
// cap_ez / cap_br cover; shx, shy (nullptr: none): per design cell sums of
// aHx bx and aHy by for the mu_r gradient (the H brackets rebuilt from the
// captured Ez; the design box must be clear of the CPML slabs).
hipError_t launch_adj2d_fused(const Prob2D &p, const Adj2D &l0, const Adj2D &l1, const int *design,
                              const int *cbox, const float *cap_ez, const float *cap_br, double *sez, double *sbr,
                              double *shx, double *shy, int seed_out, const ProbeTiles &pt, const float *rec,
                              int64_t rec_stride, int64_t seed_k, int V, int TX, hipStream_t st);
// The seed of the first adjoint step: ez[cell u] += 2 * rec[slot][k] over
// the probe entries [start[u], start[u+1]) of the nu probed cells.
hipError_t launch_adj2d_seed(float *ez, const int *seed_start, const int *seed_cell, const int *seed_slot, int nu,
                             const float *rec, int64_t rec_stride, int64_t k, hipStream_t st);

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);

}  // namespace gem

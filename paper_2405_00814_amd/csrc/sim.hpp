// Host-side simulation object behind the fdtd_sim handle.
#pragma once

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "common.hpp"

namespace gem {

// CODATA 2018
constexpr double kC0 = 299792458.0;
constexpr double kMu0 = 1.25663706212e-6;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kPi = 3.14159265358979323846;

// Error carried out of the host runtime as a status code.
struct Status {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string &msg);
void hip_check(hipError_t e, const char *what);

// Device memory through the caller's allocator (or hipMalloc).
struct DevAlloc {
    fdtd_allocator a{};
    bool has = false;
    hipStream_t st = nullptr;
    std::vector<void *> blocks;
    void *get(size_t bytes);            // zero-filled on the stream
    void put(void *p);                  // release one block
    void release_all();
};

// One axis of CPML tables in double precision before rounding.
struct AxisHost {
    int n = 0, lo = 0, hi = 0;
    std::vector<float> kE, bE, cE, kH, bH, cH;
};
AxisHost build_axis(int n, int lo, int hi, double d, double dt, const fdtd_cpml &cp);
AxisDev upload_axis(DevAlloc &al, const AxisHost &h, hipStream_t st);

// Source waveform sample for step n (added at the end of step n, t = (n+1) dt).
double source_sample(int kind, const double *par, double dt, int64_t n);
// parameters a kind reads (FDTD_SRC_*)
int src_nparams(int kind);

struct Sim {
    int ndim = 2;
    int nx = 0, ny = 0, nz = 1;
    int64_t ncell = 0;
    double dx = 0, dy = 0, dz = 0, dt = 0;
    hipStream_t st = nullptr;
    int device = 0;
    int cus = 256;  // compute units of the device
    bool split = false;      // split-field PML (2D) instead of the CPML
    float *ezy = nullptr;    // its Ezy of every cell (device)
    DevAlloc al;

    // host copies of the maps (for refolding)
    std::vector<float> eps_r, mu_r, sigma;
    bool lossy = false, mumap = false;
    fdtd_cpml cpml{};

    // device coefficients
    float *ca = nullptr, *cb = nullptr, *db = nullptr;
    float db0 = 0;
    AxisHost axh[3];
    AxisDev ax[3]{};

    // double-buffered state: fields[set][comp], psi[set][a]; set 2 is
    // allocated for the two-step pass only (state n+1 of the cells that the
    // two-step kernel does not cover)
    float *f[3][6] = {};
    float *psi[3][NPSI3] = {};
    int64_t psi_len[NPSI3] = {};
    int cur = 0;

    // source
    int src_comp = FDTD_EZ;
    int64_t src_idx = -1;                 // first cell of the source box (-1: none)
    int src_box[6] = {0, 0, 0, 0, 0, 0};  // [lo, hi) per axis (2D: z = [0, 1))
    int src_kind = -1;
    double src_par[4] = {0, 0, 0, 0};
    std::vector<float> src_table;   // TABLE kind
    float *src_dev = nullptr;
    int64_t src_cap = 0;            // entries on the device
    int64_t src_len = 0;            // valid entries (kernels add only below)

    // probes
    int probe_comp = FDTD_EZ;
    std::vector<int64_t> probe_cells;
    int *probe_dev = nullptr;          // int32 linear index (2D)
    int64_t *probe_dev64 = nullptr;    // int64 linear index (3D)
    float *rec_dev = nullptr;
    int64_t rec_cap = 0;
    int64_t n_rec = 0;
    // probes grouped by tile for the fused kernels
    int *pt_start = nullptr, *pt_cell = nullptr, *pt_slot = nullptr;
    int *tbo_any = nullptr;  // per two-step slab tile: holds a probe
    // probes of the interior two-step tiles (slab-tile mode): the single
    // step of their plane, row and z segment (step n+1, recorded; set 2
    // takes the fields), and the list read from the output set (step n+2)
    Wave3DPlan pw;
    Tile3 *pw_dev = nullptr;
    int *pg_cell = nullptr, *pg_slot = nullptr;
    int n_pg = 0;
    int pt_ntiles = -1;
    int pt_cfg[6] = {-1, -1, -1, -1, -1, -1};
    // 2D fused: tile ids clear of the CPML slabs, then the others.  Large
    // grids launch the two lists separately (the interior without the CPML
    // code); small grids take one launch, where a second launch's fixed cost
    // outweighs the gain.
    int *tl2_dev = nullptr;
    int tl2_inner = 0, tl2_outer = 0;
    bool split2d() const { return (int64_t)nx * ny >= (int64_t)4 << 20; }
    // single-step 2D configuration (variant 2's tiles; the default one for
    // the remainder steps of variant 3)
    Fused2DCfg single2d() const;
    // 2D, TB steps per pass (variant 3: tile[0] = V, tile[1] = TX, tile[2] =
    // TB): tiles clear of the slabs, then the others, and their probe groups
    Tile2T *tb2_dev = nullptr;
    int tb2_inner = 0, tb2_outer = 0;
    int *pt2_start = nullptr, *pt2_cell = nullptr, *pt2_slot = nullptr;
    int mat() const { return mumap ? 2 : (lossy ? 1 : 0); }
    // the 2D grid (no CPML, split field, mu_r map or graph) fits the
    // one-workgroup kernel with the current probes
    bool res2d_ok() const {
        return ndim == 2 && !split && !is_graph && mat() <= 1 &&
               res2d_supported(nx, ny, ax[0].lo + ax[0].hi + ax[1].lo + ax[1].hi > 0, (int)probe_cells.size());
    }
    // 3D fused: launch plan and its tile lists on the device
    Wave3DPlan plan3;
    Tile3 *tl_dev = nullptr;
    // 3D two steps per pass (variant 3): its plan and tile lists
    TwoPlan plan2;
    TileTB *tb_dev = nullptr, *tbo_dev = nullptr;
    Tile3 *p1_dev = nullptr, *p2_dev = nullptr;
    int plan2_mat = -1;

    // 2D multi-step passes replayed from a captured HIP graph (kernel
    // config tb = steps per replay, 0/1: none): the kernels read the problem
    // of the buffer parity from `probs` and the step from `step_base`, so
    // one graph serves every step range; captured again when a list or
    // table it holds is rebuilt
    struct GraphRun {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipStream_t cap_st = nullptr;
        int steps = 0;
        Prob2D *probs = nullptr;       // device [2]: set 0 -> 1, set 1 -> 0
        int64_t *step_base = nullptr;  // device step counter
        std::vector<const void *> key; // pointers the graph holds
    } gr;
    void graph_reset();
    int64_t graph_advance(int64_t n);  // steps advanced by graph replays

    int64_t n_done = 0;
    fdtd_kernel_config kcfg{};
    bool kcfg_explicit = false;

    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // second stream of the 2D multi-step pass (its CPML tiles) and the
    // events that fork it from and join it to `st`
    hipStream_t side = nullptr;
    hipEvent_t evf = nullptr, evj = nullptr;
    hipEvent_t *lev = nullptr;  // per-launch events of a profiled step (3D fused)
    bool timed = false;
    int64_t last_launches = 0;

    // explicit graph form (ndim 2)
    bool is_graph = false;
    struct Graph {
        int64_t nmain = 0, nnodes = 0;
        float *x = nullptr;  // node vector
        // per layer: the field rows, each holding the auxiliary (psi) row
        // it reads as a group of its edges (CsrLayerArgs)
        struct Layer {
            int nrows = 0, naux = 0;
            int *rowptr = nullptr, *col = nullptr, *dst = nullptr;
            float *w = nullptr;
            int4 *chunk = nullptr;
            int64_t nnz = 0;
        } h, e;
        std::vector<int64_t> ez_node;     // node of Ez(i,j) (host; split field: of Ezx)
        std::vector<int64_t> ez_node2;    // split field: node of Ezy(i,j), else empty
        int *src_nodes = nullptr;  // device: the source box's Ez nodes
        int nsrc = 0;
        int *probe_node = nullptr;
        int *probe_node2 = nullptr;  // split field: the Ezy node of each probe
        int64_t bytes = 0;
    } g;

    // adjoint scratch
    struct AdjBuf {
        bool init = false;
        Adj2D a{};
    } adj;

    ~Sim();

    Prob2D prob2d(int set_in, int set_out) const;
    Prob3D prob3d(int set_in, int set_out) const;
    void ensure_source(int64_t upto);
    void ensure_rec(int64_t upto);
    void build_probe_tiles();
    void launch_step(int64_t step);
    void launch_pair(int64_t step, hipEvent_t *ev = nullptr);
    size_t pair_launches() const;

    // frequency-domain monitor (comp < 0: none)
    struct Dft {
        int comp = -1, nf = 0;
        int box[6] = {0, 0, 0, 0, 0, 0};
        double f[kDftMaxFreq] = {};
        int64_t npts = 0, nacc = 0;
        int64_t *idx = nullptr;  // device: node index of each cell (graph form; else the box)
        double *acc = nullptr;   // device: [2 nf][npts]
        float *ring = nullptr;   // device: [kDftBatch][npts] samples not yet summed
        int nbuf = 0;            // rows of the ring in use
        DftPhases pend{};        // their phase factors
    } dft;
    void dft_accumulate(int64_t step);
    void dft_flush();
    void records_to_host(float *out, int64_t ld, int64_t m);
    void split_check() const;
    void launch_tb2d(int64_t step, const CapArgs *cap = nullptr);
    void advance(int64_t n);
    void alloc_set(int set);
    void zero_state();
    void refold(int64_t c0, int64_t c1);
};

// explicit graph form (graph.cpp)
void build_graph(Sim &s);
void graph_step(Sim &s, int64_t step);
void graph_refold(Sim &s);
void graph_set_source_probes(Sim &s);
// node of component comp at cell (i, j) in the graph's node vector
int64_t graph_node(const Sim &s, int comp, int i, int j);
void graph_get_field(Sim &s, int comp, float *host);
void graph_set_field(Sim &s, int comp, const float *host);
// nonzeros of the largest layer (graph.cpp); the row pointers are int32
int64_t graph_layer_nnz_max(int nx, int ny, int sx, int sy, bool split);

// default single-step 2D tiles for a grid, and the default kernel
// configuration of a simulation (runtime.cpp)
Fused2DCfg default_single2d(int nx, int ny);
int default_variant_tiles(const Sim &s, fdtd_kernel_config &k);

// autotuner cache: a JSON object of key -> integer list (runtime.cpp)
std::map<std::string, std::vector<int>> read_cache(const char *path);
void write_cache(const char *path, const std::map<std::string, std::vector<int>> &m);

// creation helpers (runtime.cpp)
void validate_desc(const fdtd_desc *d);
void init_sim(Sim &s, const fdtd_desc *d);

}  // namespace gem

struct fdtd_sim {
    gem::Sim s;
};

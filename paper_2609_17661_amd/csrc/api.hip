// C ABI of the pic1d library (include/pic1d.h): state, workspace carving,
// kernel launches.
#include <hip/hip_runtime.h>

#include <cstring>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/pic1d.h"
#include "kernels.h"
#include "setup.h"

using namespace pic1d;

namespace {

thread_local std::string g_init_error;

struct Carver {
    char* base;
    size_t off = 0;
    bool dry;
    explicit Carver(void* b) : base((char*)b), dry(b == nullptr) {}
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T* p = dry ? nullptr : (T*)(base + off);
        off += count * sizeof(T);
        return p;
    }
};

struct Layout {
    bool pairs = false;
    int n_lines = 0, nseg = 0;
    int64_t total_slots = 0;
    int32_t n_cells = 0, n_nodes = 0, max_nodes = 0;
    int64_t table_floats = 0;
    int32_t n_layer = 0;
    int32_t photon_region = 0;   // photon records per append region
    int32_t n_chunks = 0;        // chunks of SCAN_CELLS cells over all lines (the sort's scan)
    bool mlp = false;            // surrogate-network RICS backend
    bool mlp_fallback = false;   // ... with the table of every line as its fallback
    int32_t table_ns = 0;
};

}  // namespace

struct pic1d_state {
    pic1d_config cfg;
    std::vector<pic1d_line> lines_cfg;
    std::vector<LineHost> lines;
    Layout lay;
    hipStream_t stream = nullptr;
    int backend = 0;
    int n_cu = 0, push_blocks = 0, aux_blocks = 0;
    int frozen = 0;
    uint64_t host_step = 0;
    std::string err;
    std::vector<int64_t> seg_base_h;
    std::vector<int32_t> seg_cap_h;
    // device pointers
    int32_t *cell[2] = {nullptr, nullptr};
    float *off[2] = {nullptr, nullptr}, *u[2] = {nullptr, nullptr};
    uint64_t* id[2] = {nullptr, nullptr};
    int cur = 0;  // which particle buffer set is live
    int64_t* seg_base = nullptr;
    int32_t *seg_cap = nullptr, *n_cur = nullptr, *alloc = nullptr, *tile_prefix = nullptr, *new_count = nullptr;
    LineDev* dlines = nullptr;
    double *E = nullptr, *j_last = nullptr, *E_sum = nullptr, *j_sum = nullptr;
    float* E32 = nullptr;
    unsigned long long* J = nullptr;
    int32_t* hist[2] = {nullptr, nullptr};
    int32_t *pair_step = nullptr, *pair_last = nullptr, *cell_line = nullptr;
    int4 *bins = nullptr, *chunk_sum = nullptr;
    int32_t *chunk_line = nullptr, *line_chunk0 = nullptr;
    long long *pair_sum = nullptr, *n_sum = nullptr, *avg_count = nullptr;
    float4* nodes = nullptr;
    double* rc_nodes = nullptr;
    float4* table = nullptr;
    int32_t *ann_k = nullptr, *ann_off = nullptr, *ann_fill = nullptr, *ann_ctl = nullptr;
    int32_t *layer_cell = nullptr, *layer_line = nullptr, *layer_target = nullptr;
    unsigned long long* counters = nullptr;
    DevScalars* sc = nullptr;
    unsigned long long* rho = nullptr;
    double* mom_out = nullptr;          // [0] Gauss residual maximum; then MOM_GRID_BLOCKS pairs of partials
    unsigned long long* mom_kin = nullptr;   // kinetic energy in fixed-point chunks
    PhotonRec* photons = nullptr;
    int32_t* n_photons = nullptr;
    float* mlp_params = nullptr;
    bf16x8* mlp_ft = nullptr;
    bf16x8* mlp_bt = nullptr;
    float* mlp_bias = nullptr;
    float mlp_norm[6] = {0, 0, 0, 1, 1, 1};
    double* row_geo = nullptr;                 // MLP with table fallback: (b, mu, x) per table row
    unsigned int* mlp_err_bits = nullptr;      // ... the network's error estimate per line (float bits)
    std::vector<double> mlp_error;             // ... and on the host
    // per-kernel event timing (pic1d_profile)
    int prof_on = 0;
    // launch shape (tunable) and captured step graphs
    int xcd_walk = 1;
    int push_bpc = 0;                              // push blocks per CU
    int ppt = PUSH_PPT_DEFAULT;                    // particles per lane per tile of the push
    int ww = 0;                                    // deposit window of the push (cells)
    int sort_sub = SORT_SUB_DEFAULT;               // sort bins per cell
    int n_table_lines = 0;                         // MLP with table fallback: lines on their table
    int push_blocks_table = 0;                     // ... and the table kernel's blocks for them
    int graph_steps = 0;                           // requested steps per graph; 0 = eager
    int graph_len = 0;                             // steps per graph (a multiple of sort_interval)
    hipGraphExec_t gexec[2] = {nullptr, nullptr};  // by the live buffer set at the graph's start
    hipStream_t cap_stream = nullptr;
    std::vector<hipEvent_t> ev_pool;
    std::vector<int> ev_kernel;     // kernel id of each recorded pair (pool index 2k, 2k+1)
    double prof_ms[8] = {0};
    int64_t prof_n[8] = {0};
    void drop_graphs() {
        for (auto& g : gexec) {
            if (g) (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    }
    ~pic1d_state() {
        drop_graphs();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    }
};

namespace {

int fail(pic1d_state* st, int code, const std::string& msg) {
    if (st) st->err = msg; else g_init_error = msg;
    return code;
}

}  // namespace

namespace pic1d {
// error of a call without a state handle (pic1d_last_error(NULL))
int set_global_error(int code, const std::string& msg) { return fail(nullptr, code, msg); }
}  // namespace pic1d

namespace {

// Synchronous copy ordered on the state's stream.
hipError_t copy_sync(hipStream_t s, void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
    hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

#define HIP_TRY(st, expr)                                                                         \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail((st), PIC1D_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

bool c_pairs(const Layout& L) { return L.pairs; }

Layout plan_layout(const pic1d_config* c, std::vector<LineHost>* lines_out) {
    Layout L;
    L.pairs = c->pairs != 0;
    L.n_lines = c->n_lines;
    L.nseg = 4 * c->n_lines;
    int32_t cb = 0;
    int64_t toff = 0;
    for (int l = 0; l < c->n_lines; ++l) {
        LineHost lh;
        build_line(c, l, cb, (int32_t)(toff / 4), lh);
        cb += c->lines[l].n_cells;
        L.n_chunks += (c->lines[l].n_cells + SCAN_CELLS - 1) / SCAN_CELLS;
        L.max_nodes = std::max(L.max_nodes, c->lines[l].n_cells + 1);
        for (int s = 0; s < 4; ++s) L.total_slots += lh.cap[s];
        toff += (int64_t)lh.table.size();
        L.n_layer += (int32_t)lh.layer_cell.size();
        if (lines_out) lines_out->push_back(std::move(lh));
    }
    L.n_cells = cb;
    L.n_nodes = cb + c->n_lines;
    // photon records: up to a quarter of all particle slots per step (one event per lepton-step at most)
    L.photon_region = (int32_t)std::min<int64_t>(std::max<int64_t>(256, (L.total_slots / 4 + PHOTON_REPL - 1) / PHOTON_REPL),
                                                 (1ll << 30) / PHOTON_REPL);
    L.table_floats = toff;
    L.mlp = c->rics_backend == PIC1D_RICS_MLP;
    L.mlp_fallback = L.mlp && c->mlp_fallback_tol > 0.0;
    L.table_ns = c->table_ns;
    return L;
}

// Carve (or size, when the carver is dry) every device buffer.
void carve(Carver& cv, const Layout& L, pic1d_state* st) {
    pic1d_state dummy;
    pic1d_state* s = st ? st : &dummy;
    for (int b = 0; b < 2; ++b) {
        s->cell[b] = cv.take<int32_t>(L.total_slots);
        s->off[b] = cv.take<float>(L.total_slots);
        s->u[b] = cv.take<float>(L.total_slots);
        s->id[b] = cv.take<uint64_t>(L.total_slots);
    }
    s->seg_base = cv.take<int64_t>(L.nseg);
    s->seg_cap = cv.take<int32_t>(L.nseg);
    s->n_cur = cv.take<int32_t>(L.nseg);
    s->alloc = cv.take<int32_t>(L.nseg);
    s->new_count = cv.take<int32_t>(L.nseg);
    s->tile_prefix = cv.take<int32_t>(L.nseg + 1);
    s->dlines = cv.take<LineDev>(L.n_lines);
    s->E = cv.take<double>(L.n_cells);
    s->E32 = cv.take<float>(L.n_cells);
    s->J = cv.take<unsigned long long>(L.n_cells);
    s->j_last = cv.take<double>(L.n_cells);
    s->E_sum = cv.take<double>(L.n_cells);
    s->j_sum = cv.take<double>(L.n_cells);
    s->hist[0] = cv.take<int32_t>(4 * (size_t)L.n_cells);
    s->hist[1] = cv.take<int32_t>(4 * (size_t)L.n_cells);
    s->bins = cv.take<int4>((size_t)SORT_SUB_MAX * L.n_cells);
    s->chunk_sum = cv.take<int4>(L.n_chunks);
    s->chunk_line = cv.take<int32_t>(L.n_chunks);
    s->line_chunk0 = cv.take<int32_t>(L.n_lines + 1);
    s->pair_step = cv.take<int32_t>(L.n_cells);
    s->pair_last = cv.take<int32_t>(L.n_cells);
    s->cell_line = cv.take<int32_t>(L.n_cells);
    s->pair_sum = cv.take<long long>(L.n_cells);
    s->n_sum = cv.take<long long>(4 * (size_t)L.n_cells);
    s->avg_count = cv.take<long long>(1);
    s->nodes = cv.take<float4>(L.n_nodes);
    s->rc_nodes = cv.take<double>(L.n_nodes);
    s->table = cv.take<float4>(std::max<int64_t>(L.table_floats / 4, 1));
    s->ann_k = cv.take<int32_t>(L.n_cells);
    s->ann_off = cv.take<int32_t>(L.n_cells);
    s->ann_fill = cv.take<int32_t>(2 * (size_t)L.n_cells);
    s->ann_ctl = cv.take<int32_t>(4);
    s->layer_cell = cv.take<int32_t>(std::max(L.n_layer, 1));
    s->layer_line = cv.take<int32_t>(std::max(L.n_layer, 1));
    s->layer_target = cv.take<int32_t>(std::max(L.n_layer, 1));
    s->counters = cv.take<unsigned long long>((size_t)NCOUNT * CNT_REPL * L.n_lines);
    s->sc = cv.take<DevScalars>(1);
    s->rho = cv.take<unsigned long long>(L.max_nodes);
    s->mom_out = cv.take<double>(8 + 2 * MOM_GRID_BLOCKS);
    s->mom_kin = cv.take<unsigned long long>(4);
    s->photons = cv.take<PhotonRec>(c_pairs(L) ? (size_t)PHOTON_REPL * L.photon_region : 1);
    s->n_photons = cv.take<int32_t>(PHOTON_REPL);
    s->mlp_params = cv.take<float>(L.mlp ? MLP_NPARAM : 1);
    s->mlp_ft = cv.take<bf16x8>(L.mlp ? FT_TOTAL * 64 : 1);
    s->mlp_bt = cv.take<bf16x8>(L.mlp ? BT_TOTAL * 64 : 1);
    s->mlp_bias = cv.take<float>(L.mlp ? MLP_BIAS : 1);
    s->row_geo = cv.take<double>(L.mlp_fallback ? 3 * (size_t)L.n_lines * L.table_ns : 1);
    s->mlp_err_bits = cv.take<unsigned int>(L.mlp_fallback ? L.n_lines : 1);
}

// The particle kernel of a backend at a tile shape (particles per lane, deposit
// window in cells), or null where that shape is not built.
const void* push_kernel(int backend, int ppt, int ww) {
    switch (backend) {
        case RICS_OFF:
            if (ww == 32) return ppt == 4 ? (const void*)k_push<RICS_OFF, 4, 32, 0> : ppt == 8 ? (const void*)k_push<RICS_OFF, 8, 32, 0>
                               : ppt == 16 ? (const void*)k_push<RICS_OFF, 16, 32, 0> : nullptr;
            return (ww == 64 && ppt == 8) ? (const void*)k_push<RICS_OFF, 8, 64, 0> : nullptr;
        case RICS_EXACT:
            if (ww == 32) return ppt == 4 ? (const void*)k_push<RICS_EXACT, 4, 32, 0> : ppt == 8 ? (const void*)k_push<RICS_EXACT, 8, 32, 0>
                               : ppt == 16 ? (const void*)k_push<RICS_EXACT, 16, 32, 0> : nullptr;
            return (ww == 64 && ppt == 8) ? (const void*)k_push<RICS_EXACT, 8, 64, 0> : nullptr;
        case RICS_TABLE:
            if (ww == 128) return ppt == 4 ? (const void*)k_push<RICS_TABLE, 4, 128, 0> : ppt == 8 ? (const void*)k_push<RICS_TABLE, 8, 128, 0>
                                : ppt == 16 ? (const void*)k_push<RICS_TABLE, 16, 128, 0> : nullptr;
            return (ww == 64 && ppt == 8) ? (const void*)k_push<RICS_TABLE, 8, 64, 0> : nullptr;
        case RICS_MLP:
            return (ww == 32 && ppt == 8) ? (const void*)k_push<RICS_MLP, 8, 32, 0> : nullptr;
        default:
            return nullptr;
    }
}

int default_window(int backend) { return backend == RICS_TABLE ? 128 : 32; }

PushArgs push_args(pic1d_state* st) {
    PushArgs a{};
    const int b = st->cur;
    a.cell = st->cell[b]; a.off = st->off[b]; a.u = st->u[b]; a.id = st->id[b];
    a.seg_base = st->seg_base; a.seg_cap = st->seg_cap; a.n_cur = st->n_cur; a.alloc = st->alloc;
    a.tile_prefix = st->tile_prefix; a.nseg = st->lay.nseg; a.tile = 64 * st->ppt;
    a.nlg = st->cfg.table_nlg; a.ns = st->cfg.table_ns;
    a.pairs = st->cfg.pairs; a.conversion = st->cfg.conversion; a.emission = st->cfg.emission;
    a.gravity = st->cfg.atmosphere && st->cfg.gravity;
    a.lines = st->dlines; a.E32 = st->E32; a.J = st->J; a.nodes = st->nodes; a.rc_nodes = st->rc_nodes;
    a.table = st->table; a.hist[0] = st->hist[0]; a.hist[1] = st->hist[1];
    a.pair_step = st->pair_step; a.counters = st->counters; a.sc = st->sc;
    a.key0 = (uint32_t)(st->cfg.seed & 0xFFFFFFFFu); a.key1 = (uint32_t)(st->cfg.seed >> 32);
    a.xcd_walk = st->xcd_walk;
    a.mlp_ft = st->mlp_ft; a.mlp_bias = st->mlp_bias;
    for (int k = 0; k < 3; ++k) { a.mlp_mean[k] = st->mlp_norm[k]; a.mlp_std[k] = st->mlp_norm[3 + k]; }
    a.mlp_kTn = (float)((st->cfg.kT_keV - 0.3) * (2.0 / 0.7) - 1.0);
    a.qm_ion = (float)(1.0 / st->cfg.mass_ratio);
    a.inv_mass_ion = (float)(1.0 / st->cfg.mass_ratio);
    a.photons = st->photons;
    a.n_photons = st->n_photons;
    a.photon_region = st->lay.photon_region;
    return a;
}

BookArgs book_args(pic1d_state* st) {
    BookArgs b{};
    b.n_photons = st->n_photons;
    b.n_cur = st->n_cur; b.alloc = st->alloc; b.seg_cap = st->seg_cap; b.tile_prefix = st->tile_prefix;
    b.nseg = st->lay.nseg; b.tile = 64 * st->ppt; b.sc = st->sc;
    return b;
}

// Event pair around one kernel launch when profiling is on; returns the pair index or -1.
int prof_begin(pic1d_state* st, int kid) {
    if (!st->prof_on) return -1;
    const size_t k = st->ev_kernel.size();
    while (st->ev_pool.size() < 2 * (k + 1)) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        st->ev_pool.push_back(e);
    }
    st->ev_kernel.push_back(kid);
    (void)hipEventRecord(st->ev_pool[2 * k], st->stream);
    return (int)k;
}

void prof_end(pic1d_state* st, int k) {
    if (k >= 0) (void)hipEventRecord(st->ev_pool[2 * k + 1], st->stream);
}

// After the stream has been synchronised: accumulate the recorded durations.
void prof_collect(pic1d_state* st) {
    for (size_t k = 0; k < st->ev_kernel.size(); ++k) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, st->ev_pool[2 * k], st->ev_pool[2 * k + 1]) == hipSuccess) {
            st->prof_ms[st->ev_kernel[k]] += ms;
            st->prof_n[st->ev_kernel[k]] += 1;
        }
    }
    st->ev_kernel.clear();
}

int launch_push(pic1d_state* st) {
    PushArgs a = push_args(st);
    void* args[] = {&a};
    const int pk = prof_begin(st, 0);
    if (st->backend == RICS_MLP && st->n_table_lines > 0) {
        // the surrogate with table fallback: the lines on their tables through the table
        // kernel (its own occupancy; the MLP kernel holds one wavefront per SIMD), the
        // lines on the network through the MLP kernel
        const int n_net = st->lay.n_lines - st->n_table_lines;
        if (st->ppt != 8 || st->ww != 32) return fail(st, PIC1D_EINVAL, "push shape not built");
        const void* kt = n_net > 0 ? (const void*)k_push<RICS_TABLE, 8, 128, 1> : (const void*)k_push<RICS_TABLE, 8, 128, 0>;
        HIP_TRY(st, hipLaunchKernel(kt, dim3(st->push_blocks_table), dim3(PUSH_TPB), args, 0, st->stream));
        if (n_net > 0)
            HIP_TRY(st, hipLaunchKernel((const void*)k_push<RICS_MLP, 8, 32, 2>, dim3(st->push_blocks), dim3(PUSH_TPB_MLP),
                                        args, 0, st->stream));
    } else {
        const void* kp = push_kernel(st->backend, st->ppt, st->ww);
        if (!kp) return fail(st, PIC1D_EINVAL, "push shape not built");
        HIP_TRY(st, hipLaunchKernel(kp, dim3(st->push_blocks), dim3(st->backend == RICS_MLP ? PUSH_TPB_MLP : PUSH_TPB),
                                    args, 0, st->stream));
    }
    prof_end(st, pk);
    return PIC1D_OK;
}

int launch_plan(pic1d_state* st, int advance) {
    const int pk = prof_begin(st, 3);
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(256), 0, st->stream, book_args(st), advance);
    prof_end(st, pk);
    return PIC1D_OK;
}

int launch_hist(pic1d_state* st) {
    // recount H[step & 1] from the live particles
    HistArgs h{};
    h.cell = st->cell[st->cur]; h.seg_base = st->seg_base; h.n_cur = st->n_cur; h.tile_prefix = st->tile_prefix;
    h.nseg = st->lay.nseg; h.tile = 64 * st->ppt; h.lines = st->dlines; h.hist = st->hist[st->host_step & 1];
    HIP_TRY(st, hipMemsetAsync(h.hist, 0, 4 * sizeof(int32_t) * (size_t)st->lay.n_cells, st->stream));
    hipLaunchKernelGGL(k_hist, dim3(st->aux_blocks), dim3(PUSH_TPB), 0, st->stream, h);
    return PIC1D_OK;
}

int launch_sort(pic1d_state* st) {
    SortArgs s{};
    const int b = st->cur, o = 1 - st->cur;
    s.cell = st->cell[b]; s.off = st->off[b]; s.u = st->u[b]; s.id = st->id[b];
    s.cell2 = st->cell[o]; s.off2 = st->off[o]; s.u2 = st->u[o]; s.id2 = st->id[o];
    s.seg_base = st->seg_base; s.seg_cap = st->seg_cap; s.n_cur = st->n_cur; s.alloc = st->alloc;
    s.tile_prefix = st->tile_prefix;
    s.nseg = st->lay.nseg; s.tile = 64 * st->ppt; s.lines = st->dlines; s.hist[0] = st->hist[0]; s.hist[1] = st->hist[1];
    s.bins = st->bins; s.chunk_sum = st->chunk_sum; s.chunk_line = st->chunk_line; s.line_chunk0 = st->line_chunk0;
    s.n_chunks = st->lay.n_chunks; s.n_bins = st->sort_sub * st->lay.n_cells; s.sub = st->sort_sub;
    s.new_count = st->new_count; s.sc = st->sc;
    const int pk = prof_begin(st, 4);
    hipLaunchKernelGGL(k_sort_zero, dim3(st->aux_blocks), dim3(256), 0, st->stream, s);
    hipLaunchKernelGGL(k_sort_count, dim3(4 * st->aux_blocks), dim3(PUSH_TPB), 0, st->stream, s);
    hipLaunchKernelGGL(k_sort_chunks, dim3(st->lay.n_chunks), dim3(SCAN_CELLS), 0, st->stream, s);
    hipLaunchKernelGGL(k_sort_lines, dim3(st->lay.n_lines), dim3(256), 0, st->stream, s);
    hipLaunchKernelGGL(k_sort_cursors, dim3(st->lay.n_chunks), dim3(SCAN_CELLS), 0, st->stream, s);
    hipLaunchKernelGGL(k_sort_scatter, dim3(4 * st->aux_blocks), dim3(PUSH_TPB), 0, st->stream, s);
    hipLaunchKernelGGL(k_sort_finish, dim3((st->lay.nseg + 255) / 256), dim3(256), 0, st->stream, s);
    prof_end(st, pk);
    st->cur = o;
    return launch_plan(st, 0);
}

int check_error(pic1d_state* st) {
    DevScalars h{};
    HIP_TRY(st, hipMemcpyAsync(&h, st->sc, sizeof(h), hipMemcpyDeviceToHost, st->stream));
    HIP_TRY(st, hipStreamSynchronize(st->stream));
    if (h.err != 0) {
        st->frozen = h.err;
        return fail(st, h.err, h.err == PIC1D_ECAPACITY   ? "particle capacity exceeded (state frozen)"
                               : h.err == PIC1D_ENONFINITE ? "non-finite momentum (state frozen)"
                                                           : "cell counts and particles disagree (state frozen)");
    }
    return PIC1D_OK;
}

}  // namespace

extern "C" {

int pic1d_workspace_size(const pic1d_config* cfg, size_t* bytes) {
    const char* why = validate_config(cfg);
    if (why[0]) return fail(nullptr, PIC1D_EINVAL, why);
    if (!bytes) return fail(nullptr, PIC1D_EINVAL, "bytes is NULL");
    const Layout L = plan_layout(cfg, nullptr);
    Carver cv(nullptr);
    carve(cv, L, nullptr);
    *bytes = cv.off + 256;
    return PIC1D_OK;
}

int pic1d_init(const pic1d_config* cfg, pic1d_state** out) {
    if (!out) return fail(nullptr, PIC1D_EINVAL, "out is NULL");
    *out = nullptr;
    const char* why = validate_config(cfg);
    if (why[0]) return fail(nullptr, PIC1D_EINVAL, why);
    const bool mlp_fallback = cfg->rics_backend == PIC1D_RICS_MLP && cfg->mlp_fallback_tol > 0.0;
    if (cfg->rics_backend == PIC1D_RICS_MLP) {
        if (!cfg->mlp_weights || !cfg->mlp_norm) return fail(nullptr, PIC1D_EINVAL, "MLP backend needs mlp_weights and mlp_norm");
        for (int l = 0; l < cfg->n_lines && !mlp_fallback; ++l)
            if (cfg->lines[l].r_eq != 4.0)
                return fail(nullptr, PIC1D_EINVAL, "the surrogate network covers the R_max = 4 line only");
        if (!(cfg->kT_keV >= 0.3 && cfg->kT_keV <= 1.0))
            return fail(nullptr, PIC1D_EINVAL, "the surrogate network covers kT in [0.3, 1] keV");
        for (int k = 0; k < 6; ++k)
            if (!std::isfinite(cfg->mlp_norm[k]) || (k >= 3 && !(cfg->mlp_norm[k] > 0.0f)))
                return fail(nullptr, PIC1D_EINVAL, "mlp_norm: finite means and positive deviations");
    }
    pic1d_state* st = new pic1d_state();
    st->cfg = *cfg;
    st->lines_cfg.assign(cfg->lines, cfg->lines + cfg->n_lines);
    st->cfg.lines = st->lines_cfg.data();
    st->stream = (hipStream_t)cfg->stream;
    st->backend = cfg->rics_backend;
    st->lay = plan_layout(&st->cfg, &st->lines);
    Carver dry(nullptr);
    carve(dry, st->lay, nullptr);
    if (!cfg->workspace || cfg->workspace_bytes < dry.off + 256 || ((uintptr_t)cfg->workspace & 255)) {
        delete st;
        return fail(nullptr, PIC1D_ENOMEM, "workspace missing, misaligned or smaller than pic1d_workspace_size");
    }
    Carver cv(cfg->workspace);
    carve(cv, st->lay, st);

    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        delete st;
        return fail(nullptr, PIC1D_EDEVICE, "no HIP device");
    }
    st->n_cu = prop.multiProcessorCount;
    int occ = 0;
    st->ppt = PUSH_PPT_DEFAULT;
    st->ww = default_window(st->backend);
    const void* kp = push_kernel(st->backend, st->ppt, st->ww);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kp, st->backend == RICS_MLP ? PUSH_TPB_MLP : PUSH_TPB, 0);
    occ = std::max(1, std::min(occ, 8));
    st->push_blocks = st->n_cu * occ;
    st->aux_blocks = st->n_cu * 4;

    const hipStream_t s = st->stream;
    auto bail = [&](int code, const std::string& m) {
        g_init_error = m;
        delete st;
        return code;
    };
#define INIT_TRY(expr)                                                                       \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return bail(PIC1D_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

    INIT_TRY(hipMemsetAsync(cfg->workspace, 0, cv.off, s));
    // segments
    const int nseg = st->lay.nseg;
    st->seg_base_h.assign(nseg, 0);
    st->seg_cap_h.assign(nseg, 0);
    int64_t acc = 0;
    for (int l = 0; l < st->lay.n_lines; ++l)
        for (int sp = 0; sp < 4; ++sp) {
            st->seg_base_h[4 * l + sp] = acc;
            st->seg_cap_h[4 * l + sp] = (int32_t)st->lines[l].cap[sp];
            acc += st->lines[l].cap[sp];
        }
    std::vector<LineDev> ld(st->lay.n_lines);
    std::vector<float> nodes;
    std::vector<double> rcn;
    std::vector<float> table;
    std::vector<int32_t> lc, ll, lt, cell_line, chunk_line, line_chunk0;
    for (int l = 0; l < st->lay.n_lines; ++l) {
        const LineHost& lh = st->lines[l];
        ld[l] = lh.dev;
        nodes.insert(nodes.end(), lh.nodes.begin(), lh.nodes.end());
        rcn.insert(rcn.end(), lh.rc.begin(), lh.rc.end());
        table.insert(table.end(), lh.table.begin(), lh.table.end());
        for (size_t k = 0; k < lh.layer_cell.size(); ++k) {
            lc.push_back(lh.dev.cell_base + lh.layer_cell[k]);
            ll.push_back(l);
            lt.push_back(lh.layer_target[k]);
        }
        cell_line.insert(cell_line.end(), lh.dev.n_cells, l);
        line_chunk0.push_back((int32_t)chunk_line.size());
        chunk_line.insert(chunk_line.end(), (lh.dev.n_cells + SCAN_CELLS - 1) / SCAN_CELLS, l);
    }
    line_chunk0.push_back((int32_t)chunk_line.size());
    INIT_TRY(hipMemcpyAsync(st->seg_base, st->seg_base_h.data(), nseg * sizeof(int64_t), hipMemcpyHostToDevice, s));
    INIT_TRY(hipMemcpyAsync(st->seg_cap, st->seg_cap_h.data(), nseg * sizeof(int32_t), hipMemcpyHostToDevice, s));
    INIT_TRY(hipMemcpyAsync(st->dlines, ld.data(), ld.size() * sizeof(LineDev), hipMemcpyHostToDevice, s));
    INIT_TRY(hipMemcpyAsync(st->nodes, nodes.data(), nodes.size() * sizeof(float), hipMemcpyHostToDevice, s));
    INIT_TRY(hipMemcpyAsync(st->rc_nodes, rcn.data(), rcn.size() * sizeof(double), hipMemcpyHostToDevice, s));
    if (!table.empty())
        INIT_TRY(hipMemcpyAsync(st->table, table.data(), table.size() * sizeof(float), hipMemcpyHostToDevice, s));
    if (cfg->rics_backend == PIC1D_RICS_TABLE && cfg->photon_field == PIC1D_FIELD_DISK) {
        // the finite stellar disk's table, by its quadrature on the device
        DiskTableArgs da{};
        da.nlg = cfg->table_nlg;
        da.ns = cfg->table_ns;
        da.n_c = DISK_N_C;
        da.n_phi = DISK_N_PHI;
        gauss_legendre(DISK_N_C, da.gc, da.wc);
        gauss_legendre(DISK_N_PHI, da.gp, da.wp);
        da.b_pole = cfg->b_pole;
        da.theta = cfg->kT_keV / 510.99895000;
        for (int l = 0; l < st->lay.n_lines; ++l) {
            const LineHost& lh = st->lines[l];
            da.table = st->table + lh.dev.table_off;
            da.R = cfg->lines[l].r_eq;
            da.L = lh.L_rstar;
            da.AF = lh.AF;
            da.AN = lh.AN;
            INIT_TRY(launch_disk_table(da, s));
        }
    }
    if (!lc.empty()) {
        INIT_TRY(hipMemcpyAsync(st->layer_cell, lc.data(), lc.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        INIT_TRY(hipMemcpyAsync(st->layer_line, ll.data(), ll.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        INIT_TRY(hipMemcpyAsync(st->layer_target, lt.data(), lt.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    INIT_TRY(hipMemcpyAsync(st->cell_line, cell_line.data(), cell_line.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    INIT_TRY(hipMemcpyAsync(st->chunk_line, chunk_line.data(), chunk_line.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    INIT_TRY(hipMemcpyAsync(st->line_chunk0, line_chunk0.data(), line_chunk0.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, s));
    if (st->lay.mlp) {
        for (int k = 0; k < 6; ++k) st->mlp_norm[k] = cfg->mlp_norm[k];
        for (int l = 0; l < st->lay.n_lines && !mlp_fallback; ++l) {
            const std::vector<float>& nd = st->lines[l].nodes;      // {b, mu, x, 0} per node
            for (size_t i = 0; i < nd.size(); i += 4)
                if (!(nd[i] >= 0.01f && nd[i] <= 1000.0f))
                    return bail(PIC1D_EINVAL, "the surrogate network covers B/B_QED in [0.01, 1000] only");
        }
        INIT_TRY(hipMemcpyAsync(st->mlp_params, cfg->mlp_weights, MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_mlp_pack, dim3(64), dim3(256), 0, s, st->mlp_params, st->mlp_ft, st->mlp_bt, st->mlp_bias);
        INIT_TRY(hipGetLastError());
        st->mlp_error.assign(st->lay.n_lines, 0.0);
        if (mlp_fallback) {
            // the network's error estimate on every line, then each line's source
            std::vector<double> rg;
            for (int l = 0; l < st->lay.n_lines; ++l)
                rg.insert(rg.end(), st->lines[l].row_geo.begin(), st->lines[l].row_geo.end());
            INIT_TRY(hipMemcpyAsync(st->row_geo, rg.data(), rg.size() * sizeof(double), hipMemcpyHostToDevice, s));
            INIT_TRY(hipMemsetAsync(st->mlp_err_bits, 0, st->lay.n_lines * sizeof(unsigned int), s));
            hipLaunchKernelGGL(k_mlp_line_error, dim3(std::max(1, st->n_cu)), dim3(256), 0, s, push_args(st),
                               st->row_geo, cfg->kT_keV, st->mlp_err_bits);
            INIT_TRY(hipGetLastError());
            std::vector<unsigned int> bits(st->lay.n_lines);
            INIT_TRY(hipMemcpyAsync(bits.data(), st->mlp_err_bits, bits.size() * sizeof(unsigned int),
                                    hipMemcpyDeviceToHost, s));
            INIT_TRY(hipStreamSynchronize(s));
            for (int l = 0; l < st->lay.n_lines; ++l) {
                float e;
                std::memcpy(&e, &bits[l], sizeof(float));
                st->mlp_error[l] = e;
                ld[l].use_table = (double)e > cfg->mlp_fallback_tol ? 1 : 0;
                st->lines[l].dev.use_table = ld[l].use_table;
                st->n_table_lines += ld[l].use_table;
            }
            int occ_t = 0;
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &occ_t, push_kernel(RICS_TABLE, st->ppt, default_window(RICS_TABLE)), PUSH_TPB, 0);
            st->push_blocks_table = st->n_cu * std::max(1, std::min(occ_t, 8));
            INIT_TRY(hipMemcpyAsync(st->dlines, ld.data(), ld.size() * sizeof(LineDev), hipMemcpyHostToDevice, s));
        }
    }

    // initial pair plasma
    std::vector<int32_t> alloc0(nseg, 0);
    for (int l = 0; l < st->lay.n_lines; ++l) {
        const pic1d_line& ln = st->lines_cfg[l];
        const int64_t np = (ln.init_mode == PIC1D_INIT_EMPTY) ? 0 : (int64_t)ln.ppc_init * ln.n_cells;
        if (np == 0) continue;
        if (np > st->seg_cap_h[4 * l] || np > st->seg_cap_h[4 * l + 1]) return bail(PIC1D_EINVAL, "capacity below the initial pairs");
        InitArgs ia{};
        ia.cell = st->cell[0]; ia.off = st->off[0]; ia.u = st->u[0]; ia.id = st->id[0];
        ia.base_e = st->seg_base_h[4 * l]; ia.base_p = st->seg_base_h[4 * l + 1];
        ia.n_pairs = np; ia.ppc = ln.ppc_init; ia.line = l; ia.mode = ln.init_mode;
        ia.log10_gmax = ln.init_mode == PIC1D_INIT_HOT ? log10(ln.init_gamma_max) : 0.0;
        const double us = ln.init_beta / sqrt(1.0 - ln.init_beta * ln.init_beta);
        ia.u_stream = (cfg->j_twist >= 0.0 ? 1.0 : -1.0) * us;
        ia.id_base = (uint64_t)l << 40;
        ia.key0 = (uint32_t)(cfg->seed & 0xFFFFFFFFu); ia.key1 = (uint32_t)(cfg->seed >> 32);
        hipLaunchKernelGGL(k_init_pairs, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, ia);
        alloc0[4 * l] = alloc0[4 * l + 1] = (int32_t)np;
    }
    INIT_TRY(hipMemcpyAsync(st->alloc, alloc0.data(), nseg * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (launch_plan(st, 0) != PIC1D_OK) return bail(PIC1D_EDEVICE, st->err);
    if (launch_hist(st) != PIC1D_OK) return bail(PIC1D_EDEVICE, st->err);
    // the initial plasma in position order (its offsets are random within each cell)
    if (cfg->sort_interval > 0 && launch_sort(st) != PIC1D_OK) return bail(PIC1D_EDEVICE, st->err);
    INIT_TRY(hipStreamSynchronize(s));
    INIT_TRY(hipGetLastError());
#undef INIT_TRY
    *out = st;
    return PIC1D_OK;
}

}  // extern "C"

namespace {

// Enqueue one step on st->stream: push, conversion, atmosphere, Ampere, plan,
// and the cell sort every sort_interval steps.
int enqueue_step(pic1d_state* st) {
    const int nt = st->lay.n_cells;
    FieldArgs f{};
    {
        int rc = launch_push(st);
        if (rc) return rc;
        // pair conversion and atmosphere refill, one launch
        ConvertArgs ca{};
        AtmArgs aa{};
        int conv_blocks = 0, atm_blocks = 0;
        const int b = st->cur;
        if (st->cfg.pairs) {
            ca.cell = st->cell[b]; ca.off = st->off[b]; ca.u = st->u[b]; ca.id = st->id[b];
            ca.seg_base = st->seg_base; ca.seg_cap = st->seg_cap; ca.alloc = st->alloc; ca.lines = st->dlines;
            ca.rc_nodes = st->rc_nodes; ca.hist[0] = st->hist[0]; ca.hist[1] = st->hist[1];
            ca.pair_step = st->pair_step; ca.counters = st->counters; ca.sc = st->sc;
            ca.photons = st->photons; ca.n_photons = st->n_photons; ca.photon_region = st->lay.photon_region;
            ca.conversion = st->cfg.conversion;
            ca.key0 = (uint32_t)(st->cfg.seed & 0xFFFFFFFFu); ca.key1 = (uint32_t)(st->cfg.seed >> 32);
            // one block per CU: every block first scans the record regions' fills, which
            // is most of the launch where few photons were recorded (four per CU cost
            // 1 us more a step on a quiet line and bought nothing with 2.5e5 pairs a step)
            conv_blocks = st->n_cu;
        }
        ca.sc = st->sc;
        if (st->cfg.atmosphere && st->lay.n_layer > 0) {
            aa.cell = st->cell[b]; aa.off = st->off[b]; aa.u = st->u[b]; aa.id = st->id[b];
            aa.seg_base = st->seg_base; aa.seg_cap = st->seg_cap; aa.alloc = st->alloc; aa.lines = st->dlines;
            aa.hist[0] = st->hist[0]; aa.hist[1] = st->hist[1];
            aa.layer_cell = st->layer_cell; aa.layer_line = st->layer_line; aa.layer_target = st->layer_target;
            aa.n_layer = st->lay.n_layer; aa.counters = st->counters; aa.sc = st->sc;
            aa.key0 = (uint32_t)(st->cfg.seed & 0xFFFFFFFFu); aa.key1 = (uint32_t)(st->cfg.seed >> 32);
            aa.sig_e = (float)sqrt(st->cfg.atm_T);
            aa.sig_i = (float)sqrt(st->cfg.atm_T / st->cfg.mass_ratio);
            atm_blocks = std::max(1, std::min(st->aux_blocks, (st->lay.n_layer * 64 + 255) / 256));
        }
        if (conv_blocks + atm_blocks > 0) {
            const int pk = prof_begin(st, 1);
            hipLaunchKernelGGL(k_append, dim3(conv_blocks + atm_blocks), dim3(256), 0, st->stream, ca, aa,
                               conv_blocks);
            prof_end(st, pk);
        }
        f.E = st->E; f.E32 = st->E32; f.J = st->J; f.j_last = st->j_last; f.hist[0] = st->hist[0]; f.hist[1] = st->hist[1];
        f.pair_step = st->pair_step; f.pair_last = st->pair_last; f.E_sum = st->E_sum; f.j_sum = st->j_sum;
        f.pair_sum = st->pair_sum; f.n_sum = st->n_sum; f.avg_count = st->avg_count; f.cell_line = st->cell_line;
        f.lines = st->dlines; f.n_total = nt; f.frozen = st->cfg.frozen_field; f.avg_start = st->cfg.avg_start_step;
        f.sc = st->sc;
        if (st->cfg.annihilation) {
            // pair annihilation at the density limit: plan and candidates here, the
            // selection in k_field before Ampere
            AnnihArgs& an = f.an;
            an.cell = st->cell[b]; an.off = st->off[b]; an.u = st->u[b]; an.id = st->id[b];
            an.seg_base = st->seg_base; an.seg_cap = st->seg_cap; an.alloc = st->alloc;
            an.hist[0] = st->hist[0]; an.hist[1] = st->hist[1];
            an.cell_line = st->cell_line; an.lines = st->dlines;
            an.n_total = nt; an.n_lines = st->lay.n_lines;
            an.ann_k = st->ann_k; an.ann_off = st->ann_off; an.ann_fill = st->ann_fill; an.ann_ctl = st->ann_ctl;
            // candidate records in the other particle buffer set (written only by the sort)
            an.cand_key = st->id[1 - b];
            an.cand_slot = st->cell[1 - b];
            an.cand_cap = st->lay.total_slots;
            an.J = st->J; an.counters = st->counters;
            an.key0 = (uint32_t)(st->cfg.seed & 0xFFFFFFFFu); an.key1 = (uint32_t)(st->cfg.seed >> 32);
            an.sc = st->sc;
            f.annihilation = 1;
            const int pk = prof_begin(st, 5);
            hipLaunchKernelGGL(k_annih_plan, dim3(std::min(st->aux_blocks, (nt + 255) / 256)), dim3(256), 0,
                               st->stream, an);
            hipLaunchKernelGGL(k_annih_gather, dim3(GATHER_BLOCKS_PER_CU * st->n_cu), dim3(256), 0, st->stream, an);
            prof_end(st, pk);
        }
        // Ampere; its last block plans the next push and advances the step counter
        const int pk = prof_begin(st, 2);
        // 64 cells per wavefront, 4 with annihilation (k_field's cells per wavefront)
        const int field_cells = f.annihilation ? 16 : 256;
        // (and one more block for the bookkeeping)
        hipLaunchKernelGGL(k_field, dim3(std::min(16 * st->aux_blocks, (nt + field_cells - 1) / field_cells) + 1),
                           dim3(256), 0, st->stream, f, book_args(st));
        prof_end(st, pk);
        st->host_step += 1;
        if (st->cfg.sort_interval > 0 && st->host_step % st->cfg.sort_interval == 0) {
            rc = launch_sort(st);
            if (rc) return rc;
        }
    }
    return PIC1D_OK;
}

// Capture graph_len steps starting from the current buffer set (host_step a
// multiple of graph_len) on a private stream; the host-side step state is
// restored afterwards, the graph replays on the caller's stream.
int capture_graph(pic1d_state* st) {
    if (!st->cap_stream) HIP_TRY(st, hipStreamCreateWithFlags(&st->cap_stream, hipStreamNonBlocking));
    const hipStream_t user = st->stream;
    const uint64_t hs = st->host_step;
    const int cur0 = st->cur, prof = st->prof_on;
    st->stream = st->cap_stream;
    st->prof_on = 0;
    hipGraph_t g = nullptr;
    int rc = PIC1D_OK;
    hipError_t e = hipStreamBeginCapture(st->cap_stream, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
        for (int i = 0; i < st->graph_len && rc == PIC1D_OK; ++i) rc = enqueue_step(st);
        const hipError_t e2 = hipStreamEndCapture(st->cap_stream, &g);
        if (e2 != hipSuccess) e = e2;
    }
    st->stream = user;
    st->host_step = hs;
    st->cur = cur0;
    st->prof_on = prof;
    if (rc != PIC1D_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(st, PIC1D_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&st->gexec[cur0], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        st->gexec[cur0] = nullptr;
        return fail(st, PIC1D_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    return PIC1D_OK;
}

// Steps per graph for a request: a multiple of the sort interval, so that every
// replay starts at the same point of the sort cycle.
int graph_length(const pic1d_state* st, int requested) {
    if (requested <= 0) return 0;
    const int S = st->cfg.sort_interval;
    return S > 0 ? ((requested + S - 1) / S) * S : requested;
}

}  // namespace

extern "C" {

int pic1d_step(pic1d_state* st, int32_t n_steps) {
    if (!st || n_steps < 0) return fail(st, PIC1D_EINVAL, "bad arguments");
    if (st->frozen) return fail(st, PIC1D_ESTATE, "state frozen by an earlier error");
    int32_t i = 0;
    const int G = st->graph_len;
    if (G > 0 && !st->prof_on) {
        // eager up to the next multiple of G, then whole graphs
        while (i < n_steps && st->host_step % (uint64_t)G != 0) {
            if (int rc = enqueue_step(st)) return rc;
            ++i;
        }
        const int S = st->cfg.sort_interval;
        const int flips = S > 0 ? (G / S) & 1 : 0;
        while (n_steps - i >= G) {
            if (!st->gexec[st->cur])
                if (int rc = capture_graph(st)) return rc;
            HIP_TRY(st, hipGraphLaunch(st->gexec[st->cur], st->stream));
            st->host_step += (uint64_t)G;
            st->cur ^= flips;
            i += G;
        }
    }
    for (; i < n_steps; ++i)
        if (int rc = enqueue_step(st)) return rc;
    HIP_TRY(st, hipGetLastError());
    const int rc = check_error(st);
    prof_collect(st);
    return rc;
}

int pic1d_set_graph(pic1d_state* st, int32_t steps_per_graph) {
    if (!st || steps_per_graph < 0) return fail(st, PIC1D_EINVAL, "bad arguments");
    st->drop_graphs();
    st->graph_steps = steps_per_graph;
    st->graph_len = graph_length(st, steps_per_graph);
    return PIC1D_OK;
}

// Tile shape and block count of the particle kernel.  A new tile size re-plans the
// tiles of the live particles (the plan is in units of tiles); captured graphs hold
// the old arguments and are dropped.
int set_push_shape(pic1d_state* st, int blocks_per_cu, int ppt, int ww) {
    st->drop_graphs();
    st->push_blocks = st->n_cu * blocks_per_cu;
    const bool retile = ppt != st->ppt;
    st->ppt = ppt;
    st->ww = ww;
    if (retile) {
        if (int rc = launch_plan(st, 0)) return rc;
        HIP_TRY(st, hipGetLastError());
    }
    return PIC1D_OK;
}

int pic1d_set_push_shape(pic1d_state* st, int32_t blocks_per_cu, int32_t ppt, int32_t window) {
    if (!st || blocks_per_cu < 1 || blocks_per_cu > 32) return fail(st, PIC1D_EINVAL, "bad arguments");
    if (st->frozen) return fail(st, PIC1D_ESTATE, "state frozen by an earlier error");
    if (!push_kernel(st->backend, ppt, window)) return fail(st, PIC1D_EINVAL, "push shape not built");
    return set_push_shape(st, blocks_per_cu, ppt, window);
}

int pic1d_set_sort_granularity(pic1d_state* st, int32_t bins_per_cell) {
    if (!st || bins_per_cell < 1 || bins_per_cell > SORT_SUB_MAX || (bins_per_cell & (bins_per_cell - 1)) != 0)
        return fail(st, PIC1D_EINVAL, "bad arguments");
    if (st->frozen) return fail(st, PIC1D_ESTATE, "state frozen by an earlier error");
    // captured graphs hold the old bin count in their sort launches
    HIP_TRY(st, hipStreamSynchronize(st->stream));
    st->drop_graphs();
    st->sort_sub = bins_per_cell;
    return PIC1D_OK;
}

int pic1d_autotune(pic1d_state* st, int32_t trial_steps, pic1d_tune_out* out) {
    if (!st || trial_steps < 1 || !out) return fail(st, PIC1D_EINVAL, "bad arguments");
    if (st->frozen) return fail(st, PIC1D_ESTATE, "state frozen by an earlier error");
    hipEvent_t e0, e1;
    HIP_TRY(st, hipEventCreate(&e0));
    HIP_TRY(st, hipEventCreate(&e1));
    const int prof = st->prof_on;
    st->prof_on = 0;
    int trials = 0;
    // time `trial` real steps (at least one sort cycle) with the current shape
    // eager launches while tuning: graph capture would land in the timed steps
    auto measure = [&](double& ms_per_step) -> int {
        st->drop_graphs();
        st->graph_len = 0;
        const int S = st->cfg.sort_interval;
        const int n = std::max(trial_steps, S > 0 ? S : 0);
        if (int rc = pic1d_step(st, 1)) return rc;           // warm: capture or caches
        HIP_TRY(st, hipEventRecord(e0, st->stream));
        if (int rc = pic1d_step(st, n)) return rc;
        HIP_TRY(st, hipEventRecord(e1, st->stream));
        HIP_TRY(st, hipEventSynchronize(e1));
        float ms = 0.0f;
        HIP_TRY(st, hipEventElapsedTime(&ms, e0, e1));
        ms_per_step = ms / n;
        ++trials;
        return PIC1D_OK;
    };
    double base = 0.0;
    int rc = measure(base);
    double best = base;
    const int occ = std::max(1, st->push_blocks / std::max(st->n_cu, 1));
    // 0. tile shape of the particle kernel: particles per lane and deposit window
    {
        const int ppt0 = st->ppt, ww0 = st->ww;
        int best_ppt = ppt0, best_ww = ww0;
        double best_shape = base;
        const int cand_ppt[] = {4, 8, 16};
        // windows no smaller than the backend's own: a smaller one wins by a few percent
        // while each tile's particles stay close together, and loses half the speed once
        // the plasma heats, they spread between sorts and the tiles overflow it into
        // global atomics (the TABLE backend's 64 cells, reachable by pic1d_set_push_shape)
        const int wdef = default_window(st->backend);
        const int cand_ww[] = {wdef, 64};
        for (int p : cand_ppt)
            for (int w : cand_ww) {
                if (rc || (p == ppt0 && w == ww0) || w < wdef || !push_kernel(st->backend, p, w)) continue;
                rc = set_push_shape(st, occ, p, w);
                double t = 0.0;
                if (!rc) rc = measure(t);
                if (!rc && t < best_shape) { best_shape = t; best_ppt = p; best_ww = w; }
            }
        // the winner has to beat the starting shape again, timed alternately twice each
        if (!rc && (best_ppt != ppt0 || best_ww != ww0)) {
            double ta = 0.0, tb = 0.0;
            for (int rep = 0; rep < 2 && !rc; ++rep)
                for (int which = 0; which < 2 && !rc; ++which) {
                    rc = which ? set_push_shape(st, occ, best_ppt, best_ww) : set_push_shape(st, occ, ppt0, ww0);
                    double t = 0.0;
                    if (!rc) rc = measure(t);
                    (which ? tb : ta) += t;
                }
            if (!rc && ta <= tb) { best_ppt = ppt0; best_ww = ww0; }
            if (!rc) best = 0.5 * std::min(ta, tb);
        }
        if (!rc) rc = set_push_shape(st, occ, best_ppt, best_ww);
    }
    // 1. push blocks per CU
    const int bpc0 = occ;
    int best_bpc = bpc0;
    const int cand_bpc[] = {1, 2, 3, 4, 6, 8};
    for (int c : cand_bpc) {
        if (rc || c == bpc0 || c > 2 * occ + 2) continue;
        st->push_blocks = st->n_cu * c;
        double t = 0.0;
        rc = measure(t);
        if (!rc && t < best) { best = t; best_bpc = c; }
    }
    // the state drifts while the trials run (and one trial can be noisy): the winner
    // has to beat the starting shape again, timed alternately twice each
    if (!rc && best_bpc != bpc0) {
        double ta = 0.0, tb = 0.0;
        for (int rep = 0; rep < 2 && !rc; ++rep) {
            for (int which = 0; which < 2 && !rc; ++which) {
                st->push_blocks = st->n_cu * (which ? best_bpc : bpc0);
                double t = 0.0;
                rc = measure(t);
                (which ? tb : ta) += t;
            }
        }
        if (!rc) {
            if (ta <= tb) best_bpc = bpc0;
            best = 0.5 * std::min(ta, tb);
        }
    }
    st->push_blocks = st->n_cu * best_bpc;
    // 2. XCD-aware tile walk on or off
    if (!rc) {
        const int x0 = st->xcd_walk;
        st->xcd_walk = 1 - x0;
        double t = 0.0;
        rc = measure(t);
        if (!rc && t < best) best = t; else st->xcd_walk = x0;
    }
    // 3. sort interval (the result does not depend on the particle order)
    if (!rc) {
        const int s0 = st->cfg.sort_interval;
        int best_s = s0;
        // short intervals pay where pair creation appends many unsorted particles a step
        const int cand_s[] = {1, 2, 5, 10, 25, 50, 100};
        for (int c : cand_s) {
            if (rc || c == s0) continue;
            st->cfg.sort_interval = c;
            double t = 0.0;
            rc = measure(t);
            if (!rc && t < best) { best = t; best_s = c; }
        }
        st->cfg.sort_interval = best_s;
    }
    // 4. sort bins per cell (finer bins cost more counting but group the particles
    //    that cross a face more tightly; pays where sorts are rare)
    if (!rc && st->cfg.sort_interval > 0) {
        const int g0 = st->sort_sub;
        int best_g = g0;
        const int cand_g[] = {8, 16, 32};
        double best_t = best;
        for (int c : cand_g) {
            if (rc || c == g0) continue;
            st->sort_sub = c;
            double t = 0.0;
            rc = measure(t);
            if (!rc && t < best_t) { best_t = t; best_g = c; }
        }
        // (the gain is a percent or two: the winner has to beat the start again,
        // timed alternately twice each)
        if (!rc && best_g != g0) {
            double ta = 0.0, tb = 0.0;
            for (int rep = 0; rep < 2 && !rc; ++rep)
                for (int which = 0; which < 2 && !rc; ++which) {
                    st->sort_sub = which ? best_g : g0;
                    double t = 0.0;
                    rc = measure(t);
                    (which ? tb : ta) += t;
                }
            if (!rc) {
                if (ta <= tb) best_g = g0;
                best = std::min(best, 0.5 * std::min(ta, tb));
            }
        }
        st->sort_sub = best_g;
    }
    st->drop_graphs();
    st->graph_len = graph_length(st, st->graph_steps);
    st->prof_on = prof;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    out->push_blocks_per_cu = st->push_blocks / std::max(st->n_cu, 1);
    out->push_ppt = st->ppt;
    out->deposit_window = st->ww;
    out->xcd_walk = st->xcd_walk;
    out->sort_interval = st->cfg.sort_interval;
    out->sort_granularity = st->sort_sub;
    out->n_trials = trials;
    out->ms_per_step_before = base;
    out->ms_per_step_after = best;
    return PIC1D_OK;
}

int pic1d_profile(pic1d_state* st, int32_t enable) {
    if (!st) return fail(st, PIC1D_EINVAL, "bad arguments");
    HIP_TRY(st, hipStreamSynchronize(st->stream));
    prof_collect(st);
    for (int k = 0; k < 8; ++k) { st->prof_ms[k] = 0.0; st->prof_n[k] = 0; }
    st->prof_on = enable ? 1 : 0;
    return PIC1D_OK;
}

int pic1d_profile_read(pic1d_state* st, pic1d_profile_out* out) {
    if (!st || !out) return fail(st, PIC1D_EINVAL, "bad arguments");
    for (int k = 0; k < 8; ++k) { out->ms[k] = st->prof_ms[k]; out->launches[k] = st->prof_n[k]; }
    return PIC1D_OK;
}

int pic1d_moments(pic1d_state* st, int32_t line, int32_t flags, pic1d_moments_out* out) {
    if (!st || !out || line < 0 || line >= st->lay.n_lines) return fail(st, PIC1D_EINVAL, "bad arguments");
    const LineHost& lh = st->lines[line];
    const int n = lh.dev.n_cells, cb = lh.dev.cell_base;
    const hipStream_t s = st->stream;
    HIP_TRY(st, hipMemsetAsync(st->rho, 0, sizeof(unsigned long long) * (n + 1), s));
    HIP_TRY(st, hipMemsetAsync(st->mom_out, 0, 8 * sizeof(double), s));
    HIP_TRY(st, hipMemsetAsync(st->mom_kin, 0, 4 * sizeof(unsigned long long), s));
    MomArgs m{};
    m.cell = st->cell[st->cur]; m.off = st->off[st->cur]; m.u = st->u[st->cur];
    m.seg_base = st->seg_base; m.n_cur = st->n_cur; m.tile_prefix = st->tile_prefix; m.nseg = st->lay.nseg;
    m.tile = 64 * st->ppt;
    m.line = line; m.lines = st->dlines; m.E = st->E; m.rho = st->rho; m.out = st->mom_out;
    m.kin = st->mom_kin; m.part = st->mom_out + 8;
    const double sign[4] = {-1.0, 1.0, -1.0, 1.0};
    for (int k = 0; k < 4; ++k) m.sign[k] = sign[k];
    m.mass_ratio = st->cfg.mass_ratio;
    const int grid_blocks = std::max(1, std::min(MOM_GRID_BLOCKS, (n + 256) / 256));
    hipLaunchKernelGGL(k_moments_particles, dim3(st->aux_blocks), dim3(PUSH_TPB), 0, s, m);
    hipLaunchKernelGGL(k_moments_grid, dim3(grid_blocks), dim3(256), 0, s, m);
    double mo[8];
    std::vector<double> part(2 * (size_t)grid_blocks);
    unsigned long long kin[4];
    DevScalars sc{};
    long long avg = 0;
    std::vector<int32_t> ncur(4);
    std::vector<unsigned long long> cnt((size_t)NCOUNT * CNT_REPL);
    HIP_TRY(st, hipMemcpyAsync(mo, st->mom_out, sizeof(mo), hipMemcpyDeviceToHost, s));
    HIP_TRY(st, hipMemcpyAsync(part.data(), st->mom_out + 8, part.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(st, hipMemcpyAsync(kin, st->mom_kin, sizeof(kin), hipMemcpyDeviceToHost, s));
    HIP_TRY(st, hipMemcpyAsync(&sc, st->sc, sizeof(sc), hipMemcpyDeviceToHost, s));
    HIP_TRY(st, hipMemcpyAsync(&avg, st->avg_count, sizeof(avg), hipMemcpyDeviceToHost, s));
    HIP_TRY(st, hipMemcpyAsync(ncur.data(), st->n_cur + 4 * line, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(st, hipMemcpyAsync(cnt.data(), st->counters + (size_t)NCOUNT * CNT_REPL * line, cnt.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    const bool average = (flags & PIC1D_MOM_AVERAGE) != 0;
    std::vector<int32_t> hist(4 * (size_t)n);
    std::vector<long long> nsum, psum;
    std::vector<int32_t> plast;
    std::vector<double> E(n), jv(n);
    if (average) {
        nsum.resize(4 * (size_t)n);
        psum.resize(n);
        HIP_TRY(st, hipMemcpyAsync(nsum.data(), st->n_sum + 4 * (size_t)cb, nsum.size() * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(st, hipMemcpyAsync(psum.data(), st->pair_sum + cb, psum.size() * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(st, hipMemcpyAsync(E.data(), st->E_sum + cb, n * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(st, hipMemcpyAsync(jv.data(), st->j_sum + cb, n * 8, hipMemcpyDeviceToHost, s));
    } else {
        plast.resize(n);
        HIP_TRY(st, hipStreamSynchronize(s));
        HIP_TRY(st, hipMemcpyAsync(hist.data(), st->hist[sc.step & 1] + 4 * (size_t)cb, hist.size() * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(st, hipMemcpyAsync(plast.data(), st->pair_last + cb, n * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(st, hipMemcpyAsync(E.data(), st->E + cb, n * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(st, hipMemcpyAsync(jv.data(), st->j_last + cb, n * 8, hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(st, hipStreamSynchronize(s));
    const double Q = lh.dev.Q, C = lh.dev.C, ppc0 = st->cfg.ppc0;
    const double jn = ppc0 * Q * C;   // n0 e c in code units
    const double na = average ? (double)std::max(avg, 1ll) : 1.0;
    for (int sp = 0; sp < 4; ++sp)
        if (out->n_cell[sp])
            for (int c = 0; c < n; ++c)
                out->n_cell[sp][c] = (average ? (double)nsum[4 * (size_t)c + sp] : (double)hist[4 * (size_t)c + sp]) / (na * ppc0);
    if (out->j) for (int c = 0; c < n; ++c) out->j[c] = jv[c] / (na * jn);
    if (out->E) for (int c = 0; c < n; ++c) out->E[c] = E[c] / na;
    if (out->pair_rate)
        for (int c = 0; c < n; ++c) out->pair_rate[c] = average ? (double)psum[c] / na : (double)plast[c];
    // partial sums in block order (the same bits on every call)
    double esum = 0.0, e2 = 0.0;
    for (int b = 0; b < grid_blocks; ++b) {
        esum += part[2 * (size_t)b];
        e2 += part[2 * (size_t)b + 1];
    }
    // kinetic energy: the three 32-bit chunk sums of sum m (gamma - 1) / m_e * 2^48
    const unsigned __int128 ksum = (unsigned __int128)kin[0] + ((unsigned __int128)kin[1] << 32) +
                                   ((unsigned __int128)kin[2] << 64);
    out->gauss_residual = mo[0] / (4.0 * M_PI * Q * ppc0);
    out->v_circuit = -esum / (C * C);
    out->energy_kinetic = (double)ksum * 0x1.0p-48 * Q * C * C;
    out->energy_field = e2 / (8.0 * M_PI);
    for (int k = 0; k < 4; ++k) out->count[k] = 0;
    out->step = (int64_t)sc.step;
    out->avg_steps = avg;
    for (int k = 0; k < NCOUNT; ++k) {
        out->counters[k] = 0;
        for (int r = 0; r < CNT_REPL; ++r) out->counters[k] += (int64_t)cnt[(size_t)r * NCOUNT + k];
    }
    // live counts: the histogram of the current particles (absorbed ones excluded)
    {
        std::vector<int32_t> hc(4 * (size_t)n);
        HIP_TRY(st, copy_sync(st->stream, hc.data(), st->hist[sc.step & 1] + 4 * (size_t)cb, hc.size() * 4, hipMemcpyDeviceToHost));
        for (int c = 0; c < n; ++c)
            for (int k = 0; k < 4; ++k) out->count[k] += hc[4 * (size_t)c + k];
    }
    if (flags & PIC1D_MOM_RESET) {
        HIP_TRY(st, hipMemsetAsync(st->n_sum, 0, 4 * 8 * (size_t)st->lay.n_cells, s));
        HIP_TRY(st, hipMemsetAsync(st->pair_sum, 0, 8 * (size_t)st->lay.n_cells, s));
        HIP_TRY(st, hipMemsetAsync(st->E_sum, 0, 8 * (size_t)st->lay.n_cells, s));
        HIP_TRY(st, hipMemsetAsync(st->j_sum, 0, 8 * (size_t)st->lay.n_cells, s));
        HIP_TRY(st, hipMemsetAsync(st->avg_count, 0, 8, s));
        HIP_TRY(st, hipStreamSynchronize(s));
    }
    (void)ncur;
    return PIC1D_OK;
}

void pic1d_free(pic1d_state* st) { delete st; }

const char* pic1d_last_error(const pic1d_state* st) { return st ? st->err.c_str() : g_init_error.c_str(); }

int pic1d_get_particles(pic1d_state* st, int32_t line, int32_t species, int64_t capacity, int64_t* count,
                        int32_t* cell, float* offset, float* u, uint64_t* id) {
    if (!st || !count || line < 0 || line >= st->lay.n_lines || species < 0 || species > 3)
        return fail(st, PIC1D_EINVAL, "bad arguments");
    const int seg = 4 * line + species;
    int32_t n = 0;
    HIP_TRY(st, hipMemcpyAsync(&n, st->n_cur + seg, 4, hipMemcpyDeviceToHost, st->stream));
    HIP_TRY(st, hipStreamSynchronize(st->stream));
    const int64_t b = st->seg_base_h[seg];
    std::vector<int32_t> c(n);
    std::vector<float> o(n), uu(n);
    std::vector<uint64_t> ii(n);
    const int k = st->cur;
    if (n > 0) {
        HIP_TRY(st, copy_sync(st->stream, c.data(), st->cell[k] + b, 4 * (size_t)n, hipMemcpyDeviceToHost));
        HIP_TRY(st, copy_sync(st->stream, o.data(), st->off[k] + b, 4 * (size_t)n, hipMemcpyDeviceToHost));
        HIP_TRY(st, copy_sync(st->stream, uu.data(), st->u[k] + b, 4 * (size_t)n, hipMemcpyDeviceToHost));
        HIP_TRY(st, copy_sync(st->stream, ii.data(), st->id[k] + b, 8 * (size_t)n, hipMemcpyDeviceToHost));
    }
    int64_t live = 0;
    for (int32_t i = 0; i < n; ++i) live += (c[i] != DEAD_CELL);
    *count = live;
    if (live > capacity) return fail(st, PIC1D_EINVAL, "capacity of the output arrays too small");
    int64_t w = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (c[i] == DEAD_CELL) continue;
        if (cell) cell[w] = c[i];
        if (offset) offset[w] = o[i];
        if (u) u[w] = uu[i];
        if (id) id[w] = ii[i];
        ++w;
    }
    return PIC1D_OK;
}

int pic1d_set_particles(pic1d_state* st, int32_t line, int32_t species, int64_t count, const int32_t* cell,
                        const float* offset, const float* u, const uint64_t* id) {
    if (!st || line < 0 || line >= st->lay.n_lines || species < 0 || species > 3 || count < 0)
        return fail(st, PIC1D_EINVAL, "bad arguments");
    if (count > 0 && (!cell || !offset || !u || !id)) return fail(st, PIC1D_EINVAL, "NULL particle array");
    const int seg = 4 * line + species;
    if (count > st->seg_cap_h[seg]) return fail(st, PIC1D_ECAPACITY, "more particles than the species capacity");
    const int n = st->lines[line].dev.n_cells;
    for (int64_t i = 0; i < count; ++i)
        if (cell[i] < 0 || cell[i] >= n || !(offset[i] >= 0.0f && offset[i] < 1.0f) || !isfinite(u[i]))
            return fail(st, PIC1D_EINVAL, "particle outside the line or non-finite");
    const int64_t b = st->seg_base_h[seg];
    const int k = st->cur;
    if (count > 0) {
        HIP_TRY(st, copy_sync(st->stream, st->cell[k] + b, cell, 4 * (size_t)count, hipMemcpyHostToDevice));
        HIP_TRY(st, copy_sync(st->stream, st->off[k] + b, offset, 4 * (size_t)count, hipMemcpyHostToDevice));
        HIP_TRY(st, copy_sync(st->stream, st->u[k] + b, u, 4 * (size_t)count, hipMemcpyHostToDevice));
        HIP_TRY(st, copy_sync(st->stream, st->id[k] + b, id, 8 * (size_t)count, hipMemcpyHostToDevice));
    }
    const int32_t c32 = (int32_t)count;
    HIP_TRY(st, copy_sync(st->stream, st->alloc + seg, &c32, 4, hipMemcpyHostToDevice));
    launch_plan(st, 0);
    int rc = launch_hist(st);
    if (rc) return rc;
    HIP_TRY(st, hipStreamSynchronize(st->stream));
    return PIC1D_OK;
}

int pic1d_get_field(pic1d_state* st, int32_t line, double* E) {
    if (!st || !E || line < 0 || line >= st->lay.n_lines) return fail(st, PIC1D_EINVAL, "bad arguments");
    const LineDev& d = st->lines[line].dev;
    HIP_TRY(st, hipStreamSynchronize(st->stream));
    HIP_TRY(st, copy_sync(st->stream, E, st->E + d.cell_base, 8 * (size_t)d.n_cells, hipMemcpyDeviceToHost));
    return PIC1D_OK;
}

int pic1d_set_field(pic1d_state* st, int32_t line, const double* E) {
    if (!st || !E || line < 0 || line >= st->lay.n_lines) return fail(st, PIC1D_EINVAL, "bad arguments");
    const LineDev& d = st->lines[line].dev;
    for (int i = 0; i < d.n_cells; ++i)
        if (!isfinite(E[i])) return fail(st, PIC1D_EINVAL, "non-finite field value");
    HIP_TRY(st, hipStreamSynchronize(st->stream));
    HIP_TRY(st, copy_sync(st->stream, st->E + d.cell_base, E, 8 * (size_t)d.n_cells, hipMemcpyHostToDevice));
    std::vector<float> e32(E, E + d.n_cells);
    HIP_TRY(st, copy_sync(st->stream, st->E32 + d.cell_base, e32.data(), 4 * (size_t)d.n_cells, hipMemcpyHostToDevice));
    return PIC1D_OK;
}

int pic1d_set_step(pic1d_state* st, int64_t step) {
    if (!st || step < 0) return fail(st, PIC1D_EINVAL, "bad arguments");
    // the per-cell counts live in H[step & 1]; move them along with the counter
    HIP_TRY(st, hipStreamSynchronize(st->stream));
    DevScalars sc{};
    HIP_TRY(st, copy_sync(st->stream, &sc, st->sc, sizeof(sc), hipMemcpyDeviceToHost));
    const int from = (int)(sc.step & 1), to = (int)(step & 1);
    if (from != to) {
        const size_t bytes = 4 * sizeof(int32_t) * (size_t)st->lay.n_cells;
        HIP_TRY(st, copy_sync(st->stream, st->hist[to], st->hist[from], bytes, hipMemcpyDeviceToDevice));
        HIP_TRY(st, hipMemsetAsync(st->hist[from], 0, bytes, st->stream));
    }
    sc.step = (uint64_t)step;
    HIP_TRY(st, copy_sync(st->stream, st->sc, &sc, sizeof(sc), hipMemcpyHostToDevice));
    st->host_step = (uint64_t)step;
    return PIC1D_OK;
}

int pic1d_rics_line_info(pic1d_state* st, int32_t line, double* error, int32_t* uses_table) {
    if (!st || !error || !uses_table || line < 0 || line >= st->lay.n_lines) return fail(st, PIC1D_EINVAL, "bad arguments");
    *error = (st->lay.mlp_fallback && line < (int)st->mlp_error.size()) ? st->mlp_error[line] : -1.0;
    *uses_table = st->lines[line].dev.use_table;
    return PIC1D_OK;
}

int pic1d_rics_eval(pic1d_state* st, int32_t line, int64_t n, const float* s_cells, const float* u, float* F,
                    float* ndot, float* eps) {
    if (!st || line < 0 || line >= st->lay.n_lines || n < 0 || (n > 0 && (!s_cells || !u || !F || !ndot || !eps)))
        return fail(st, PIC1D_EINVAL, "bad arguments");
    if (n == 0) return PIC1D_OK;
    PushArgs a = push_args(st);
    const dim3 grid((unsigned)((n + 255) / 256));
    switch (st->backend) {
        case RICS_OFF: hipLaunchKernelGGL(k_rics_eval<RICS_OFF>, grid, dim3(256), 0, st->stream, a, line, n, s_cells, u, F, ndot, eps); break;
        case RICS_EXACT: hipLaunchKernelGGL(k_rics_eval<RICS_EXACT>, grid, dim3(256), 0, st->stream, a, line, n, s_cells, u, F, ndot, eps); break;
        case RICS_TABLE: hipLaunchKernelGGL(k_rics_eval<RICS_TABLE>, grid, dim3(256), 0, st->stream, a, line, n, s_cells, u, F, ndot, eps); break;
        case RICS_MLP: hipLaunchKernelGGL(k_rics_eval_mlp, grid, dim3(256), 0, st->stream, a, line, n, s_cells, u, F, ndot, eps); break;
        default: return fail(st, PIC1D_EINVAL, "unknown RICS backend");
    }
    HIP_TRY(st, hipGetLastError());
    HIP_TRY(st, hipStreamSynchronize(st->stream));
    return PIC1D_OK;
}

}  // extern "C"

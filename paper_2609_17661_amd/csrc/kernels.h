// Kernel argument blocks and launch constants shared by kernels.hip and api.hip.
#pragma once

#include "mlp_dev.h"
#include "pic1d_dev.h"

namespace pic1d {

enum { RICS_OFF = 0, RICS_EXACT = 1, RICS_TABLE = 2, RICS_MLP = 3 };

constexpr int PUSH_TPB = 256;                   // threads per block of the particle kernels
constexpr int PUSH_TPB_MLP = 256;               // ... with the surrogate network: one block per CU (its
                                                // weights fill the LDS), one wavefront per SIMD
constexpr int PUSH_PPT_DEFAULT = 8;             // consecutive particles per thread per tile: 4, 8 or 16
                                                // (a tile, 64 ppt particles, is one wavefront's work item;
                                                // the other particle kernels take a tile per block)
constexpr int CNT_REPL = 64;                    // replicas of every counter (spreads same-address atomics)
constexpr int SORT_SUB_DEFAULT = 8;             // sort key: cell and offset in eighths of a cell ...
constexpr int SORT_SUB_MAX = 32;                // ... or in up to 32 parts (a power of two)
constexpr int SCAN_CELLS = 256;                 // cells per chunk of the sort's scan (one block)

constexpr int GATHER_U = 4;                     // particles per thread and pass of the annihilation gather
constexpr int GATHER_BLOCKS_PER_CU = 16;        // its blocks per CU

constexpr int PHOTON_REPL = 256;                // append regions of the photon buffer (one per wavefront
                                                // slot of a block and block mod 64: spreads the reservations)

// A photon above the pair threshold, recorded by the pusher for the conversion kernel.
struct PhotonRec {
    uint64_t pid;     // emitting lepton
    int32_t line;
    int32_t cell;     // emission point: cell and offset (x^n)
    float off;
    float u_pre;      // lepton momentum before the recoil (sets gamma and eps)
    float b;          // B / B_QED at the emission point
    float mu;         // rest-frame emission cosine from the lepton's motion (0: perpendicular)
};

struct PushArgs {
    int32_t* cell;
    float* off;
    float* u;
    uint64_t* id;
    const int64_t* seg_base;
    const int32_t* seg_cap;
    const int32_t* n_cur;
    int32_t* alloc;
    const int32_t* tile_prefix;
    int32_t nseg;
    int32_t tile;              // particles per tile (64 ppt)
    int32_t nlg, ns;
    int32_t pairs, conversion, gravity;
    int32_t emission;          // PIC1D_EMIT_*
    const LineDev* lines;
    const float* E32;          // float32 copy of E (the gather needs no more)
    unsigned long long* J;
    const float4* nodes;
    const double* rc_nodes;
    const float4* table;       // RICS tables, [line][ns][nlg] {F(i), F(i+1), Ndot(i), Ndot(i+1)}
    int32_t* hist[2];          // per-cell counts, ping-pong by step parity
    int32_t* pair_step;
    unsigned long long* counters;   // [line][CNT_REPL][NCOUNT]
    DevScalars* sc;
    uint32_t key0, key1;
    float qm_ion;              // charge / mass of an ion (units of e/m_e)
    float inv_mass_ion;        // m_e / m_i
    PhotonRec* photons;        // PHOTON_REPL regions of photon_region slots
    int32_t* n_photons;        // [PHOTON_REPL] fill of each region
    int32_t photon_region;
    // surrogate network (RICS_MLP): bfloat16 forward tiles and biases, output normalisation
    const bf16x8* mlp_ft;
    const float* mlp_bias;
    float mlp_mean[3], mlp_std[3];
    float mlp_kTn;             // kT input, normalised to [-1, 1]
    int32_t xcd_walk;          // 1: each XCD walks a contiguous range of tiles (its own L2)
};

struct ConvertArgs {
    int32_t* cell;
    float* off;
    float* u;
    uint64_t* id;
    const int64_t* seg_base;
    const int32_t* seg_cap;
    int32_t* alloc;
    const LineDev* lines;
    const double* rc_nodes;
    int32_t* hist[2];
    int32_t* pair_step;
    unsigned long long* counters;
    DevScalars* sc;
    const PhotonRec* photons;
    const int32_t* n_photons;
    int32_t photon_region;
    int32_t conversion;
    uint32_t key0, key1;
};

struct AtmArgs {
    int32_t* cell;
    float* off;
    float* u;
    uint64_t* id;
    const int64_t* seg_base;
    const int32_t* seg_cap;
    int32_t* alloc;
    const LineDev* lines;
    int32_t* hist[2];
    const int32_t* layer_cell;     // global cells of all atmosphere layers
    const int32_t* layer_line;
    const int32_t* layer_target;   // hydrostatic target count per cell and species
    int32_t n_layer;
    unsigned long long* counters;
    DevScalars* sc;
    uint32_t key0, key1;
    float sig_e, sig_i;            // thermal spread of u for electrons and ions
};

struct BookArgs {
    int32_t* n_photons;        // reset to 0 for the next step (may be null)
    int32_t* n_cur;
    int32_t* alloc;
    const int32_t* seg_cap;
    int32_t* tile_prefix;
    int32_t nseg;
    int32_t tile;              // particles per tile (64 ppt)
    DevScalars* sc;
};

// Pair annihilation at the density limit (Sec. 3).  Per step, after the appends:
// k_annih_plan sizes every cell's annihilation from its end-of-step counts,
// k_annih_gather records the candidates (every e-/e+ of a cell over the limit),
// and k_field selects and removes them before Ampere.  The candidate records
// live in the particle buffer set the sort scatters into, idle between sorts.
struct AnnihArgs {
    int32_t* cell;              // the live particle buffer set
    float* off;
    float* u;
    const uint64_t* id;
    const int64_t* seg_base;
    const int32_t* seg_cap;
    const int32_t* alloc;       // slots in use per segment, appends included
    int32_t* hist[2];           // per-cell counts, ping-pong by step parity
    const int32_t* cell_line;
    const LineDev* lines;
    int32_t n_total;            // cells over all lines
    int32_t n_lines;
    int32_t* ann_k;             // per global cell: pairs to annihilate this step, 0 if none
    int32_t* ann_off;           // per global cell: first candidate record (e- then e+)
    int32_t* ann_fill;          // per global cell and species 0/1: candidates recorded
    int32_t* ann_ctl;           // [0] records allocated, [1] cells over the limit (this step),
                                //   [2] its copy for the field kernel
    uint64_t* cand_key;         // candidate records: ranking key ...
    int32_t* cand_slot;         // ... and slot within its species segment
    int64_t cand_cap;           // records available
    unsigned long long* J;
    unsigned long long* counters;
    uint32_t key0, key1;
    DevScalars* sc;
};

struct FieldArgs {
    double* E;
    float* E32;
    unsigned long long* J;
    double* j_last;
    int32_t* hist[2];
    int32_t* pair_step;
    int32_t* pair_last;
    double* E_sum;
    double* j_sum;
    long long* pair_sum;
    long long* n_sum;
    long long* avg_count;
    const int32_t* cell_line;
    const LineDev* lines;
    int32_t n_total;
    int32_t frozen;
    int64_t avg_start;
    DevScalars* sc;
    int32_t annihilation;       // 1: select and remove the planned annihilations first
    int32_t pad;
    AnnihArgs an;
};

struct SortArgs {
    int32_t* cell;
    float* off;
    float* u;
    uint64_t* id;
    int32_t* cell2;
    float* off2;
    float* u2;
    uint64_t* id2;
    const int64_t* seg_base;
    const int32_t* seg_cap;
    int32_t* n_cur;
    int32_t* alloc;
    const int32_t* tile_prefix;
    int32_t nseg;
    int32_t tile;              // particles per tile (64 ppt)
    const LineDev* lines;
    int32_t* hist[2];          // counts per cell and species; current = hist[step & 1]
    int4* bins;                // [cells * sub]: counts, then cursors, per species
    int4* chunk_sum;           // [n_chunks]: counts per chunk, then its first slot per species
    const int32_t* chunk_line; // [n_chunks]: line of each chunk of SCAN_CELLS cells
    const int32_t* line_chunk0;// [n_lines + 1]: first chunk of each line
    int32_t n_chunks;
    int32_t n_bins;            // cells * sub
    int32_t sub;               // sort bins per cell: a power of two up to SORT_SUB_MAX
    int32_t* new_count;        // [nseg]
    DevScalars* sc;
};

struct InitArgs {
    int32_t* cell;
    float* off;
    float* u;
    uint64_t* id;
    int64_t base_e, base_p;
    int64_t n_pairs;
    int32_t ppc, line, mode;
    double log10_gmax, u_stream;
    uint64_t id_base;
    uint32_t key0, key1;
};

struct HistArgs {
    const int32_t* cell;
    const int64_t* seg_base;
    const int32_t* n_cur;
    const int32_t* tile_prefix;
    int32_t nseg;
    int32_t tile;              // particles per tile (64 ppt)
    const LineDev* lines;
    int32_t* hist;
};

struct MomArgs {
    const int32_t* cell;
    const float* off;
    const float* u;
    const int64_t* seg_base;
    const int32_t* n_cur;
    const int32_t* tile_prefix;
    int32_t nseg;
    int32_t tile;              // particles per tile (64 ppt)
    int32_t line;
    const LineDev* lines;
    const double* E;
    unsigned long long* rho;   // fixed point, nodes of the line
    double* out;               // [0] maximum Gauss residual (bits, atomic max)
    unsigned long long* kin;   // [3]: sum of m (gamma - 1) / m_e at 2^-48, in 32-bit chunks (exact, any order)
    double* part;              // [MOM_GRID_BLOCKS][2]: per block sum E, sum E^2 (summed in block order on the host)
    double sign[4];
    double mass_ratio;
};

constexpr int MOM_GRID_BLOCKS = 256;          // blocks of k_moments_grid at most

// Finite-disk RICS table of one line (disk.hip): Gauss-Legendre product rule of
// n_c x n_phi nodes over the stellar disk, float64, written as float32 records.
constexpr int DISK_MAX_NODES = 32;
struct DiskTableArgs {
    float4* table;              // the line's [ns][nlg] records
    double R, b_pole, L;        // R_max / R*, B* / B_QED, line length (R*)
    double theta, AF, AN;       // kT / m_e c^2 and the prefactors of the radial beam
    int32_t nlg, ns, n_c, n_phi;
    double gc[DISK_MAX_NODES], wc[DISK_MAX_NODES];   // Gauss-Legendre on [-1, 1]: cos t
    double gp[DISK_MAX_NODES], wp[DISK_MAX_NODES];   // ... and phi
};
void gauss_legendre(int n, double* x, double* w);
hipError_t launch_disk_table(const DiskTableArgs& a, hipStream_t s);
constexpr int DISK_N_C = 24, DISK_N_PHI = 24;

// KIND: 0 every line; 1 only the lines on their table; 2 only the lines on the network
template <int BACKEND, int PPT, int WW, int KIND> __global__ void k_push(PushArgs a);
__global__ void k_mlp_pack(const float* p, bf16x8* ft, bf16x8* bt, float* bias);
// The surrogate's error estimate on every line: the largest relative error of
// F_hat and Ndot_hat against the float64 closed forms over the line's table nodes,
// as float bits in err[line] (0 before the launch).  row_geo: per line, per table
// row, (b, mu, x) at the row centre.
__global__ void k_mlp_line_error(PushArgs a, const double* row_geo, double kT_keV, unsigned int* err);
__global__ void k_rics_eval_mlp(PushArgs a, int line, int64_t n, const float* s_cells, const float* u, float* F,
                                float* N, float* eps);
__global__ void k_append(ConvertArgs ca, AtmArgs aa, int conv_blocks);
__global__ void k_plan(BookArgs b, int advance_step);
__global__ void k_field(FieldArgs f, BookArgs b);
__global__ void k_annih_plan(AnnihArgs a);
__global__ void k_annih_gather(AnnihArgs a);
__global__ void k_sort_zero(SortArgs s);
__global__ void k_sort_count(SortArgs s);
__global__ void k_sort_chunks(SortArgs s);
__global__ void k_sort_lines(SortArgs s);
__global__ void k_sort_cursors(SortArgs s);
__global__ void k_sort_scatter(SortArgs s);
__global__ void k_sort_finish(SortArgs s);
__global__ void k_init_pairs(InitArgs a);
__global__ void k_hist(HistArgs h);
__global__ void k_moments_particles(MomArgs m);
__global__ void k_moments_grid(MomArgs m);
template <int BACKEND>
__global__ void k_rics_eval(PushArgs a, int line, int64_t n, const float* s_cells, const float* u, float* F,
                            float* N, float* eps);

}  // namespace pic1d

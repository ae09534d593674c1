// Kernel argument blocks and launch constants shared by kernels.hip and api.hip.
#pragma once

#include "pic1d_dev.h"

namespace pic1d {

enum { RICS_OFF = 0, RICS_EXACT = 1, RICS_TABLE = 2, RICS_MLP = 3 };

constexpr int PUSH_TPB = 256;                   // threads per block of the particle kernels
constexpr int PUSH_PPT = 4;                     // particles per thread per tile
constexpr int PUSH_TILE = PUSH_TPB * PUSH_PPT;  // particles per tile

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
    int32_t nlg, ns;
    int32_t pairs, conversion, gravity;
    const LineDev* lines;
    const double* E;
    unsigned long long* J;
    const float4* nodes;
    const double* rc_nodes;
    const float* table;
    int32_t* hist[2];          // per-cell counts, ping-pong by step parity
    const int32_t* hist_in;    // set in the kernel: counts at the start of the step
    int32_t* hist_out;         // set in the kernel: counts of the new positions
    int32_t* pair_step;
    unsigned long long* counters;   // [line][8]
    DevScalars* sc;
    uint64_t step;             // set in the kernel from sc->step
    uint32_t key0, key1;
    float qm[4];               // charge / mass per species (units of e/m_e)
    double sign[4];            // charge sign per species
    float inv_mass[4];         // m_e / m per species
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
    int32_t* n_cur;
    int32_t* alloc;
    const int32_t* seg_cap;
    int32_t* tile_prefix;
    int32_t nseg;
    DevScalars* sc;
};

struct FieldArgs {
    double* E;
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
    const LineDev* lines;
    int32_t* hist[2];          // counts per cell and species; current = hist[step & 1]
    int32_t* cursor;           // [cells][4]
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
    int32_t line;
    const LineDev* lines;
    const double* E;
    unsigned long long* rho;   // fixed point, nodes of the line
    double* out;               // [0] residual max, [1] sum E, [2] kinetic energy, [3] sum E^2
    double sign[4];
    double mass_ratio;
};

template <int BACKEND> __global__ void k_push(PushArgs a);
__global__ void k_atmosphere(AtmArgs a);
__global__ void k_plan(BookArgs b, int advance_step);
__global__ void k_field(FieldArgs f);
__global__ void k_sort_scan(SortArgs s);
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

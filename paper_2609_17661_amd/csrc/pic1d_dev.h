// Device-side data layout and small device helpers of the pic1d library.
//
// Memory layout in HBM (all carved from the caller's workspace):
//   particles, structure of arrays over all (line, species) segments:
//     cell  int32   cell index within the line, DEAD_CELL once absorbed
//     off   float   offset in [0, 1) inside the cell
//     u     float   gamma * beta along +s
//     id    uint64  particle id (keys the Philox draws)
//   segment k = 4 * line + species owns slots [seg_base[k], seg_base[k] + seg_cap[k]).
//   grid, concatenated over lines (global cell g = cell_base[line] + local cell):
//     E     double  field at cell centres (faces k + 1/2)
//     J     int64   current deposit of the running step, fixed point 2^-32 cell
//     hist  int32[2][cells][4]  live particles per cell and species (ping-pong by step parity)
//   nodes (n_cells + 1 per line): float4 {b, mu, x = r/R*, R_curv in R*} and R_curv as double.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic1d {

constexpr int32_t DEAD_CELL = INT32_MIN;
constexpr int NSPEC = 4;
constexpr int NCOUNT = 16;                        // counters per line
constexpr double FIX_SCALE = 4294967296.0;        // 2^32: fixed point of the current deposit
constexpr double FIX_INV = 1.0 / 4294967296.0;
// Positions enter the deposit and the charge density quantised to 2^-28 cell
// (exact for offsets >= 1/16, where float32 spacing is at least that); one
// quantum is 2^4 fixed-point units of the current.
constexpr int POS_BITS = 28;
constexpr float POS_SCALE = 268435456.0f;          // 2^28
constexpr int POS_TO_FIX = 4;                      // 2^(32 - POS_BITS) as a shift
constexpr float Y_CUT = 80.0f;                    // Planck factors vanish beyond y = 80

// Philox stream tags (fourth counter word of each draw).
constexpr uint32_t STREAM_INIT = 1, STREAM_RICS = 2, STREAM_CHILD = 3,
                   STREAM_ATM_A = 4, STREAM_ATM_B = 5, STREAM_ATM_ID = 6, STREAM_ANNIH = 7;
constexpr uint64_t HASHED_ID_BIT = 1ull << 63;

// Per-line constants, precomputed on the host in FP64.
struct LineDev {
    int32_t cell_base;    // first global cell
    int32_t n_cells;
    int32_t node_base;    // first global node = cell_base + line index
    int32_t table_off;    // float4 offset of this line's RICS table
    float C, invC;        // cells per step at c, and its inverse
    float h;              // one step in R*/c
    float tau_hat;        // tau_min in R*/c
    float damp;           // 1 - exp(-1/(2 tau_min[steps])) of the damping branch
    float A_F, A_N;       // RICS prefactors r_e R* Theta^{3,2} / (4 lambdabar^2)
    float inv_theta;      // m_e c^2 / kT
    float b_thr;
    float grav;           // T C / h_atm: |du| per step of a unit-mass particle in the layer
    float nmax;           // n_max per cell (all species)
    float half_n;         // n_cells / 2
    int32_t use_table;    // 1: the line's RICS comes from its table (TABLE backend, or the
                          //    MLP backend where the network's error estimate exceeds the tolerance)
    int32_t pad_ut;
    float lgk;            // table: (nlg - 1)/16 log10(2): fractional column per unit log2 gamma^2
    float pad_lgk[2];
    float s_scale_f;      // table: s_scale in float32 (rows per cell)
    double s_scale;       // table: ns / n_cells
    double lg_scale;      // table: (nlg - 1) / 8
    double atm_depth;     // gravity layer depth (cells from each wall)
    double inv_ds;        // cells per R*
    double j_tw;          // twist current, code units
    double Q;             // macro-particle charge
    double amp_scale;     // 4 pi Q 2^-32: Ampere increment per fixed-point unit
};

struct DevScalars {
    uint64_t step;        // steps taken; keys Philox
    int32_t err;          // first error code (pic1d_status), 0 if none
    int32_t pad;
    uint64_t step_field;  // the running step, as k_field reads it (k_field advances `step`)
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32->64 multiplies
// by 0xD2511F53 and 0xCD9E8D57 with the key bumped by the Weyl constants
// 0x9E3779B9 / 0xBB67AE85 between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ float uniform24(uint32_t w) { return (float)(w >> 8) * 0x1.0p-24f; }
__device__ __forceinline__ float uniform24_open0(uint32_t w) { return (float)((w >> 8) + 1u) * 0x1.0p-24f; }
__device__ __forceinline__ uint64_t id_from_words(uint32_t lo, uint32_t hi) {
    return ((uint64_t)hi << 32 | lo) | HASHED_ID_BIT;
}

__device__ __forceinline__ void set_error(int* err, int code) { atomicCAS(err, 0, code); }

}  // namespace pic1d

// HIP kernels (gfx950) of one PIC step and its bookkeeping.
//
// Step pipeline on one stream:
//   k_push        gather, RICS drag / events, kick, move, fixed-point current
//                 deposit (LDS window per tile), per-cell histogram of the new
//                 positions, pair injection by append
//   k_append      photon conversion into pairs and refill of the surface
//                 layers, both by append
//   k_field       Ampere E -= 4 pi (j - j_twist), averages
//   k_plan        live counts, tile plan of the next push, step counter
//   k_sort_*      every sort_interval steps: counting sort by position (cell and
//                 eighth of a cell) per segment, dropping absorbed particles
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.h"
#include "rics_dev.h"

namespace pic1d {

// ---------------------------------------------------------------------------
// small wave / block reductions (wavefront of 64 lanes)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Data that the running kernel never writes (segment tables, line constants),
// read at a wave-uniform index: through the constant address space the compiler
// issues scalar loads into SGPRs instead of holding the values in VGPRs.
template <typename T>
__device__ __forceinline__ auto kconst(const T* p) {
#if defined(__HIP_DEVICE_COMPILE__)
    return (const __attribute__((address_space(4))) T*)(p);
#else
    return p;
#endif
}

// Segment of a global tile index by binary search over the tile prefix.
template <typename P>
__device__ __forceinline__ int find_segment(P prefix, int nseg, int t) {
    int lo = 0, hi = nseg;           // prefix[lo] <= t < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// XCD-aware tile walk: the 8 XCDs each take a contiguous range of tiles (blocks
// are dispatched round-robin over XCDs, so block b runs on XCD b % 8).
// Same walk at wavefront granularity: wavefront w of block b takes tile slots of
// its XCD's range.
struct WaveWalk {
    int t, end, stride;
    __device__ WaveWalk(int total, int xcd = 1) {
        const int wpb = blockDim.x >> 6;
        const int nb = gridDim.x >> 3;
        // wave-uniform: keeps every per-tile quantity in scalar registers
        const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        if (!xcd || nb == 0 || (gridDim.x & 7) != 0) {
            t = blockIdx.x * wpb + wid; end = total; stride = gridDim.x * wpb;
            return;
        }
        const int x = blockIdx.x & 7, lw = (blockIdx.x >> 3) * wpb + wid;
        const int chunk = (total + 7) >> 3;
        t = x * chunk + lw;
        end = min(total, (x + 1) * chunk);
        stride = nb * wpb;
    }
};

struct TileWalk {
    int t, end, stride;
    __device__ TileWalk(int total) {
        const int nb = gridDim.x >> 3;
        const int x = blockIdx.x & 7, lb = blockIdx.x >> 3;
        if (nb == 0 || (gridDim.x & 7) != 0) { t = blockIdx.x; end = total; stride = gridDim.x; return; }
        const int chunk = (total + 7) >> 3;
        t = x * chunk + lb;
        end = min(total, (x + 1) * chunk);
        stride = nb;
    }
};

// Geometry of a particle at cell c0, offset f: linear between the two nodes.
__device__ __forceinline__ Geo geo_lerp(const LineDev& L, const float4& a, const float4& b, float f) {
    Geo g;
    g.b = fmaf(f, b.x - a.x, a.x);
    g.mu = fmaf(f, b.y - a.y, a.y);
    const float xr = fmaf(f, b.z - a.z, a.z);
    g.ix2 = frcp(xr * xr);
    g.by = g.b * L.inv_theta;
    return g;
}

__device__ __forceinline__ Geo geo_at(const LineDev& L, const float4* __restrict__ nodes, int node, float f) {
    const float4 a = nodes[node];
    const float4 b = nodes[node + 1];
    Geo g;
    g.b = fmaf(f, b.x - a.x, a.x);
    g.mu = fmaf(f, b.y - a.y, a.y);
    const float xr = fmaf(f, b.z - a.z, a.z);
    g.ix2 = frcp(xr * xr);
    g.by = g.b * L.inv_theta;
    return g;
}

// What the RICS evaluations of one particle share: its geometry and (table
// backend) its table rows.
struct PartGeo {
    Geo g;
    TabRows rows;
    TabMemo memo;
};

// The line's table and its second row (row j0 + 1 at the same byte offset).
__device__ __forceinline__ const char* tab_base(const PushArgs& a, const LineDev& L) {
    return reinterpret_cast<const char*>(a.table + L.table_off);
}

// F_hat at u with what dF/du needs (evaluated only where the midpoint asks for it).
template <int BACKEND>
__device__ __forceinline__ auto rics_eval(const PushArgs& a, const LineDev& L, float u, PartGeo& pg) {
    if constexpr (BACKEND == RICS_TABLE) {
        const char* tb = tab_base(a, L);
        return table_eval(L, tb, tb + 16 * a.nlg, a.nlg, pg.rows, u, pg.memo);
    } else {
        return exact_eval(L, u, pg.g);
    }
}
__device__ __forceinline__ float eval_dF(const LineDev& L, const TableEval& e) { return e.dF(L); }
__device__ __forceinline__ float eval_dF(const LineDev&, const ExactEval& e) { return e.dF(); }

template <int BACKEND>
__device__ __forceinline__ float rics_N(const PushArgs& a, const LineDev& L, float u, PartGeo& pg) {
    if constexpr (BACKEND == RICS_TABLE) {
        const char* tb = tab_base(a, L);
        return table_N(L, tb, tb + 16 * a.nlg, a.nlg, pg.rows, u, pg.memo);
    } else {
        return exact_N(L, u, pg.g);
    }
}

// Geometry and table rows of a particle at x = c0 + o0 in float64 (the general
// form; the pusher forms the rows per cell where it can).
template <int BACKEND>
__device__ __forceinline__ PartGeo part_geo(const PushArgs& a, const LineDev& L, const float4& n0, const float4& n1,
                                            int c0, float o0) {
    PartGeo pg;
    pg.g = geo_lerp(L, n0, n1, o0);
    if constexpr (BACKEND == RICS_TABLE) pg.rows = table_rows(L, a.ns, 16 * a.nlg, (double)c0 + (double)o0);
    return pg;
}

// Newton-Raphson on u1 - u0 - (h/4)(F(u0) + F(u1)) = 0 from the explicit start
// (kept out of line: it is rarely needed at these step sizes).
template <int BACKEND>
__device__ __forceinline__ float newton_midpoint(const PushArgs& a, const LineDev& L, float u0, float F0, float u1,
                                              PartGeo& g) {
    const float hq = 0.25f * L.h;
#pragma unroll 1
    for (int it = 0; it < 4; ++it) {
        const auto e1 = rics_eval<BACKEND>(a, L, u1, g);
        const float G = u1 - u0 - hq * (F0 + e1.F);
        const float del = G / (1.0f - hq * eval_dF(L, e1));
        u1 -= del;
        if (fabsf(del) <= 0x1.0p-24f * fabsf(u1)) break;
    }
    return u1;
}

// One drag update over h/2 (Sec. 3): implicit midpoint where |F(p0)| tau_min <= |p0|,
// solved by Newton from the explicit start p0 + (h/2) F(p0) -- needed only when
// the predicted correction (h/4)|F'|(h/2)|F0| exceeds half an ulp of the result,
// F' taken at p0 -- and exponential relaxation towards p_tilde = mu / (1 - mu^2)^(1/2)
// otherwise.
template <int BACKEND>
__device__ __forceinline__ float drag_half(const PushArgs& a, const LineDev& L, float u0, PartGeo& g,
                                           float ptilde, bool alive, int& n_limited, int& n_newton) {
    const auto e0 = rics_eval<BACKEND>(a, L, u0, g);
    const float F0 = e0.F;
    const bool implicit = fabsf(F0) * L.tau_hat <= fabsf(u0);
    float u1 = implicit ? fmaf(0.5f * L.h, F0, u0) : fmaf(-(u0 - ptilde), L.damp, u0);
    n_limited += (alive && !implicit) ? 1 : 0;
    // F = 0 beyond the Planck cutoff (cold particles): the explicit start is the root
    if (implicit && F0 != 0.0f &&
        0.25f * L.h * fabsf(eval_dF(L, e0)) * 0.5f * L.h * fabsf(F0) > 0x1.0p-25f * fabsf(u1)) {
        n_newton += alive ? 1 : 0;
        u1 = newton_midpoint<BACKEND>(a, L, u0, F0, u1, g);
    }
    return u1;
}

// Per-tile constants of the pusher (species of the tile, step, count buffers).
struct TileCtx {
    uint64_t step;
    const int32_t* hist_in;     // counts at the start of the step
    int32_t* hist_out;          // counts of the new positions
    float qm;                   // charge / mass of the species (units of e/m_e)
    float inv_mass;             // m_e / m
    bool negative;              // negative charge
    bool gravity;               // the tile touches an atmosphere layer
};

// Append one particle to a segment; returns false (and flags ECAPACITY) if full.
__device__ __forceinline__ bool append_particle(const PushArgs& a, int seg, int cell, float off, float u,
                                                uint64_t id) {
    const int slot = atomicAdd(&a.alloc[seg], 1);
    if (slot >= a.seg_cap[seg]) {
        set_error(&a.sc->err, -3);
        return false;
    }
    const int64_t k = a.seg_base[seg] + slot;
    a.cell[k] = cell;
    a.off[k] = off;
    a.u[k] = u;
    a.id[k] = id;
    return true;
}

struct Counts {
    int events = 0, pairs = 0, escaped = 0, absorbed = 0, clipped = 0, limited = 0, newton = 0, pushed = 0,
        draws = 0, mlp = 0, pushed_ion = 0, mlp_need = 0;
};

// Stochastic regime (b >= b_thr, Sec. 3): after the kick, a scattering event with
// probability min(Ndot h, 1) from the Philox draw keyed by (step, id); the event
// emits eps = gamma (1 - (1+2b)^-1/2) and leaves gamma / (1+2b)^1/2 (Appendix A), or,
// with an angular emission pattern, the photon leaves the excited lepton's rest frame
// at the cosine drawn from the block's other words.
__device__ __forceinline__ float stochastic_step(const PushArgs& a, const LineDev& L, const TileCtx& T, int line,
                                              int64_t k, int c0, float o0, float u, const Geo& g, float ndot,
                                              Counts& cnt) {
    const float lam = ndot * L.h;
    if (lam > 1.0f) ++cnt.clipped;
    if (!(lam > 0.0f)) return u;
    ++cnt.draws;
    const uint64_t pid = a.id[k];
    const uint4 w = philox4x32_10(make_uint4((uint32_t)T.step, (uint32_t)pid, (uint32_t)(pid >> 32), STREAM_RICS),
                                  a.key0, a.key1);
    if (!(uniform24(w.x) < fminf(lam, 1.0f))) return u;
    ++cnt.events;
    const float gam = fsqrt(fmaf(u, u, 1.0f));
    const float dir = (u >= 0.0f) ? 1.0f : -1.0f;
    const float u_pre = u;
    float eps, mu_r = 0.0f;
    if (a.emission == 0) {
        eps = photon_energy(gam, g.b);
        const float gnew = gam * frsq(fmaf(2.0f, g.b, 1.0f));
        u = dir * fsqrt(fmaxf((gnew - 1.0f) * (gnew + 1.0f), 0.0f));
    } else {
        mu_r = emission_cosine(w, a.emission);
        eps = angled_event(gam, g.b, mu_r, dir, u);
    }
    if (a.pairs && eps >= 2.0f) {
        // record for the conversion kernel; lanes of a wavefront reserve their slots together
        const unsigned long long m = __ballot(1);
        const int lane = threadIdx.x & 63;
        const int leader = __ffsll((long long)m) - 1;
        const int r = (int)((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) & (PHOTON_REPL - 1));
        int slot0 = 0;
        if (lane == leader) slot0 = atomicAdd(&a.n_photons[r], __popcll(m));
        const int slot = __shfl(slot0, leader, 64) + __popcll(m & ((1ull << lane) - 1ull));
        if (slot < a.photon_region) {
            PhotonRec& p = a.photons[(size_t)r * a.photon_region + slot];
            p.pid = pid;
            p.line = line;
            p.cell = c0;
            p.off = o0;
            p.u_pre = u_pre;
            p.b = g.b;
            p.mu = mu_r;
        } else {
            set_error(&a.sc->err, -3);
        }
    } else {
        ++cnt.escaped;
    }
    return u;
}

// ---------------------------------------------------------------------------
// Surrogate-network RICS (RICS_MLP).  The network runs on the matrix cores for
// the 64 particles of a wavefront at once (four groups of 16 samples), so every
// lane must reach each evaluation: the callers below are wave-uniform.
// ---------------------------------------------------------------------------
struct MlpRics {
    float F, N;
};

// F_hat and Ndot_hat at momentum u of a particle with geometry g at arc-length
// fraction sl (x / n): the network gives G = |F_hat| / |gamma mu - u| and Ndot at
// (log10 gamma, s/L of the particle or of its mirror point, log10 b, kT);
// F_hat = (gamma mu - u) G, and both vanish beyond the Planck cutoff.
__device__ __forceinline__ MlpRics mlp_rics(const PushArgs& a, const bf16x8* W, const float* Wb, float u,
                                            const Geo& g, float sl, int& n_eval) {
    const int lane = threadIdx.x & 63, g4 = lane >> 4, r = lane & 15;
    ++n_eval;
    const float ua = fabsf(u);
    const float gam = fsqrt(fmaf(ua, ua, 1.0f));
    constexpr float LOG10_2 = 0.301029995663981f;
    float xn[4];
    xn[0] = __builtin_amdgcn_logf(gam) * (LOG10_2 * 0.25f) - 1.0f;
    xn[1] = fmaf(u >= 0.0f ? sl : 1.0f - sl, 2.0f, -1.0f);
    xn[2] = fmaf(__builtin_amdgcn_logf(g.b) * LOG10_2 + 2.0f, 0.4f, -1.0f);
    xn[3] = a.mlp_kTn;
    float o0 = 0.0f, o1 = 0.0f;
#pragma unroll 1
    for (int G = 0; G < 4; ++G) {
        float xg[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) xg[k] = __shfl(xn[k], 16 * G + r, 64);
        const bf16x8 bin = mlp_input_operand(xg, g4);
        const f32x4 out = mlp_group_forward<false>(W, Wb, bin, nullptr, 0, 0);
        const float v0 = __shfl(out[0], r, 64), v1 = __shfl(out[1], r, 64);
        if (g4 == G) {
            o0 = v0;
            o1 = v1;
        }
    }
    constexpr float LOG2_10 = 3.32192809488736f;
    const float y = g.by * frcp(fmaf(-u, g.mu, gam));
    const bool inside = y <= Y_CUT;
    MlpRics res;
    res.F = inside ? fmaf(gam, g.mu, -u) * exp2f(fmaf(a.mlp_std[0], o0, a.mlp_mean[0]) * LOG2_10) : 0.0f;
    res.N = inside ? exp2f(fmaf(a.mlp_std[1], o1, a.mlp_mean[1]) * LOG2_10) : 0.0f;
    return res;
}

// Drag half step with the surrogate force F0 = F(u0) (Sec. 3): damping branch where
// |F0| tau_min > |u0|; otherwise the implicit midpoint u1 = u0 + (h/4)(F0 + F(u1)),
// from the explicit start and refined by fixed-point iteration (contraction
// (h/4)|F'| << 1 on this branch) where (h/2)|F0| exceeds 2^-12 |u0|, until the
// next correction, predicted from the secant slope, is below half an ulp.  The
// network gives no derivative without another evaluation, so the gate is on F0
// alone: a skipped correction is (h/4)|F'| (h/2)|F0| / (1 - (h/4)|F'|), at most
// 2^-12 (|F'| h/4) / (1 - |F'| h/4) |u0| -- below half an ulp of u0 while
// |F'| h/4 < 2^-13, and within the 1e-5 momentum budget while |F'| h/4 < 0.04.
// Lanes with active == false return u0 but still take part in the network
// evaluations.
__device__ __forceinline__ float mlp_drag_half(const PushArgs& a, const bf16x8* W, const float* Wb, const LineDev& L,
                                               float u0, float F0, const Geo& g, float sl, float ptilde, bool active,
                                               bool alive, Counts& cnt) {
    const bool implicit = fabsf(F0) * L.tau_hat <= fabsf(u0);
    float u1 = implicit ? fmaf(0.5f * L.h, F0, u0) : fmaf(-(u0 - ptilde), L.damp, u0);
    cnt.limited += (active && alive && !implicit) ? 1 : 0;
    bool refine = active && implicit && F0 != 0.0f && 0.5f * L.h * fabsf(F0) > 0x1.0p-12f * fabsf(u0);
    cnt.newton += (refine && alive) ? 1 : 0;
#pragma unroll 1
    for (int it = 0; it < 4; ++it) {
        if (__ballot(refine) == 0ull) break;
        cnt.mlp_need += (refine && alive) ? 1 : 0;
        const float F1 = mlp_rics(a, W, Wb, u1, g, sl, cnt.mlp).F;
        const float un = fmaf(0.25f * L.h, F0 + F1, u0);
        // the next correction would be (h/4) F' (un - u1); F' from the secant through
        // the evaluations at u0 and u1.  Stop once it is below half an ulp of un.
        const float du = u1 - u0;
        const float slope = du != 0.0f ? (F1 - F0) / du : 0.0f;
        const bool more = 0.25f * L.h * fabsf(slope) * fabsf(un - u1) > 0x1.0p-25f * fabsf(un);
        u1 = refine ? un : u1;
        refine = refine && more;
    }
    return active ? u1 : u0;
}

// Field and geometry of the cell a lane is working in.  A lane's particles are
// consecutive in cell order, so the cache is reloaded only when the cell changes.
// The kick q E / (m C) is kept as its value at the cell centre and its change per
// cell towards the neighbouring centres, whose E is clamped at the walls (the
// gather is constant beyond the outermost cell centres).  The table backend
// keeps the per-cell part of the particle's table rows: for offset o the row
// position is rows0.pos.wj + o s_scale (u >= 0) and rows0.neg.wj - o s_scale
// (mirrored), valid for the whole cell where rows_simple (the cell lies between
// two rows, clear of the clamped ends).
struct CellCache {
    int cell;
    float K0, KsL, KsU;
    float4 n0, n1;          // geometry nodes c, c+1
    TabRows rows0;
    bool rows_simple;
    TabMemo memo;           // the lane's last table record (reset per tile)
};

template <int BACKEND>
__device__ __forceinline__ void cache_load(CellCache& cc, const PushArgs& a, const LineDev& L, float qmC, int c0) {
    cc.cell = c0;
    const float* E = a.E32 + L.cell_base;
    const float Em = E[max(c0 - 1, 0)];
    const float E0 = E[c0];
    const float Ep = E[min(c0 + 1, L.n_cells - 1)];
    cc.K0 = qmC * E0;
    cc.KsL = qmC * (E0 - Em);
    cc.KsU = qmC * (Ep - E0);
    if constexpr (BACKEND != RICS_OFF) {
        cc.n0 = a.nodes[L.node_base + c0];
        cc.n1 = a.nodes[L.node_base + c0 + 1];
    }
    if constexpr (BACKEND == RICS_TABLE) {
        const double sc = L.s_scale;
        const double fp = fma((double)c0, sc, -0.5);
        const double fn = fma((double)(L.n_cells - c0), sc, -0.5);
        const double jp = floor(fp), jn = floor(fn);
        const double top = (double)(a.ns - 2);
        constexpr double M = 0x1.0p-20;      // margin for the float32 row weight
        cc.rows_simple = jp >= 0.0 && jp <= top && fp + sc <= jp + 1.0 - M &&
                         jn >= 0.0 && jn <= top && fn - sc >= jn + M;
        const int nlg16 = 16 * a.nlg;
        cc.rows0.pos.off = cc.rows_simple ? (int)jp * nlg16 : 0;
        cc.rows0.pos.wj = (float)(fp - jp);
        cc.rows0.neg.off = cc.rows_simple ? (int)jn * nlg16 : 0;
        cc.rows0.neg.wj = (float)(fn - jn);
    }
}

// Everything one particle does in one step: gather, RICS, kick, move, and the
// deposit of its path in fixed point.  Written without data-dependent branches on
// the common path.  Dead slots (absorbed particles and the padding of a partial
// tile) enter at o0 = 1/2, u = 0, are held at u = 0, and so stay in their cell and
// deposit nothing.  c0 is the cached cell.
// Returns the new cell (DEAD_CELL when absorbed or dead) in c1, d = c1 - c0 in
// {-1, 0, 1}, and the path's overlaps with cells c0-1, c0, c0+1 in units of 2^-28
// cell (unsigned by the charge; jm and jp vanish unless the path leaves the cell).
template <int BACKEND>
__device__ __forceinline__ void advance_particle(const PushArgs& a, const LineDev& L, const TileCtx& T,
                                                 CellCache& cc, bool alive, int line, int sp, int64_t k,
                                                 int c0, float o0, float& u, Counts& cnt, int& c1, float& o1,
                                                 int& jm, int& j0, int& jp, int& d, bool& gone, const bf16x8* W,
                                                 const float* Wb) {
    const int n = L.n_cells;
    constexpr bool RICS = BACKEND != RICS_OFF;

    // field gather: E at x^n, linear between cell centres (as the kick per step)
    const float ws = o0 - 0.5f;
    float kick = fmaf(ws, ws >= 0.0f ? cc.KsU : cc.KsL, cc.K0);
    if (T.gravity) {
        const double x = (double)c0 + (double)o0;
        const double dw = fmin(x, (double)n - x);
        const float gk = ((x < (double)L.half_n) ? -1.0f : 1.0f) * L.grav * T.inv_mass;
        kick += (dw <= L.atm_depth) ? gk : 0.0f;
    }

    if constexpr (BACKEND == RICS_MLP) {
        if (sp != 3) {            // wave-uniform: a tile holds one species
            const Geo g = geo_lerp(L, cc.n0, cc.n1, o0);
            const float sl = (float)(((double)c0 + (double)o0) / (double)n);
            const bool cont = g.b < L.b_thr;
            const float pt = g.mu * frsq(fmaxf(fmaf(-g.mu, g.mu, 1.0f), 1e-30f));
            // the force at u^n is needed only in the continuous regime: a wavefront with
            // no live lane there skips the first evaluation (the step needs F at u^n and
            // at the kicked u in that regime, Ndot at the kicked u in the stochastic one)
            const bool any_cont = __ballot(cont && alive) != 0ull;
            cnt.mlp_need += alive ? (cont ? 2 : 1) : 0;
            if (any_cont) {
                const MlpRics ra = mlp_rics(a, W, Wb, u, g, sl, cnt.mlp);
                u = mlp_drag_half(a, W, Wb, L, u, ra.F, g, sl, pt, cont, alive, cnt);
            }
            u += kick;
            const MlpRics rb = mlp_rics(a, W, Wb, u, g, sl, cnt.mlp);
            if (any_cont) u = mlp_drag_half(a, W, Wb, L, u, rb.F, g, sl, pt, cont, alive, cnt);
            if (!cont && alive) u = stochastic_step(a, L, T, line, k, c0, o0, u, g, rb.N, cnt);
        } else {
            u += kick;
        }
    } else if (RICS && sp != 3) {
        PartGeo pg;
        pg.g = geo_lerp(L, cc.n0, cc.n1, o0);
        if constexpr (BACKEND == RICS_TABLE) {
            pg.memo = cc.memo;
            if (cc.rows_simple) {
                pg.rows.pos.off = cc.rows0.pos.off;
                pg.rows.pos.wj = fmaf(o0, L.s_scale_f, cc.rows0.pos.wj);
                pg.rows.neg.off = cc.rows0.neg.off;
                pg.rows.neg.wj = fmaf(-o0, L.s_scale_f, cc.rows0.neg.wj);
            } else {
                pg.rows = table_rows(L, a.ns, 16 * a.nlg, (double)c0 + (double)o0);
            }
        }
        if (pg.g.b < L.b_thr) {
            // continuous regime: Strang splitting drag h/2, Lorentz kick, drag h/2, both
            // at x^n; the damping branch relaxes towards p_tilde = mu / (1 - mu^2)^(1/2)
            const float pt = pg.g.mu * frsq(fmaxf(fmaf(-pg.g.mu, pg.g.mu, 1.0f), 1e-30f));
            u = drag_half<BACKEND>(a, L, u, pg, pt, alive, cnt.limited, cnt.newton);
            u += kick;
            u = drag_half<BACKEND>(a, L, u, pg, pt, alive, cnt.limited, cnt.newton);
        } else {
            u += kick;
            if (alive) u = stochastic_step(a, L, T, line, k, c0, o0, u, pg.g, rics_N<BACKEND>(a, L, u, pg), cnt);
        }
        if constexpr (BACKEND == RICS_TABLE) cc.memo = pg.memo;
    } else {
        u += kick;
    }
    u = alive ? u : 0.0f;      // (a non-finite u is reported once per tile by the caller)

    // move x^{n+1} = x^n + C u / gamma with the offset carried into the cell index
    // (|C u / gamma| < 1/2, so the carry is -1, 0 or 1 and o1 - carry is exact; o1 + 1
    // may round up to 1)
    const float o1r = fmaf(L.C * u, frsq(fmaf(u, u, 1.0f)), o0);
    const float carry = floorf(o1r);
    o1 = o1r - carry;
    const bool fix = o1 >= 1.0f;
    o1 = fix ? 0.0f : o1;
    d = (int)carry + (fix ? 1 : 0);
    c1 = c0 + d;
    // fixed-point deposit of the path from the stored old and new offsets quantised
    // to 2^-28 cell: X1 is the new position relative to the old cell's left face.
    // Differences of quantised stored positions telescope, so the deposit equals the
    // change of the quantised charge density exactly.  The parts beyond a wall land
    // in cells -1 or n, which the flush drops.
    constexpr int ONE = 1 << POS_BITS;
    const int f0 = (int)(o0 * POS_SCALE);
    const int X1 = d * ONE + (int)(o1 * POS_SCALE);
    jm = min(X1, 0);
    j0 = min(max(X1, 0), ONE) - f0;
    jp = max(X1 - ONE, 0);
    const bool out = (unsigned)c1 >= (unsigned)n;
    cnt.absorbed += (alive && out) ? 1 : 0;
    gone = out || !alive;
    c1 = gone ? DEAD_CELL : c1;
}

__device__ __forceinline__ void counts_flush(unsigned long long* counters, int line, Counts& c) {
    const int v[12] = {c.events, c.pairs, c.escaped, c.absorbed, c.clipped, c.limited, c.newton, c.pushed, c.draws,
                       c.mlp, c.pushed_ion, c.mlp_need};
    const int slot[12] = {0, 1, 2, 3, 4, 5, 6, 8, 9, 10, 12, 13};
    const size_t rep = ((size_t)line * CNT_REPL + (blockIdx.x & (CNT_REPL - 1))) * NCOUNT;
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        const int s = wave_sum_i(v[i]);
        if ((threadIdx.x & 63) == 0 && s != 0) atomicAdd(&counters[rep + slot[i]], (unsigned long long)s);
    }
    c = Counts();
}

// Waves per SIMD the particle kernel is compiled for, per backend.  A wavefront's
// LDS is its staged tile (768 bytes per particle per lane: 6 KB at 8) plus its
// deposit window (12 bytes per cell): at 8 particles per lane and 128 cells five
// 256-thread blocks fit a CU (five waves per SIMD, what the table backend's
// registers allow), at 32 cells six (the closed-form and field-only backends, in
// 80 registers with at most a few spilled).  The tile (4, 8 or 16 particles per
// lane) and the window (cells) are template parameters picked by the autotuner;
// tiles whose cells span more than the window deposit through global atomics.
constexpr int push_waves(int backend) {
    return backend == RICS_MLP ? 1 : backend == RICS_TABLE ? 5 : 6;
}

// Sorting network on PPT keys (ascending): the 19-comparator network for 8, five
// comparators for 4, Batcher's bitonic network for 16.
template <int PPT>
__device__ __forceinline__ void sort_keys(uint32_t* k) {
    auto cx = [&](int i, int j) {
        const uint32_t x = k[i], y = k[j];
        k[i] = min(x, y);
        k[j] = max(x, y);
    };
    if constexpr (PPT == 4) {
        cx(0, 1); cx(2, 3); cx(0, 2); cx(1, 3); cx(1, 2);
    } else if constexpr (PPT == 8) {
        constexpr int NET[19][2] = {{0, 2}, {1, 3}, {4, 6}, {5, 7}, {0, 4}, {1, 5}, {2, 6}, {3, 7}, {0, 1}, {2, 3},
                                    {4, 5}, {6, 7}, {2, 4}, {3, 5}, {1, 4}, {3, 6}, {1, 2}, {3, 4}, {5, 6}};
#pragma unroll
        for (int e = 0; e < 19; ++e) cx(NET[e][0], NET[e][1]);
    } else {
#pragma unroll
        for (int size = 2; size <= PPT; size <<= 1)
#pragma unroll
            for (int stride = size >> 1; stride > 0; stride >>= 1)
#pragma unroll
                for (int i = 0; i < PPT; ++i) {
                    const int j = i ^ stride;
                    if (j > i) {
                        if ((i & size) == 0) cx(i, j);
                        else cx(j, i);
                    }
                }
    }
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// The particle kernel.  Work is split into tiles of 64 PPT consecutive particles
// of one (line, species) segment, one tile per wavefront at a time, PPT
// consecutive particles per lane (128-bit loads and stores).  Each lane
// accumulates its deposit and new-cell counts over runs of particles in the same
// cell (three cells wide: the run's cell and its neighbours); each wavefront
// merges its lanes in a private LDS window and flushes the window to the global
// fixed-point current with one atomic per touched cell.  No block-level
// synchronisation.
template <int BACKEND, int PPT, int WW, int KIND>
__global__ __launch_bounds__(BACKEND == RICS_MLP ? PUSH_TPB_MLP : PUSH_TPB)
__attribute__((amdgpu_waves_per_eu(push_waves(BACKEND)))) void k_push(PushArgs a) {
    static_assert(PPT == 4 || PPT == 8 || PPT == 16, "4, 8 or 16 particles per lane");
    constexpr int TILE = 64 * PPT;
    constexpr int TPB = BACKEND == RICS_MLP ? PUSH_TPB_MLP : PUSH_TPB;
    __shared__ unsigned long long sJ[TPB / 64][WW];
    __shared__ int sH[TPB / 64][WW];
    __shared__ int sPc[TPB / 64][PPT][64];      // the wave's tile: cell, offset, momentum
    __shared__ float sPo[TPB / 64][PPT][64];
    __shared__ float sPu[TPB / 64][PPT][64];
    // surrogate weights, staged once per block (the network runs on them for every particle)
    __shared__ bf16x8 sW[BACKEND == RICS_MLP ? FT_TOTAL * 64 : 1];
    __shared__ float sWb[BACKEND == RICS_MLP ? MLP_BIAS : 1];
    if constexpr (BACKEND == RICS_MLP) {
        // before the error check: every wave of the block reaches the barrier
        for (int e = threadIdx.x; e < FT_TOTAL * 64; e += TPB) sW[e] = a.mlp_ft[e];
        for (int e = threadIdx.x; e < MLP_BIAS; e += TPB) sWb[e] = a.mlp_bias[e];
        __syncthreads();
    }
    if (a.sc->err != 0) return;
    const uint64_t step = a.sc->step;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.sc->step_field = step;
    const int32_t* hist_in = (step & 1) ? a.hist[1] : a.hist[0];
    int32_t* hist_out = (step & 1) ? a.hist[0] : a.hist[1];
    const int total = a.tile_prefix[a.nseg];
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    Counts cnt;
    int cur_line = -1;
    int seg = 0, seg_t0 = 0, seg_t1 = 0;       // segment of the previous tile and its tile range
    // The next tile's particles are fetched (vector loads into registers) before the
    // current tile's results are stored and its deposit window flushed, so that the
    // loads are in flight while the stores and atomics drain.
    WaveWalk ww(total, a.xcd_walk);
    int f_seg = 0, f_ib = 0, f_nv = 0;
    bool f_full = false;
    int64_t f_base = 0;
    int4 fc[PPT / 4];
    float4 fo[PPT / 4], fu[PPT / 4];
    // (every call assigns all fetched values, so that none stays live across the loop)
    auto fetch = [&](int t) {
        const bool have = t < ww.end;
        if (have && (t < seg_t0 || t >= seg_t1)) {
            seg = find_segment(kconst(a.tile_prefix), a.nseg, t);
            seg_t0 = kconst(a.tile_prefix)[seg];
            seg_t1 = kconst(a.tile_prefix)[seg + 1];
        }
        f_seg = seg;
        f_base = kconst(a.seg_base)[seg];
        // this lane's PPT consecutive particles (vector loads; slots up to the
        // capacity, a multiple of 256, always exist)
        const int t0 = (t - seg_t0) * TILE;
        const int ncur = kconst(a.n_cur)[seg];
        f_full = have && ncur - t0 >= TILE;        // wave-uniform
        f_ib = t0 + lane * PPT;
        f_nv = have ? max(0, min(PPT, ncur - f_ib)) : 0;
        const int4* cp = reinterpret_cast<const int4*>(a.cell + f_base + f_ib);
        const float4* op = reinterpret_cast<const float4*>(a.off + f_base + f_ib);
        const float4* up = reinterpret_cast<const float4*>(a.u + f_base + f_ib);
#pragma unroll
        for (int h = 0; h < PPT / 4; ++h) {
            fc[h] = make_int4(DEAD_CELL, DEAD_CELL, DEAD_CELL, DEAD_CELL);
            fo[h] = make_float4(0.5f, 0.5f, 0.5f, 0.5f);
            fu[h] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (f_nv > 0) { fc[h] = cp[h]; fo[h] = op[h]; fu[h] = up[h]; }
        }
    };
    fetch(ww.t);
    for (; ww.t < ww.end; ww.t += ww.stride) {
        const int tseg = f_seg, ib = f_ib, nv = f_nv;
        const int64_t base = f_base;
        const int line = tseg >> 2, sp = tseg & 3;
        if (line != cur_line) {
            if (cur_line >= 0) counts_flush(a.counters, cur_line, cnt);
            cur_line = line;
        }
        const LineDev L = kconst(a.lines)[line];
        // the surrogate's states with lines on both sources push them in two launches
        // (table lines at the table kernel's occupancy): a tile of the other kind is
        // left to the other launch
        if constexpr (KIND != 0) {
            if ((L.use_table != 0) != (KIND == 1)) {
                fetch(ww.t + ww.stride);
                continue;
            }
        }
        // the fetched particles, staged in the wave's LDS slots [q][lane] so the
        // particle loop indexes them freely without bank conflicts.  Dead slots are
        // stored as (DEAD_CELL, 1/2, 0); the padding of a partial tile is made so.
        // The lane's cell range: DEAD_CELL is the largest cell as unsigned and the
        // smallest as signed, so neither bound sees it.
        unsigned lo_u = 0xffffffffu;
        int hi_s = INT32_MIN;
        int cst[PPT];
        auto stage = [&](auto full) {
#pragma unroll
            for (int h = 0; h < PPT / 4; ++h) {
                const int4 ci = fc[h];
                const float4 oi = fo[h], ui = fu[h];
                const int cv[4] = {ci.x, ci.y, ci.z, ci.w};
                const float ov[4] = {oi.x, oi.y, oi.z, oi.w}, uv[4] = {ui.x, ui.y, ui.z, ui.w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int q = 4 * h + i;
                    const bool valid = decltype(full)::value || q < nv;
                    const int c = valid ? cv[i] : DEAD_CELL;
                    cst[q] = c;
                    lo_u = min(lo_u, (unsigned)c);
                    hi_s = max(hi_s, c);
                    sPc[wid][q][lane] = c;
                    sPo[wid][q][lane] = valid ? ov[i] : 0.5f;
                    sPu[wid][q][lane] = valid ? uv[i] : 0.0f;
                }
            }
        };
        if (f_full) stage(std::true_type{});
        else stage(std::false_type{});
        const bool lane_any = hi_s >= 0;
        const int first = lane_any ? (int)lo_u : 0;
        // the first cell's cache, loaded early so that its latency hides under the
        // tile set-up below
        const float qmC = ((sp == 0 || sp == 2) ? -1.0f : (sp == 1 ? 1.0f : a.qm_ion)) * L.invC;
        CellCache cc;
        cache_load<BACKEND>(cc, a, L, qmC, first);
        // The order in which the lane visits its slots: by cell (dead slots last), so
        // that the run accumulator and the cell cache see each cell once however the
        // particles of a cell are ordered in memory.  A sorting network on keys
        // (cell - first) * 2^VB + slot; the slot order is packed in VB-bit fields.
        // Slots already in that order (as unsigned, DEAD_CELL is the largest) keep
        // it; the network runs when any lane of the wavefront needs it.
        constexpr int VB = PPT == 4 ? 2 : PPT == 8 ? 3 : 4;
        using Visit = std::conditional_t<PPT == 16, uint64_t, uint32_t>;
        constexpr Visit IN_ORDER = [] {
            Visit v = 0;
            for (int q = 0; q < PPT; ++q) v |= (Visit)q << (VB * q);
            return v;
        }();
        Visit visit = IN_ORDER;
        bool ordered = true;
#pragma unroll
        for (int q = 1; q < PPT; ++q) ordered = ordered && (uint32_t)cst[q] >= (uint32_t)cst[q - 1];
        if (__ballot(!ordered) != 0ull) {
            visit = 0;
            uint32_t k[PPT];
#pragma unroll
            for (int q = 0; q < PPT; ++q)
                k[q] = (cst[q] == DEAD_CELL ? (0xffffffffu << VB) : (uint32_t)(cst[q] - first) << VB) | (uint32_t)q;
            sort_keys<PPT>(k);
#pragma unroll
            for (int q = 0; q < PPT; ++q) visit |= (Visit)(k[q] & ((1u << VB) - 1u)) << (VB * q);
        }
        // window [lo, hi] of cells this wavefront's deposit can touch: in a tile in
        // position order, the first lane's lowest and the last lane's highest cell;
        // checked, and reduced over the wavefront where that guess fails
        const int lane_lo = lane_any ? (int)lo_u - 1 : INT32_MAX;
        const int lane_hi = lane_any ? hi_s + 1 : INT32_MIN;
        int lo = __builtin_amdgcn_readfirstlane(lane_lo);
        int hi = __builtin_amdgcn_readlane(lane_hi, 63);
        if (__ballot(lane_lo < lo || lane_hi > hi) != 0ull) {
            lo = wave_min_i(lane_lo);
            hi = wave_max_i(lane_hi);
        }
        const bool any = lo <= hi;
        lo = any ? max(lo, 0) : 0;
        hi = any ? min(hi, L.n_cells - 1) : -1;
        const bool use_lds = any && (hi - lo + 1) <= WW;
        const int span = use_lds ? (hi - lo + 1) : 0;
        for (int cc = lane; cc < span; cc += 64) {
            sJ[wid][cc] = 0ull;
            sH[wid][cc] = 0;
        }
        wave_sync();

        TileCtx T;
        T.step = step;
        T.hist_in = hist_in;
        T.hist_out = hist_out;
        T.negative = (sp == 0 || sp == 2);
        T.qm = T.negative ? -1.0f : (sp == 1 ? 1.0f : a.qm_ion);
        T.inv_mass = (sp == 3) ? a.inv_mass_ion : 1.0f;
        T.gravity = a.gravity && any && ((double)lo <= L.atm_depth + 1.0 ||
                                         (double)(L.n_cells - 1 - hi) <= L.atm_depth + 1.0);
        unsigned long long* Jg = a.J + L.cell_base;
        int* Hg = hist_out + 4 * (size_t)L.cell_base + sp;
        // per-lane run accumulator over consecutive particles of one cell: deposits
        // (2^-28 cell) into cells key-1, key, key+1 and the new-cell counts of the same
        // three cells packed in 10-bit fields of hc
        int key = cc.cell;
        int jv0 = 0, jv1 = 0, jv2 = 0, hc = 0;
        // flush the lowest `ncells` cells of the run's three (all of them, or only
        // key-1 when the next run starts in key+1 and the other two carry over)
        auto flush_run = [&](int ncells) {
            const int jv[3] = {jv0, jv1, jv2};
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const int cell = key - 1 + r;
                const int hv = (hc >> (10 * r)) & 1023;
                if (r < ncells && cell >= 0 && cell < L.n_cells) {
                    const long long j = (long long)(T.negative ? -jv[r] : jv[r]) << POS_TO_FIX;
                    if (use_lds) {
                        if (j != 0) atomicAdd(&sJ[wid][cell - lo], (unsigned long long)j);
                        if (hv != 0) atomicAdd(&sH[wid][cell - lo], hv);
                    } else {
                        if (j != 0) atomicAdd(&Jg[cell], (unsigned long long)j);
                        if (hv != 0) atomicAdd(&Hg[4 * (size_t)cell], hv);
                    }
                }
            }
        };
        bool nonfinite = false;
#pragma unroll 1
        for (int q = 0; q < PPT; ++q) {
            const int slot = (int)(visit >> (VB * q)) & ((1 << VB) - 1);
            const int c0 = sPc[wid][slot][lane];
            const bool alive = c0 != DEAD_CELL;
            if (alive && c0 != cc.cell) {
                if (c0 == key + 1) {
                    // slide the run one cell up: key and key+1 carry over
                    flush_run(1);
                    jv0 = jv1;
                    jv1 = jv2;
                    jv2 = 0;
                    hc >>= 10;
                } else {
                    flush_run(3);
                    jv0 = jv1 = jv2 = hc = 0;
                }
                cache_load<BACKEND>(cc, a, L, qmC, c0);
                key = c0;
            }
            float uq = sPu[wid][slot][lane];
            const float oq = sPo[wid][slot][lane];
            int c1, d, jm, j0, jp;
            float o1;
            bool gone;
            advance_particle<BACKEND>(a, L, T, cc, alive, line, sp, base + ib + slot, cc.cell, oq, uq, cnt, c1, o1,
                                      jm, j0, jp, d, gone, sW, sWb);
            nonfinite = nonfinite || !isfinite(uq);
            cnt.pushed += alive ? 1 : 0;
            cnt.pushed_ion += (alive && sp == 3) ? 1 : 0;
            jv0 += jm;
            jv1 += j0;
            jv2 += jp;
            hc += alive ? (1 << (10 * (d + 1))) : 0;
            sPc[wid][slot][lane] = c1;
            sPo[wid][slot][lane] = gone ? 0.5f : o1;
            sPu[wid][slot][lane] = gone ? 0.0f : uq;
        }
        flush_run(3);
        if (nonfinite) set_error(&a.sc->err, -5);
        // write back (vector stores for full groups; never touch slots >= ncur, where
        // appended particles may be landing)
        if (nv == PPT) {
            int4* cp = reinterpret_cast<int4*>(a.cell + base + ib);
            float4* op = reinterpret_cast<float4*>(a.off + base + ib);
            float4* up = reinterpret_cast<float4*>(a.u + base + ib);
#pragma unroll
            for (int h = 0; h < PPT / 4; ++h) {
                cp[h] = make_int4(sPc[wid][4 * h][lane], sPc[wid][4 * h + 1][lane], sPc[wid][4 * h + 2][lane],
                                  sPc[wid][4 * h + 3][lane]);
                op[h] = make_float4(sPo[wid][4 * h][lane], sPo[wid][4 * h + 1][lane], sPo[wid][4 * h + 2][lane],
                                    sPo[wid][4 * h + 3][lane]);
                up[h] = make_float4(sPu[wid][4 * h][lane], sPu[wid][4 * h + 1][lane], sPu[wid][4 * h + 2][lane],
                                    sPu[wid][4 * h + 3][lane]);
            }
        } else {
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                if (q < nv) {
                    a.cell[base + ib + q] = sPc[wid][q][lane];
                    a.off[base + ib + q] = sPo[wid][q][lane];
                    a.u[base + ib + q] = sPu[wid][q][lane];
                }
            }
        }
        fetch(ww.t + ww.stride);
        // flush the window
        wave_sync();
        for (int cc2 = lane; cc2 < span; cc2 += 64) {
            const unsigned long long sj = sJ[wid][cc2];
            if (sj != 0ull) atomicAdd(&Jg[lo + cc2], sj);
            const int sh = sH[wid][cc2];
            if (sh != 0) atomicAdd(&Hg[4 * (size_t)(lo + cc2)], sh);
        }
        wave_sync();
    }
    if (cur_line >= 0) counts_flush(a.counters, cur_line, cnt);
}

// the shapes the autotuner chooses from: 4, 8 or 16 particles per lane, and two
// deposit windows per backend
template __global__ void k_push<RICS_OFF, 4, 32, 0>(PushArgs);
template __global__ void k_push<RICS_OFF, 8, 32, 0>(PushArgs);
template __global__ void k_push<RICS_OFF, 16, 32, 0>(PushArgs);
template __global__ void k_push<RICS_OFF, 8, 64, 0>(PushArgs);
template __global__ void k_push<RICS_EXACT, 4, 32, 0>(PushArgs);
template __global__ void k_push<RICS_EXACT, 8, 32, 0>(PushArgs);
template __global__ void k_push<RICS_EXACT, 16, 32, 0>(PushArgs);
template __global__ void k_push<RICS_EXACT, 8, 64, 0>(PushArgs);
template __global__ void k_push<RICS_TABLE, 4, 128, 0>(PushArgs);
template __global__ void k_push<RICS_TABLE, 8, 128, 0>(PushArgs);
template __global__ void k_push<RICS_TABLE, 16, 128, 0>(PushArgs);
template __global__ void k_push<RICS_TABLE, 8, 64, 0>(PushArgs);
template __global__ void k_push<RICS_MLP, 8, 32, 0>(PushArgs);
// the surrogate's states with lines on both sources: the table lines alone, the
// network lines alone
template __global__ void k_push<RICS_TABLE, 8, 128, 1>(PushArgs);
template __global__ void k_push<RICS_MLP, 8, 32, 2>(PushArgs);

// ---------------------------------------------------------------------------
// Photon conversion (Sec. 3): every recorded photon with E >= 2 m_e c^2 turns into
// an e-/e+ pair at gamma = eps/2 each where it converts -- at the emission point,
// or where the straight photon leaves the curved line by arcsin(2 m_e c^2/E) --
// if that point lies on the line and the cell's count at the start of the step
// is below n_max.  Float64 throughout: the member momenta are ill-conditioned in
// eps when eps/2 is close to 1.
// ---------------------------------------------------------------------------
// The records of all regions form one index space (regions in order); a block
// takes CONV_CHUNK consecutive records at a time, CONV_K per thread.  The slots of
// a chunk's pairs are reserved with one atomic per (block, line) on each
// allocation counter: those counters are single addresses that every block
// hits, and device-wide atomics on one address serialise.
constexpr int CONV_K = 4;
constexpr int CONV_CHUNK = 256 * CONV_K;
static_assert(PHOTON_REPL % 64 == 0 && PHOTON_REPL <= 256, "region fills: PHOTON_REPL / 64 per lane of one wave");

struct ConvRec {
    int line, cell;
    float off, up;
    uint64_t pid;
    bool valid, convert;
};

// The lab photon energy of an angled event in float64 (the arithmetic of
// angled_event); dir turns into the photon's direction along s, the lepton's sign
// times that of c + beta_e.
__device__ __forceinline__ double angled_photon(double gam, double q, double c, double& dir) {
    const double ge = gam / q;
    const double g2m1 = (ge - 1.0) * (ge + 1.0);
    const bool boost = g2m1 > 0.0;
    const double be = boost ? sqrt(g2m1) / ge : 0.0;
    const double omb = boost ? 1.0 / (ge * ge * (1.0 + be)) : 1.0;
    const double eg = (q - 1.0 / q) / (1.0 + sqrt(c * c + (1.0 - c) * (1.0 + c) / (q * q)));
    const double dopp = c >= 0.0 ? fma(be, c, 1.0) : fma(be, 1.0 + c, omb);
    if (c + be < 0.0) dir = -dir;
    return ge * eg * dopp;
}

__device__ __forceinline__ ConvRec convert_record(const ConvertArgs& a, const int32_t* hist_in, const PhotonRec& p,
                                                  bool valid) {
    ConvRec c;
    c.valid = valid;
    c.convert = false;
    c.line = valid ? p.line : INT32_MAX;
    c.cell = p.cell;
    c.off = p.off;
    c.up = 0.0f;
    c.pid = p.pid;
    if (!valid) return c;
    const LineDev& L = a.lines[p.line];
    const int n = L.n_cells;
    const double ud = (double)p.u_pre;
    const double qd = sqrt(1.0 + 2.0 * (double)p.b);
    double dir = ud >= 0.0 ? 1.0 : -1.0;
    const double eps = p.mu == 0.0f ? sqrt(1.0 + ud * ud) * (2.0 * (double)p.b) / (qd * (1.0 + qd))
                                    : angled_photon(sqrt(1.0 + ud * ud), qd, (double)p.mu, dir);
    bool ok = true;
    if (a.conversion != 0) {
        const double* rc = a.rc_nodes + L.node_base + p.cell;
        const double rcx = fma((double)p.off, rc[1] - rc[0], rc[0]);
        const double sp = (double)p.cell + (double)p.off + dir * rcx * L.inv_ds * asin(fmin(2.0 / eps, 1.0));
        ok = (sp >= 0.0) && (sp < (double)n);
        c.cell = ok ? (int)floor(sp) : 0;
        c.off = ok ? (float)(sp - (double)c.cell) : 0.0f;
        if (c.off >= 1.0f) { c.off = 0.0f; c.cell += 1; ok = ok && c.cell < n; }
    }
    if (ok) {
        const int* hc = hist_in + 4 * (size_t)(L.cell_base + c.cell);
        c.convert = (float)(hc[0] + hc[1] + hc[2] + hc[3]) < L.nmax;
        const double gp = 0.5 * eps;
        c.up = (float)(dir * sqrt(fmax((gp - 1.0) * (gp + 1.0), 0.0)));
    }
    return c;
}

// block-wide sum and exclusive prefix (in thread order) of one int per thread
__device__ __forceinline__ int block_scan(int v, int& total, int* s_part) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) s_part[w] = inc;
    __syncthreads();
    int before = 0;
    total = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int pk = s_part[k];
        before += (k < w) ? pk : 0;
        total += pk;
    }
    __syncthreads();
    return before + inc - v;
}

__device__ __forceinline__ void convert_photons(const ConvertArgs& a, int blk, int nblk) {
    __shared__ int s_pref[PHOTON_REPL + 1];    // exclusive prefix of the region fills
    __shared__ int s_part[4];
    __shared__ int s_base[2];
    const uint64_t step = a.sc->step;
    const int32_t* hist_in = (step & 1) ? a.hist[1] : a.hist[0];
    int32_t* hist_out = (step & 1) ? a.hist[0] : a.hist[1];
    const int lane = threadIdx.x & 63;
    constexpr int RPL = PHOTON_REPL / 64;      // regions per lane
    if (threadIdx.x < 64) {
        int f[RPL], sum = 0;
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            f[k] = min(a.n_photons[lane * RPL + k], a.photon_region);
            sum += f[k];
        }
        int inc = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(inc, o, 64);
            if (lane >= o) inc += t;
        }
        int run = inc - sum;
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            s_pref[lane * RPL + k] = run;
            run += f[k];
        }
        if (lane == 63) s_pref[PHOTON_REPL] = inc;
    }
    __syncthreads();
    const int total = s_pref[PHOTON_REPL];
    for (int c0 = blk * CONV_CHUNK; c0 < total; c0 += nblk * CONV_CHUNK) {
        ConvRec rec[CONV_K];
#pragma unroll
        for (int k = 0; k < CONV_K; ++k) {
            const int g = c0 + k * 256 + (int)threadIdx.x;
            const bool valid = g < total;
            PhotonRec p{};
            if (valid) {
                int lo = 0, hi = PHOTON_REPL;          // s_pref[lo] <= g < s_pref[hi]
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_pref[mid] <= g) lo = mid; else hi = mid;
                }
                p = a.photons[(size_t)lo * a.photon_region + (g - s_pref[lo])];
            }
            rec[k] = convert_record(a, hist_in, p, valid);
        }
        // one reservation per line present in the chunk, lowest line first
        while (true) {
            int m = INT32_MAX;
#pragma unroll
            for (int k = 0; k < CONV_K; ++k) m = min(m, rec[k].line);
            m = wave_min_i(m);
            if (lane == 0) s_part[threadIdx.x >> 6] = m;
            __syncthreads();
            const int gl = min(min(s_part[0], s_part[1]), min(s_part[2], s_part[3]));
            __syncthreads();
            if (gl == INT32_MAX) break;
            int mine = 0, seen = 0;
#pragma unroll
            for (int k = 0; k < CONV_K; ++k) {
                mine += (rec[k].line == gl && rec[k].convert) ? 1 : 0;
                seen += (rec[k].line == gl) ? 1 : 0;
            }
            int nconv = 0;
            const int before = block_scan(mine, nconv, s_part);
            int nseen = 0;
            block_scan(seen, nseen, s_part);
            if (threadIdx.x == 0) {
                s_base[0] = nconv > 0 ? atomicAdd(&a.alloc[4 * gl + 0], nconv) : 0;
                s_base[1] = nconv > 0 ? atomicAdd(&a.alloc[4 * gl + 1], nconv) : 0;
            }
            __syncthreads();
            const int base_e = s_base[0] + before, base_p = s_base[1] + before;
            __syncthreads();
            int made = 0, j = 0;
#pragma unroll
            for (int k = 0; k < CONV_K; ++k) {
                if (rec[k].line != gl) continue;
                if (rec[k].convert) {
                    const int se = base_e + j, spp = base_p + j;
                    ++j;
                    const bool e_ok = se < a.seg_cap[4 * gl + 0], p_ok = spp < a.seg_cap[4 * gl + 1];
                    if (!e_ok || !p_ok) set_error(&a.sc->err, -3);
                    const uint4 wc = philox4x32_10(make_uint4((uint32_t)step, (uint32_t)rec[k].pid,
                                                              (uint32_t)(rec[k].pid >> 32), STREAM_CHILD),
                                                   a.key0, a.key1);
                    if (e_ok) {
                        const int64_t q = a.seg_base[4 * gl + 0] + se;
                        a.cell[q] = rec[k].cell; a.off[q] = rec[k].off; a.u[q] = rec[k].up;
                        a.id[q] = id_from_words(wc.x, wc.y);
                    }
                    if (p_ok) {
                        const int64_t q = a.seg_base[4 * gl + 1] + spp;
                        a.cell[q] = rec[k].cell; a.off[q] = rec[k].off; a.u[q] = rec[k].up;
                        a.id[q] = id_from_words(wc.z, wc.w);
                    }
                    if (e_ok && p_ok) {
                        const LineDev& L = a.lines[gl];
                        int* ho = hist_out + 4 * (size_t)(L.cell_base + rec[k].cell);
                        atomicAdd(&ho[0], 1);
                        atomicAdd(&ho[1], 1);
                        atomicAdd(&a.pair_step[L.cell_base + rec[k].cell], 1);
                        ++made;
                    }
                }
                rec[k].line = INT32_MAX;      // done with this record
            }
            int n_made = 0;
            block_scan(made, n_made, s_part);
            if (threadIdx.x == 0) {
                const size_t rep = ((size_t)gl * CNT_REPL + (blk & (CNT_REPL - 1))) * NCOUNT;
                if (n_made) atomicAdd(&a.counters[rep + 1], (unsigned long long)n_made);
                if (nseen - n_made) atomicAdd(&a.counters[rep + 2], (unsigned long long)(nseen - n_made));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Atmosphere (Appendix B.1): every layer cell is refilled to its hydrostatic
// target with co-located (e-, ion) pairs; one wavefront per layer cell.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void refill_atmosphere(const AtmArgs& a, int blk, int nblk) {
    const uint64_t step = a.sc->step;
    int32_t* hist_out = a.hist[(step & 1) ^ 1];
    const int lane = threadIdx.x & 63;
    const int wglob = (blk * blockDim.x + threadIdx.x) >> 6;
    const int nw = (nblk * blockDim.x) >> 6;
    for (int e = wglob; e < a.n_layer; e += nw) {
        const int g = a.layer_cell[e];         // global cell
        const int line = a.layer_line[e];
        const int target = a.layer_target[e];
        int* h = hist_out + 4 * (size_t)g;
        const int have = min(h[2], h[3]);
        const int D = max(target - have, 0);
        if (D == 0) continue;
        const LineDev& L = a.lines[line];
        const int segE = 4 * line + 2, segI = 4 * line + 3;
        int baseE = 0, baseI = 0;
        if (lane == 0) {
            baseE = atomicAdd(&a.alloc[segE], D);
            baseI = atomicAdd(&a.alloc[segI], D);
        }
        baseE = __shfl(baseE, 0, 64);
        baseI = __shfl(baseI, 0, 64);
        if (baseE + D > a.seg_cap[segE] || baseI + D > a.seg_cap[segI]) {
            if (lane == 0) set_error(&a.sc->err, -3);
            continue;
        }
        const int c = g - L.cell_base;
        for (int kk = lane; kk < D; kk += 64) {
            const uint4 wa = philox4x32_10(make_uint4((uint32_t)step, (uint32_t)g, (uint32_t)kk, STREAM_ATM_A), a.key0, a.key1);
            const uint4 wb = philox4x32_10(make_uint4((uint32_t)step, (uint32_t)g, (uint32_t)kk, STREAM_ATM_B), a.key0, a.key1);
            const uint4 wc = philox4x32_10(make_uint4((uint32_t)step, (uint32_t)g, (uint32_t)kk, STREAM_ATM_ID), a.key0, a.key1);
            const float off = uniform24(wa.x);
            const float ue = a.sig_e * sqrtf(-2.0f * logf(uniform24_open0(wa.y))) * cospif(2.0f * uniform24(wa.z));
            const float ui = a.sig_i * sqrtf(-2.0f * logf(uniform24_open0(wb.x))) * cospif(2.0f * uniform24(wb.y));
            const int64_t ke = a.seg_base[segE] + baseE + kk;
            const int64_t ki = a.seg_base[segI] + baseI + kk;
            a.cell[ke] = c; a.off[ke] = off; a.u[ke] = ue; a.id[ke] = id_from_words(wc.x, wc.y);
            a.cell[ki] = c; a.off[ki] = off; a.u[ki] = ui; a.id[ki] = id_from_words(wc.z, wc.w);
        }
        if (lane == 0) {
            h[2] += D;
            h[3] += D;
            atomicAdd(&a.counters[((size_t)line * CNT_REPL + (blk & (CNT_REPL - 1))) * NCOUNT + 7],
                      (unsigned long long)D);
        }
    }
}

// The step's appends in one launch: blocks [0, conv_blocks) convert the recorded
// photons into pairs (species 0 and 1), the rest refill the atmosphere (species 2
// and 3).  The two touch different segments and different species counts, so they
// run side by side.
__global__ __launch_bounds__(256) void k_append(ConvertArgs ca, AtmArgs aa, int conv_blocks) {
    if (ca.sc->err != 0) return;
    if ((int)blockIdx.x < conv_blocks) convert_photons(ca, blockIdx.x, conv_blocks);
    else refill_atmosphere(aa, blockIdx.x - conv_blocks, gridDim.x - conv_blocks);
}

// Block-wide (256 threads) exclusive scan of one int; writes the block total.
__device__ __forceinline__ int block_excl_scan(int v, int& total) {
    __shared__ int sWave[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) sWave[w] = inc;
    __syncthreads();
    int before = 0;
    total = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int t = sWave[i];
        before += i < w ? t : 0;
        total += t;
    }
    __syncthreads();
    return before + inc - v;
}

// ---------------------------------------------------------------------------
// Per-step bookkeeping shared by k_field and k_plan: live counts <- allocation
// counters (clamped to capacity), tile plan of the next push.
// ---------------------------------------------------------------------------
__device__ void bookkeeping(const BookArgs& b) {
    if (b.sc->err != 0) return;
    if (b.n_photons && threadIdx.x < PHOTON_REPL) b.n_photons[threadIdx.x] = 0;
    const int nseg = b.nseg;
    const int per = (nseg + 255) / 256;
    const int s0 = threadIdx.x * per, s1 = min(s0 + per, nseg);
    int sum = 0, n_last = 0;
    for (int s = s0; s < s1; ++s) {
        const int n = min(b.alloc[s], b.seg_cap[s]);
        b.n_cur[s] = n;
        b.alloc[s] = n;
        n_last = n;
        sum += (n + b.tile - 1) / b.tile;
    }
    int total;
    int run = block_excl_scan(sum, total);
    for (int s = s0; s < s1; ++s) {
        b.tile_prefix[s] = run;
        // (one segment per thread up to 256 segments: its count is still in a register)
        run += ((per == 1 ? n_last : b.n_cur[s]) + b.tile - 1) / b.tile;
    }
    if (threadIdx.x == 255) b.tile_prefix[nseg] = total;
}

// Bookkeeping kernel of every step (and after init, sort, set_particles): one block.
__global__ __launch_bounds__(256) void k_plan(BookArgs b, int advance_step) {
    bookkeeping(b);
    if (advance_step && threadIdx.x == 0 && b.sc->err == 0) b.sc->step += 1;
}

// ---------------------------------------------------------------------------
// Pair annihilation at the density limit (Sec. 3: pairs annihilate where the
// total density approaches n_max, which keeps the skin depth resolved; the paper
// gives no mechanics, so these are readings).  A cell whose end-of-step count N
// of all particles exceeds n_max loses k = min(N-, N+, ceil((N - n_max)/2))
// e-/e+ pairs (species 0 and 1): the k of each species with the smallest
// (key, id), key the 64-bit Philox draw (step, id, STREAM_ANNIH), so the choice
// does not depend on where the particles sit in memory.  Each pair annihilates
// as if its positron first moved to its electron: the cell's face current gains
// sum q(x-) - sum q(x+) in the deposit's fixed point (the same quantised
// positions the push deposits from), and the neutral pair leaves no charge.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t annih_key(uint64_t step, uint64_t id, uint32_t k0, uint32_t k1) {
    const uint4 w = philox4x32_10(make_uint4((uint32_t)step, (uint32_t)id, (uint32_t)(id >> 32), STREAM_ANNIH),
                                  k0, k1);
    return ((uint64_t)w.y << 32) | (uint64_t)w.x;
}


// Every cell's k from its end-of-step counts, and for the cells over the limit a
// run of candidate records (their e- then their e+), one allocation per block.
__global__ __launch_bounds__(256) void k_annih_plan(AnnihArgs a) {
    if (a.sc->err != 0) return;
    const uint64_t step = a.sc->step;
    const int32_t* hist_out = a.hist[(step & 1) ^ 1];
    __shared__ int s_base;
    for (int g0 = blockIdx.x * 256; g0 < a.n_total; g0 += gridDim.x * 256) {
        const int g = g0 + (int)threadIdx.x;
        int k = 0, need = 0;
        if (g < a.n_total) {
            const int* h = hist_out + 4 * (size_t)g;
            const int h0 = h[0], h1 = h[1];
            const int N = h0 + h1 + h[2] + h[3];
            const double nmax = (double)a.lines[a.cell_line[g]].nmax;
            if ((double)N > nmax) k = (int)fmin(fmin((double)h0, (double)h1), ceil(((double)N - nmax) * 0.5));
            need = k > 0 ? h0 + h1 : 0;
        }
        int total = 0;
        const int excl = block_excl_scan(need, total);
        if (total > 0 && threadIdx.x == 0) {
            s_base = atomicAdd(&a.ann_ctl[0], total);
            atomicOr(&a.ann_ctl[1], 1);
        }
        __syncthreads();
        if (k > 0) {
            const int64_t off = (int64_t)s_base + excl;
            if (off + need > a.cand_cap || off + need > (int64_t)INT32_MAX) {
                set_error(&a.sc->err, -3);
                k = 0;
            } else {
                a.ann_off[g] = (int)off;
                a.ann_fill[2 * (size_t)g] = 0;
                a.ann_fill[2 * (size_t)g + 1] = 0;
            }
        }
        if (g < a.n_total) a.ann_k[g] = k;
        __syncthreads();
    }
}

__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}

// Candidates per lane held in registers by the register selection (at most
// 64 * ANNIH_KPL candidates of a species); larger cells take the radix select
// over the records in memory.
constexpr int ANNIH_KPL = 8;
constexpr int ANNIH_EXTRACT_K = 8;

// The `k` smallest (key, id) of one species' m candidates, with the keys in
// registers: for k <= ANNIH_EXTRACT_K extracted one at a time by wave-wide
// minima, else an 8-bit radix select on a per-wavefront LDS histogram `hist`
// (256 ints) followed by the keys below the k-th.  Ids are read only where keys
// tie exactly.  Bit j of the result: the lane's j-th candidate (record
// lane + 64 j) is taken.
__device__ uint32_t annih_select_regs(const AnnihArgs& a, int64_t rec0, int64_t base, int m, int k, int* hist) {
    const int lane = threadIdx.x & 63;
    uint64_t key[ANNIH_KPL];
#pragma unroll
    for (int j = 0; j < ANNIH_KPL; ++j) {
        const int r = lane + 64 * j;
        key[j] = r < m ? a.cand_key[rec0 + r] : ~0ull;
    }
    auto valid = [&](int j) { return lane + 64 * j < m; };
    uint32_t taken = 0;
    // take `n` more of the untaken candidates whose key is kmin, smallest id first
    auto take_ties = [&](uint64_t kmin, int n) {
        for (int t = 0; t < n; ++t) {
            uint64_t idmin = ~0ull;
            int jmin = -1;
#pragma unroll
            for (int j = 0; j < ANNIH_KPL; ++j) {
                if (!((taken >> j) & 1u) && valid(j) && key[j] == kmin) {
                    const uint64_t id = a.id[base + a.cand_slot[rec0 + lane + 64 * j]];
                    if (id < idmin) { idmin = id; jmin = j; }
                }
            }
            const uint64_t wid = wave_min_u64(idmin);
            if (jmin >= 0 && idmin == wid) taken |= 1u << jmin;
        }
    };
    if (k <= ANNIH_EXTRACT_K) {
        for (int round = 0; round < k; ++round) {
            uint64_t mine = ~0ull;
#pragma unroll
            for (int j = 0; j < ANNIH_KPL; ++j)
                if (!((taken >> j) & 1u) && valid(j) && key[j] < mine) mine = key[j];
            const uint64_t kmin = wave_min_u64(mine);
            int ties = 0;
#pragma unroll
            for (int j = 0; j < ANNIH_KPL; ++j) ties += (!((taken >> j) & 1u) && valid(j) && key[j] == kmin) ? 1 : 0;
            if (wave_sum_i(ties) == 1) {
#pragma unroll
                for (int j = 0; j < ANNIH_KPL; ++j)
                    if (valid(j) && key[j] == kmin) taken |= 1u << j;
            } else {
                take_ties(kmin, 1);
            }
        }
        return taken;
    }
    // radix select, most significant byte first: kth ends as the k-th smallest key
    uint64_t kth = 0;
    int want = k;
    for (int p = 7; p >= 0; --p) {
        const int sh = 8 * p;
        for (int i = lane; i < 256; i += 64) hist[i] = 0;
        wave_sync();
#pragma unroll
        for (int j = 0; j < ANNIH_KPL; ++j) {
            const bool match = valid(j) && (p == 7 || (key[j] >> (sh + 8)) == (kth >> (sh + 8)));
            if (match) atomicAdd(&hist[(int)((key[j] >> sh) & 255ull)], 1);
        }
        wave_sync();
        const int c0 = hist[4 * lane], c1 = hist[4 * lane + 1], c2 = hist[4 * lane + 2], c3 = hist[4 * lane + 3];
        const int t = c0 + c1 + c2 + c3;
        int inc = t;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(inc, o, 64);
            if (lane >= o) inc += v;
        }
        const int excl = inc - t;
        const unsigned long long hb = __ballot(excl < want && want <= inc);
        const int L = __ffsll((long long)hb) - 1;
        int d = 0, below = excl;
        if (lane == L) {
            const int w = want - excl;
            if (w <= c0) { d = 0; }
            else if (w <= c0 + c1) { d = 1; below += c0; }
            else if (w <= c0 + c1 + c2) { d = 2; below += c0 + c1; }
            else { d = 3; below += c0 + c1 + c2; }
        }
        d = __shfl(d, L, 64);
        below = __shfl(below, L, 64);
        kth |= (uint64_t)(4 * L + d) << sh;
        want -= below;
        wave_sync();
    }
    int eq = 0;
#pragma unroll
    for (int j = 0; j < ANNIH_KPL; ++j) {
        if (valid(j) && key[j] < kth) taken |= 1u << j;
        eq += (valid(j) && key[j] == kth) ? 1 : 0;
    }
    if (wave_sum_i(eq) == want) {
#pragma unroll
        for (int j = 0; j < ANNIH_KPL; ++j)
            if (valid(j) && key[j] == kth) taken |= 1u << j;
    } else {
        take_ties(kth, want);
    }
    return taken;
}

// One wavefront removes cell g's k annihilating pairs (every lane calls it with
// the same g and k): per species a most-significant-bit-first radix select finds
// the k-th smallest key, keys below it are taken and keys equal to it (in
// practice only itself) by rank of id.  Returns (to every lane) the annihilation
// current in the deposit's units (2^-28 cell); the caller adds it to J[g] and
// takes k off the cell's e-/e+ counts.
__device__ long long annihilate_cell(const AnnihArgs& a, const int32_t* hist_out, int g, int k, int* hist) {
    const int lane = threadIdx.x & 63;
    const int line = a.cell_line[g];
    const int* h = hist_out + 4 * (size_t)g;
    const int h0 = h[0], h1 = h[1];
    // every e- and e+ of the cell must have been recorded (records beyond those
    // written hold stale data of the other buffer set and are never read)
    if (a.ann_fill[2 * (size_t)g] != h0 || a.ann_fill[2 * (size_t)g + 1] != h1) {
        if (lane == 0) set_error(&a.sc->err, -4);
        return 0;
    }
    long long dq = 0;
    for (int s = 0; s < 2; ++s) {
        const int m = s ? h1 : h0;
        const int64_t rec0 = (int64_t)a.ann_off[g] + (s ? h0 : 0);
        const int64_t base = a.seg_base[4 * line + s];
        if (m <= 64 * ANNIH_KPL) {
            const uint32_t taken = annih_select_regs(a, rec0, base, m, k, hist);
#pragma unroll
            for (int j = 0; j < ANNIH_KPL; ++j) {
                if ((taken >> j) & 1u) {
                    const int64_t kidx = base + a.cand_slot[rec0 + lane + 64 * j];
                    const long long q = (long long)(int)(a.off[kidx] * POS_SCALE);
                    dq += s == 0 ? q : -q;
                    a.cell[kidx] = DEAD_CELL;
                    a.off[kidx] = 0.5f;
                    a.u[kidx] = 0.0f;
                }
            }
            continue;
        }
        uint64_t kth = 0;
        int want = k;                 // rank sought among the keys that match kth so far
        for (int b = 63; b >= 0; --b) {
            const uint64_t above = b == 63 ? 0ull : (~0ull << (b + 1));
            int c = 0;
            for (int r = lane; r < m; r += 64) {
                const uint64_t key = a.cand_key[rec0 + r];
                c += ((key & above) == kth && ((key >> b) & 1ull) == 0ull) ? 1 : 0;
            }
            c = wave_sum_i(c);
            if (want > c) {
                want -= c;
                kth |= 1ull << b;
            }
        }
        // kth is the k-th smallest key; `want` of the keys equal to it are taken
        for (int r = lane; r < m; r += 64) {
            const uint64_t key = a.cand_key[rec0 + r];
            const int slot = a.cand_slot[rec0 + r];
            bool take = key < kth;
            if (key == kth) {
                const uint64_t id = a.id[base + slot];
                int below = 0;
                for (int r2 = 0; r2 < m; ++r2)
                    below += (a.cand_key[rec0 + r2] == kth && a.id[base + a.cand_slot[rec0 + r2]] < id) ? 1 : 0;
                take = below < want;
            }
            if (take) {
                const int64_t kidx = base + slot;
                const long long q = (long long)(int)(a.off[kidx] * POS_SCALE);
                dq += s == 0 ? q : -q;
                a.cell[kidx] = DEAD_CELL;
                a.off[kidx] = 0.5f;
                a.u[kidx] = 0.0f;
            }
        }
    }
    if (lane == 0)
        atomicAdd(&a.counters[((size_t)line * CNT_REPL + (blockIdx.x & (CNT_REPL - 1))) * NCOUNT + 11],
                  (unsigned long long)k);
    return wave_sum_ll(dq);
}

// Ampere's law with the static twist current (Sec. 3): E -= 4 pi (j - j_twist),
// plus time averages and the reset of the step's accumulators.  Block 0 also does
// the step's bookkeeping (live counts, the next push's tile plan) and advances the
// step counter; the cells read the running step from the copy the push left.
__global__ __launch_bounds__(256) void k_field(FieldArgs f, BookArgs b) {
    if (f.sc->err != 0) return;
    const uint64_t step = f.sc->step_field;
    const int n = f.n_total;
    const int hin = (int)(step & 1);
    int* hist_in = f.hist[hin];
    int* hist_out = f.hist[hin ^ 1];
    const bool averaging = f.avg_start >= 0 && step >= (uint64_t)f.avg_start;
    // the last block plans the next push and advances the step counter, beside the
    // cells' blocks rather than before one of them (none of them reads what it writes)
    const int nb = gridDim.x - 1;
    if ((int)blockIdx.x == nb) {
        bookkeeping(b);
        if (threadIdx.x == 0) {
            if (b.sc->err == 0) b.sc->step += 1;
            if (f.annihilation) {
                // the plan of the next step allocates from zero (no other block reads these)
                f.an.ann_ctl[0] = 0;
                f.an.ann_ctl[1] = 0;
            }
            if (averaging) f.avg_count[0] += 1;
        }
        return;
    }
    // Each wavefront takes cpw consecutive cells per iteration: all 64 lanes, or 4
    // in a step where some cell is over the limit, so that the selections, which a
    // wavefront runs one after another, spread over many wavefronts (the grid is
    // sized for 4; with 64 most of its blocks find no cells).
    __shared__ int sHist[4][256];            // per wavefront: the radix histogram of the selection
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int cpw = (f.annihilation && f.an.ann_ctl[2] != 0) ? 4 : 64;
    const int wpb = blockDim.x >> 6;
    for (int gw = (blockIdx.x * wpb + wid) * cpw; gw < n; gw += nb * wpb * cpw) {
        const int g = gw + lane;
        const bool own = lane < cpw && g < n;
        long long dJ = 0;        // this lane's cell: annihilation current and pairs removed
        int k_own = 0;
        if (f.annihilation) {
            // this wavefront's cells over the limit, one at a time, before their Ampere
            const int k = own ? f.an.ann_k[g] : 0;
            unsigned long long m = __ballot(k > 0);
            while (m != 0ull) {
                const int lead = __ffsll((long long)m) - 1;
                m &= m - 1ull;
                const long long d = annihilate_cell(f.an, hist_out, __shfl(g, lead, 64), __shfl(k, lead, 64),
                                                    sHist[wid]);
                if (lane == lead) {
                    dJ = d;
                    k_own = k;
                }
            }
            if (k_own > 0) {
                hist_out[4 * (size_t)g] -= k_own;
                hist_out[4 * (size_t)g + 1] -= k_own;
            }
        }
        if (!own) continue;
        const int line = f.cell_line[g];
        const LineDev& L = f.lines[line];
        const long long J = (long long)f.J[g] + dJ * (1ll << POS_TO_FIX);
        const double j = (double)J * FIX_INV * L.Q;
        f.J[g] = 0ull;
        f.j_last[g] = j;
        if (!f.frozen) {
            const double En = f.E[g] - 4.0 * 3.14159265358979323846 * (j - L.j_tw);
            f.E[g] = En;
            f.E32[g] = (float)En;
        }
        const int ps = f.pair_step[g];
        f.pair_step[g] = 0;
        if (averaging) {
            f.E_sum[g] += f.E[g];
            f.j_sum[g] += j;
            f.pair_sum[g] += ps;
#pragma unroll
            for (int s = 0; s < 4; ++s) f.n_sum[4 * (size_t)g + s] += hist_out[4 * (size_t)g + s];
        }
        f.pair_last[g] = ps;
#pragma unroll
        for (int s = 0; s < 4; ++s) hist_in[4 * (size_t)g + s] = 0;
    }
}

// ---------------------------------------------------------------------------
// Sort by position (counting sort per segment on the key cell * sub +
// floor(offset * sub), sub bins per cell, eight unless the launch tuner picks
// another power of two), dropping absorbed particles.  Ordering by parts of a
// cell, not only by cell, keeps a lane's consecutive particles together in
// space, so that after a step the ones that crossed a face are grouped instead
// of spread through every lane's slots.  Counts live in bins[cell * sub + k] as
// one int4 (the four species):
//   k_sort_zero     clears the bins
//   k_sort_count    counts the live particles per bin
//   k_sort_chunks   per chunk of SCAN_CELLS cells: its counts
//   k_sort_lines    per line: exclusive scan over its chunks, and the new counts
//   k_sort_cursors  per chunk: each bin's first slot
//   k_sort_scatter  every particle takes the next slot of its bin
// ---------------------------------------------------------------------------
__device__ __forceinline__ int sort_bin(int cell_base, int c, float off, int sub) {
    return (cell_base + c) * sub + min((int)(off * (float)sub), sub - 1);    // off * sub is exact
}

__device__ __forceinline__ int& int4_at(int4& v, int k) {
    return k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w;
}

// For each lane: the lanes of the wavefront (among `active`) with the same key, and
// the lowest of them.
__device__ __forceinline__ unsigned long long match_key(int key, bool active, int& leader) {
    unsigned long long act = __ballot(active), mine = 0ull;
    leader = 0;
    while (act) {
        const int l = __ffsll((long long)act) - 1;
        const int k = __shfl(key, l, 64);
        const unsigned long long m = __ballot(active && key == k);
        if (active && key == k) {
            mine = m;
            leader = l;
        }
        act &= ~m;
    }
    return mine;
}

// The candidates: every live e- and e+ (appends included) in a cell over the
// limit records its key and slot.  Exits at once when no cell is over it.  Lanes
// of a wavefront in the same cell reserve their records with one atomic.
__global__ __launch_bounds__(256) void k_annih_gather(AnnihArgs a) {
    if (a.sc->err != 0) return;
    // a copy of the over-limit flag for k_field, which clears [1] for the next step
    // while its other blocks still need to know
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ann_ctl[2] = a.ann_ctl[1];
    if (a.ann_ctl[1] == 0) return;
    const uint64_t step = a.sc->step;
    const int32_t* hist_out = a.hist[(step & 1) ^ 1];
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    // a thread takes GATHER_U particles per pass and issues their cell and per-cell
    // loads together, so that several loads are in flight per lane
    constexpr int U = GATHER_U;
    const int64_t stride = (int64_t)gridDim.x * 256 * U;     // (a segment may hold nearly 2^31 slots)
    for (int l = 0; l < a.n_lines; ++l) {
        const int cb = a.lines[l].cell_base;
        for (int s = 0; s < 2; ++s) {
            const int seg = 4 * l + s;
            const int n = min(a.alloc[seg], a.seg_cap[seg]);
            const int64_t base = a.seg_base[seg];
            for (int64_t i0 = (int64_t)blockIdx.x * 256 * U; i0 < n; i0 += stride) {   // block-uniform trip count
                int cu[U], ku[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t i = i0 + u * 256 + (int)threadIdx.x;
                    cu[u] = i < n ? a.cell[base + i] : DEAD_CELL;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) ku[u] = cu[u] != DEAD_CELL ? a.ann_k[cb + cu[u]] : 0;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int i = (int)(i0 + u * 256 + (int)threadIdx.x);    // < n where used
                    const int g = cu[u] != DEAD_CELL ? cb + cu[u] : 0;
                    const bool cand = cu[u] != DEAD_CELL && ku[u] != 0;
                    if (__ballot(cand) == 0ull) continue;                     // wave-uniform
                    int leader;
                    const unsigned long long mm = match_key(g, cand, leader);
                    int r0 = 0;
                    if (cand && lane == leader) r0 = atomicAdd(&a.ann_fill[2 * (size_t)g + s], __popcll(mm));
                    const int r = __shfl(r0, leader, 64) + __popcll(mm & below);
                    if (!cand) continue;
                    const int* h = hist_out + 4 * (size_t)g;
                    if (r >= h[s]) {              // counts and particles disagree: cannot happen
                        set_error(&a.sc->err, -4);
                        continue;
                    }
                    const int64_t rec = (int64_t)a.ann_off[g] + (s ? h[0] : 0) + r;
                    a.cand_key[rec] = annih_key(step, a.id[base + i], a.key0, a.key1);
                    a.cand_slot[rec] = i;
                }
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_sort_zero(SortArgs s) {
    if (s.sc->err != 0) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < s.n_bins; i += gridDim.x * blockDim.x)
        s.bins[i] = make_int4(0, 0, 0, 0);
}

__global__ __launch_bounds__(256) void k_sort_count(SortArgs s) {
    if (s.sc->err != 0) return;
    const int total = s.tile_prefix[s.nseg];
    const int lane = threadIdx.x & 63;
    for (TileWalk tw(total); tw.t < tw.end; tw.t += tw.stride) {
        const int t = tw.t;
        const int seg = find_segment(s.tile_prefix, s.nseg, t);
        const int sp = seg & 3;
        const LineDev& L = s.lines[seg >> 2];
        const int ncur = s.n_cur[seg];
        const int64_t base = s.seg_base[seg];
        const int i0 = (t - s.tile_prefix[seg]) * s.tile;
        for (int q = 0; q < s.tile / PUSH_TPB; ++q) {
            const int i = i0 + q * PUSH_TPB + threadIdx.x;
            const int c = (i < ncur) ? s.cell[base + i] : DEAD_CELL;
            const bool live = c != DEAD_CELL;
            const int bin = live ? sort_bin(L.cell_base, c, s.off[base + i], s.sub) : 0;
            int leader;
            const unsigned long long m = match_key(bin, live, leader);
            if (live && lane == leader) atomicAdd(&int4_at(s.bins[bin], sp), __popcll(m));
        }
    }
}

// Block-wide exclusive scan of one int4 per thread (256 threads); returns the
// thread's prefix and writes the block total.
__device__ __forceinline__ int4 block_scan_int4(int4 v, int4& total) {
    __shared__ int4 sPart[256];
    const int t = threadIdx.x;
    sPart[t] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int4 w = t >= o ? sPart[t - o] : make_int4(0, 0, 0, 0);
        __syncthreads();
        if (t >= o) sPart[t] = make_int4(sPart[t].x + w.x, sPart[t].y + w.y, sPart[t].z + w.z, sPart[t].w + w.w);
        __syncthreads();
    }
    const int4 inc = sPart[t];
    total = sPart[255];
    __syncthreads();
    return make_int4(inc.x - v.x, inc.y - v.y, inc.z - v.z, inc.w - v.w);
}

// Counts of one cell (thread) of a chunk (block), summed over its bins.
__device__ __forceinline__ int4 cell_counts(const SortArgs& s, int chunk, int& gcell, bool& in) {
    const int line = s.chunk_line[chunk];
    const LineDev& L = s.lines[line];
    const int c = (chunk - s.line_chunk0[line]) * SCAN_CELLS + (int)threadIdx.x;
    in = c < L.n_cells;
    gcell = L.cell_base + c;
    int4 n = make_int4(0, 0, 0, 0);
    if (in) {
        const int4* bc = s.bins + (size_t)gcell * s.sub;
#pragma unroll 8
        for (int k = 0; k < s.sub; ++k) {
            const int4 b = bc[k];
            n.x += b.x; n.y += b.y; n.z += b.z; n.w += b.w;
        }
    }
    return n;
}

__global__ __launch_bounds__(256) void k_sort_chunks(SortArgs s) {
    if (s.sc->err != 0) return;
    int gcell;
    bool in;
    const int4 n = cell_counts(s, blockIdx.x, gcell, in);
    int4 total;
    (void)block_scan_int4(n, total);
    if (threadIdx.x == 0) s.chunk_sum[blockIdx.x] = total;
}

// One block per line: the chunks' first slots (exclusive scan over the line's
// chunks, per species) and the line's new live counts.
__global__ __launch_bounds__(256) void k_sort_lines(SortArgs s) {
    if (s.sc->err != 0) return;
    const int line = blockIdx.x;
    const int c0 = s.line_chunk0[line], c1 = s.line_chunk0[line + 1];
    int4 run = make_int4(0, 0, 0, 0);
    for (int b = c0; b < c1; b += 256) {
        const int k = b + (int)threadIdx.x;
        const int4 v = k < c1 ? s.chunk_sum[k] : make_int4(0, 0, 0, 0);
        int4 total;
        const int4 ex = block_scan_int4(v, total);
        if (k < c1) s.chunk_sum[k] = make_int4(run.x + ex.x, run.y + ex.y, run.z + ex.z, run.w + ex.w);
        run = make_int4(run.x + total.x, run.y + total.y, run.z + total.z, run.w + total.w);
    }
    if (threadIdx.x < 4) s.new_count[4 * line + threadIdx.x] = int4_at(run, threadIdx.x);
}

__global__ __launch_bounds__(256) void k_sort_cursors(SortArgs s) {
    if (s.sc->err != 0) return;
    int gcell;
    bool in;
    const int4 n = cell_counts(s, blockIdx.x, gcell, in);
    int4 total;
    const int4 ex = block_scan_int4(n, total);
    if (!in) return;
    const int4 c0 = s.chunk_sum[blockIdx.x];
    int4 run = make_int4(c0.x + ex.x, c0.y + ex.y, c0.z + ex.z, c0.w + ex.w);
    int4* bc = s.bins + (size_t)gcell * s.sub;
#pragma unroll 8
    for (int k = 0; k < s.sub; ++k) {
        const int4 b = bc[k];
        bc[k] = run;
        run = make_int4(run.x + b.x, run.y + b.y, run.z + b.z, run.w + b.w);
    }
}

// Every live particle takes the next slot of its bin: the lanes of a wavefront
// that share a bin reserve their slots with one atomic, all bins at once.
__global__ __launch_bounds__(256) void k_sort_scatter(SortArgs s) {
    if (s.sc->err != 0) return;
    const int total = s.tile_prefix[s.nseg];
    const int lane = threadIdx.x & 63;
    for (TileWalk tw(total); tw.t < tw.end; tw.t += tw.stride) {
        const int t = tw.t;
        const int seg = find_segment(s.tile_prefix, s.nseg, t);
        const int sp = seg & 3;
        const LineDev& L = s.lines[seg >> 2];
        const int ncur = s.n_cur[seg];
        const int cap = s.seg_cap[seg];
        const int64_t base = s.seg_base[seg];
        const int i0 = (t - s.tile_prefix[seg]) * s.tile;
        for (int q = 0; q < s.tile / PUSH_TPB; ++q) {
            const int i = i0 + q * PUSH_TPB + threadIdx.x;
            const int c = (i < ncur) ? s.cell[base + i] : DEAD_CELL;
            const bool live = c != DEAD_CELL;
            float pof = 0.0f, puv = 0.0f;
            uint64_t pid = 0;
            if (live) {
                pof = s.off[base + i];
                puv = s.u[base + i];
                pid = s.id[base + i];
            }
            const int bin = live ? sort_bin(L.cell_base, c, pof, s.sub) : 0;
            int leader;
            const unsigned long long m = match_key(bin, live, leader);
            int first = 0;
            if (live && lane == leader) first = atomicAdd(&int4_at(s.bins[bin], sp), __popcll(m));
            first = __shfl(first, leader, 64);
            if (live) {
                const int pos = first + __popcll(m & ((1ull << lane) - 1ull));
                if (pos < cap) {
                    const int64_t dst = base + pos;
                    s.cell2[dst] = c;
                    s.off2[dst] = pof;
                    s.u2[dst] = puv;
                    s.id2[dst] = pid;
                } else {
                    set_error(&s.sc->err, -3);
                }
            }
        }
    }
}

__global__ void k_sort_finish(SortArgs s) {
    const int seg = blockIdx.x * blockDim.x + threadIdx.x;
    if (s.sc->err == 0 && seg < s.nseg) {
        s.n_cur[seg] = s.new_count[seg];
        s.alloc[seg] = s.new_count[seg];
    }
}

// ---------------------------------------------------------------------------
// Initial pair plasma: pair i of a line in cell i / ppc at offset U24(w0) of the
// Philox block (0, i, line, STREAM_INIT).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_init_pairs(InitArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_pairs) return;
    const uint4 w = philox4x32_10(make_uint4(0u, (uint32_t)i, (uint32_t)a.line, STREAM_INIT), a.key0, a.key1);
    const int cell = (int)(i / a.ppc);
    const float off = uniform24(w.x);
    float ue = 0.0f, up = 0.0f;
    if (a.mode == 1) {
        const double gam = pow(10.0, (double)uniform24(w.y) * a.log10_gmax);
        const double uu = sqrt(fmax(gam * gam - 1.0, 0.0));
        const float s = (w.z >> 31) ? -1.0f : 1.0f;
        ue = up = s * (float)uu;
    } else if (a.mode == 2) {
        up = (float)a.u_stream;
        ue = -(float)a.u_stream;
    }
    const int64_t ke = a.base_e + i, kp = a.base_p + i;
    a.cell[ke] = cell; a.off[ke] = off; a.u[ke] = ue; a.id[ke] = a.id_base + 2 * (uint64_t)i;
    a.cell[kp] = cell; a.off[kp] = off; a.u[kp] = up; a.id[kp] = a.id_base + 2 * (uint64_t)i + 1;
}

// Sum of v over the run of consecutive lanes that share this lane's key, in the
// run's first lane (head = true there).  Every lane of the wavefront must take part.
// Keys need not be sorted: equal keys that are not adjacent form runs of their own.
__device__ __forceinline__ long long wave_run_sum(int key, long long v, bool& head) {
    const int lane = threadIdx.x & 63;
    const int prev = __shfl_up(key, 1, 64);
    const int next = __shfl_down(key, 1, 64);
    head = lane == 0 || prev != key;
    const bool tail = lane == 63 || next != key;
    long long p = v;                                  // inclusive prefix sum
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long y = __shfl_up(p, o, 64);
        if (lane >= o) p += y;
    }
    const unsigned long long T = __ballot(tail);      // bit 63 always set
    const int e = lane + __builtin_ctzll(T >> lane);  // the run's last lane
    const long long pe = __shfl(p, e, 64);
    const long long pb = __shfl(p, lane > 0 ? lane - 1 : 0, 64);
    return pe - (lane > 0 ? pb : 0ll);
}

// Histogram of live particles per cell and species (after init / set_particles).
__global__ __launch_bounds__(256) void k_hist(HistArgs h) {
    const int total = h.tile_prefix[h.nseg];
    for (TileWalk tw(total); tw.t < tw.end; tw.t += tw.stride) {
        const int t = tw.t;
        const int seg = find_segment(h.tile_prefix, h.nseg, t);
        const int sp = seg & 3;
        const LineDev& L = h.lines[seg >> 2];
        const int ncur = h.n_cur[seg];
        const int64_t base = h.seg_base[seg];
        const int i0 = (t - h.tile_prefix[seg]) * h.tile;
        for (int q = 0; q < h.tile / PUSH_TPB; ++q) {
            // one atomic per run of lanes in the same cell (every lane takes part)
            const int i = i0 + q * PUSH_TPB + threadIdx.x;
            const int c = i < ncur ? h.cell[base + i] : DEAD_CELL;
            bool head;
            const long long n = wave_run_sum(c == DEAD_CELL ? -1 : c, c == DEAD_CELL ? 0 : 1, head);
            if (head && c != DEAD_CELL) atomicAdd(&h.hist[4 * (size_t)(L.cell_base + c) + sp], (int)n);
        }
    }
}

// ---------------------------------------------------------------------------
// Moments: cloud-in-cell charge on nodes (fixed point), kinetic energy.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_moments_particles(MomArgs m) {
    __shared__ unsigned long long sK[4][3];
    // only the tiles of the requested line's four segments
    const int t_first = m.tile_prefix[4 * m.line], t_last = m.tile_prefix[4 * m.line + 4];
    // kinetic energy sum m (gamma - 1) / m_e in fixed point: v 2^48 split exactly into
    // three 32-bit chunks, each summed as an integer, so the total does not depend on
    // the order in which particles are visited (bits below 2^-48 of a term dropped)
    unsigned long long k0 = 0, k1 = 0, k2 = 0;
    for (TileWalk tw(t_last - t_first); tw.t < tw.end; tw.t += tw.stride) {
        const int t = t_first + tw.t;
        const int seg = find_segment(m.tile_prefix, m.nseg, t);
        const int sp = seg & 3;
        const int ncur = m.n_cur[seg];
        const int64_t base = m.seg_base[seg];
        const int i0 = (t - m.tile_prefix[seg]) * m.tile;
        const double qs = m.sign[sp] * FIX_SCALE;
        const double mass = (sp == 3) ? m.mass_ratio : 1.0;
        for (int q = 0; q < m.tile / PUSH_TPB; ++q) {
            // every lane takes part in the run sums: absent and dead slots carry key -1
            const int i = i0 + q * PUSH_TPB + threadIdx.x;
            const int c0 = i < ncur ? m.cell[base + i] : DEAD_CELL;
            const bool live = c0 != DEAD_CELL;
            const int c = live ? c0 : -1;
            // cloud-in-cell weights of the position quantised as in the deposit (2^-28 cell)
            const long long f = live ? (long long)(int)(m.off[base + i] * POS_SCALE) << POS_TO_FIX : 0ll;
            const long long sg = (qs < 0.0) ? -1 : 1;
            const double u = live ? (double)m.u[base + i] : 0.0;
            // the charge of a run of particles in one cell, added by the run's first lane
            // (same-address atomics from every particle of a cell would serialise)
            bool head;
            const long long a0 = wave_run_sum(c, live ? sg * (4294967296ll - f) : 0ll, head);
            const long long a1 = wave_run_sum(c, sg * f, head);
            if (head && live) {
                atomicAdd(&m.rho[c], (unsigned long long)a0);
                atomicAdd(&m.rho[c + 1], (unsigned long long)a1);
            }
            // gamma - 1 = u^2 / (gamma + 1), free of cancellation at small u
            const double v = mass * (u * u / (sqrt(fma(u, u, 1.0)) + 1.0));
            const double sv = v * 0x1.0p48;
            const double h2 = floor(sv * 0x1.0p-64);
            const double r = fma(-h2, 0x1.0p64, sv);          // exact: the bits of sv below 2^64
            const double h1 = floor(r * 0x1.0p-32);
            const double h0 = floor(fma(-h1, 0x1.0p32, r));
            k0 += (unsigned long long)h0;
            k1 += (unsigned long long)h1;
            k2 += (unsigned long long)h2;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        k0 += __shfl_xor(k0, o, 64);
        k1 += __shfl_xor(k1, o, 64);
        k2 += __shfl_xor(k2, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sK[threadIdx.x >> 6][0] = k0;
        sK[threadIdx.x >> 6][1] = k1;
        sK[threadIdx.x >> 6][2] = k2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const unsigned long long s = sK[0][threadIdx.x] + sK[1][threadIdx.x] + sK[2][threadIdx.x] + sK[3][threadIdx.x];
        if (s != 0ull) atomicAdd(&m.kin[threadIdx.x], s);
    }
}

// Gauss residual on interior nodes, and the per-block partial sums of E and E^2 of
// one line (the host adds the partials in block order: the circuit potential and
// the field energy are the same bits on every run).
__global__ __launch_bounds__(256) void k_moments_grid(MomArgs m) {
    __shared__ double sE[4][2];
    const LineDev& L = m.lines[m.line];
    const int n = L.n_cells;
    double rmax = 0.0, esum = 0.0, e2 = 0.0;
    const double* E = m.E + L.cell_base;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += gridDim.x * blockDim.x) {
        if (i < n) { esum += E[i]; e2 = fma(E[i], E[i], e2); }
        if (i >= 1 && i <= n - 1) {
            const double rho = (double)(long long)m.rho[i] * FIX_INV * L.Q;
            rmax = fmax(rmax, fabs(E[i] - E[i - 1] - 4.0 * 3.14159265358979323846 * rho));
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        rmax = fmax(rmax, __shfl_xor(rmax, o, 64));
        esum += __shfl_xor(esum, o, 64);
        e2 += __shfl_xor(e2, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax((unsigned long long*)&m.out[0], (unsigned long long)__double_as_longlong(rmax));
        sE[threadIdx.x >> 6][0] = esum;
        sE[threadIdx.x >> 6][1] = e2;
    }
    __syncthreads();
    if (threadIdx.x < 2)
        m.part[2 * blockIdx.x + threadIdx.x] =
            ((sE[0][threadIdx.x] + sE[1][threadIdx.x]) + sE[2][threadIdx.x]) + sE[3][threadIdx.x];
}

// RICS backend evaluation at given points (diagnostics and surrogate error).
template <int BACKEND>
__device__ __forceinline__ void rics_eval_point(const PushArgs& a, int line, int64_t n, const float* s_cells,
                                                const float* uin, float* F, float* N, float* eps) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const LineDev L = a.lines[line];
    const float s = fminf(fmaxf(s_cells[i], 0.0f), (float)L.n_cells);
    const int c0 = min((int)floorf(s), L.n_cells - 1);
    const float o0 = s - (float)c0;
    PartGeo pg = part_geo<BACKEND>(a, L, a.nodes[L.node_base + c0], a.nodes[L.node_base + c0 + 1], c0, o0);
    const Geo& g = pg.g;
    const float u = uin[i];
    float f = 0.0f, nd = 0.0f;
    if constexpr (BACKEND != RICS_OFF) {
        f = rics_eval<BACKEND>(a, L, u, pg).F;
        nd = rics_N<BACKEND>(a, L, u, pg);
    }
    F[i] = f;
    N[i] = nd;
    eps[i] = photon_energy(fsqrt(fmaf(u, u, 1.0f)), g.b);
}
template <int BACKEND>
__global__ __launch_bounds__(256) void k_rics_eval(PushArgs a, int line, int64_t n, const float* s_cells,
                                                   const float* uin, float* F, float* N, float* eps) {
    rics_eval_point<BACKEND>(a, line, n, s_cells, uin, F, N, eps);
}
template __global__ void k_rics_eval<RICS_OFF>(PushArgs, int, int64_t, const float*, const float*, float*, float*, float*);
template __global__ void k_rics_eval<RICS_EXACT>(PushArgs, int, int64_t, const float*, const float*, float*, float*, float*);
template __global__ void k_rics_eval<RICS_TABLE>(PushArgs, int, int64_t, const float*, const float*, float*, float*, float*);

// The surrogate at n points (one per lane; the whole wavefront evaluates the
// network together, lanes past n on a dummy point).
__global__ __launch_bounds__(256) void k_rics_eval_mlp(PushArgs a, int line, int64_t n, const float* s_cells,
                                                       const float* uin, float* F, float* N, float* eps) {
    if (a.lines[line].use_table) {           // this line takes its table (uniform over the launch)
        rics_eval_point<RICS_TABLE>(a, line, n, s_cells, uin, F, N, eps);
        return;
    }
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = i < n;
    const LineDev L = a.lines[line];
    const float s = ok ? fminf(fmaxf(s_cells[i], 0.0f), (float)L.n_cells) : 0.5f;
    const int c0 = min((int)floorf(s), L.n_cells - 1);
    const float o0 = s - (float)c0;
    const double x = (double)c0 + (double)o0;
    const Geo g = geo_lerp(L, a.nodes[L.node_base + c0], a.nodes[L.node_base + c0 + 1], o0);
    const float u = ok ? uin[i] : 0.0f;
    int n_eval = 0;
    const MlpRics rr = mlp_rics(a, a.mlp_ft, a.mlp_bias, u, g, (float)(x / (double)L.n_cells), n_eval);
    if (ok) {
        F[i] = rr.F;
        N[i] = rr.N;
        eps[i] = photon_energy(fsqrt(fmaf(u, u, 1.0f)), g.b);
    }
}

// The surrogate's error estimate on each line (MLP backend with table fallback):
// every table node (log10 gamma_i, row centre s_j) of every line is evaluated by
// the network as the pusher evaluates it (float32 geometry, inputs at s_j / L) and
// by the closed forms of Eqs. contdrag and scatteringNdot in float64; the line's
// estimate is the largest relative error of F and Ndot where they are significant
// (|F| h >= 1e-9 max(u, 1) and Ndot h >= 1e-9).  One node per lane; the whole wavefront
// evaluates the network together.
__global__ __launch_bounds__(256) void k_mlp_line_error(PushArgs a, const double* row_geo, double kT_keV,
                                                        unsigned int* err) {
    __shared__ bf16x8 sW[FT_TOTAL * 64];
    __shared__ float sWb[MLP_BIAS];
    for (int e = threadIdx.x; e < FT_TOTAL * 64; e += blockDim.x) sW[e] = a.mlp_ft[e];
    for (int e = threadIdx.x; e < MLP_BIAS; e += blockDim.x) sWb[e] = a.mlp_bias[e];
    __syncthreads();
    const int nlg = a.nlg, ns = a.ns;
    const int64_t per_line = (int64_t)nlg * ns;
    const int n_lines = a.nseg >> 2;
    const int64_t total = per_line * n_lines;
    const double theta = kT_keV / 510.99895000;
    const double base = 2.8179403262e-13 * 1.0e6 / (4.0 * 3.8615926796e-11 * 3.8615926796e-11);
    const double AF = base * theta * theta * theta, AN = base * theta * theta;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // every lane of a wavefront runs the same number of iterations (the network needs all 64)
    const int64_t rounds = (total + stride - 1) / stride;
    for (int64_t it = 0; it < rounds; ++it) {
        const int64_t e = it * stride + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        const bool valid = e < total;
        const int64_t ee = valid ? e : 0;
        const int line = (int)(ee / per_line);
        const int rem = (int)(ee % per_line);
        const int j = rem / nlg, i = rem % nlg;
        const LineDev& L = a.lines[line];
        const double* rg = row_geo + 3 * ((size_t)line * ns + j);
        const double b = rg[0], mu = rg[1], x = rg[2];
        const double gam = pow(10.0, 8.0 * i / (nlg - 1));
        const double u = sqrt(fmax(gam * gam - 1.0, 0.0));
        Geo g;
        g.b = (float)b;
        g.mu = (float)mu;
        g.ix2 = frcp((float)x * (float)x);
        g.by = g.b * L.inv_theta;
        int dummy = 0;
        const MlpRics r = mlp_rics(a, sW, sWb, (float)u, g, (float)((j + 0.5) / ns), dummy);
        // closed forms (float64)
        const double y = b / (theta * (gam - u * mu));
        double Fe = 0.0, Ne = 0.0;
        if (y <= 80.0) {
            const double em1 = expm1(y);
            Fe = AF / (x * x) * (gam * mu - u) * y * y * y / em1;
            Ne = AN / (x * x * gam) * y * y / em1;
        }
        const double h = (double)L.h;
        double worst = 0.0;
        if (valid && fabs(Fe) * h >= 1e-9 * fmax(u, 1.0) && Fe != 0.0) worst = fabs((double)r.F - Fe) / fabs(Fe);
        if (valid && Ne * h >= 1e-9) worst = fmax(worst, fabs((double)r.N - Ne) / Ne);
        if (!(worst <= 3.0e38)) worst = 3.0e38;        // non-finite network output: no trust
        const float wf = (float)worst;
        if (valid && wf > 0.0f) atomicMax(&err[line], __float_as_uint(wf));
    }
}

}  // namespace pic1d

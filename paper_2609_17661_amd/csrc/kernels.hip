// HIP kernels (gfx950) of one PIC step and its bookkeeping.
//
// Step pipeline on one stream:
//   k_push        gather, RICS drag / events, kick, move, fixed-point current
//                 deposit (LDS window per tile), per-cell histogram of the new
//                 positions, pair injection by append
//   k_atmosphere  refill of the surface layers by append
//   k_field       Ampere E -= 4 pi (j - j_twist), averages, per-step bookkeeping
//                 (counts, tile plan, step counter)
//   k_sort_*      every sort_interval steps: counting sort by cell per segment,
//                 dropping absorbed particles
#include <hip/hip_runtime.h>

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

// Segment of a global tile index by binary search over the tile prefix.
__device__ __forceinline__ int find_segment(const int32_t* __restrict__ prefix, int nseg, int t) {
    int lo = 0, hi = nseg;           // prefix[lo] <= t < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// XCD-aware tile walk: the 8 XCDs each take a contiguous range of tiles (blocks
// are dispatched round-robin over XCDs, so block b runs on XCD b % 8).
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

__device__ __forceinline__ Geo geo_at(const float4* __restrict__ nodes, int node, float f) {
    const float4 a = nodes[node];
    const float4 b = nodes[node + 1];
    Geo g;
    g.b = fmaf(f, b.x - a.x, a.x);
    g.mu = fmaf(f, b.y - a.y, a.y);
    g.xr = fmaf(f, b.z - a.z, a.z);
    g.rc = fmaf(f, b.w - a.w, a.w);
    return g;
}

template <int BACKEND>
__device__ __forceinline__ RicsOut rics_eval(const PushArgs& a, const LineDev& L, float u, const Geo& g,
                                             int c0, float o0) {
    if constexpr (BACKEND == RICS_TABLE) {
        double x = (double)c0 + (double)o0;
        if (u < 0.0f) x = (double)L.n_cells - x;
        return rics_table(L, a.table + L.table_off, a.nlg, a.ns, u, x);
    } else {
        return rics_exact(L, u, g);
    }
}

// One drag update over h/2 (Sec. 3): implicit midpoint where |F(p0)| tau_min <= |p0|,
// solved by Newton from the explicit start p0 + (h/2) F(p0) and stopped once the
// step falls below float32 resolution; exponential relaxation towards
// p_tilde = mu / (1 - mu^2)^(1/2) otherwise.
template <int BACKEND>
__device__ __forceinline__ float drag_half(const PushArgs& a, const LineDev& L, float u0, const Geo& g,
                                           int c0, float o0, int& n_limited, int& n_newton) {
    const RicsOut r0 = rics_eval<BACKEND>(a, L, u0, g, c0, o0);
    if (fabsf(r0.F) * L.tau_hat <= fabsf(u0)) {
        const float hq = 0.25f * L.h;
        float u1 = fmaf(0.5f * L.h, r0.F, u0);
        // predicted Newton correction of the explicit start: (h/4)|F'| (h/2)|F0|
        if (hq * fabsf(r0.dF) * 0.5f * L.h * fabsf(r0.F) > 0x1.0p-25f * fabsf(u1)) {
            ++n_newton;
#pragma unroll 1
            for (int it = 0; it < 4; ++it) {
                const RicsOut r1 = rics_eval<BACKEND>(a, L, u1, g, c0, o0);
                const float G = u1 - u0 - hq * (r0.F + r1.F);
                const float dG = 1.0f - hq * r1.dF;
                const float del = G / dG;
                u1 -= del;
                if (fabsf(del) <= 0x1.0p-24f * fabsf(u1)) break;
            }
        }
        return u1;
    }
    ++n_limited;
    const float pt = g.mu * rsqrtf(fmaxf(fmaf(-g.mu, g.mu, 1.0f), 1e-30f));
    return fmaf(-(u0 - pt), L.damp, u0);
}

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
        draws = 0;
};

// Everything one particle does in one step.  Returns its new cell (DEAD_CELL if it
// left the line) and writes the deposit contributions (cell, fixed-point value).
template <int BACKEND>
__device__ __forceinline__ void advance_particle(const PushArgs& a, const LineDev& L, int line, int sp,
                                                 int64_t k, int c0, Counts& cnt, int& ca, long long& da,
                                                 int& cb, long long& db, int& cnew) {
    const int n = L.n_cells;
    const float o0 = a.off[k];
    float u = a.u[k];

    // field gather: E at x^n, linear between cell centres, constant beyond the outer ones
    double Ep;
    {
        int kk;
        float w;
        if (o0 >= 0.5f) { kk = c0; w = o0 - 0.5f; } else { kk = c0 - 1; w = o0 + 0.5f; }
        const double* E = a.E + L.cell_base;
        if (kk < 0) Ep = E[0];
        else if (kk >= n - 1) Ep = E[n - 1];
        else Ep = fma((double)w, E[kk + 1] - E[kk], E[kk]);
    }
    float kick = a.qm[sp] * (float)Ep * L.invC;
    if (a.gravity) {
        const double x = (double)c0 + (double)o0;
        const double dw = fmin(x, (double)n - x);
        if (dw <= (double)L.atm_depth) kick += ((x < (double)L.half_n) ? -1.0f : 1.0f) * L.grav * a.inv_mass[sp];
    }

    if (BACKEND != RICS_OFF && sp != 3) {
        const Geo g = geo_at(a.nodes, L.node_base + c0, o0);
        if (g.b < L.b_thr) {
            // continuous regime: Strang splitting drag h/2, Lorentz kick, drag h/2
            u = drag_half<BACKEND>(a, L, u, g, c0, o0, cnt.limited, cnt.newton);
            u += kick;
            u = drag_half<BACKEND>(a, L, u, g, c0, o0, cnt.limited, cnt.newton);
        } else {
            // stochastic regime: kick, then a scattering event with probability min(Ndot h, 1)
            u += kick;
            const RicsOut r = rics_eval<BACKEND>(a, L, u, g, c0, o0);
            const float lam = r.N * L.h;
            if (lam > 1.0f) ++cnt.clipped;
            if (lam > 0.0f) {
                ++cnt.draws;
                const uint64_t pid = a.id[k];
                const uint4 w = philox4x32_10(make_uint4((uint32_t)a.step, (uint32_t)pid, (uint32_t)(pid >> 32),
                                                         STREAM_RICS), a.key0, a.key1);
                if (uniform24(w.x) < fminf(lam, 1.0f)) {
                    ++cnt.events;
                    const float gam = sqrtf(fmaf(u, u, 1.0f));
                    const float dir = (u >= 0.0f) ? 1.0f : -1.0f;
                    const float eps = photon_energy(gam, g.b);
                    const float gnew = gam / sqrtf(fmaf(2.0f, g.b, 1.0f));
                    const float u_pre = u;
                    u = dir * sqrtf(fmaxf((gnew - 1.0f) * (gnew + 1.0f), 0.0f));
                    // photon conversion into an e-/e+ pair (Sec. 3), limited by n_max
                    bool made = false;
                    if (a.pairs && eps >= 2.0f) {
                        int cs;
                        float os;
                        bool ok;
                        if (a.conversion == 0) {
                            cs = c0; os = o0; ok = true;
                        } else {
                            // eps in float64 from the post-kick momentum on this rare path
                            const double ud = (double)u_pre;
                            const double epsd = sqrt(1.0 + ud * ud) * (1.0 - 1.0 / sqrt(1.0 + 2.0 * (double)g.b));
                            const double rc = fma((double)o0, a.rc_nodes[L.node_base + c0 + 1] - a.rc_nodes[L.node_base + c0],
                                                  a.rc_nodes[L.node_base + c0]);
                            const double sp_ = (double)c0 + (double)o0 +
                                               (double)dir * rc * L.inv_ds * asin(fmin(2.0 / epsd, 1.0));
                            ok = (sp_ >= 0.0) && (sp_ < (double)n);
                            cs = ok ? (int)floor(sp_) : 0;
                            os = ok ? (float)(sp_ - (double)cs) : 0.0f;
                            if (os >= 1.0f) { os = 0.0f; cs += 1; ok = ok && cs < n; }
                        }
                        if (ok) {
                            const int* hc = a.hist_in + 4 * (size_t)(L.cell_base + cs);
                            const int tot = hc[0] + hc[1] + hc[2] + hc[3];
                            if ((float)tot < L.nmax) {
                                // pair members at gamma = eps/2 each, in float64 on this rare path
                                // (u is ill-conditioned in eps when eps/2 is close to 1)
                                const double ud = (double)u_pre;
                                const double gpd = 0.5 * sqrt(1.0 + ud * ud) * (2.0 * (double)g.b) /
                                                   (sqrt(1.0 + 2.0 * (double)g.b) * (1.0 + sqrt(1.0 + 2.0 * (double)g.b)));
                                const float up = dir * (float)sqrt(fmax((gpd - 1.0) * (gpd + 1.0), 0.0));
                                const uint64_t pid = a.id[k];
                                const uint4 wc = philox4x32_10(make_uint4((uint32_t)a.step, (uint32_t)pid,
                                                                          (uint32_t)(pid >> 32), STREAM_CHILD),
                                                               a.key0, a.key1);
                                const bool e_ok = append_particle(a, 4 * line + 0, cs, os, up, id_from_words(wc.x, wc.y));
                                const bool p_ok = append_particle(a, 4 * line + 1, cs, os, up, id_from_words(wc.z, wc.w));
                                if (e_ok && p_ok) {
                                    int* ho = a.hist_out + 4 * (size_t)(L.cell_base + cs);
                                    atomicAdd(&ho[0], 1);
                                    atomicAdd(&ho[1], 1);
                                    atomicAdd(&a.pair_step[L.cell_base + cs], 1);
                                    ++cnt.pairs;
                                    made = true;
                                }
                            }
                        }
                    }
                    if (!made) ++cnt.escaped;
                }
            }
        }
    } else {
        u += kick;
    }
    if (!isfinite(u)) set_error(&a.sc->err, -5);

    // move x^{n+1} = x^n + C u / gamma with the offset carried into the cell index
    const float gam = sqrtf(fmaf(u, u, 1.0f));
    const float dx = L.C * u / gam;
    float o1 = o0 + dx;
    int c1 = c0;
    if (o1 >= 1.0f) {
        o1 -= 1.0f;
        c1 += 1;
    } else if (o1 < 0.0f) {
        o1 += 1.0f;
        c1 -= 1;
        if (o1 >= 1.0f) { o1 = 0.0f; c1 += 1; }
    }
    // charge-conserving deposit of the path [x^n, x^{n+1}] clipped to [0, n],
    // from the stored old and new positions (exact in float64)
    ca = c0;
    cb = -1;
    db = 0;
    double va, vb = 0.0;
    if (c1 == c0) {
        va = (double)o1 - (double)o0;
    } else if (c1 > c0) {
        va = 1.0 - (double)o0;
        cb = c1;
        vb = (double)o1;
    } else {
        va = -(double)o0;
        cb = c1;
        vb = (double)o1 - 1.0;
    }
    const double qs = a.sign[sp] * FIX_SCALE;
    da = __double2ll_rn(va * qs);
    if (cb >= 0 && cb < n) db = __double2ll_rn(vb * qs); else cb = -1;

    if (c1 < 0 || c1 >= n) {
        ++cnt.absorbed;
        cnew = DEAD_CELL;
        a.cell[k] = DEAD_CELL;
    } else {
        cnew = c1;
        a.cell[k] = c1;
        a.off[k] = o1;
    }
    a.u[k] = u;
}

__device__ void flush_counts(const PushArgs& a, int line, Counts& c) {
    int v[9] = {c.events, c.pairs, c.escaped, c.absorbed, c.clipped, c.limited, c.newton, c.pushed, c.draws};
    const int slot[9] = {0, 1, 2, 3, 4, 5, 6, 8, 9};
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int s = wave_sum_i(v[i]);
        if ((threadIdx.x & 63) == 0 && s != 0)
            atomicAdd(&a.counters[line * NCOUNT + slot[i]], (unsigned long long)s);
    }
    c = Counts();
}

constexpr int WMAX = 384;     // LDS window of the deposit, cells
constexpr int NCOPY = 4;      // privatised copies of the window (fewer same-address LDS atomics)

template <int BACKEND>
__global__ __launch_bounds__(PUSH_TPB) void k_push(PushArgs a) {
    __shared__ unsigned long long sJ[NCOPY][WMAX];
    __shared__ int sH[WMAX];
    __shared__ int sRed[2][PUSH_TPB / 64];
    if (a.sc->err != 0) return;
    a.step = a.sc->step;
    a.hist_in = a.hist[a.step & 1];
    a.hist_out = a.hist[(a.step & 1) ^ 1];
    const int total = a.tile_prefix[a.nseg];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int copy = lane & (NCOPY - 1);
    for (TileWalk tw(total); tw.t < tw.end; tw.t += tw.stride) {
        const int t = tw.t;
        const int seg = find_segment(a.tile_prefix, a.nseg, t);
        const int line = seg >> 2, sp = seg & 3;
        const LineDev L = a.lines[line];
        const int nseg_cur = a.n_cur[seg];
        const int64_t base = a.seg_base[seg];
        const int i0 = (t - a.tile_prefix[seg]) * PUSH_TILE;

        // pass 1: cells of the tile -> window [lo, hi] of cells the deposit can touch
        int cl[PUSH_PPT];
        int lo = INT32_MAX, hi = INT32_MIN;
#pragma unroll
        for (int q = 0; q < PUSH_PPT; ++q) {
            const int i = i0 + q * PUSH_TPB + threadIdx.x;
            cl[q] = (i < nseg_cur) ? a.cell[base + i] : DEAD_CELL;
            if (cl[q] != DEAD_CELL) {
                lo = min(lo, cl[q] - 1);
                hi = max(hi, cl[q] + 1);
            }
        }
        lo = wave_min_i(lo);
        hi = wave_max_i(hi);
        if (lane == 0) { sRed[0][wid] = lo; sRed[1][wid] = hi; }
        __syncthreads();
        lo = sRed[0][0]; hi = sRed[1][0];
#pragma unroll
        for (int w = 1; w < PUSH_TPB / 64; ++w) { lo = min(lo, sRed[0][w]); hi = max(hi, sRed[1][w]); }
        const bool any = lo <= hi;
        lo = any ? max(lo, 0) : 0;
        hi = any ? min(hi, L.n_cells - 1) : -1;
        const bool use_lds = any && (hi - lo + 1) <= WMAX;
        const int span = use_lds ? (hi - lo + 1) : 0;
        for (int c = threadIdx.x; c < span; c += PUSH_TPB) {
#pragma unroll
            for (int r = 0; r < NCOPY; ++r) sJ[r][c] = 0ull;
            sH[c] = 0;
        }
        __syncthreads();

        // pass 2: advance every particle, deposit into the window (or global memory)
        Counts cnt;
        unsigned long long* Jg = a.J + L.cell_base;
        int* Hg = a.hist_out + 4 * (size_t)L.cell_base + sp;
#pragma unroll 1
        for (int q = 0; q < PUSH_PPT; ++q) {
            if (cl[q] == DEAD_CELL) continue;
            const int64_t k = base + i0 + q * PUSH_TPB + threadIdx.x;
            ++cnt.pushed;
            int ca, cb, cnew;
            long long da, db;
            advance_particle<BACKEND>(a, L, line, sp, k, cl[q], cnt, ca, da, cb, db, cnew);
            if (use_lds) {
                if (ca >= 0 && ca < L.n_cells && da != 0) atomicAdd(&sJ[copy][ca - lo], (unsigned long long)da);
                if (cb >= 0 && db != 0) atomicAdd(&sJ[copy][cb - lo], (unsigned long long)db);
                if (cnew != DEAD_CELL) atomicAdd(&sH[cnew - lo], 1);
            } else {
                if (ca >= 0 && ca < L.n_cells && da != 0) atomicAdd(&Jg[ca], (unsigned long long)da);
                if (cb >= 0 && db != 0) atomicAdd(&Jg[cb], (unsigned long long)db);
                if (cnew != DEAD_CELL) atomicAdd(&Hg[4 * (size_t)cnew], 1);
            }
        }
        flush_counts(a, line, cnt);
        __syncthreads();
        // flush the window
        for (int c = threadIdx.x; c < span; c += PUSH_TPB) {
            unsigned long long s = 0;
#pragma unroll
            for (int r = 0; r < NCOPY; ++r) s += sJ[r][c];
            if (s != 0ull) atomicAdd(&Jg[lo + c], s);
            if (sH[c] != 0) atomicAdd(&Hg[4 * (size_t)(lo + c)], sH[c]);
        }
        __syncthreads();
    }
}

template __global__ void k_push<RICS_OFF>(PushArgs);
template __global__ void k_push<RICS_EXACT>(PushArgs);
template __global__ void k_push<RICS_TABLE>(PushArgs);

// ---------------------------------------------------------------------------
// Atmosphere (Appendix B.1): every layer cell is refilled to its hydrostatic
// target with co-located (e-, ion) pairs; one wavefront per layer cell.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_atmosphere(AtmArgs a) {
    if (a.sc->err != 0) return;
    const uint64_t step = a.sc->step;
    int32_t* hist_out = a.hist[(step & 1) ^ 1];
    const int lane = threadIdx.x & 63;
    const int wglob = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nw = (gridDim.x * blockDim.x) >> 6;
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
            atomicAdd(&a.counters[line * NCOUNT + 7], (unsigned long long)D);
        }
    }
}

// ---------------------------------------------------------------------------
// Per-step bookkeeping shared by k_field and k_plan: live counts <- allocation
// counters (clamped to capacity), tile plan of the next push.
// ---------------------------------------------------------------------------
__device__ void bookkeeping(const BookArgs& b) {
    if (b.sc->err != 0) return;
    __shared__ int sPart[256];
    const int nseg = b.nseg;
    const int per = (nseg + 255) / 256;
    const int s0 = threadIdx.x * per;
    int sum = 0;
    for (int s = s0; s < min(s0 + per, nseg); ++s) {
        const int n = min(b.alloc[s], b.seg_cap[s]);
        b.n_cur[s] = n;
        b.alloc[s] = n;
        sum += (n + PUSH_TILE - 1) / PUSH_TILE;
    }
    sPart[threadIdx.x] = sum;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int v = (threadIdx.x >= o) ? sPart[threadIdx.x - o] : 0;
        __syncthreads();
        sPart[threadIdx.x] += v;
        __syncthreads();
    }
    int run = sPart[threadIdx.x] - sum;     // exclusive prefix
    for (int s = s0; s < min(s0 + per, nseg); ++s) {
        b.tile_prefix[s] = run;
        run += (b.n_cur[s] + PUSH_TILE - 1) / PUSH_TILE;
    }
    if (threadIdx.x == 255) b.tile_prefix[nseg] = sPart[255];
}

// Bookkeeping kernel of every step (and after init, sort, set_particles): one block.
__global__ __launch_bounds__(256) void k_plan(BookArgs b, int advance_step) {
    bookkeeping(b);
    if (advance_step && threadIdx.x == 0 && b.sc->err == 0) b.sc->step += 1;
}

// Ampere's law with the static twist current (Sec. 3): E -= 4 pi (j - j_twist),
// plus time averages and the reset of the step's accumulators.
__global__ __launch_bounds__(256) void k_field(FieldArgs f) {
    if (f.sc->err != 0) return;
    const int n = f.n_total;
    const int hin = (int)(f.sc->step & 1);
    int* hist_in = f.hist[hin];
    const int* hist_out = f.hist[hin ^ 1];
    const bool averaging = f.avg_start >= 0 && f.sc->step >= (uint64_t)f.avg_start;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n; g += gridDim.x * blockDim.x) {
        const int line = f.cell_line[g];
        const LineDev& L = f.lines[line];
        const long long J = (long long)f.J[g];
        const double j = (double)J * FIX_INV * L.Q;
        f.J[g] = 0ull;
        f.j_last[g] = j;
        if (!f.frozen) f.E[g] -= 4.0 * 3.14159265358979323846 * (j - L.j_tw);
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
    if (averaging && blockIdx.x == 0 && threadIdx.x == 0) f.avg_count[0] += 1;
}

// ---------------------------------------------------------------------------
// Sort by cell (counting sort per segment), dropping absorbed particles.
// k_sort_scan: one block per segment, exclusive scan of the per-cell counts of
// that species into cursor[cell][species]; also the new live count.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_sort_scan(SortArgs s) {
    __shared__ long long sPart[1024];
    if (s.sc->err != 0) return;
    const int seg = blockIdx.x;
    const int line = seg >> 2, sp = seg & 3;
    const LineDev& L = s.lines[line];
    const int n = L.n_cells;
    const int per = (n + 1023) / 1024;
    const int c0 = threadIdx.x * per;
    const int32_t* hist = s.hist[s.sc->step & 1];
    long long sum = 0;
    for (int c = c0; c < min(c0 + per, n); ++c) sum += hist[4 * (size_t)(L.cell_base + c) + sp];
    sPart[threadIdx.x] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const long long v = (threadIdx.x >= o) ? sPart[threadIdx.x - o] : 0;
        __syncthreads();
        sPart[threadIdx.x] += v;
        __syncthreads();
    }
    long long run = sPart[threadIdx.x] - sum;
    for (int c = c0; c < min(c0 + per, n); ++c) {
        s.cursor[4 * (size_t)(L.cell_base + c) + sp] = (int)run;
        run += hist[4 * (size_t)(L.cell_base + c) + sp];
    }
    if (threadIdx.x == 1023) s.new_count[seg] = (int)sPart[1023];
}

// k_sort_scatter: every live particle takes the next slot of its cell; lanes of a
// wavefront that share a cell reserve their slots with one atomic.
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
        const int i0 = (t - s.tile_prefix[seg]) * PUSH_TILE;
        for (int q = 0; q < PUSH_PPT; ++q) {
            const int i = i0 + q * PUSH_TPB + threadIdx.x;
            const int c = (i < ncur) ? s.cell[base + i] : DEAD_CELL;
            bool pending = (c != DEAD_CELL);
            int pos = 0;
            unsigned long long act = __ballot(pending);
            while (act) {
                const int leader = __ffsll((long long)act) - 1;
                const int cl = __shfl(c, leader, 64);
                const unsigned long long m = __ballot(pending && c == cl);
                int basepos = 0;
                if (lane == leader) basepos = atomicAdd(&s.cursor[4 * (size_t)(L.cell_base + cl) + sp], __popcll(m));
                basepos = __shfl(basepos, leader, 64);
                if (pending && c == cl) {
                    pos = basepos + __popcll(m & ((1ull << lane) - 1ull));
                    pending = false;
                    if (pos < cap) {
                        const int64_t src = base + i, dst = base + pos;
                        s.cell2[dst] = c;
                        s.off2[dst] = s.off[src];
                        s.u2[dst] = s.u[src];
                        s.id2[dst] = s.id[src];
                    } else {
                        set_error(&s.sc->err, -3);
                    }
                }
                act &= ~m;
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
        const int i0 = (t - h.tile_prefix[seg]) * PUSH_TILE;
        for (int q = 0; q < PUSH_PPT; ++q) {
            const int i = i0 + q * PUSH_TPB + threadIdx.x;
            if (i >= ncur) continue;
            const int c = h.cell[base + i];
            if (c != DEAD_CELL) atomicAdd(&h.hist[4 * (size_t)(L.cell_base + c) + sp], 1);
        }
    }
}

// ---------------------------------------------------------------------------
// Moments: cloud-in-cell charge on nodes (fixed point), kinetic energy.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_moments_particles(MomArgs m) {
    __shared__ double sK[4];
    const int total = m.tile_prefix[m.nseg];
    double kin = 0.0;
    for (TileWalk tw(total); tw.t < tw.end; tw.t += tw.stride) {
        const int t = tw.t;
        const int seg = find_segment(m.tile_prefix, m.nseg, t);
        const int line = seg >> 2, sp = seg & 3;
        if (line != m.line) continue;
        const LineDev& L = m.lines[line];
        const int ncur = m.n_cur[seg];
        const int64_t base = m.seg_base[seg];
        const int i0 = (t - m.tile_prefix[seg]) * PUSH_TILE;
        const double qs = m.sign[sp] * FIX_SCALE;
        const double mass = (sp == 3) ? m.mass_ratio : 1.0;
        for (int q = 0; q < PUSH_PPT; ++q) {
            const int i = i0 + q * PUSH_TPB + threadIdx.x;
            if (i >= ncur) continue;
            const int c = m.cell[base + i];
            if (c == DEAD_CELL) continue;
            const double o = (double)m.off[base + i];
            const double u = (double)m.u[base + i];
            atomicAdd(&m.rho[c], (unsigned long long)__double2ll_rn((1.0 - o) * qs));
            atomicAdd(&m.rho[c + 1], (unsigned long long)__double2ll_rn(o * qs));
            kin += mass * L.Q * (double)L.C * (double)L.C * (sqrt(1.0 + u * u) - 1.0);
        }
    }
    for (int o = 32; o > 0; o >>= 1) kin += __shfl_xor(kin, o, 64);
    if ((threadIdx.x & 63) == 0) sK[threadIdx.x >> 6] = kin;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double s = sK[0] + sK[1] + sK[2] + sK[3];
        if (s != 0.0) atomicAdd(&m.out[2], s);
    }
}

// Gauss residual on interior nodes, circuit potential and field energy of one line.
__global__ __launch_bounds__(256) void k_moments_grid(MomArgs m) {
    const LineDev& L = m.lines[m.line];
    const int n = L.n_cells;
    double rmax = 0.0, esum = 0.0, e2 = 0.0;
    const double* E = m.E + L.cell_base;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += gridDim.x * blockDim.x) {
        if (i < n) { esum += E[i]; e2 += E[i] * E[i]; }
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
        atomicAdd(&m.out[1], esum);
        atomicAdd(&m.out[3], e2);
    }
}

// RICS backend evaluation at given points (diagnostics and surrogate error).
template <int BACKEND>
__global__ __launch_bounds__(256) void k_rics_eval(PushArgs a, int line, int64_t n, const float* s_cells,
                                                   const float* uin, float* F, float* N, float* eps) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const LineDev L = a.lines[line];
    const float s = fminf(fmaxf(s_cells[i], 0.0f), (float)L.n_cells);
    int c0 = min((int)floorf(s), L.n_cells - 1);
    const float o0 = s - (float)c0;
    const Geo g = geo_at(a.nodes, L.node_base + c0, o0);
    const float u = uin[i];
    RicsOut r;
    if constexpr (BACKEND == RICS_OFF) { r.F = 0.0f; r.dF = 0.0f; r.N = 0.0f; }
    else r = rics_eval<BACKEND>(a, L, u, g, c0, o0);
    F[i] = r.F;
    N[i] = r.N;
    eps[i] = photon_energy(sqrtf(fmaf(u, u, 1.0f)), g.b);
}
template __global__ void k_rics_eval<RICS_OFF>(PushArgs, int, int64_t, const float*, const float*, float*, float*, float*);
template __global__ void k_rics_eval<RICS_EXACT>(PushArgs, int, int64_t, const float*, const float*, float*, float*, float*);
template __global__ void k_rics_eval<RICS_TABLE>(PushArgs, int, int64_t, const float*, const float*, float*, float*, float*);

}  // namespace pic1d

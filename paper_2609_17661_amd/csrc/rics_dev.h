// RICS drag force, scattering rate and photon energy as evaluated inside the
// pusher (float32).
//
// Closed forms (Sec. 2.2, Eqs. scatteringNdot and contdrag, with the radial
// beam subtending pi/x^2 sr; normalised to m_e c^2/R* and c/R*):
//   y     = b / (Theta gamma (1 - beta mu))
//   F_hat = A_F / x^2 * (gamma mu - u) * y^3 / (e^y - 1)
//   Ndot  = A_N / (x^2 gamma) * y^2 / (e^y - 1)
// and the perpendicular-emission photon energy of Appendix A.3 (Eq. perpemit)
//   eps = gamma (1 - (1 + 2b)^(-1/2)) = gamma 2b / (q (1 + q)),  q = (1 + 2b)^(1/2).
// The table backend interpolates F_hat and Ndot bilinearly in (log10 gamma, s)
// for u >= 0 and mirrors u < 0 through F(-u, s) = -F(u, L - s).
//
// The hardware square root, reciprocal and log2 (1 ulp) are used directly; the
// comparisons with the float64 oracle budget for them.
#pragma once

#include "pic1d_dev.h"

namespace pic1d {

__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }

// Geometry of a particle (linear between the nodes of its cell), in the form the
// RICS functions use it.
struct Geo {
    float b;      // B / B_QED
    float mu;     // photon-field cosine
    float by;     // b / Theta
    float ix2;    // (R* / r)^2
};

// F_hat of the closed form at u, with what dF/du needs.  With w = gamma mu - u and
// d = gamma - u mu: dw/du = -(d/gamma), dy/du = y w / (gamma d),
// d(y^3/(e^y-1))/dy = g3 (3/y - 1 - 1/(e^y - 1)).
struct ExactEval {
    float F;
    float gam, d, y, r, w, Ag3;     // (Ag3 = A_F x^-2 y^3 / (e^y - 1))
    bool inside;                    // below the Planck cutoff (else F = dF/du = 0)
    __device__ __forceinline__ float dF() const {
        if (!inside) return 0.0f;
        const float ig = frcp(gam);
        const float dy = y * w * ig * frcp(d);
        return Ag3 * (-(d * ig) + w * (3.0f * frcp(y) - 1.0f - r) * dy);
    }
};

__device__ __forceinline__ ExactEval exact_eval(const LineDev& L, float u, const Geo& g) {
    ExactEval e;
    e.gam = fsqrt(fmaf(u, u, 1.0f));
    e.d = fmaf(-u, g.mu, e.gam);
    e.y = g.by * frcp(e.d);
    e.inside = e.y <= Y_CUT;
    e.r = e.w = e.Ag3 = 0.0f;
    e.F = 0.0f;
    if (e.inside) {
        e.r = frcp(expm1f(e.y));
        e.Ag3 = L.A_F * g.ix2 * (e.y * e.y * e.y * e.r);
        e.w = fmaf(e.gam, g.mu, -u);
        e.F = e.Ag3 * e.w;
    }
    return e;
}

__device__ __forceinline__ float exact_N(const LineDev& L, float u, const Geo& g) {
    const float gam = fsqrt(fmaf(u, u, 1.0f));
    const float y = g.by * frcp(fmaf(-u, g.mu, gam));
    if (!(y <= Y_CUT)) return 0.0f;
    return L.A_N * g.ix2 * y * y * frcp(expm1f(y) * gam);
}

// Table rows of a particle: byte offset of row j0 within the line's table and the
// weight wj of row j0 + 1, for the u >= 0 half at x (cells) and for the mirrored
// u < 0 half at L - x.  Row j sits at x = (j + 1/2) / s_scale.
struct TabRow {
    int off;        // j0 * nlg * 16
    float wj;
};

struct TabRows {
    TabRow pos, neg;
};

// General form, in float64 from the position x (the pusher takes it only where
// a cell straddles a row or the clamped ends; elsewhere the rows are per cell).
__device__ __forceinline__ TabRow table_row(const LineDev& L, int ns, int nlg16, double xm) {
    double fj = fma(xm, L.s_scale, -0.5);
    fj = fmin(fmax(fj, 0.0), (double)(ns - 1));
    const int j0 = min((int)fj, ns - 2);
    TabRow r;
    r.off = j0 * nlg16;
    r.wj = (float)(fj - (double)j0);
    return r;
}

__device__ __forceinline__ TabRows table_rows(const LineDev& L, int ns, int nlg16, double x) {
    TabRows r;
    r.pos = table_row(L, ns, nlg16, x);
    r.neg = table_row(L, ns, nlg16, (double)L.n_cells - x);
    return r;
}

// Column position along log10 gamma: i0 and weight wi, from the fractional column
// lgk log2(gamma^2) with the hardware log2 (1 ulp: an absolute error of the weight
// below 2e-5 over the table's 8 decades).
struct TabCol {
    int i0;
    float wi;
    float g2;         // gamma^2
    bool inside;      // strictly inside the table (derivative non-zero)
};

__device__ __forceinline__ TabCol table_col(const LineDev& L, int nlg, float ua) {
    TabCol c;
    c.g2 = fmaf(ua, ua, 1.0f);
    const float r = fmaxf(__builtin_amdgcn_logf(c.g2) * L.lgk, 0.0f);
    const float fr = floorf(r);
    const int i = (int)fr;
    const int i0 = min(i, nlg - 2);
    // above the table the weight clamps to 1
    const float wi = fminf((r - fr) + (float)(i - i0), 1.0f);
    c.inside = (i == i0) && !(i == 0 && wi == 0.0f);
    c.i0 = i0;
    c.wi = wi;
    return c;
}

// The last table record a lane read: its byte offset (row j0, column i0, half)
// and the two row pairs.  Consecutive evaluations of a lane often read the same
// record (particles of one cell at similar gamma); they reuse it without a load.
struct TabMemo {
    uint32_t o = 0xffffffffu;
    float2 a, b;
};

// The table is stored as [ns][nlg] float4 {F(i), F(i+1), Ndot(i), Ndot(i+1)} so that
// one gather per row brings both columns of a quantity.  tb is the line's table,
// tb1 = tb + nlg * 16 bytes (row j0 + 1 at the same offset).
template <int HALF>      // 0: F, 1: Ndot
__device__ __forceinline__ float2 table_pair(const char* __restrict__ tb, const char* __restrict__ tb1,
                                             const TabRow& rw, const TabCol& cl, float& slope, TabMemo& m) {
    const uint32_t o = (uint32_t)rw.off + ((uint32_t)cl.i0 << 4) + 8u * HALF;
    float2 a, b;
    if (o == m.o) {
        a = m.a;
        b = m.b;
    } else {
        a = *reinterpret_cast<const float2*>(tb + o);      // row j0
        b = *reinterpret_cast<const float2*>(tb1 + o);     // row j0 + 1
        m.o = o;
        m.a = a;
        m.b = b;
    }
    const float fa = fmaf(rw.wj, b.x - a.x, a.x);                    // at column i0
    const float fc = fmaf(rw.wj, b.y - a.y, a.y);                    // at column i0 + 1
    slope = fc - fa;
    return make_float2(fa, fc);
}

// F_hat from the table at u, with what dF/du needs (the slope per column).
struct TableEval {
    float F, slope, ua, g2;
    bool inside;
    // d(fractional column)/d|u| = (nlg-1)/8 |u| / (gamma^2 ln 10); for u < 0,
    // d(-F(|u|))/du = +dF/d|u|
    __device__ __forceinline__ float dF(const LineDev& L) const {
        return inside ? slope * (float)L.lg_scale * ua * frcp(g2 * 2.302585093f) : 0.0f;
    }
};

__device__ __forceinline__ TableEval table_eval(const LineDev& L, const char* tb, const char* tb1, int nlg,
                                                const TabRows& rows, float u, TabMemo& m) {
    TableEval e;
    e.ua = fabsf(u);
    const TabCol cl = table_col(L, nlg, e.ua);
    const float2 f = table_pair<0>(tb, tb1, u < 0.0f ? rows.neg : rows.pos, cl, e.slope, m);
    const float F = fmaf(cl.wi, e.slope, f.x);
    e.F = u < 0.0f ? -F : F;
    e.g2 = cl.g2;
    e.inside = cl.inside;
    return e;
}

__device__ __forceinline__ float table_N(const LineDev& L, const char* tb, const char* tb1, int nlg,
                                         const TabRows& rows, float u, TabMemo& m) {
    const TabCol cl = table_col(L, nlg, fabsf(u));
    float slope;
    const float2 n = table_pair<1>(tb, tb1, u < 0.0f ? rows.neg : rows.pos, cl, slope, m);
    return fmaf(cl.wi, slope, n.x);
}

__device__ __forceinline__ float photon_energy(float gam, float b) {
    const float q = fsqrt(fmaf(2.0f, b, 1.0f));
    return gam * (2.0f * b) * frcp(q * (1.0f + q));
}

// Rest-frame emission cosine from words 2-4 of the event's Philox block (the first
// decides the event).  Pattern 1: uniform on [-1, 1], 2 U1 - 1.  Pattern 2: density
// 3/8 (1 + c^2), sampled as the mixture of the uniform (weight 3/4) and, when bits 0
// and 1 of the second word are clear (weight 1/4), the density 3/2 c^2, whose |c| is
// the largest of three uniforms and whose sign is bit 2.  Every draw is exact in
// float32.
__device__ __forceinline__ float emission_cosine(const uint4& w, int pattern) {
    const float u1 = uniform24(w.y);
    if (pattern == 1 || (w.y & 3u) != 0u) return fmaf(2.0f, u1, -1.0f);
    const float top = fmaxf(u1, fmaxf(uniform24(w.z), uniform24(w.w)));
    return (w.y & 4u) ? -top : top;
}

// One event whose photon leaves the excited lepton's rest frame at cosine c from its
// motion (Appendix A.2-A.3).  Rest frame: E_gamma(theta) = (q - 1/q) / (1 + (c^2 +
// (1 - c^2)/q^2)^1/2), the printed form without its 0/0 at c = +-1 (q = E_B/m_e c^2 =
// (1+2b)^1/2); the lepton keeps E_e = q - E_gamma and momentum -E_gamma c along the
// motion.  Both are boosted back with gamma_e = gamma / q (Eq. scatlim1; no boost where
// gamma_e < 1).  1 - beta_e = 1/(gamma_e^2 (1 + beta_e)) keeps the Doppler factors
// exact where they cancel: 1 + beta_e c for c < 0, and E_e - beta_e E_gamma c =
// 1/(E_e + E_gamma c) + E_gamma c (1 - beta_e) for c >= 0 (rest-frame mass shell).
// Returns the lab photon energy; u receives the lepton's momentum (dir = its sign
// before the event).
__device__ __forceinline__ float angled_event(float gam, float b, float c, float dir, float& u) {
    const float q2 = fmaf(2.0f, b, 1.0f);
    const float iq = frsq(q2), q = q2 * iq;
    const float ge = gam * iq;
    const float g2m1 = (ge - 1.0f) * (ge + 1.0f);
    const bool boost = g2m1 > 0.0f;
    const float be = boost ? fsqrt(g2m1) * frcp(ge) : 0.0f;
    const float omb = boost ? frcp(ge * ge * (1.0f + be)) : 1.0f;
    const float s2 = (1.0f - c) * (1.0f + c);
    const float eg = (q - iq) * frcp(1.0f + fsqrt(fmaf(c, c, s2 * iq * iq)));
    const float ee = q - eg, egc = eg * c;
    const bool fwd = c >= 0.0f;
    const float dopp = fwd ? fmaf(be, c, 1.0f) : fmaf(be, 1.0f + c, omb);
    const float gn = ge * (fwd ? fmaf(egc, omb, frcp(ee + egc)) : fmaf(-be, egc, ee));
    const float m = fsqrt(fmaxf((gn - 1.0f) * (gn + 1.0f), 0.0f));
    u = (fmaf(be, ee, -egc) >= 0.0f) ? dir * m : -dir * m;
    return ge * eg * dopp;
}

}  // namespace pic1d

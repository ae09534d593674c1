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

// F_hat and, if DF, dF/du of the closed form.  With w = gamma mu - u and
// d = gamma - u mu: dw/du = -(d/gamma), dy/du = y w / (gamma d),
// d(y^3/(e^y-1))/dy = g3 (3/y - 1 - 1/(e^y - 1)).
template <bool DF>
__device__ __forceinline__ float exact_F(const LineDev& L, float u, const Geo& g, float& dF) {
    const float gam = fsqrt(fmaf(u, u, 1.0f));
    const float d = fmaf(-u, g.mu, gam);
    const float y = g.by * frcp(d);
    if (!(y <= Y_CUT)) {
        if (DF) dF = 0.0f;
        return 0.0f;
    }
    const float r = frcp(expm1f(y));
    const float g3 = y * y * y * r;
    const float w = fmaf(gam, g.mu, -u);
    const float A = L.A_F * g.ix2;
    if (DF) {
        const float ig = frcp(gam);
        const float dy = y * w * ig * frcp(d);
        dF = A * g3 * (-(d * ig) + w * (3.0f * frcp(y) - 1.0f - r) * dy);
    }
    return A * w * g3;
}

__device__ __forceinline__ float exact_N(const LineDev& L, float u, const Geo& g) {
    const float gam = fsqrt(fmaf(u, u, 1.0f));
    const float y = g.by * frcp(fmaf(-u, g.mu, gam));
    if (!(y <= Y_CUT)) return 0.0f;
    return L.A_N * g.ix2 * y * y * frcp(expm1f(y) * gam);
}

// Table position along s of a particle at x (cells): row j0 and weight wj, for the
// u >= 0 half (x) and for the mirrored u < 0 half (L - x).  Formed once per
// particle in float64 (the position does not change during the push).
struct TabRow {
    int j0;
    float wj;
};

__device__ __forceinline__ TabRow table_row(const LineDev& L, int ns, double xm) {
    double fj = fma(xm, L.s_scale, -0.5);
    fj = fmin(fmax(fj, 0.0), (double)(ns - 1));
    TabRow r;
    r.j0 = min((int)fj, ns - 2);
    r.wj = (float)(fj - (double)r.j0);
    return r;
}

// Column position along log10 gamma: i0 and weight wi.  log2 gamma is split into
// the exponent ex and log2 of the mantissa; ex * K is formed exactly from a
// 10-fraction-bit head of K = (nlg-1)/8 * log10(2), so that the weight carries an
// absolute error of about 1e-6 in float32.
struct TabCol {
    int i0;
    float wi;
    bool inside;      // strictly inside the table (derivative non-zero)
};

__device__ __forceinline__ TabCol table_col(const LineDev& L, int nlg, float ua) {
    const float gam = fsqrt(fmaf(ua, ua, 1.0f));
    const unsigned bits = __float_as_uint(gam);
    const int ex = (int)((bits >> 23) & 0xffu) - 126;                          // gam = man 2^ex
    const float man = __uint_as_float((bits & 0x007fffffu) | 0x3f000000u);      // man in [0.5, 1)
    const float l2m = __builtin_amdgcn_logf(man);                                // in [-1, 0)
    const float head = (float)ex * L.lgk_hi;                                     // exact
    const float ih = floorf(head);
    const float r = (head - ih) + fmaf((float)ex, L.lgk_lo, l2m * L.lgk);
    const float fr = floorf(r);
    int i0 = (int)ih + (int)fr;
    float wi = r - fr;
    TabCol c;
    c.inside = (i0 >= 0) && (i0 < nlg - 1) && !(i0 == 0 && wi == 0.0f);
    if (i0 < 0) { i0 = 0; wi = 0.0f; }
    if (i0 > nlg - 2) { i0 = nlg - 2; wi = 1.0f; }
    c.i0 = i0;
    c.wi = wi;
    return c;
}

// The table is stored as [ns][nlg] float4 {F(i), F(i+1), Ndot(i), Ndot(i+1)} so that
// one 16-byte gather per row brings both columns of both quantities.
struct TabVal {
    float F, slopeF, N;
};

__device__ __forceinline__ TabVal table_interp(const float4* __restrict__ T, int nlg, const TabRow& rw,
                                               const TabCol& cl) {
    const float4* t = T + (rw.j0 * nlg + cl.i0);
    const float4 a = t[0];        // row j0
    const float4 b = t[nlg];      // row j0 + 1
    const float fa = fmaf(rw.wj, b.x - a.x, a.x);      // F at i0
    const float fc = fmaf(rw.wj, b.y - a.y, a.y);      // F at i0 + 1
    const float na = fmaf(rw.wj, b.z - a.z, a.z);
    const float nc = fmaf(rw.wj, b.w - a.w, a.w);
    TabVal v;
    v.slopeF = fc - fa;
    v.F = fmaf(cl.wi, fc - fa, fa);
    v.N = fmaf(cl.wi, nc - na, na);
    return v;
}

// Table rows of a particle for both signs of u.
struct TabRows {
    TabRow pos, neg;
};

__device__ __forceinline__ TabRows table_rows(const LineDev& L, int ns, double x) {
    TabRows r;
    r.pos = table_row(L, ns, x);
    r.neg = table_row(L, ns, (double)L.n_cells - x);
    return r;
}

template <bool DF>
__device__ __forceinline__ float table_F(const LineDev& L, const float4* __restrict__ tab, int nlg, const TabRows& rows,
                                         float u, float& dF) {
    const float ua = fabsf(u);
    const TabCol cl = table_col(L, nlg, ua);
    const TabVal v = table_interp(tab, nlg, u < 0.0f ? rows.neg : rows.pos, cl);
    if (DF) {
        // d(fractional index)/d|u| = (nlg-1)/8 |u| / (gamma^2 ln 10); for u < 0,
        // d(-F(|u|))/du = +dF/d|u|
        dF = cl.inside ? v.slopeF * (float)L.lg_scale * ua * frcp(fmaf(ua, ua, 1.0f) * 2.302585093f) : 0.0f;
    }
    return u < 0.0f ? -v.F : v.F;
}

__device__ __forceinline__ float table_N(const LineDev& L, const float4* __restrict__ tab, int nlg,
                                         const TabRows& rows, float u) {
    const TabCol cl = table_col(L, nlg, fabsf(u));
    return table_interp(tab, nlg, u < 0.0f ? rows.neg : rows.pos, cl).N;
}

__device__ __forceinline__ float photon_energy(float gam, float b) {
    const float q = fsqrt(fmaf(2.0f, b, 1.0f));
    return gam * (2.0f * b) * frcp(q * (1.0f + q));
}

}  // namespace pic1d

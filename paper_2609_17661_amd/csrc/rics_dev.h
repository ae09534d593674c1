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
#pragma once

#include "pic1d_dev.h"

namespace pic1d {

struct Geo {
    float b, mu, xr, rc;
};

struct RicsOut {
    float F, dF, N;
};

// dF/du of the closed form: with w = gamma mu - u and d = gamma - u mu,
// dw/du = -(d/gamma), dy/du = y w / (gamma d), g3' = g3 (3/y - 1 - 1/(e^y - 1)).
__device__ __forceinline__ RicsOut rics_exact(const LineDev& L, float u, const Geo& g) {
    RicsOut o;
    const float gam = sqrtf(fmaf(u, u, 1.0f));
    const float d = fmaf(-u, g.mu, gam);
    const float y = g.b * L.inv_theta / d;
    if (!(y <= Y_CUT)) {
        o.F = 0.0f; o.dF = 0.0f; o.N = 0.0f;
        return o;
    }
    const float em1 = expm1f(y);
    const float r = 1.0f / em1;
    const float g2 = y * y * r;
    const float g3 = g2 * y;
    const float ix2 = 1.0f / (g.xr * g.xr);
    const float w = fmaf(gam, g.mu, -u);
    const float ig = 1.0f / gam;
    o.F = L.A_F * ix2 * w * g3;
    o.N = L.A_N * ix2 * g2 * ig;
    const float dy = y * w * ig / d;
    o.dF = L.A_F * ix2 * (-(d * ig) * g3 + w * g3 * (3.0f / y - 1.0f - r) * dy);
    return o;
}

// Table lookup.  tab points at this line's F table ([ns][nlg], log10 gamma
// fastest), followed by the Ndot table.  x_mirror is the arc length in cells
// already mirrored to L - s for u < 0.  The fractional table indices are formed
// in float64 (log2 gamma split into exponent and mantissa) so that their
// rounding stays far below the interpolation weights' resolution.
__device__ __forceinline__ RicsOut rics_table(const LineDev& L, const float* __restrict__ tab,
                                              int nlg, int ns, float u, double x_mirror) {
    RicsOut o;
    const float ua = fabsf(u);
    const float gam = sqrtf(fmaf(ua, ua, 1.0f));
    int ex;
    const float man = frexpf(gam, &ex);                       // gam = man 2^ex, man in [0.5, 1)
    const double lg2 = (double)ex + (double)log2f(man);
    double fi = lg2 * (L.lg_scale * 0.30102999566398120);   // log10(gamma) (nlg-1)/8
    const bool inside_i = (fi > 0.0) && (fi < (double)(nlg - 1));
    fi = fmin(fmax(fi, 0.0), (double)(nlg - 1));
    double fj = fma(x_mirror, L.s_scale, -0.5);
    fj = fmin(fmax(fj, 0.0), (double)(ns - 1));
    const int i0 = min((int)fi, nlg - 2);
    const int j0 = min((int)fj, ns - 2);
    const float wi = (float)(fi - (double)i0);
    const float wj = (float)(fj - (double)j0);
    const float* F = tab + (size_t)j0 * nlg + i0;
    const float* N = F + (size_t)nlg * ns;
    const float f00 = F[0], f01 = F[1], f10 = F[nlg], f11 = F[nlg + 1];
    const float n00 = N[0], n01 = N[1], n10 = N[nlg], n11 = N[nlg + 1];
    const float fa = fmaf(wj, f10 - f00, f00);      // at i0
    const float fc = fmaf(wj, f11 - f01, f01);      // at i0 + 1
    const float na = fmaf(wj, n10 - n00, n00);
    const float nc = fmaf(wj, n11 - n01, n01);
    const float Ft = fmaf(wi, fc - fa, fa);
    o.N = fmaf(wi, nc - na, na);
    const float dfi = inside_i ? (float)L.lg_scale * ua / (gam * gam * 2.302585093f) : 0.0f;
    o.dF = (fc - fa) * dfi;
    o.F = (u < 0.0f) ? -Ft : Ft;
    return o;
}

__device__ __forceinline__ float photon_energy(float gam, float b) {
    const float q = sqrtf(fmaf(2.0f, b, 1.0f));
    return gam * (2.0f * b) / (q * (1.0f + q));
}

}  // namespace pic1d

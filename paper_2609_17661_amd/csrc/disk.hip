// RICS table of the finite stellar disk (PIC1D_FIELD_DISK), built on the device
// in float64.
//
// Sec. 2.2 evaluates the scattering rate (Eq. scatteringNdot) and the drag force
// (Eq. contdrag) for photons streaming radially from the star; Sec. 5 notes that
// the real field differs.  Here the star is a uniform disk filling the cone of
// half-angle theta_d = asin(1/x) around the radial direction.  A photon at polar
// angle t from the radial direction and azimuth phi about it crosses the field at
//   mu' = mu cos t + (1 - mu^2)^(1/2) sin t cos phi,
// resonates at y = b / (Theta gamma (1 - beta mu')), and the table stores
//   F_hat    = A_F / pi * sum_k w_k gamma (mu'_k - beta) y_k^3 / (e^y_k - 1)
//   Ndot_hat = A_N / (pi gamma) * sum_k w_k y_k^2 / (e^y_k - 1)
// over the product rule of n_c Gauss-Legendre nodes in cos t on [cos theta_d, 1]
// and n_phi in phi on [0, pi] (weights doubled: the integrand is even in phi).
// Taking the cone to pi/x^2 directions at mu' = mu gives back the radial beam.
// The table has the layout of the radial one: [ns][nlg] records
// {F(i), F(i+1), Ndot(i), Ndot(i+1)} at log10 gamma_i = 8 i/(nlg - 1) and row
// centres s_j = (j + 1/2) L / ns, u >= 0 (u < 0 by the mirror of the lookup).
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace pic1d {

namespace {

// cos(theta) at arc length s (R*) from the northern footpoint of r = R sin^2(theta):
// s(v) = (R/2)(P(v0) - P(v)), P(v) = v (1 + 3 v^2)^(1/2) + asinh(3^(1/2) v) / 3^(1/2)
// (Appendix B.2), by Newton safeguarded by the bracket [-v0, v0].
__device__ double disk_cos_at(double R, double s) {
    const double r3 = 1.7320508075688772;
    auto P = [&](double v) { return v * sqrt(1.0 + 3.0 * v * v) + asinh(r3 * v) / r3; };
    const double v0 = sqrt(1.0 - 1.0 / R);
    const double Pv0 = P(v0);
    const double L = R * Pv0;
    double lo = -v0, hi = v0;
    double v = v0 - 2.0 * v0 * s / L;
    for (int it = 0; it < 100; ++it) {
        const double f = 0.5 * R * (Pv0 - P(v)) - s;
        if (f > 0.0) lo = fmax(lo, v); else hi = fmin(hi, v);
        double vn = v + f / (R * sqrt(1.0 + 3.0 * v * v));
        if (!(vn > lo && vn < hi)) vn = 0.5 * (lo + hi);
        if (fabs(vn - v) <= 1e-16 * (1.0 + fabs(v))) { v = vn; break; }
        v = vn;
    }
    return v;
}

__global__ __launch_bounds__(256) void k_disk_table(DiskTableArgs a) {
    const int64_t total = (int64_t)a.ns * a.nlg;
    float* tab = reinterpret_cast<float*>(a.table);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e / a.nlg), i = (int)(e % a.nlg);
        // geometry at the row centre
        const double v = disk_cos_at(a.R, (j + 0.5) * a.L / a.ns);
        const double q = sqrt(1.0 + 3.0 * v * v);
        const double x = a.R * (1.0 - v * v);
        const double b = a.b_pole * q / (2.0 * x * x * x);
        const double mu = 2.0 * v / q;
        const double sm = sqrt(fmax(1.0 - mu * mu, 0.0));
        const double cd = sqrt(fmax(1.0 - 1.0 / (x * x), 0.0));
        // the column's momentum
        const double gam = pow(10.0, 8.0 * i / (a.nlg - 1));
        const double u = sqrt(fmax(gam * gam - 1.0, 0.0));
        const double beta = u / gam;
        double F = 0.0, N = 0.0;
        for (int k = 0; k < a.n_c; ++k) {
            const double c = 0.5 * (1.0 - cd) * a.gc[k] + 0.5 * (1.0 + cd);
            const double wc = 0.5 * (1.0 - cd) * a.wc[k];
            const double st = sqrt(fmax(1.0 - c * c, 0.0));
            for (int l = 0; l < a.n_phi; ++l) {
                const double phi = 0.5 * 3.14159265358979323846 * (a.gp[l] + 1.0);
                const double w = wc * (3.14159265358979323846 * a.wp[l]);
                const double mup = mu * c + sm * st * cos(phi);
                const double y = b / (a.theta * gam * (1.0 - beta * mup));
                if (!(y <= 80.0)) continue;
                const double p2 = y * y / expm1(y);
                F += w * gam * (mup - beta) * (p2 * y);
                N += w * p2;
            }
        }
        F *= a.AF / 3.14159265358979323846;
        N *= a.AN / (3.14159265358979323846 * gam);
        // record i holds columns i and i + 1: this column is the first of record i and
        // the second of record i - 1 (the last record repeats it, as the clamp needs)
        float* r = tab + 4 * ((size_t)j * a.nlg + i);
        r[0] = (float)F;
        r[2] = (float)N;
        if (i > 0) {
            r[-3] = (float)F;
            r[-1] = (float)N;
        }
        if (i == a.nlg - 1) {
            r[1] = (float)F;
            r[3] = (float)N;
        }
    }
}

}  // namespace

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on the three-term recurrence
// of P_n from the asymptotic first guesses), float64.
void gauss_legendre(int n, double* x, double* w) {
    for (int i = 0; i < n; ++i) {
        double z = cos(3.14159265358979323846 * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) <= 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

hipError_t launch_disk_table(const DiskTableArgs& a, hipStream_t s) {
    const int64_t total = (int64_t)a.ns * a.nlg;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_disk_table, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace pic1d

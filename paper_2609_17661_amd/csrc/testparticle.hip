// Test particles under RICS drag along dipole field lines (Appendix A.4, Fig. 6):
// one thread per field line integrates a lepton injected at the northern
// footpoint with gamma_0, moving away from the star under the drag force of
// Eq. contdrag alone, and reads off the minimum Lorentz factor the drag imposes
// on the way to the equator, where its first scattering happens (the expected
// number of scatterings, the integral of Ndot along the path, reaching 1;
// Eq. scatteringNdot) and the extent of the pair-production zone from there to
// where b drops below the pair threshold.
//
// Equations in t_hat = c t / R*, the position as v = cos(theta) on
// r = R sin^2(theta) (ds = -R (1 + 3 v^2)^(1/2) dv, Appendix B.2):
//   dv/dt = -beta / (R (1 + 3 v^2)^(1/2)),  du/dt = F_hat(u, v),  dN/dt = Ndot_hat(u, v),
// by the classical fourth-order Runge-Kutta method with the step limited by the
// drag's stiffness (|dF/du| dt), the relative change of u, the scatterings per
// step and the geometry's scale along the path; float64 throughout.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "../../include/pic1d.h"
#include "kernels.h"

namespace pic1d {

namespace {

struct TpLine {
    double R, b_pole, theta, AF, AN;
};

struct TpEval {
    double dv, F, dF, N, x;
};

__device__ __forceinline__ TpEval tp_eval(const TpLine& p, double v, double u) {
    const double q = sqrt(1.0 + 3.0 * v * v);
    const double x = p.R * (1.0 - v * v);
    const double b = p.b_pole * q / (2.0 * x * x * x);
    const double mu = 2.0 * v / q;
    const double gam = sqrt(1.0 + u * u);
    const double beta = u / gam;
    TpEval e;
    e.x = x;
    e.dv = -beta / (p.R * q);
    const double d = gam - u * mu;            // gamma (1 - beta mu)
    const double y = b / (p.theta * d);
    if (!(y <= 80.0)) {                       // the Planck cutoff of the radial beam
        e.F = e.dF = e.N = 0.0;
        return e;
    }
    const double em1 = expm1(y);
    const double g3 = y * y * y / em1;
    const double ix2 = 1.0 / (x * x);
    const double w = gam * mu - u;            // gamma (mu - beta)
    e.F = p.AF * ix2 * w * g3;
    e.N = p.AN * ix2 / gam * y * y / em1;
    // dF/du: dw/du = -(d / gamma), dy/du = y w / (gamma d), g3' = g3 (3/y - 1 - 1/(e^y - 1))
    const double dg3 = g3 * (3.0 / y - 1.0 - 1.0 / em1);
    e.dF = p.AF * ix2 * (-(d / gam) * g3 + w * dg3 * (y * w / (gam * d)));
    return e;
}

// v where b first falls to b_pp from the northern footpoint, or -1 if b >= b_pp on
// the whole line (b decreases monotonically towards the equator), by bisection
__device__ double tp_threshold_cos(double R, double b_pole, double b_pp) {
    auto bof = [&](double v) {
        const double r = R * (1.0 - v * v);
        return b_pole * sqrt(1.0 + 3.0 * v * v) / (2.0 * r * r * r);
    };
    if (bof(0.0) >= b_pp) return -1.0;
    double lo = 0.0, hi = sqrt(1.0 - 1.0 / R);
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (bof(mid) < b_pp) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

// arc length from the northern footpoint to cos(theta) = v
__device__ __forceinline__ double tp_s_of(double R, double v) {
    const double r3 = 1.7320508075688772;
    auto P = [&](double w) { return w * sqrt(1.0 + 3.0 * w * w) + asinh(r3 * w) / r3; };
    return 0.5 * R * (P(sqrt(1.0 - 1.0 / R)) - P(v));
}

__global__ __launch_bounds__(64) void k_testparticle(pic1d_tp_config c, int n, const double* r_eq,
                                                    pic1d_tp_result* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double R = r_eq[i];
    const double theta = c.kT_keV / 510.99895000;
    const double base = 2.8179403262e-13 * 1.0e6 / (4.0 * 3.8615926796e-11 * 3.8615926796e-11);
    const TpLine p{R, c.b_pole, theta, base * theta * theta * theta, base * theta * theta};
    const double v0 = sqrt(1.0 - 1.0 / R);
    const double L = tp_s_of(R, -v0);
    double v = v0, u = sqrt(fmax(c.gamma0 * c.gamma0 - 1.0, 0.0)), N = 0.0, t = 0.0;
    double gmin = sqrt(1.0 + u * u), s_first = -1.0;
    int crossed = 0;
    long long steps = 0;
    const double t_end = c.t_max * L;
    while (t < t_end && steps < c.max_steps) {
        const TpEval e = tp_eval(p, v, u);
        // step: stiffness, relative change of u, scatterings, geometry scale
        double dt = c.dt_max;
        if (e.dF != 0.0) dt = fmin(dt, c.tol_stiff / fabs(e.dF));
        if (e.F != 0.0) dt = fmin(dt, c.tol * fmax(fabs(u), 1e-2) / fabs(e.F));
        if (e.N > 0.0 && s_first < 0.0) dt = fmin(dt, c.tol / e.N);   // until the first scattering
        if (e.dv != 0.0) dt = fmin(dt, c.tol * fmax(fabs(v), 1e-3) / fabs(e.dv));
        dt = fmin(dt, t_end - t);
        const TpEval k2 = tp_eval(p, v + 0.5 * dt * e.dv, u + 0.5 * dt * e.F);
        const TpEval k3 = tp_eval(p, v + 0.5 * dt * k2.dv, u + 0.5 * dt * k2.F);
        const TpEval k4 = tp_eval(p, v + dt * k3.dv, u + dt * k3.F);
        const double vn = v + dt / 6.0 * (e.dv + 2.0 * k2.dv + 2.0 * k3.dv + k4.dv);
        const double un = u + dt / 6.0 * (e.F + 2.0 * k2.F + 2.0 * k3.F + k4.F);
        const double Nn = N + dt / 6.0 * (e.N + 2.0 * k2.N + 2.0 * k3.N + k4.N);
        ++steps;
        if (s_first < 0.0 && Nn >= 1.0) {
            // the first scattering inside the step, by linear interpolation in N
            const double w = (1.0 - N) / (Nn - N);
            s_first = tp_s_of(R, v + w * (vn - v));
        }
        if (vn < 0.0) {
            // the equator inside the step: u there by linear interpolation in v
            const double w = v / (v - vn);
            const double ue = u + w * (un - u);
            gmin = fmin(gmin, sqrt(1.0 + ue * ue));
            crossed = 1;
            break;
        }
        v = vn;
        u = un;
        N = Nn;
        t += dt;
        gmin = fmin(gmin, sqrt(1.0 + u * u));
    }
    const double vb = tp_threshold_cos(R, c.b_pole, c.b_pp);
    const double s_b = vb >= 0.0 ? tp_s_of(R, vb) : -1.0;
    double l_pp = 0.0;
    if (s_first >= 0.0) l_pp = s_b >= 0.0 ? fmax(s_b - s_first, 0.0) : fmax(L - 2.0 * s_first, 0.0);
    pic1d_tp_result r;
    r.gamma_min = gmin;
    r.s_first = s_first;
    r.s_b = s_b;
    r.l_pp = l_pp;
    r.L = L;
    r.crossed = crossed;
    r.pad = 0;
    r.steps = steps;
    out[i] = r;
}

}  // namespace

int set_global_error(int code, const std::string& msg);

}  // namespace pic1d

using namespace pic1d;

namespace {
size_t tp_align(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

extern "C" {

int pic1d_testparticle_workspace_size(int32_t n, size_t* bytes) {
    if (n < 1 || !bytes) return set_global_error(PIC1D_EINVAL, "bad arguments");
    *bytes = tp_align(sizeof(double) * (size_t)n) + tp_align(sizeof(pic1d_tp_result) * (size_t)n);
    return PIC1D_OK;
}

int pic1d_testparticle_sweep(const pic1d_tp_config* cfg, int32_t n, const double* r_eq, pic1d_tp_result* out,
                             void* workspace, size_t workspace_bytes, void* stream) {
    if (!cfg || n < 1 || !r_eq || !out) return set_global_error(PIC1D_EINVAL, "bad arguments");
    if (!(cfg->gamma0 >= 1.0) || !(cfg->kT_keV > 0.0) || !(cfg->b_pole > 0.0) || !(cfg->b_pp > 0.0) ||
        !(cfg->t_max > 0.0) || !(cfg->dt_max > 0.0) || !(cfg->tol > 0.0) || !(cfg->tol_stiff > 0.0) ||
        cfg->max_steps < 1)
        return set_global_error(PIC1D_EINVAL, "invalid test-particle config");
    for (int k = 0; k < n; ++k)
        if (!(r_eq[k] > 1.0)) return set_global_error(PIC1D_EINVAL, "r_eq must exceed 1");
    size_t need = 0;
    pic1d_testparticle_workspace_size(n, &need);
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255) || workspace_bytes < need)
        return set_global_error(PIC1D_ENOMEM, "workspace missing, misaligned or too small");
    double* d_r = static_cast<double*>(workspace);
    pic1d_tp_result* d_out =
        reinterpret_cast<pic1d_tp_result*>(static_cast<char*>(workspace) + tp_align(sizeof(double) * (size_t)n));
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(d_r, r_eq, sizeof(double) * (size_t)n, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_testparticle, dim3((n + 63) / 64), dim3(64), 0, s, *cfg, n, d_r, d_out);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, d_out, sizeof(pic1d_tp_result) * (size_t)n, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_global_error(PIC1D_EDEVICE, std::string("test-particle sweep: ") + hipGetErrorString(e));
    return PIC1D_OK;
}

}  // extern "C"

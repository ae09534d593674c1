// Host-side FP64 set-up of the per-line constants (see setup.h).
#include "setup.h"

#include <math.h>

#include <algorithm>

namespace pic1d {

namespace {

// CODATA 2018 (cgs) and the stellar radius used by the paper (Sec. 2.2).
constexpr double kRe = 2.8179403262e-13;        // classical electron radius, cm
constexpr double kLambdaBar = 3.8615926796e-11; // reduced Compton wavelength, cm
constexpr double kMeC2keV = 510.99895000;       // electron rest energy, keV
constexpr double kRstar = 1.0e6;                // cm
constexpr double kPi = 3.14159265358979323846;

// Arc length along r = R sin^2(theta): ds = R sqrt(1 + 3 cos^2) sin dtheta, so with
// v = cos(theta) the length from the northern footpoint v0 is (R/2) (P(v0) - P(v)),
// P(v) = v sqrt(1 + 3 v^2) + asinh(sqrt(3) v) / sqrt(3).
double P(double v) { return v * sqrt(1.0 + 3.0 * v * v) + asinh(sqrt(3.0) * v) / sqrt(3.0); }

struct NodeGeo {
    double b, mu, x, rc;
};

NodeGeo geometry_at(double R, double b_pole, double v) {
    NodeGeo g;
    const double q = sqrt(1.0 + 3.0 * v * v);
    const double r = R * (1.0 - v * v);
    g.x = r;
    g.b = b_pole * q / (2.0 * r * r * r);            // dipole |B| / B_QED
    g.mu = 2.0 * v / q;                              // B^r / |B|
    g.rc = R * sqrt(fmax(1.0 - v * v, 0.0)) * q * q * q / (3.0 * (1.0 + v * v));
    return g;
}

// Closed forms of the normalised drag force and scattering rate with the
// cutoff y > 80 -> 0 (float64).
void rics_closed(double u, double b, double mu, double x, double theta, double AF, double AN, double& F,
                 double& N) {
    const double gam = sqrt(1.0 + u * u);
    const double y = b / (theta * (gam - u * mu));
    if (!(y <= 80.0)) {
        F = 0.0;
        N = 0.0;
        return;
    }
    const double em1 = expm1(y);
    F = AF / (x * x) * (gam * mu - u) * y * y * y / em1;
    N = AN / (x * x * gam) * y * y / em1;
}

}  // namespace

double line_length_rstar(double R) { return R * P(sqrt(1.0 - 1.0 / R)); }

double cos_theta_at(double R, double s) {
    // Newton on f(v) = (R/2)(P(v0) - P(v)) - s, f'(v) = -R sqrt(1 + 3 v^2), from a
    // linear first guess, safeguarded by the bracket [-v0, v0].
    const double v0 = sqrt(1.0 - 1.0 / R);
    const double L = R * P(v0);
    double lo = -v0, hi = v0;
    double v = v0 - 2.0 * v0 * s / L;
    for (int it = 0; it < 100; ++it) {
        const double f = 0.5 * R * (P(v0) - P(v)) - s;
        if (f > 0.0) lo = std::max(lo, v); else hi = std::min(hi, v);   // s(v) > s: v too small
        const double d = f / (-R * sqrt(1.0 + 3.0 * v * v));
        double vn = v - d;
        if (!(vn > lo && vn < hi)) vn = 0.5 * (lo + hi);
        if (fabs(vn - v) <= 1e-16 * (1.0 + fabs(v))) { v = vn; break; }
        v = vn;
    }
    return v;
}

bool config_has_table(const pic1d_config* c) {
    return c->rics_backend == 2 || (c->rics_backend == 3 && c->mlp_fallback_tol > 0.0);
}

const char* validate_config(const pic1d_config* c) {
    if (!c) return "config is NULL";
    if (c->n_lines < 1 || c->n_lines > 4096 || !c->lines) return "n_lines must be in [1, 4096] with lines given";
    if (!(c->cfl > 0.0 && c->cfl <= 0.5)) return "cfl must be in (0, 0.5]";
    if (!(c->d0_cells > 0.0) || !(c->ppc0 > 0.0)) return "d0_cells and ppc0 must be positive";
    if (!(c->kT_keV > 0.0) || !(c->b_pole > 0.0)) return "kT_keV and b_pole must be positive";
    if (c->annihilation != 0 && c->annihilation != 1) return "annihilation must be 0 or 1";
    if (!(c->mass_ratio >= 1.0)) return "mass_ratio must be >= 1";
    if (!(c->eta_min > 0.0)) return "eta_min must be positive";
    if (c->rics_backend < 0 || c->rics_backend > 3) return "unknown rics_backend";
    if (!(c->mlp_fallback_tol >= 0.0)) return "mlp_fallback_tol must be >= 0";
    if (config_has_table(c) && (c->table_nlg < 2 || c->table_ns < 2 || c->table_nlg > 4096 || c->table_ns > 65536))
        return "table dimensions out of range";
    if (config_has_table(c) && (int64_t)c->table_nlg * c->table_ns > (1ll << 27))
        return "table_nlg * table_ns must not exceed 2^27";
    if (c->conversion != 0 && c->conversion != 1) return "unknown conversion mode";
    if (c->photon_field != 0 && c->photon_field != 1) return "unknown photon_field";
    if (c->emission < 0 || c->emission > 2) return "unknown emission pattern";
    if (c->photon_field == 1 && c->rics_backend != 2 && c->rics_backend != 0)
        return "the finite-disk photon field needs the TABLE backend";
    if (c->sort_interval < 0) return "sort_interval must be >= 0";
    int64_t cells = 0;
    for (int l = 0; l < c->n_lines; ++l) {
        const pic1d_line& ln = c->lines[l];
        if (!(ln.r_eq > 1.0)) return "r_eq must exceed 1";
        if (ln.n_cells < 2 || ln.n_cells > (1 << 26)) return "n_cells must be in [2, 2^26]";
        if (ln.ppc_init < 0) return "ppc_init must be >= 0";
        if (ln.init_mode < 0 || ln.init_mode > 3) return "unknown init_mode";
        if (ln.init_mode == 2 && !(fabs(ln.init_beta) < 1.0)) return "init_beta must be below 1";
        if (ln.init_mode == 1 && !(ln.init_gamma_max >= 1.0)) return "init_gamma_max must be >= 1";
        if ((int64_t)ln.ppc_init * ln.n_cells >= (1ll << 31)) return "too many initial pairs on a line";
        for (int s = 0; s < 4; ++s)
            if (ln.capacity[s] < 0 || ln.capacity[s] >= (1ll << 31)) return "capacity per species must be < 2^31";
        cells += ln.n_cells;
    }
    if (cells > (1ll << 27)) return "too many cells in total (at most 2^27)";
    return "";
}

void build_line(const pic1d_config* c, int line, int32_t cell_base, int32_t table_off, LineHost& o) {
    const pic1d_line& ln = c->lines[line];
    const double R = ln.r_eq;
    const int n = ln.n_cells;
    const double C = c->cfl;
    o.L_rstar = line_length_rstar(R);
    o.ds = o.L_rstar / n;
    const double h = C * o.ds;
    const double wp0 = C / c->d0_cells;
    const double Q = wp0 * wp0 / (4.0 * kPi * c->ppc0);
    const double npsi = fabs(c->j_twist);
    o.tau_steps = (npsi > 0.0 ? c->eta_min * sqrt(npsi) : c->eta_min) / wp0;
    const double theta = c->kT_keV / kMeC2keV;
    const double base = kRe * kRstar / (4.0 * kLambdaBar * kLambdaBar);
    const double AF = base * theta * theta * theta, AN = base * theta * theta;
    o.AF = AF;
    o.AN = AN;

    LineDev& d = o.dev;
    d.cell_base = cell_base;
    d.n_cells = n;
    d.node_base = cell_base + line;
    d.table_off = table_off;
    d.C = (float)C;
    d.invC = (float)(1.0 / C);
    d.h = (float)h;
    d.tau_hat = (float)(o.tau_steps * h);
    d.damp = (float)(-expm1(-0.5 / o.tau_steps));
    d.A_F = (float)AF;
    d.A_N = (float)AN;
    d.inv_theta = (float)(1.0 / theta);
    d.b_thr = (float)c->b_thr;
    const bool table = config_has_table(c);
    d.s_scale = table ? (double)c->table_ns / n : 0.0;
    d.lg_scale = table ? (c->table_nlg - 1) / 8.0 : 0.0;
    d.use_table = c->rics_backend == 2 ? 1 : 0;     // the MLP backend's lines decide at init
    d.s_scale_f = (float)d.s_scale;
    d.lgk = (float)(0.5 * d.lg_scale * log10(2.0));
    const double nmax = (c->nmax_over_n0 > 0.0 ? c->nmax_over_n0 : c->d0_cells * c->d0_cells) * c->ppc0;
    d.nmax = (float)nmax;
    d.half_n = 0.5f * (float)n;
    d.inv_ds = 1.0 / o.ds;
    d.j_tw = c->j_twist * c->ppc0 * Q * C;
    d.Q = Q;
    d.amp_scale = 4.0 * kPi * Q / 4294967296.0;

    // atmosphere (Appendix B.1): n/n0 = a0 exp(-d/h) near both walls
    double a0 = c->atm_a0 > 0.0 ? c->atm_a0 : 18.0 * npsi;
    if (a0 <= 0.0) a0 = c->atm_cut;
    const double hat = c->atm_h_cells > 0.0 ? c->atm_h_cells : 3.0 * c->d0_cells / sqrt(a0);
    d.atm_depth = (c->atmosphere && c->gravity && a0 > c->atm_cut) ? hat * log(a0 / c->atm_cut) : -1.0;
    d.grav = (float)(c->atm_T * C / hat);
    o.layer_cell.clear();
    o.layer_target.clear();
    int64_t atm_total = 0;
    if (c->atmosphere) {
        for (int k = 0; k < n; ++k) {
            const double dw = std::min(k + 0.5, n - k - 0.5);
            const double prof = a0 * exp(-dw / hat);
            if (prof >= c->atm_cut) {
                const int tgt = (int)floor(prof * c->ppc0);
                if (tgt > 0) {
                    o.layer_cell.push_back(k);
                    o.layer_target.push_back(tgt);
                    atm_total += tgt;
                }
            }
        }
    }

    // nodes s_i = i L / n
    o.nodes.resize(4 * (size_t)(n + 1));
    o.rc.resize(n + 1);
    const double v0 = sqrt(1.0 - 1.0 / R);
    for (int i = 0; i <= n; ++i) {
        double v = (i == 0) ? v0 : (i == n) ? -v0 : cos_theta_at(R, i * o.ds);
        const NodeGeo g = geometry_at(R, c->b_pole, v);
        o.nodes[4 * (size_t)i + 0] = (float)g.b;
        o.nodes[4 * (size_t)i + 1] = (float)g.mu;
        o.nodes[4 * (size_t)i + 2] = (float)g.x;
        o.nodes[4 * (size_t)i + 3] = (float)g.rc;
        o.rc[i] = g.rc;
    }

    // RICS table for u >= 0 at log10 gamma_i = 8 i/(nlg-1), s_j = (j + 1/2) L/ns, stored as
    // [ns][nlg] records {F(i), F(i+1), Ndot(i), Ndot(i+1)} (column i+1 clamped at the end)
    o.table.clear();
    o.row_geo.clear();
    if (table && c->photon_field == 1) {
        // the finite disk: built on the device by its quadrature (disk.hip)
        o.table.assign(4 * (size_t)c->table_nlg * c->table_ns, 0.0f);
    } else if (table) {
        const int nlg = c->table_nlg, ns = c->table_ns;
        std::vector<double> Fr(nlg), Nr(nlg);
        o.table.assign(4 * (size_t)nlg * ns, 0.0f);
        o.row_geo.assign(3 * (size_t)ns, 0.0);
        for (int j = 0; j < ns; ++j) {
            const double s = (j + 0.5) * o.L_rstar / ns;
            const NodeGeo g = geometry_at(R, c->b_pole, cos_theta_at(R, s));
            o.row_geo[3 * (size_t)j + 0] = g.b;
            o.row_geo[3 * (size_t)j + 1] = g.mu;
            o.row_geo[3 * (size_t)j + 2] = g.x;
            for (int i = 0; i < nlg; ++i) {
                const double gam = pow(10.0, 8.0 * i / (nlg - 1));
                const double u = sqrt(fmax(gam * gam - 1.0, 0.0));
                rics_closed(u, g.b, g.mu, g.x, theta, AF, AN, Fr[i], Nr[i]);
            }
            for (int i = 0; i < nlg; ++i) {
                const int i1 = std::min(i + 1, nlg - 1);
                float* rec = &o.table[4 * ((size_t)j * nlg + i)];
                rec[0] = (float)Fr[i];
                rec[1] = (float)Fr[i1];
                rec[2] = (float)Nr[i];
                rec[3] = (float)Nr[i1];
            }
        }
    }

    // capacities
    const int64_t pairs0 = (int64_t)ln.ppc_init * n;
    int64_t defcap[4];
    defcap[0] = defcap[1] = (ln.init_mode == 3 ? 0 : pairs0) + (c->pairs ? 16 * (int64_t)n + 4096 : 0) + 64;
    defcap[2] = defcap[3] = c->atmosphere ? 4 * atm_total + 4096 : 64;
    for (int s = 0; s < 4; ++s) {
        o.cap[s] = ln.capacity[s] > 0 ? ln.capacity[s] : defcap[s];
        // multiples of 256 slots keep every segment aligned for vector loads
        o.cap[s] = std::min<int64_t>((o.cap[s] + 255) / 256 * 256, (1ll << 31) - 256);
    }
}

}  // namespace pic1d

// Host-side FP64 set-up of the per-line constants: dipole geometry at the grid
// nodes (Appendix B.2), RICS table (Sec. 2.2 closed forms), atmosphere layers
// (Appendix B.1) and the code-unit derivations.
#pragma once

#include <stdint.h>

#include <vector>

#include "../../include/pic1d.h"
#include "pic1d_dev.h"

namespace pic1d {

struct LineHost {
    LineDev dev;                       // constants uploaded to the device
    double L_rstar = 0, ds = 0;        // line length and cell length in R*
    double tau_steps = 0;
    double AF = 0, AN = 0;             // RICS prefactors in float64
    std::vector<float> nodes;          // 4 floats per node: b, mu, x, R_curv
    std::vector<double> rc;            // R_curv per node, double
    std::vector<float> table;          // F table then Ndot table, [ns][nlg]
    std::vector<double> row_geo;       // b, mu, x at the table's row centres (radial table)
    std::vector<int32_t> layer_cell;   // local cells of the atmosphere layers
    std::vector<int32_t> layer_target; // their hydrostatic targets
    int64_t cap[4] = {0, 0, 0, 0};
};

// Whether the config gives every line a RICS table (TABLE backend, or the MLP
// backend with its table fallback).
bool config_has_table(const pic1d_config* cfg);

// Validate cfg; returns an empty string if valid, else the reason.
const char* validate_config(const pic1d_config* cfg);

// Build every per-line quantity in FP64.
void build_line(const pic1d_config* cfg, int line, int32_t cell_base, int32_t table_off, LineHost& out);

// Dipole geometry helpers (exposed for tests of the library's own set-up).
double line_length_rstar(double R);
double cos_theta_at(double R, double s_rstar);

}  // namespace pic1d

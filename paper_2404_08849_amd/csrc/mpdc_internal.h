// Internal structures of the mpdc library (host + device).
//
// Device tables are fixed-width per entity so that a kernel thread reaches
// its stencil with one multiply-add: cells carry 6 slots (pentagons pad the
// sixth with -1 and zero weights), edges carry 10 TRiSK slots, vertices 3.
// Geometry weights come in FP64 (every policy's FP64 terms) and FP32 (the
// FP32 advective terms of the mixed policy); both are derived in FP64 on the
// host and the FP32 copy is a rounding of the FP64 value.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mpdc.h"

namespace mpdc {

constexpr int kCellSlots = 6;
constexpr int kTriskSlots = 10;

// Device view of the mesh tables (pointers into the caller's workspace).
struct DevMesh {
    int N, E, V;
    // cells: 6 slots, counter-clockwise, pentagons padded
    const int *c_edge;      // [N][6] edge of slot j (-1 pad)
    const int *c_nbr;       // [N][6] neighbour across slot j (self for pads)
    const int *c_vert;      // [N][6] vertex j, between edges j-1 and j (pentagon pad = vertex 0)
    const double *c_div;    // [N][6] s_{e,i} l_e / A_i
    const float *c_div32;
    const double *c_ke;     // [N][6] l_e d_e / (4 A_i)
    const float *c_ke32;
    const double *c_gk;     // [N][6] s_{e,i} / d_e   (cell i's share of -grad K on edge j)
    const float *c_gk32;
    const double *c_hess;   // [N][3][6] slot differences -> (Hxx, Hxy, Hyy)
    const float *c_hess32;
    const double *c_hd;     // [N][6][8] third-order flux of slot j: neighbour direction in i's frame
                            // (u^2, 2uv, v^2), direction of i in the neighbour's frame, -d_e^2/6, 0
    const float *c_hd32;
    const double *c_tk;     // [N][6][6] TRiSK half-stencil: w_{e_j,e_j'} l_{e_j'} / (4 d_{e_j}) from cell i
    const float *c_tk32;
    const double *c_area;   // [N]
    // edges
    const int *e_cell;      // [E][2]
    const int *e_vert;      // [E][2]
    const double *e_dinv;   // [E] 1/d_e
    const float *e_dinv32;
    const double *e_d2;     // [E] d_e^2/12
    const float *e_d2_32;
    const double *e_hdir;   // [E][2][3] (c^2, 2cs, s^2) of the neighbour direction in c1's / c2's frame
    const float *e_hdir32;
    // vertices (padded to 4)
    const int *v_edge;      // [V][4]
    const int *v_cell;      // [V][4]
    const double *v_curl;   // [V][4] s'_{e,v} d_e / A_v
    const float *v_curl32;
    const double *v_kite;   // [V][4] R_{i,v} / A_v
    const double *v_f;      // [V]
    const double *v_area;   // [V] dual-cell areas (diagnostics)
};

}  // namespace mpdc

struct mpdc_mesh {
    int N, E, V;
    double radius;
    mpdc::DevMesh dev;
    hipStream_t stream;
    // FP64 host copies of the exported tables
    std::vector<int> cells_on_cell;
    std::vector<double> edge_sign, vertex_sign;
    std::vector<int> trisk_off, trisk_edge;
    std::vector<double> trisk_w;
    std::vector<double> hessian;   // [2E][6]
    std::vector<double> area_cell; // host copy for diagnostics weights
};

namespace mpdc {

// Layout helpers
struct Dims {
    int N, E, V, K, M, T;
    long long KM() const { return (long long)K * M; }
};

// Kernel launch shape
// Launch shape per kernel class (dycore: cell_a, vertex, cell_b, edge;
// tracer: low, limit, update).  Any legal shape gives bitwise identical results.
struct Launch {
    int cpb[4] = {0, 0, 0, 0};            // column kernels: cells per work-group (0 = auto)
    int flat[4] = {256, 256, 256, 256};   // flat kernels: threads per work-group
    int vpl[4] = {0, 0, 0, 0};            // (k, m) or tracer values per lane (0 = auto)
};

// Thread-local error message
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

// Table derivation (host, FP64); returns "" or an error message.
struct HostTables {
    std::vector<int> c_edge, c_nbr, c_vert;
    std::vector<double> c_div, c_ke, c_gk, c_hess, c_hd, c_tk, c_area;
    std::vector<int> e_cell, e_vert;
    std::vector<double> e_dinv, e_d2, e_hdir;
    std::vector<int> v_edge, v_cell;              // [V][4]
    std::vector<double> v_curl, v_kite, v_f, v_area;   // [V][4], [V][4], [V], [V]
    // exported (reference-form) tables
    std::vector<int> cells_on_cell, trisk_off, trisk_edge;
    std::vector<double> edge_sign, vertex_sign, trisk_w, hessian;
};
std::string validate_mesh(const mpdc_mesh_desc *d);
std::string derive_tables(const mpdc_mesh_desc *d, HostTables &t);

}  // namespace mpdc

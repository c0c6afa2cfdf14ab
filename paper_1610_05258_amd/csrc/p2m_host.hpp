// Host-only pieces of the library: the problem geometry, the validation of
// problems and solve options, and the line format of the plan file.  Plain C++
// (no HIP): the library compiles them with its kernels, and the host compiler
// builds them alone for the sanitizer test.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>

#include "../../include/p2m.h"

namespace p2m {

// Geometry of one periodic structured problem, computed once on the host in FP64.
struct Mesh {
    int dim;          // 1 or 2
    int nx, ny;       // ny == 1 in 1D
    int nn;           // nodes = cells = nx*ny
    int np;           // particles
    double inv_hx;    // nx / lx   (one FP64 division on the host)
    double inv_hy;    // ny / ly
    double cell_measure;  // hx*hy (2D) or hx (1D): the mesh volume v_i of every node
    double v_uniform;     // lx*ly/np (2D) or lx/np (1D): particle volume when none is given
};

// The checks every entry point applies to a problem (and fills m from it) and to
// solve options; the status the entry point then returns.
p2m_status check_problem(const p2m_problem* p, Mesh& m);
p2m_status check_opts(const p2m_solve_opts* opts);

// Plan file: a JSON object, one plan per line,
//   "key": {"solver": S, "groups": G, "scatter_tile": T, "inner_rtol": R, "time_ms": M}
// A line without a quote is skipped (the braces); a plan line with a key longer
// than 127 characters, a missing field or a value outside its range is rejected.
enum PlanLine { kPlanSkip = 0, kPlanOk = 1, kPlanBad = 2 };
PlanLine parse_plan_line(const char* line, std::string& key, p2m_plan& plan);
// The line for one plan (with a trailing comma unless last); the number of
// characters written, or -1 if cap is too small.
int format_plan_line(char* buf, size_t cap, const std::string& key, const p2m_plan& plan,
                     bool last);

}  // namespace p2m

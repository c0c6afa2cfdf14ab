#include "p2m_host.hpp"

#include <math.h>
#include <stdio.h>
#include <string.h>

namespace p2m {

p2m_status check_problem(const p2m_problem* p, Mesh& m) {
    if (!p) return P2M_ERR_INVALID_ARG;
    if (p->dim != 1 && p->dim != 2) return P2M_ERR_INVALID_ARG;
    if (p->dtype != P2M_F32 && p->dtype != P2M_F64) return P2M_ERR_INVALID_ARG;
    if (p->nx < 2 || (p->dim == 2 && p->ny < 2)) return P2M_ERR_INVALID_ARG;
    if (p->np < 0) return P2M_ERR_INVALID_ARG;
    if (!isfinite(p->lx) || (p->dim == 2 && !isfinite(p->ly))) return P2M_ERR_NONFINITE;
    if (!(p->lx > 0.0) || (p->dim == 2 && !(p->ly > 0.0))) return P2M_ERR_RANGE;
    const int ny = (p->dim == 2) ? p->ny : 1;
    const int64_t nn = (int64_t)p->nx * ny;
    if (nn >= ((int64_t)1 << 31) - 1 || p->np >= ((int64_t)1 << 31) - 1) return P2M_ERR_UNSUPPORTED;
    if (p->np > 0 && (!p->x || (p->dim == 2 && !p->y))) return P2M_ERR_INVALID_ARG;
    m.dim = p->dim;
    m.nx = p->nx;
    m.ny = ny;
    m.nn = (int)nn;
    m.np = (int)p->np;
    m.inv_hx = (double)p->nx / p->lx;
    m.inv_hy = (p->dim == 2) ? (double)p->ny / p->ly : 1.0;
    m.cell_measure = (p->dim == 2) ? (p->lx / p->nx) * (p->ly / p->ny) : p->lx / p->nx;
    const double area = (p->dim == 2) ? p->lx * p->ly : p->lx;
    m.v_uniform = (p->np > 0) ? area / (double)p->np : 0.0;
    return P2M_OK;
}

p2m_status check_opts(const p2m_solve_opts* opts) {
    if (!opts) return P2M_ERR_INVALID_ARG;
    if (!isfinite(opts->tol) || !isfinite(opts->inner_rtol)) return P2M_ERR_NONFINITE;
    if (!(opts->tol > 0.0) || opts->inner_rtol < 0.0 || opts->inner_rtol >= 1.0) return P2M_ERR_RANGE;
    if (opts->maxit < 0 || opts->max_refine < 0 || opts->reserved != 0) return P2M_ERR_INVALID_ARG;
    if (opts->start < P2M_START_FLIP || opts->start > P2M_START_DELTA1D) return P2M_ERR_INVALID_ARG;
    return P2M_OK;
}

PlanLine parse_plan_line(const char* line, std::string& key, p2m_plan& p) {
    if (!line) return kPlanSkip;
    const char* q = strchr(line, '"');
    if (!q) return kPlanSkip;
    char k[128];
    memset(&p, 0, sizeof(p));
    if (sscanf(q,
               "\"%127[^\"]\": {\"solver\": %d, \"groups\": %d, \"scatter_tile\": %d, "
               "\"inner_rtol\": %lf, \"time_ms\": %lf}",
               k, &p.solver, &p.groups, &p.scatter_tile, &p.inner_rtol, &p.time_ms) != 6)
        return kPlanBad;
    if (p.solver < P2M_SOLVER_AUTO || p.solver > P2M_SOLVER_RESIDENT_CHEB || p.groups < 0 ||
        (p.scatter_tile != 0 && p.scatter_tile != 8) || !(p.inner_rtol < 1.0) ||
        !isfinite(p.inner_rtol) || !isfinite(p.time_ms))
        return kPlanBad;
    key.assign(k);
    return kPlanOk;
}

int format_plan_line(char* buf, size_t cap, const std::string& key, const p2m_plan& p, bool last) {
    const int n = snprintf(buf, cap,
                           "  \"%s\": {\"solver\": %d, \"groups\": %d, \"scatter_tile\": %d, "
                           "\"inner_rtol\": %.17g, \"time_ms\": %.6f}%s\n",
                           key.c_str(), p.solver, p.groups, p.scatter_tile, p.inner_rtol, p.time_ms,
                           last ? "" : ",");
    return (n < 0 || (size_t)n >= cap) ? -1 : n;
}

}  // namespace p2m

// Host-side checks of the library's pure C++ parts (problem and option validation,
// the plan-file line format), built with the host compiler under AddressSanitizer
// and UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py.  Exits 0 when
// every expectation holds; any memory or UB error aborts through the sanitizers.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <random>
#include <string>

#include "../paper_1610_05258_amd/csrc/p2m_host.hpp"

using namespace p2m;

static int failures = 0;
#define EXPECT(cond)                                                    \
    do {                                                                \
        if (!(cond)) {                                                  \
            fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                 \
        }                                                               \
    } while (0)

static p2m_problem good() {
    static float xs[4] = {0.1f, 0.2f, 0.3f, 0.4f};
    p2m_problem p;
    memset(&p, 0, sizeof p);
    p.dim = 2;
    p.nx = 8;
    p.ny = 4;
    p.lx = 1.0;
    p.ly = 0.5;
    p.np = 4;
    p.dtype = P2M_F32;
    p.x = xs;
    p.y = xs;
    return p;
}

static void problems() {
    Mesh m;
    EXPECT(check_problem(nullptr, m) == P2M_ERR_INVALID_ARG);
    p2m_problem p = good();
    EXPECT(check_problem(&p, m) == P2M_OK);
    EXPECT(m.nn == 32 && m.np == 4 && m.inv_hx == 8.0 && m.inv_hy == 8.0);
    EXPECT(fabs(m.cell_measure - 0.125 * 0.125) < 1e-18 && fabs(m.v_uniform - 0.125) < 1e-18);
    struct Case {
        void (*edit)(p2m_problem&);
        p2m_status want;
    } cases[] = {
        {[](p2m_problem& q) { q.dim = 3; }, P2M_ERR_INVALID_ARG},
        {[](p2m_problem& q) { q.dtype = 7; }, P2M_ERR_INVALID_ARG},
        {[](p2m_problem& q) { q.nx = 1; }, P2M_ERR_INVALID_ARG},
        {[](p2m_problem& q) { q.ny = 0; }, P2M_ERR_INVALID_ARG},
        {[](p2m_problem& q) { q.np = -1; }, P2M_ERR_INVALID_ARG},
        {[](p2m_problem& q) { q.lx = NAN; }, P2M_ERR_NONFINITE},
        {[](p2m_problem& q) { q.ly = INFINITY; }, P2M_ERR_NONFINITE},
        {[](p2m_problem& q) { q.lx = -1.0; }, P2M_ERR_RANGE},
        {[](p2m_problem& q) { q.ly = 0.0; }, P2M_ERR_RANGE},
        {[](p2m_problem& q) { q.nx = 65536; q.ny = 65536; }, P2M_ERR_UNSUPPORTED},
        {[](p2m_problem& q) { q.np = (int64_t)1 << 40; }, P2M_ERR_UNSUPPORTED},
        {[](p2m_problem& q) { q.x = nullptr; }, P2M_ERR_INVALID_ARG},
        {[](p2m_problem& q) { q.y = nullptr; }, P2M_ERR_INVALID_ARG},
        {[](p2m_problem& q) { q.dim = 1; q.ny = 0; q.y = nullptr; }, P2M_OK},
        {[](p2m_problem& q) { q.np = 0; q.x = q.y = nullptr; }, P2M_OK},
        {[](p2m_problem& q) { q.nx = 2147483647; q.dim = 1; }, P2M_ERR_UNSUPPORTED},
    };
    for (const Case& c : cases) {
        p2m_problem q = good();
        c.edit(q);
        EXPECT(check_problem(&q, m) == c.want);
    }
}

static void options() {
    p2m_solve_opts o;
    memset(&o, 0, sizeof o);
    o.tol = 1e-8;
    o.inner_rtol = 1e-4;
    o.maxit = 100;
    o.max_refine = 5;
    o.start = P2M_START_FLIP;
    EXPECT(check_opts(nullptr) == P2M_ERR_INVALID_ARG);
    EXPECT(check_opts(&o) == P2M_OK);
    p2m_solve_opts q = o;
    q.tol = NAN;
    EXPECT(check_opts(&q) == P2M_ERR_NONFINITE);
    q = o;
    q.tol = 0.0;
    EXPECT(check_opts(&q) == P2M_ERR_RANGE);
    q = o;
    q.inner_rtol = 1.0;
    EXPECT(check_opts(&q) == P2M_ERR_RANGE);
    q = o;
    q.inner_rtol = -INFINITY;
    EXPECT(check_opts(&q) == P2M_ERR_NONFINITE);
    q = o;
    q.maxit = -1;
    EXPECT(check_opts(&q) == P2M_ERR_INVALID_ARG);
    q = o;
    q.reserved = 3;
    EXPECT(check_opts(&q) == P2M_ERR_INVALID_ARG);
    q = o;
    q.start = 99;
    EXPECT(check_opts(&q) == P2M_ERR_INVALID_ARG);
}

static void plan_lines() {
    p2m_plan p;
    memset(&p, 0, sizeof p);
    p.solver = P2M_SOLVER_RESIDENT_CHEB;
    p.groups = 3;
    p.scatter_tile = 8;
    p.inner_rtol = 3e-5;
    p.time_ms = 0.4834;
    char buf[512];
    const std::string key = "2d-f32-F3-nx10-ny10-ppc3";
    const int n = format_plan_line(buf, sizeof buf, key, p, false);
    EXPECT(n > 0 && buf[n - 2] == ',');
    std::string k2;
    p2m_plan q;
    EXPECT(parse_plan_line(buf, k2, q) == kPlanOk);
    EXPECT(k2 == key && q.solver == p.solver && q.groups == 3 && q.scatter_tile == 8 &&
           q.inner_rtol == p.inner_rtol && fabs(q.time_ms - p.time_ms) < 1e-6);
    EXPECT(format_plan_line(buf, 16, key, p, true) == -1);   // too small: no overflow
    EXPECT(parse_plan_line("{\n", k2, q) == kPlanSkip);
    EXPECT(parse_plan_line(nullptr, k2, q) == kPlanSkip);
    EXPECT(parse_plan_line("  \"k\": {\"solver\": 2}\n", k2, q) == kPlanBad);
    EXPECT(parse_plan_line("  \"k\": {\"solver\": 9, \"groups\": 0, \"scatter_tile\": 0, "
                           "\"inner_rtol\": 0, \"time_ms\": 1}\n", k2, q) == kPlanBad);
    EXPECT(parse_plan_line("  \"k\": {\"solver\": 2, \"groups\": 0, \"scatter_tile\": 0, "
                           "\"inner_rtol\": nan, \"time_ms\": 1}\n", k2, q) == kPlanBad);
    EXPECT(parse_plan_line("  \"k\": {\"solver\": 2, \"groups\": -1, \"scatter_tile\": 0, "
                           "\"inner_rtol\": 0, \"time_ms\": 1}\n", k2, q) == kPlanBad);
    // a key longer than the 127-character field: rejected, nothing written past it
    std::string longline = "  \"" + std::string(300, 'a') +
                            "\": {\"solver\": 2, \"groups\": 0, \"scatter_tile\": 0, "
                            "\"inner_rtol\": 0, \"time_ms\": 1}\n";
    EXPECT(parse_plan_line(longline.c_str(), k2, q) == kPlanBad);
    // random bytes and random cuts of a valid line: any result, no memory error
    std::mt19937 g(12345);
    for (int t = 0; t < 20000; ++t) {
        std::string s;
        const int len = (int)(g() % 200);
        if (t % 2) {
            for (int i = 0; i < len; ++i) s.push_back((char)(1 + g() % 255));
        } else {
            s.assign(buf, buf + (len < n ? len : n));
            if (!s.empty()) s[g() % s.size()] = (char)(1 + g() % 255);
        }
        (void)parse_plan_line(s.c_str(), k2, q);
    }
}

int main() {
    problems();
    options();
    plan_lines();
    if (failures) {
        fprintf(stderr, "%d failure(s)\n", failures);
        return 1;
    }
    printf("host checks passed\n");
    return 0;
}

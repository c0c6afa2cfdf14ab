// Internal declarations shared by the HIP translation units of libp2m.
// Not part of the public ABI (see include/p2m.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/p2m.h"
#include "p2m_host.hpp"   // Mesh, the problem and option checks, the plan-file line format

namespace p2m {

constexpr int kMaxFields = 8;
constexpr size_t kAlign = 256;

template <typename T>
struct Particles {
    const T* x;
    const T* y;
    const T* vol;     // may be null
};

// Launch geometry shared by the host planner and the kernels.
constexpr int kBinBlock = 256;       // particles per block of the locate / place kernels
constexpr int kSolveTileX = 128;     // node tile of the tile solvers (one workgroup per tile)
constexpr int kSolveTileY = 32;

// Node tile of the 2D scatter for F fields of element size tsize: 15 x 15 (its
// 16 x 16 cells, one thread each, make a workgroup of exactly four waves, one per
// SIMD, so four workgroups share a compute unit whatever their wave placement)
// unless the per-cell parts of those cells exceed 64 KB of LDS, then 8 x 8.
constexpr int assemble_tile(int F, int tsize) {
    return (size_t)(13 + 4 * F) * 16 * 16 * tsize <= 65536 ? 15 : 8;
}

// One instance of a batch of independent 2D FP32 problems (an entry of the
// device-side instance table).  Particles, cells / nodes and tiles of all
// instances are numbered in one space each; an instance owns the contiguous
// ranges starting at po (particles), no (nodes = cells), lb (locate blocks),
// at (scatter tiles) and rt (solver tiles).  Node-sized work arrays hold the
// instance's block of F * nn values at F * no.
struct BatchInst {
    Mesh m;
    Particles<float> P;
    const float* values;   // [F][np]
    float* out;            // [F][nn] start (USER) on entry, result on exit
    p2m_report* rep;
    int32_t po, no, lb;
    int32_t at, atx;       // first scatter tile, scatter tiles per row
    int32_t rt, rtx, nrt;  // first solver tile, solver tiles per row, solver tiles
};

// ---------------------------------------------------------------------------
// locate: cell of a coordinate and the offset inside it, in FP64.
// t = x * (n/L); c = floor(t); xi = t - c (exact); c == n wraps to 0.
// Valid iff t is finite and 0 <= t < n + 1.  Same operations, same rounding as
// a plain FP64 evaluation, so the cell key is bit-exact.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool locate_axis(double x, int n, double inv, int& c, double& xi,
                                            bool& finite) {
    double t = __dmul_rn(x, inv);
    finite = __builtin_isfinite(t);
    bool valid = finite && t >= 0.0 && t < (double)n + 1.0;
    if (!valid) t = 0.0;
    double cf = floor(t);
    xi = __dsub_rn(t, cf);
    c = (int)cf;
    if (c == n) c = 0;
    return valid;
}

// P1 weights of the four corners of a cell for a particle at offsets (xi, eta)
// on the "/"-split square: xi >= eta is the lower triangle (n00, n10, n11) with
// barycentrics (1-xi, xi-eta, eta); otherwise the upper triangle (n00, n11, n01)
// with (1-eta, xi, eta-xi).  The corner not in the triangle gets 0.  The
// differences are taken in FP64 and rounded once to T.
template <typename T>
__device__ __forceinline__ void corner_weights(double xi, double eta, T& c00, T& c10, T& c11,
                                               T& c01) {
    // selects rather than branches: the branchy form was lowered through a local
    // array in scratch memory
    const bool lower = xi >= eta;  // lower-right triangle of the "/" split
    c00 = (T)__dsub_rn(1.0, lower ? xi : eta);
    c10 = lower ? (T)__dsub_rn(xi, eta) : (T)0;
    c11 = (T)(lower ? eta : xi);
    c01 = lower ? (T)0 : (T)__dsub_rn(eta, xi);
}

// ---------------------------------------------------------------------------
// Launchers implemented in the .hip translation units.  All are asynchronous on
// `stream`; they return hipSuccess or the launch error.
// ---------------------------------------------------------------------------

// report: zero it (a fill kernel, so the call stays capturable into graphs)
hipError_t launch_report_clear(p2m_report* rep, hipStream_t stream);
// fill n ints with value; with rep, the same launch zeroes that report
hipError_t launch_fill_i32(int32_t* p, int32_t value, size_t n, hipStream_t stream,
                           p2m_report* rep = nullptr);

// binning
template <typename T>
// key [np] (cell or -1), rank [np] (slot within the cell, -1 when not located),
// counts [nn] (zeroed by the caller, incremented)
hipError_t launch_locate_count(const Mesh& m, Particles<T> P, int32_t* key, int32_t* rank,
                               int32_t* counts, p2m_report* rep, hipStream_t stream);
// single-pass scan: scan_ws (scan_workspace_bytes(n)) must be zero on entry;
// out[0..n] receives the exclusive prefix sums and the total.  spin_max bounds
// the wait for a predecessor tile (< 0: no wait, a test hook); a scan that gives
// up raises P2M_FLAG_BIN_TIMEOUT in reps[0..nrep) and sets an abort word in
// scan_ws that the place kernels read
constexpr long kScanSpinDefault = 1L << 26;
constexpr long kSolveSpinDefault = 1L << 22;   // polls of a solve's grid-barrier wait
size_t scan_workspace_bytes(int n);
hipError_t launch_exclusive_scan(const int32_t* counts, int32_t* out, int n, void* scan_ws,
                                 long spin_max, p2m_report* reps, int nrep, hipStream_t stream);
// perm[cell_start[key] + rank] = particle; slots after the valid particles -1.
// After an aborted scan (scan_ws as given to the scan): every cell empty
// (cell_start[0..nn] = 0, perm = -1)
hipError_t launch_place(const Mesh& m, const int32_t* key, const int32_t* rank, int32_t* cell_start,
                        int32_t* perm, const void* scan_ws, hipStream_t stream);
hipError_t launch_segment_sort(const Mesh& m, const int32_t* cell_start, int32_t* perm,
                               hipStream_t stream);

// scatter-assemble: b [F][nn], w [nn], coef [c_M][nn] or null; tile 0 = the default
// 2D node tile, 8 = 8 x 8
template <typename T>
hipError_t launch_assemble(const Mesh& m, Particles<T> P, const T* values, int F,
                           const int32_t* perm, const int32_t* cell_start, T* b, T* w, T* coef,
                           hipStream_t stream, int tile = 0);

// finalize: FLIP (divide by w, orphans 0) or PIC (divide by the mesh volume)
template <typename T>
hipError_t launch_finalize(const Mesh& m, int F, const T* b, const T* w, int pic, T* out,
                           p2m_report* rep, hipStream_t stream);

// M2P gather in caller order.  ws (optional, >= F * nn elements): 2D gathers of
// 2-4 fields read a node-major copy built there
template <typename T>
hipError_t launch_gather(const Mesh& m, Particles<T> P, const T* nodal, int F, T* out,
                         p2m_report* rep, hipStream_t stream, void* ws = nullptr,
                         size_t ws_bytes = 0);

// 1D delta P2M from the binned particles
template <typename T>
hipError_t launch_delta1d(const Mesh& m, Particles<T> P, const T* values, int F,
                          const int32_t* perm, const int32_t* cell_start, T* out,
                          hipStream_t stream);

// paper-exact 1D (k_exact1d.hip), FP64.  N = located particles (binned order in
// perm[0..N)); key / idx [N] receive the positions and particle numbers in
// position order; gap, vol_s [N] sorted order, vol_c [np] caller order, As [F][N]
hipError_t x1d_sort(const Mesh& m, int N, const double* x, const int32_t* perm,
                    const int32_t* cs, double* key, int32_t* idx, hipStream_t stream);
hipError_t x1d_setup(int N, double L, const double* key, const int32_t* idx, const double* values,
                     int F, int np, double* gap, double* vol_s, double* vol_c, double* As,
                     hipStream_t stream);
// c [F][n] = int A psi_j over the mesh hats (quad: P2M_QUAD_*); fn [F][n] receives the
// particle interpolant at the nodes (the delta P2M), fm [F][n] at the element
// midpoints; t_lo, t_hi [F][n] scratch
hipError_t x1d_p2m_overlap(const Mesh& m, int N, const double* key, const double* As, int F,
                           int quad, double* fn, double* fm, double* t_lo, double* t_hi,
                           double* c, hipStream_t stream);
// c [F][N] = int Abar psi_mu over the particle hats (sorted order); fk, fmid, t_lo,
// t_hi [F][N] scratch
hipError_t x1d_m2p_overlap(const Mesh& m, int N, const double* key, const double* gap,
                           const double* nodal, int F, int quad, double* fk, double* fmid,
                           double* t_lo, double* t_hi, double* c, hipStream_t stream);
hipError_t x1d_mass_mesh(int n, double L, double* coef, double* w, hipStream_t stream);
hipError_t x1d_mass_part(int N, const double* gap, double* coef, hipStream_t stream);
hipError_t x1d_div(int K, int F, const double* c, const double* d, double s, double* out,
                   hipStream_t stream);
// out [F][np] caller order: NaN, then xs [F][N] (sorted order) at idx
hipError_t x1d_scatter(int N, int F, int np, const int32_t* idx, const double* xs, double* out,
                       hipStream_t stream);

// paper-exact 2D (k_x2d.hip); slot k = position in the binned order, N located
struct X2dArgs {
    Mesh m;
    int N, F;
    double lx, ly;
    const int32_t* perm;   // [np] binned order
    const int32_t* cs;     // [nn + 1] cell starts
    const double* x;
    const double* y;
    const double* values;  // [F][np] or null
    double* xs;            // [N] wrapped positions
    double* ys;
    int32_t* cell;         // [N]
    double* As;            // [F][N] values in binned order
    int32_t* deg;          // [N]
    int32_t* nbr;          // [N][P2M_X2D_MAXDEG] neighbour slots, counter-clockwise
    int32_t* nsh;          // [N][P2M_X2D_MAXDEG] packed image shifts
    double* vol;           // [N] int psi_mu
    p2m_report* rep;
};
hipError_t x2d_triangulate(const X2dArgs& a, hipStream_t stream);
hipError_t x2d_export(const X2dArgs& a, int32_t* deg_out, int32_t* nbr_out, int32_t* sh_out,
                      hipStream_t stream);
// particle interpolant at the nodes (half = false: out [F][nn]) or on the
// half-spacing grid (half = true: out [F][2ny][2nx])
hipError_t x2d_locate(const X2dArgs& a, bool half, double* out, hipStream_t stream);
hipError_t x2d_rhs_mesh(const X2dArgs& a, const double* H, double* b, hipStream_t stream);
hipError_t x2d_mass_mesh(const X2dArgs& a, double* coef, double* w, hipStream_t stream);
hipError_t x2d_rhs_part(const X2dArgs& a, const double* nodal, double* c, hipStream_t stream);
hipError_t x2d_mass_part(const X2dArgs& a, double* coef, int32_t* ecol, hipStream_t stream);

// mass solve
struct CgWorkspace {
    void* r;          // [F][nn] T
    void* p0;         // [F][nn] T   (ping)
    void* p1;         // [F][nn] T   (pong)
    void* q;          // [F][nn] T
    double* x64;      // [2][F][nn] FP64 solution (ping-pong)
    double* partials; // [2][blocks][3*kMaxFields]
    void* dinv;       // [nn] T, inverse of the regularised diagonal
    int blocks;       // grid size of the persistent kernel
    long spin = kSolveSpinDefault;   // bound of a grid-barrier wait (< 0: every wait ends at once)
    const int32_t* ell_col = nullptr;  // sparse-row matrix (Mesh::dim == 3): columns [ell_w][nn]
    int ell_w = 0;
};
size_t cg_partials_bytes(int blocks);
// One persistent kernel with its own grid barrier: orphan regularisation of
// (coef, b) in place, the start vector (FLIP b/w, zero, or the values in x), then
// the solve; x receives the result.
template <typename T>
hipError_t launch_cg(const Mesh& m, int F, T* coef, T* b, const T* w, T* x, int start,
                     const CgWorkspace& ws, const p2m_solve_opts& opts, p2m_report* rep,
                     hipStream_t stream);
template <typename T>
int cg_max_blocks(int device);

// register-resident solve for 2D FP32 problems whose tiles fit one workgroup per
// tile on the device (k_cgr.hip)
constexpr int kResidentMaxFields = 3;
size_t cgr_workspace_bytes(const Mesh& m, int F, int blocks);
int cgr_tiles(const Mesh& m);
bool cgr_supported(const Mesh& m, int F, int device);
// clear_rep: the report the kernel writes is zeroed first (by the counter clear)
hipError_t launch_cg_resident(const Mesh& m, int F, float* coef, float* b, const float* w,
                              float* x, int start, void* ws, const p2m_solve_opts& opts,
                              p2m_report* rep, bool clear_rep, long spin, hipStream_t stream);

// the register-resident solve with the degree-2 Chebyshev polynomial preconditioner
// (k_cgrc.hip): same workspace as the Jacobi one (cgr_workspace_bytes)
bool cgrc_supported(const Mesh& m, int F, int device);
hipError_t launch_cg_resident_cheb(const Mesh& m, int F, float* coef, float* b, const float* w,
                                   float* x, int start, void* ws, const p2m_solve_opts& opts,
                                   p2m_report* rep, bool clear_rep, long spin, hipStream_t stream);

// ---------------------------------------------------------------------------
// batches (k_bin.hip, k_assemble.hip, k_cgb.hip)
// ---------------------------------------------------------------------------
hipError_t launch_report_clear_n(p2m_report* reps, int n, hipStream_t stream);
// locate + count of every particle of the batch; block b belongs to instance
// lmap[b]; keys are batch cell numbers (or -1)
hipError_t launch_locate_count_batch(const BatchInst* inst, const int32_t* lmap, int nblocks,
                                     int32_t* key, int32_t* rank, int32_t* counts,
                                     hipStream_t stream);
// place / segment sort over the whole batch (keys and cell_start in batch numbering,
// perm receives batch particle numbers); no tail is written
hipError_t launch_place_flat(int np, int ncells, const int32_t* key, const int32_t* rank,
                             int32_t* cell_start, int32_t* perm, const void* scan_ws,
                             hipStream_t stream);
hipError_t launch_segment_sort_flat(int ncells, const int32_t* cell_start, int32_t* perm,
                                    hipStream_t stream);
// scatter of every instance: tile t belongs to instance amap[t]; b, w, coef hold
// the instances' blocks (b at F*no, w at no, coef at 4*no)
hipError_t launch_assemble_batch(int F, const BatchInst* inst, const int32_t* amap, int ntiles,
                                 const int32_t* perm, const int32_t* cell_start, float* b,
                                 float* w, float* coef, hipStream_t stream);

// Batched mass solve: one persistent kernel for all instances, several solver
// tiles per workgroup with the CG state streamed from owner-only arrays.
constexpr int kBatchMaxInstances = 128;
constexpr int kBatchMaxPairs = 256;      // instances x fields
constexpr int kBatchMaxOwn = 32;         // solver tiles per workgroup
struct BatchSolveBufs {
    const BatchInst* inst;
    int nprob;
    const int32_t* rmap;   // solver tile -> instance
    const int32_t* order = nullptr;  // dealing order of the solver tiles (null: 0, 1, 2, ...)
    int ntiles;
    float* coef;           // instance blocks [4][nn] at 4*no
    float* b;              // [F][nn] at F*no
    const float* w;        // [nn] at no
    void* ws;              // cgb_workspace_bytes of scratch
    long spin = kSolveSpinDefault;   // bound of a grid-barrier wait (< 0: every wait ends at once)
};
int cgb_grid(int F, int ntiles, int device);   // 0: does not fit
size_t cgb_workspace_bytes(int F, int nprob, int ntiles, size_t nodes);
hipError_t launch_cg_batch(int F, const BatchSolveBufs& bb, size_t nodes, int grid, int start,
                           const p2m_solve_opts& opts, hipStream_t stream);
const void* cgb_kernel(int F);
// a single 2D FP32 problem (F <= 3) through the tile-streaming solve: any mesh
// size; groups = workgroups (0 or more than fit: one per compute unit)
size_t cgt_workspace_bytes(const Mesh& m, int F);
int cgt_grid(const Mesh& m, int F, int groups, int device);   // 0: not available
hipError_t launch_cg_tiles(const Mesh& m, int F, float* coef, float* b, const float* w, float* x,
                           int start, void* ws, const p2m_solve_opts& opts, p2m_report* rep,
                           int groups, int device, long spin, hipStream_t stream);

// learned warm start (k_learn.hip); X rows are BF16 [.][160]
hipError_t launch_learn_features(const Mesh& m, Particles<float> P, const float* values, int F,
                                 const int32_t* perm, const int32_t* cs, const float* b,
                                 const float* w, const int32_t* nodes, int nrows, void* X,
                                 float* base, float* scale, hipStream_t stream);
hipError_t launch_learn_forward(const float* params, const void* X, int nrows, float* y,
                                hipStream_t stream);
size_t learn_workspace_bytes(int batch);
hipError_t launch_learn_train(float* params, float* am, float* av, int step, float lr,
                              const void* X, const float* target, const int32_t* rows, int batch,
                              float* loss_out, float* grad_out, int apply, void* ws,
                              hipStream_t stream);
// the start vector x0 [F][nn] from the network, judged against the FLIP start
size_t learned_start_workspace_bytes(const Mesh& m, int F);
hipError_t launch_learned_start(const Mesh& m, Particles<float> P, const float* values, int F,
                                const int32_t* perm, const int32_t* cs, const float* b,
                                const float* w, const float* coef, const float* params, float* x0,
                                void* ws, p2m_report* rep, hipStream_t stream);

// particle fluid solver (k_ns.hip): stencil arrays of the viscous system I + s K and of
// the pressure system K (node 0 held), the pressure right-hand side -(1/dt) D U*, the
// projection U* - dt M_L^-1 G p, and the mid-point advection of the particles
hipError_t launch_ns_coef(const Mesh& m, float s, float* cv, float* wv, float* cp, float* wp,
                          hipStream_t stream);
hipError_t launch_ns_div(const Mesh& m, double scale, int pin, const float* U, float* rhs,
                         hipStream_t stream);
// direct solve of nb right-hand sides of the viscous (I + s K, pressure = 0) or the
// pressure system (K, zero-mean solution) by 2D FFT; power-of-two sides <= 2048
// the same 2D FFT solve for nb right-hand sides of type R (mode: kFftViscous
// (I + s K), kFftPressure (K, zero mean), kFftMass (the consistent P1 mass matrix
// of the "/" split with s = hx hy)); workspace fft_workspace_bytes(m, nb)
// Sides: powers of two up to 2048, other lengths up to 1024 (fft_supported).
enum { kFftViscous = 0, kFftPressure = 1, kFftMass = 2 };
bool fft_supported(const Mesh& m);
size_t fft_workspace_bytes(const Mesh& m, int nb);
template <typename R>
hipError_t launch_fft_solve(const Mesh& m, int nb, double s, int mode, const R* rhs, R* x,
                            void* ws, hipStream_t stream);
hipError_t launch_ns_fft_solve(const Mesh& m, int nb, double s, int pressure, const float* rhs,
                               float* x, void* ws, hipStream_t stream);   // workspace for nb <= 2
hipError_t launch_ns_correct(const Mesh& m, double factor, const float* Us, const float* p,
                             float* Un, hipStream_t stream);
hipError_t launch_ns_advect(const Mesh& m, double lx, double ly, double dt, const float* x,
                            const float* y, const float* a, const float* U, float* xo, float* yo,
                            p2m_report* rep, hipStream_t stream);

}  // namespace p2m

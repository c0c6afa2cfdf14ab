// Learned warm start: node features, a per-node MLP on BF16 matrix cores, its
// training step, and the start vector of the mass solve.
//
// Features of node i come from the particles of the four cells sharing the node
// (the support of psi_i): cells a = (ix, iy), b = (ix-1, iy), c = (ix-1, iy-1),
// d = (ix, iy-1), each in binned order, the first kLMax kept.  A kept particle
// contributes its offset from the node in cell units (xi - [cell left of the
// node], eta - [cell below the node]) and (A - base) / s, where base = b_i / w_i
// is the FLIP value and s the RMS of A - base over the kept particles; the row
// ends with n / kLMax and zero padding to kLIn = 160 entries.  The network is
// 160 -> 64 -> 64 -> 64 (ReLU) -> 1; x0_i = base + s * y.  A node is used when
// 1 <= n <= kLMax, w_i > 0 and s exceeds 2^-20 max |A| of its kept particles;
// any other node keeps the FLIP value.
//
// Matrix products use v_mfma_f32_16x16x32_bf16 (BF16 operands, FP32
// accumulation).  Operand layout of one 16x16x32 step, lane l, r = l % 16,
// q = l / 16: A (16 x 32) row r, k = 8q .. 8q+7; B (32 x 16) column r, the same
// k; D (16 x 16) column r, rows 4q .. 4q+3.  A wave owns 16 rows (samples); every
// operand is one 16-byte LDS read from a row-major [rows][k] array.
#include "p2m_internal.hpp"

namespace p2m {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kLMax = 48;
constexpr int kLIn = 160;
constexpr int kLH = 64;
constexpr int XS = kLIn + 8;      // LDS row stride of 160-wide rows (bf16)
constexpr int HS = kLH + 8;       // LDS row stride of 64-wide rows
constexpr float kSFloor = 0x1p-20f;
// parameter offsets (FP32 vector)
constexpr int oW1 = 0, ob1 = oW1 + kLH * kLIn, oW2 = ob1 + kLH, ob2 = oW2 + kLH * kLH,
              oW3 = ob2 + kLH, ob3 = oW3 + kLH * kLH, oW4 = ob3 + kLH, ob4 = oW4 + kLH,
              kNParam = ob4 + 1;
static_assert(kNParam == P2M_LEARNED_NPARAM, "parameter count");

__device__ __forceinline__ f32x4 mfma16(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ bf16x8 ld8(const __bf16* p) { return *(const bf16x8*)p; }

// Weights in LDS: W1 [64][XS], W2, W3 [64][HS] as BF16; b1, b2, b3, W4 FP32.
struct LWeights {
    __bf16* W1;
    __bf16* W2;
    __bf16* W3;
    float* b1;
    float* b2;
    float* b3;
    float* W4;
    float b4;
};

__device__ void load_weights(const float* __restrict__ th, const LWeights& w, __bf16* W2T,
                             __bf16* W3T) {
    for (int i = threadIdx.x; i < kLH * kLIn; i += blockDim.x)
        w.W1[(i / kLIn) * XS + i % kLIn] = (__bf16)th[oW1 + i];
    for (int i = threadIdx.x; i < kLH * kLH; i += blockDim.x) {
        const int o = i / kLH, n = i % kLH;
        const __bf16 a = (__bf16)th[oW2 + i], c = (__bf16)th[oW3 + i];
        w.W2[o * HS + n] = a;
        w.W3[o * HS + n] = c;
        if (W2T) W2T[n * HS + o] = a;
        if (W3T) W3T[n * HS + o] = c;
    }
    for (int i = threadIdx.x; i < kLH; i += blockDim.x) {
        w.b1[i] = th[ob1 + i];
        w.b2[i] = th[ob2 + i];
        w.b3[i] = th[ob3 + i];
        w.W4[i] = th[oW4 + i];
    }
}

// Synchronisation of the forward pass: the whole workgroup, or (kWave) only the
// wave, when every buffer it touches besides the read-only weights is the wave's
// own (a wave's LDS accesses execute in program order; the fences keep the
// compiler from moving them across the point).
template <bool kWave>
__device__ __forceinline__ void fwd_sync() {
    if constexpr (kWave) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// One hidden layer for the wave's 16 rows: out[row][n] = bf16(relu(in . W[n] + b[n])),
// K = 32 * KS.  Lane holds rows 4q .. 4q+3 of columns 16t + r.  Every product is
// formed before the barrier and written after it, so out may be the input.
template <int KS, bool kWave = false>
__device__ __forceinline__ void dense_relu_bf16(const __bf16* in, int in_stride, const __bf16* W,
                                                int w_stride, const float* b, __bf16* out) {
    const int l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        acc[t] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < KS; ++s)
            acc[t] = mfma16(ld8(in + r * in_stride + 32 * s + 8 * q),
                            ld8(W + (16 * t + r) * w_stride + 32 * s + 8 * q), acc[t]);
    }
    fwd_sync<kWave>();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const float bb = b[16 * t + r];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            out[(4 * q + i) * HS + 16 * t + r] = (__bf16)fmaxf(acc[t][i] + bb, 0.f);
    }
}

// Forward of the wave's 16 rows of x (row stride XS).  h1, h2: [16][HS] scratch of
// this wave (they may be the same buffer).  Returns h3 (FP32, [t][i] = row 4q+i,
// column 16t+r) and y for rows 4q .. 4q+3 (every lane of a 16-lane group holds
// its group's four y).
template <bool kWave = false>
__device__ __forceinline__ void forward16(const __bf16* x, const LWeights& w, __bf16* h1,
                                          __bf16* h2, float (&h3)[4][4], float (&y)[4]) {
    const int l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    dense_relu_bf16<kLIn / 32, kWave>(x, XS, w.W1, XS, w.b1, h1);
    fwd_sync<kWave>();
    dense_relu_bf16<kLH / 32, kWave>(h1, HS, w.W2, HS, w.b2, h2);
    fwd_sync<kWave>();
    float yp[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < kLH / 32; ++s)
            acc = mfma16(ld8(h2 + r * HS + 32 * s + 8 * q),
                         ld8(w.W3 + (16 * t + r) * HS + 32 * s + 8 * q), acc);
        const float bb = w.b3[16 * t + r], w4 = w.W4[16 * t + r];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            h3[t][i] = fmaxf(acc[i] + bb, 0.f);
            yp[i] = fmaf(w4, h3[t][i], yp[i]);
        }
    }
    // sum over the 16 columns held by the 16 lanes of the group
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        float v = yp[i];
#pragma unroll
        for (int d = 8; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
        y[i] = v + w.b4;
    }
}

// ---------------------------------------------------------------------------
// feature gather for 16 nodes (one wave) into an LDS tile x [16][XS]
// ---------------------------------------------------------------------------
struct GatherIn {
    Mesh m;
    Particles<float> P;
    const float* values;      // [F][np]
    const int32_t* perm;      // binned particle numbers
    const int32_t* cs;        // cell_start
    const float* b;           // [F][nn]
    const float* w;           // [nn]
};

constexpr int kSlots = kLMax / 4;   // slots per lane (4 lanes per node)

// Positions part: lane (r = node of the 16, q = slot group) fills the offsets of
// slots q, q+4, ... of its node and keeps their particle numbers.  Returns n.
__device__ __forceinline__ int gather_positions(const GatherIn& g, int node, __bf16* x,
                                                int (&pidx)[kSlots]) {
    const int l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    const Mesh& m = g.m;
    int n = 0;
    int st[4] = {0, 0, 0, 0}, off[5] = {0, 0, 0, 0, 0};
    if (node >= 0) {
        const int ix = node % m.nx, iy = node / m.nx;
        const int ixm = ix == 0 ? m.nx - 1 : ix - 1, iym = iy == 0 ? m.ny - 1 : iy - 1;
        const int cells[4] = {ix + m.nx * iy, ixm + m.nx * iy, ixm + m.nx * iym, ix + m.nx * iym};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            st[c] = g.cs[cells[c]];
            off[c + 1] = off[c] + (g.cs[cells[c] + 1] - st[c]);
        }
        n = off[4];
    }
    const int k = n < kLMax ? n : kLMax;
#pragma unroll
    for (int j = 0; j < kSlots; ++j) {
        const int s = q + 4 * j;
        float dx = 0.f, dy = 0.f;
        pidx[j] = -1;
        if (s < k) {
            const int role = s < off[1] ? 0 : s < off[2] ? 1 : s < off[3] ? 2 : 3;
            const int i = g.perm[st[role] + (s - off[role])];
            int cx, cy;
            double xi, eta;
            bool fx, fy;
            locate_axis((double)g.P.x[i], m.nx, m.inv_hx, cx, xi, fx);
            locate_axis((double)g.P.y[i], m.ny, m.inv_hy, cy, eta, fy);
            dx = (float)(xi - ((role == 1 || role == 2) ? 1.0 : 0.0));
            dy = (float)(eta - ((role == 2 || role == 3) ? 1.0 : 0.0));
            pidx[j] = i;
        }
        x[r * XS + 3 * s] = (__bf16)dx;
        x[r * XS + 3 * s + 1] = (__bf16)dy;
    }
    if (q == 0) x[r * XS + 3 * kLMax] = (__bf16)((float)k / (float)kLMax);
    if (q == 1)
        for (int c = 3 * kLMax + 1; c < kLIn; ++c) x[r * XS + c] = (__bf16)0.f;
    return n;
}

// Value part of field f, loads: the kept particles' values of the lane's slots
// and the node's b and w (so that several fields' loads can be in flight at once).
struct ValLoads {
    float a[kSlots];
    float bk, wk;
};

__device__ __forceinline__ void load_values(const GatherIn& g, int f, int node,
                                            const int (&pidx)[kSlots], ValLoads& vl) {
    const Mesh& m = g.m;
    vl.wk = 0.f;
    vl.bk = 0.f;
    if (node >= 0) {
        vl.wk = g.w[node];
        vl.bk = g.b[(size_t)f * m.nn + node];
    }
#pragma unroll
    for (int j = 0; j < kSlots; ++j)
        vl.a[j] = pidx[j] >= 0 ? g.values[(size_t)f * m.np + pidx[j]] : 0.f;
}

// Value part of field f from its loads: base, s and the usable flag of the lane's
// node (the same in its four lanes); writes (A - base) / s into the tile.
__device__ __forceinline__ void apply_values(int node, int n, const int (&pidx)[kSlots],
                                             const ValLoads& vl, __bf16* x, float& base,
                                             float& scale, bool& usable) {
    const int l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    const float wk = vl.wk;
    base = 0.f;
    if (node >= 0) base = wk > 0.f ? vl.bk / wk : 0.f;
    float d[kSlots];
    float ss = 0.f, amax = 0.f;
#pragma unroll
    for (int j = 0; j < kSlots; ++j) {
        d[j] = 0.f;
        if (pidx[j] >= 0) {
            const float a = vl.a[j];
            d[j] = a - base;
            ss = fmaf(d[j], d[j], ss);
            amax = fmaxf(amax, fabsf(a));
        }
    }
    ss += __shfl_xor(ss, 16, 64);
    ss += __shfl_xor(ss, 32, 64);
    amax = fmaxf(amax, __shfl_xor(amax, 16, 64));
    amax = fmaxf(amax, __shfl_xor(amax, 32, 64));
    const int k = n < kLMax ? n : kLMax;
    const float s = k > 0 ? sqrtf(ss / (float)k) : 0.f;
    usable = node >= 0 && n >= 1 && n <= kLMax && wk > 0.f && s > kSFloor * amax;
    scale = s;
#pragma unroll
    for (int j = 0; j < kSlots; ++j) {
        const int sl = q + 4 * j;
        x[r * XS + 3 * sl + 2] = (__bf16)(s > 0.f && pidx[j] >= 0 ? d[j] / s : 0.f);
    }
}

// Both parts for one field.
__device__ __forceinline__ void gather_values(const GatherIn& g, int f, int node, int n,
                                              const int (&pidx)[kSlots], __bf16* x, float& base,
                                              float& scale, bool& usable) {
    ValLoads vl;
    load_values(g, f, node, pidx, vl);
    apply_values(node, n, pidx, vl, x, base, scale, usable);
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
constexpr int kWaves = 4;

// Feature rows for a list of nodes (or all nodes): X [row][F][160] BF16, base and
// scale [row][F] (scale 0 where the node is not usable).
__global__ __launch_bounds__(64 * kWaves) void k_learn_features(GatherIn g, int F,
                                                               const int32_t* __restrict__ nodes,
                                                               int nrows, __bf16* __restrict__ X,
                                                               float* __restrict__ base_out,
                                                               float* __restrict__ scale_out) {
    __shared__ __align__(16) __bf16 xt[kWaves][16 * XS];
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    const int row = (blockIdx.x * kWaves + wave) * 16 + r;
    const int node = row < nrows ? (nodes ? nodes[row] : row) : -1;
    int pidx[kSlots];
    __bf16* x = xt[wave];
    const int n = gather_positions(g, node, x, pidx);
    for (int f = 0; f < F; ++f) {
        float base, scale;
        bool usable;
        gather_values(g, f, node, n, pidx, x, base, scale, usable);
        __syncthreads();
        // copy the wave's 16 rows out: lane (r, q) copies 40 entries of row r
        if (row < nrows) {
            __bf16* dst = X + ((size_t)row * F + f) * kLIn;
            for (int c = q * 40; c < q * 40 + 40; c += 8) *(bf16x8*)(dst + c) = ld8(x + r * XS + c);
            if (q == 0) {
                base_out[(size_t)row * F + f] = base;
                scale_out[(size_t)row * F + f] = usable ? scale : 0.f;
            }
        }
        __syncthreads();
    }
}

// Network outputs of feature rows X [nrows][160].
__global__ __launch_bounds__(64 * kWaves) void k_learn_forward(const float* __restrict__ th,
                                                              const __bf16* __restrict__ X,
                                                              int nrows, float* __restrict__ y_out) {
    __shared__ __align__(16) __bf16 W1[kLH * XS], W2[kLH * HS], W3[kLH * HS];
    __shared__ float b1[kLH], b2[kLH], b3[kLH], W4[kLH];
    __shared__ __align__(16) __bf16 xt[kWaves][16 * XS], h1[kWaves][16 * HS], h2[kWaves][16 * HS];
    LWeights w{W1, W2, W3, b1, b2, b3, W4, th[ob4]};
    load_weights(th, w, nullptr, nullptr);
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    const int row0 = (blockIdx.x * kWaves + wave) * 16;
    for (int c = q * 40; c < q * 40 + 40; c += 8) {
        bf16x8 v = {};
        if (row0 + r < nrows) v = ld8(X + (size_t)(row0 + r) * kLIn + c);
        *(bf16x8*)(xt[wave] + r * XS + c) = v;
    }
    __syncthreads();
    float h3[4][4], y[4];
    forward16(xt[wave], w, h1[wave], h2[wave], h3, y);
    if (r == 0)
        for (int i = 0; i < 4; ++i)
            if (row0 + 4 * q + i < nrows) y_out[row0 + 4 * q + i] = y[i];
}

// Learned start of every node and field: x0 = base + s y where usable, the FLIP
// value elsewhere; the per-field usable count goes to used[f].
// Persistent over node groups (kWaves * 16 nodes each, group grp, grp + gridDim,
// ...): the weights are converted into LDS once per workgroup.
__global__ __launch_bounds__(64 * kWaves) void k_learned_start(GatherIn g, int F,
                                                              const float* __restrict__ th,
                                                              float* __restrict__ x0,
                                                              float* __restrict__ xflip,
                                                              int ngroups) {
    __shared__ __align__(16) __bf16 W1[kLH * XS], W2[kLH * HS], W3[kLH * HS];
    __shared__ float b1[kLH], b2[kLH], b3[kLH], W4[kLH];
    __shared__ __align__(16) __bf16 xt[kWaves][16 * XS], h1[kWaves][16 * HS];
    __shared__ float sbase[kWaves][16], sscale[kWaves][16];
    __shared__ int suse[kWaves][16];
    LWeights w{W1, W2, W3, b1, b2, b3, W4, th[ob4]};
    load_weights(th, w, nullptr, nullptr);
    __syncthreads();
    // from here on a wave touches only its own tiles (and the read-only weights):
    // wave-level synchronisation, so the waves of a workgroup run independently
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    for (int grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
        const int node0 = (grp * kWaves + wave) * 16;
        const int node = node0 + r < g.m.nn ? node0 + r : -1;
        int pidx[kSlots];
        const int n = gather_positions(g, node, xt[wave], pidx);
        // the values of up to kFieldLoads fields are loaded together
        constexpr int kFieldLoads = 4;
        for (int f0 = 0; f0 < F; f0 += kFieldLoads) {
            ValLoads vl[kFieldLoads];
#pragma unroll
            for (int e = 0; e < kFieldLoads; ++e)
                if (f0 + e < F) load_values(g, f0 + e, node, pidx, vl[e]);
#pragma unroll
            for (int e = 0; e < kFieldLoads; ++e) {
                const int f = f0 + e;
                if (f >= F) break;
                float base, scale;
                bool usable;
                apply_values(node, n, pidx, vl[e], xt[wave], base, scale, usable);
                if (q == 0) {
                    sbase[wave][r] = base;
                    sscale[wave][r] = scale;
                    suse[wave][r] = usable ? 1 : 0;
                }
                fwd_sync<true>();
                float h3[4][4], y[4];
                forward16<true>(xt[wave], w, h1[wave], h1[wave], h3, y);
                if (r == 0) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int rr = 4 * q + i, nd = node0 + rr;
                        if (nd >= g.m.nn) continue;
                        const float bs = sbase[wave][rr];
                        x0[(size_t)f * g.m.nn + nd] =
                            suse[wave][rr] ? fmaf(sscale[wave][rr], y[i], bs) : bs;
                        xflip[(size_t)f * g.m.nn + nd] = bs;
                    }
                }
                fwd_sync<true>();
            }
        }
    }
}

// Training step, part 1: forward and backward of 64 rows per workgroup; the
// workgroup's gradient (sum over its rows of the per-row gradient of
// (1/B) sum (y - t)^2) goes to gpart[blockIdx.x][kNParam] and its squared error
// sum to lpart[blockIdx.x].  Rows beyond the batch count as absent.
__global__ __launch_bounds__(256) void k_learn_grad(const float* __restrict__ th,
                                                   const __bf16* __restrict__ X,
                                                   const float* __restrict__ target,
                                                   const int32_t* __restrict__ rows, int batch,
                                                   float* __restrict__ gpart,
                                                   float* __restrict__ lpart) {
    __shared__ __align__(16) __bf16 W1[kLH * XS], W2[kLH * HS], W3[kLH * HS], W2T[kLH * HS],
        W3T[kLH * HS];
    __shared__ float b1[kLH], b2[kLH], b3[kLH], W4[kLH];
    __shared__ __align__(16) __bf16 Xs[64 * XS], XT[kLIn * HS];
    // H1 / H2 row-major during the forward, then the deltas (row-major Q and
    // transposed P); H1T / H2T hold the transposed activations for the backward
    __shared__ __align__(16) __bf16 Pb[64 * HS], Qb[64 * HS], H1T[kLH * HS], H2T[kLH * HS];
    __shared__ float dys[64];
    __shared__ float red[4][kWaves][kLH];   // db1, db2, db3 / dW4 partials per wave
    __shared__ float lsum[kWaves];
    LWeights w{W1, W2, W3, b1, b2, b3, W4, th[ob4]};
    load_weights(th, w, W2T, W3T);
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, r = l & 15, q = l >> 4;
    const int b0 = blockIdx.x * 64;
    // rows of the batch: row-major and transposed copies of the inputs
    for (int c = threadIdx.x; c < 64 * (kLIn / 8); c += 256) {
        const int rr = c / (kLIn / 8), cc = (c % (kLIn / 8)) * 8;
        bf16x8 v = {};
        if (b0 + rr < batch) v = ld8(X + (size_t)rows[b0 + rr] * kLIn + cc);
        *(bf16x8*)(Xs + rr * XS + cc) = v;
#pragma unroll
        for (int e = 0; e < 8; ++e) XT[(cc + e) * HS + rr] = v[e];
    }
    __syncthreads();
    // forward: this wave's 16 rows; H1 rows land in Pb, H2 rows in Qb
    const int rw = 16 * wave;
    float h3[4][4], y[4];
    forward16(Xs + rw * XS, w, Pb + rw * HS, Qb + rw * HS, h3, y);
    // transposed activations for the weight gradients
    for (int c = l; c < 16 * kLH; c += 64) {
        const int rr = c / kLH, n = c % kLH;
        H1T[n * HS + rw + rr] = Pb[(rw + rr) * HS + n];
        H2T[n * HS + rw + rr] = Qb[(rw + rr) * HS + n];
    }
    // dy = 2 (y - t) / B per row; squared error
    float le = 0.f;
    if (r == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rr = rw + 4 * q + i;
            float dy = 0.f;
            if (b0 + rr < batch) {
                const float e = y[i] - target[rows[b0 + rr]];
                dy = 2.f * e / (float)batch;
                le = fmaf(e, e, le);
            }
            dys[rr] = dy;
        }
    }
    le += __shfl_xor(le, 16, 64);
    le += __shfl_xor(le, 32, 64);
    if (l == 0) lsum[wave] = le;
    __syncthreads();
    // ---- layer 3: dz3 = dy W4 [z3 > 0]; dW4 = sum dy h3 -----------------------
    float dz3[4][4];
    {
        float pb[4], pw[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            pb[t] = 0.f;
            pw[t] = 0.f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float dy = dys[rw + 4 * q + i];
                dz3[t][i] = h3[t][i] > 0.f ? dy * W4[16 * t + r] : 0.f;
                pb[t] += dz3[t][i];
                pw[t] = fmaf(dy, h3[t][i], pw[t]);
            }
            pb[t] += __shfl_xor(pb[t], 16, 64);
            pb[t] += __shfl_xor(pb[t], 32, 64);
            pw[t] += __shfl_xor(pw[t], 16, 64);
            pw[t] += __shfl_xor(pw[t], 32, 64);
            if (q == 0) {
                red[2][wave][16 * t + r] = pb[t];
                red[3][wave][16 * t + r] = pw[t];
            }
        }
    }
    __syncthreads();   // H1, H2 rows (Pb, Qb) are no longer read
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rr = rw + 4 * q + i, n = 16 * t + r;
            const __bf16 v = (__bf16)dz3[t][i];
            Qb[rr * HS + n] = v;     // dZ3 [row][out]
            Pb[n * HS + rr] = v;     // dZ3T [out][row]
        }
    __syncthreads();
    float* G = gpart + (size_t)blockIdx.x * kNParam;
    // dW3 [out][in] = dZ3T . H2 (K = 64 rows); wave = out tile
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 2; ++s)
            acc = mfma16(ld8(Pb + (rw + r) * HS + 32 * s + 8 * q),
                         ld8(H2T + (16 * t + r) * HS + 32 * s + 8 * q), acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) G[oW3 + (rw + 4 * q + i) * kLH + 16 * t + r] = acc[i];
    }
    // dz2 = (dZ3 . W3) [z2 > 0] for this wave's rows
    float dz2[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 2; ++s)
            acc = mfma16(ld8(Qb + (rw + r) * HS + 32 * s + 8 * q),
                         ld8(W3T + (16 * t + r) * HS + 32 * s + 8 * q), acc);
        float pb = 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rr = rw + 4 * q + i, n = 16 * t + r;
            dz2[t][i] = (float)H2T[n * HS + rr] > 0.f ? acc[i] : 0.f;
            pb += dz2[t][i];
        }
        pb += __shfl_xor(pb, 16, 64);
        pb += __shfl_xor(pb, 32, 64);
        if (q == 0) red[1][wave][16 * t + r] = pb;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rr = rw + 4 * q + i, n = 16 * t + r;
            const __bf16 v = (__bf16)dz2[t][i];
            Qb[rr * HS + n] = v;
            Pb[n * HS + rr] = v;
        }
    __syncthreads();
    // dW2 = dZ2T . H1
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 2; ++s)
            acc = mfma16(ld8(Pb + (rw + r) * HS + 32 * s + 8 * q),
                         ld8(H1T + (16 * t + r) * HS + 32 * s + 8 * q), acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) G[oW2 + (rw + 4 * q + i) * kLH + 16 * t + r] = acc[i];
    }
    // dz1 = (dZ2 . W2) [z1 > 0]
    float dz1[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 2; ++s)
            acc = mfma16(ld8(Qb + (rw + r) * HS + 32 * s + 8 * q),
                         ld8(W2T + (16 * t + r) * HS + 32 * s + 8 * q), acc);
        float pb = 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rr = rw + 4 * q + i, n = 16 * t + r;
            dz1[t][i] = (float)H1T[n * HS + rr] > 0.f ? acc[i] : 0.f;
            pb += dz1[t][i];
        }
        pb += __shfl_xor(pb, 16, 64);
        pb += __shfl_xor(pb, 32, 64);
        if (q == 0) red[0][wave][16 * t + r] = pb;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) Pb[(16 * t + r) * HS + rw + 4 * q + i] = (__bf16)dz1[t][i];
    __syncthreads();
    // dW1 [out][160] = dZ1T . X
    for (int t = 0; t < kLIn / 16; ++t) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 2; ++s)
            acc = mfma16(ld8(Pb + (rw + r) * HS + 32 * s + 8 * q),
                         ld8(XT + (16 * t + r) * HS + 32 * s + 8 * q), acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) G[oW1 + (rw + 4 * q + i) * kLIn + 16 * t + r] = acc[i];
    }
    // biases, W4, b4 and the loss: the waves' partials in a fixed order
    for (int n = threadIdx.x; n < kLH; n += 256) {
        float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
        for (int wv = 0; wv < kWaves; ++wv) {
            s0 += red[0][wv][n];
            s1 += red[1][wv][n];
            s2 += red[2][wv][n];
            s3 += red[3][wv][n];
        }
        G[ob1 + n] = s0;
        G[ob2 + n] = s1;
        G[ob3 + n] = s2;
        G[oW4 + n] = s3;
    }
    if (threadIdx.x == 0) {
        float s = 0.f, le2 = 0.f;
        for (int rr = 0; rr < 64; ++rr) s += dys[rr];
        for (int wv = 0; wv < kWaves; ++wv) le2 += lsum[wv];
        G[ob4] = s;
        lpart[blockIdx.x] = le2;
    }
}

// Training step, part 2: sum of the workgroup gradients in workgroup order, the
// optional gradient output and the Adam update (FP32 master parameters).
__global__ void k_learn_adam(float* __restrict__ th, float* __restrict__ am,
                             float* __restrict__ av, const float* __restrict__ gpart, int nwg,
                             const float* __restrict__ lpart, int batch, float lr, float bc1,
                             float bc2, int apply, float* __restrict__ grad_out,
                             float* __restrict__ loss_out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kNParam) {
        float g = 0.f;
        for (int k = 0; k < nwg; ++k) g += gpart[(size_t)k * kNParam + p];
        if (grad_out) grad_out[p] = g;
        if (apply) {
            const float m = 0.9f * am[p] + 0.1f * g;
            const float v = 0.999f * av[p] + 0.001f * g * g;
            am[p] = m;
            av[p] = v;
            th[p] -= lr * (m / bc1) / (sqrtf(v / bc2) + 1e-8f);
        }
    }
    if (p == 0 && loss_out) {
        float s = 0.f;
        for (int k = 0; k < nwg; ++k) s += lpart[k];
        loss_out[0] = s / (float)batch;
    }
}

// ---------------------------------------------------------------------------
// judge of the learned start: FP64 residual norms of the learned and of the FLIP
// start, per field, then the choice
// ---------------------------------------------------------------------------
constexpr int kJBlock = 256;

__global__ __launch_bounds__(kJBlock) void k_start_resid(Mesh m, int F, const float* __restrict__ coef,
                                                        const float* __restrict__ b,
                                                        const float* __restrict__ w,
                                                        const float* __restrict__ xl,
                                                        const float* __restrict__ xf,
                                                        double* __restrict__ part) {
    __shared__ double sh[kJBlock / 64][2 * kMaxFields];
    const int k = blockIdx.x * kJBlock + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int f = 0; f < F; ++f) {
        double rl = 0.0, rf = 0.0;
        if (k < m.nn) {
            const int ix = k % m.nx, iy = k / m.nx;
            const int ie = ix + 1 == m.nx ? 0 : ix + 1, iw = ix == 0 ? m.nx - 1 : ix - 1;
            const int jn = iy + 1 == m.ny ? 0 : iy + 1, js = iy == 0 ? m.ny - 1 : iy - 1;
            const int kE = ie + m.nx * iy, kW = iw + m.nx * iy, kN = ix + m.nx * jn,
                      kS = ix + m.nx * js, kNE = ie + m.nx * jn, kSW = iw + m.nx * js;
            const size_t nn = m.nn;
            const float cD = w[k] > 0.f ? coef[k] : 1.f;
            const float cE = coef[nn + k], cEw = coef[nn + kW], cN = coef[2 * nn + k],
                        cNs = coef[2 * nn + kS], cNE = coef[3 * nn + k], cNEsw = coef[3 * nn + kSW];
            const double bk = w[k] > 0.f ? (double)b[f * nn + k] : 0.0;
            const float* L = xl + f * nn;
            const float* X = xf + f * nn;
            const double ml = (double)cD * L[k] + (double)cE * L[kE] + (double)cEw * L[kW] +
                              (double)cN * L[kN] + (double)cNs * L[kS] + (double)cNE * L[kNE] +
                              (double)cNEsw * L[kSW];
            const double mf = (double)cD * X[k] + (double)cE * X[kE] + (double)cEw * X[kW] +
                              (double)cN * X[kN] + (double)cNs * X[kS] + (double)cNE * X[kNE] +
                              (double)cNEsw * X[kSW];
            rl = (bk - ml) * (bk - ml);
            rf = (bk - mf) * (bk - mf);
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            rl += __shfl_down(rl, d, 64);
            rf += __shfl_down(rf, d, 64);
        }
        if (lane == 0) {
            sh[wave][2 * f] = rl;
            sh[wave][2 * f + 1] = rf;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * F) {
        double s = 0.0;
        for (int wv = 0; wv < kJBlock / 64; ++wv) s += sh[wv][threadIdx.x];
        part[(size_t)blockIdx.x * 2 * kMaxFields + threadIdx.x] = s;
    }
}

// One workgroup of kJBlock threads: per field, keep the learned start unless its
// residual exceeds the FLIP start's; a replaced field is flagged.  Thread t sums
// the partials of blocks t, t + kJBlock, ... (all 2F values of a block in one
// pass), then a fixed tree over the threads: a deterministic order.
__global__ __launch_bounds__(kJBlock) void k_start_choose(int F, const double* __restrict__ part,
                                                          int nblocks, int* __restrict__ use_flip,
                                                          p2m_report* __restrict__ rep) {
    __shared__ double sh[2 * kMaxFields][kJBlock];
    const int t = threadIdx.x;
    double acc[2 * kMaxFields];
#pragma unroll
    for (int v = 0; v < 2 * kMaxFields; ++v) acc[v] = 0.0;
    for (int k = t; k < nblocks; k += kJBlock) {
        const double* pk = part + (size_t)k * 2 * kMaxFields;
#pragma unroll
        for (int v = 0; v < 2 * kMaxFields; ++v)
            if (v < 2 * F) acc[v] += pk[v];
    }
#pragma unroll
    for (int v = 0; v < 2 * kMaxFields; ++v) sh[v][t] = acc[v];
    __syncthreads();
    for (int d = kJBlock / 2; d >= 1; d >>= 1) {
        if (t < d)
            for (int v = 0; v < 2 * F; ++v) sh[v][t] += sh[v][t + d];
        __syncthreads();
    }
    if (t >= F) return;
    const double rl = sh[2 * t][0], rf = sh[2 * t + 1][0];
    const int flip = !(rl <= rf);
    use_flip[t] = flip;
    if (flip && rep) atomicOr(&rep->flags, (uint32_t)P2M_FLAG_LEARNED_FALLBACK);
}

__global__ void k_start_apply(int nn, int F, const int* __restrict__ use_flip,
                              const float* __restrict__ xf, float* __restrict__ x0) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)nn * F) return;
    if (use_flip[i / nn]) x0[i] = xf[i];
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static GatherIn gather_in(const Mesh& m, Particles<float> P, const float* values,
                          const int32_t* perm, const int32_t* cs, const float* b, const float* w) {
    GatherIn g;
    g.m = m;
    g.P = P;
    g.values = values;
    g.perm = perm;
    g.cs = cs;
    g.b = b;
    g.w = w;
    return g;
}

hipError_t launch_learn_features(const Mesh& m, Particles<float> P, const float* values, int F,
                                 const int32_t* perm, const int32_t* cs, const float* b,
                                 const float* w, const int32_t* nodes, int nrows, void* X,
                                 float* base, float* scale, hipStream_t stream) {
    if (nrows == 0) return hipSuccess;
    const int grid = (nrows + 16 * kWaves - 1) / (16 * kWaves);
    hipLaunchKernelGGL(k_learn_features, dim3(grid), dim3(64 * kWaves), 0, stream,
                       gather_in(m, P, values, perm, cs, b, w), F, nodes, nrows, (__bf16*)X, base,
                       scale);
    return hipGetLastError();
}

hipError_t launch_learn_forward(const float* params, const void* X, int nrows, float* y,
                                hipStream_t stream) {
    if (nrows == 0) return hipSuccess;
    const int grid = (nrows + 16 * kWaves - 1) / (16 * kWaves);
    hipLaunchKernelGGL(k_learn_forward, dim3(grid), dim3(64 * kWaves), 0, stream, params,
                       (const __bf16*)X, nrows, y);
    return hipGetLastError();
}

size_t learn_workspace_bytes(int batch) {
    const size_t nwg = (size_t)(batch + 63) / 64;
    return (nwg * kNParam * sizeof(float) + 255) / 256 * 256 + (nwg * sizeof(float) + 255) / 256 * 256;
}

hipError_t launch_learn_train(float* params, float* am, float* av, int step, float lr,
                              const void* X, const float* target, const int32_t* rows, int batch,
                              float* loss_out, float* grad_out, int apply, void* ws,
                              hipStream_t stream) {
    const int nwg = (batch + 63) / 64;
    float* gpart = (float*)ws;
    float* lpart = (float*)((char*)ws + ((size_t)nwg * kNParam * sizeof(float) + 255) / 256 * 256);
    hipLaunchKernelGGL(k_learn_grad, dim3(nwg), dim3(256), 0, stream, params, (const __bf16*)X,
                       target, rows, batch, gpart, lpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const float bc1 = 1.f - powf(0.9f, (float)step), bc2 = 1.f - powf(0.999f, (float)step);
    hipLaunchKernelGGL(k_learn_adam, dim3((kNParam + 255) / 256), dim3(256), 0, stream, params, am,
                       av, gpart, nwg, lpart, batch, lr, bc1, bc2, apply, grad_out, loss_out);
    return hipGetLastError();
}

size_t learned_start_workspace_bytes(const Mesh& m, int F) {
    const size_t nb = (size_t)(m.nn + kJBlock - 1) / kJBlock;
    return ((size_t)F * m.nn * sizeof(float) + 255) / 256 * 256 +
           (nb * 2 * kMaxFields * sizeof(double) + 255) / 256 * 256 + 256;
}

hipError_t launch_learned_start(const Mesh& m, Particles<float> P, const float* values, int F,
                                const int32_t* perm, const int32_t* cs, const float* b,
                                const float* w, const float* coef, const float* params, float* x0,
                                void* ws, p2m_report* rep, hipStream_t stream) {
    char* p = (char*)ws;
    float* xf = (float*)p;
    p += ((size_t)F * m.nn * sizeof(float) + 255) / 256 * 256;
    const int nb = (m.nn + kJBlock - 1) / kJBlock;
    double* part = (double*)p;
    p += ((size_t)nb * 2 * kMaxFields * sizeof(double) + 255) / 256 * 256;
    int* use_flip = (int*)p;
    const int ngroups = (m.nn + 16 * kWaves - 1) / (16 * kWaves);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        cus = 256;
    const int grid = ngroups < 2 * cus ? ngroups : 2 * cus;  // two workgroups fit a CU's LDS
    hipLaunchKernelGGL(k_learned_start, dim3(grid), dim3(64 * kWaves), 0, stream,
                       gather_in(m, P, values, perm, cs, b, w), F, params, x0, xf, ngroups);
    hipLaunchKernelGGL(k_start_resid, dim3(nb), dim3(kJBlock), 0, stream, m, F, coef, b, w, x0, xf,
                       part);
    hipLaunchKernelGGL(k_start_choose, dim3(1), dim3(kJBlock), 0, stream, F, part, nb, use_flip, rep);
    const size_t tot = (size_t)m.nn * F;
    hipLaunchKernelGGL(k_start_apply, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, stream, m.nn,
                       F, use_flip, xf, x0);
    return hipGetLastError();
}

}  // namespace p2m

// Adjoint of the ETac step on gfx950.
//
// Two persistent kernels over (env, patch) items, like the forward step:
// k_bwd_decay recomputes contact (nothing is kept from the forward call) and
// runs steps 1-2 below with a small LDS footprint, several workgroups per
// CU; k_bwd takes the contacted items and runs steps 3-4.  For
// L = sum_i g_i . U_i:
//   1. active nodes: dL/du_hat_j = g_j                        (U_j = u_hat_j)
//   2. Eq. 1 adjoint, transposed pair loop over passive nodes i:
//        dL/du_hat_j += sum_i w_ij g_i,
//        dL/dalpha_k += sum_ij (-d_ij w_ij) (g_i . u_hat_j)
//   3. residual-network adjoint on split-FP16 MFMA over the passive nodes
//      (the only nodes whose residual is used); every layer is evaluated in
//      both register layouts, so the weight gradients (contractions over
//      nodes) take their operands straight from registers; the max-pool
//      routes its gradient to the arg-max node of each channel (lowest index
//      on ties), which reaches u_hat of active arg-max nodes through W1;
//   4. contact adjoint: dL/d(R, t) of every winning object from dL/du_hat
//      of its active nodes, in FP64.
// Per-item partials (network parameters, alpha, poses) go to plan scratch and
// are summed by the reduction kernels in a fixed order, so results do not
// depend on which workgroup processed which item.
#include "etac_device.h"

namespace etac {

constexpr int kBChunk = 1024;  // passive nodes staged per pass of the decay adjoint
constexpr int kPhiSegs = 64;   // segments of the parameter-gradient reduction

enum BwdKind { BWD_STEP = 0, BWD_PROP = 1, BWD_CONTACT = 2 };

struct BwdParams {
    MeshDev mesh;
    SceneDev scene;
    ModelDev model;
    Scratch scr;
    BwdScratch bwd;
    int E, n_items;
    int batch;                    // queue positions claimed per atomic (all items)
    int net_batch;                // live-list positions claimed per atomic (k_bwd)
    int n_seg;                    // 1024-position segments of the queue
    const int8_t *cobj_in;        // BWD_PROP
    const float *uhat_in;         // BWD_PROP
    const float *grad_u;          // [3][E][N]   BWD_STEP, BWD_PROP
    const float *grad_uhat_in;    // [3][E][N]   BWD_CONTACT
    float *grad_uhat_out;         // [3][E][N]   BWD_PROP
    const uint32_t *saved;        // [E K][kSavedWords] pooling record of the forward, or null
};

constexpr int kTrRow = 20;     // padded row of the block transpose buffer: conflict-free stores, aligned loads
// ---------------------------------------------------------------------------
// item record of the parameter gradients
//
// For every item with contact k_bwd writes the four waves' summed
// accumulators as 40 blocks of 16 x 16 in MFMA output order (block b at
// floats [256 b, 256 b + 256), lane l's registers r at 256 b + 4 l + r):
// dW4[:, :64] (blocks 0-15, row block ob, column block ib at 4 ob + ib), dW2
// (16-31, same order), dW1 with db1 as input column 9 (32-35, row blocks) and
// dW5 (36-39, column blocks, rows 0-2), then the vectors db2, db4 (= s4),
// db3 (= dpre3), db5, g' and g.  The global-MLP weight gradients are rank one
// per item, dW4[:, 64:] = s4 g'^T and dW3 = dpre3 g^T: only their factors are
// stored and the reduction forms the products.
// ---------------------------------------------------------------------------
constexpr int kRecBlocks = 40;
constexpr int kRecB2 = kRecBlocks * 256, kRecB4 = kRecB2 + 64, kRecB3 = kRecB4 + 64, kRecB5 = kRecB3 + 64,
              kRecGp = kRecB5 + 4, kRecG = kRecGp + 64;
static_assert(kRecWords == kRecG + 64, "record size");
static_assert(kRecWords % 4 == 0, "16-byte aligned records");

__host__ __device__ constexpr int rec_block_slot(int b, int row, int col) {
    return b * 256 + (16 * (row >> 2) + col) * 4 + (row & 3);
}

// The parameter reduction sums "columns": record slots 0 .. kRecWords - 1
// (padded to kRedPlain), then the 2 x 64 x 64 rank-one entries, column
// kRedPlain + 4096 w + 64 o + i for w = 0 (dW4[o][64 + i] = s4[o] g'[i]) and
// w = 1 (dW3[o][i] = dpre3[o] g[i]).
constexpr int kRedPlain = (kRecWords + 63) / 64 * 64;
constexpr int kRedCols = kRedPlain + 2 * 4096;
static_assert(kRedCols == kRedColsMax, "reduction columns");

// Reduction column of parameter c.
__device__ int record_column(int c) {
    if (c < kB1) {
        const int o = c / 9, i = c % 9;
        return rec_block_slot(32 + (o >> 4), o & 15, i);
    }
    if (c < kW2) {
        const int o = c - kB1;
        return rec_block_slot(32 + (o >> 4), o & 15, 9);
    }
    if (c < kB2) {
        const int o = (c - kW2) >> 6, i = (c - kW2) & 63;
        return rec_block_slot(16 + 4 * (o >> 4) + (i >> 4), o & 15, i & 15);
    }
    if (c < kW3) return kRecB2 + (c - kB2);
    if (c < kB3) return kRedPlain + 4096 + (c - kW3);
    if (c < kW4) return kRecB3 + (c - kB3);
    if (c < kB4) {
        const int o = (c - kW4) >> 7, i = (c - kW4) & 127;
        if (i < 64) return rec_block_slot(4 * (o >> 4) + (i >> 4), o & 15, i & 15);
        return kRedPlain + 64 * o + (i - 64);
    }
    if (c < kW5) return kRecB4 + (c - kB4);
    if (c < kB5) {
        const int row = (c - kW5) >> 6, i = (c - kW5) & 63;
        return rec_block_slot(36 + (i >> 4), row, i & 15);
    }
    return kRecB5 + (c - kB5);
}

#ifndef ETAC_BWD_NET_ONLY
__global__ __launch_bounds__(256) void k_record_map(int *map) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c < kPhiN) map[c] = record_column(c);
}
#endif

// Staging area of the decay adjoint.
struct DecayStage {
    float4 a[kBChunk];            // (px, py, pz, gx) of staged passive nodes
    float2 b[kBChunk];            // (gy, gz)
    float4 bb[2 * (kBChunk / 32)]; // boxes of the blocks of 32 staged passive nodes
    double part[kWG][12];         // per-thread partial dL/du_hat of its (up to four) active nodes
};

// LDS of the decay kernel (contact, decay adjoint, hand-over).
struct DecayLds {
    DecayStage st;
    double dred[kWaves][12];
    int wcnt[3][kWaves];
    int gmx[kWaves];
    ItemBatch batch;
};

// Power-of-two scales of one item's adjoint: the activations' as in the
// forward (ItemScale) and the gradients': dL/dU of the passive nodes staged
// at 2^dre (dre from their largest |component|), which puts dL/dpre4 at
// 2^d4 = 2^(dre + c5t), dL/dpre2 at 2^d2 = 2^(d4 + s4t) and dL/dpre1 at
// 2^d1 = 2^(d2 + s2t), each below T (see stage_net).  In LDS, read into
// scalar registers where used.
struct BwdScale {
    float fone;          // the constant input 1 of the N-form inputs at the inputs' scale (2^ax)
    int dre, d4, d2, d1;
};

// Chunks of kWG nodes per pass of compact_given.
constexpr int kGivenChunks = 4;

struct BwdLds {
    NetLds net;
    half8 w2th[4 * 2 * 64], w2tl[4 * 2 * 64];   // [it][s][lane] split fragments of W2^T
    half8 w4th[4 * 2 * 64], w4tl[4 * 2 * 64];   // [it][s][lane] split fragments of W4[:, :64]^T
    float w1u[3][64];                           // W1[:, 6..8]: the u_hat inputs
    float w5t[3 * 64];                          // W5 2^c5t (dL/dpre4 = W5^T dL/dr)
    union {
        floatx4 red[kWaves][8][64];        // eight record blocks of every wave's gradient accumulators
        StageBuf xs;                       // node inputs of the network passes
    } u;
    floatx4 acc15[kWaves][8 * 64]; // per-wave dW1 (blocks 0-3) and dW5 (4-7) accumulators [block][lane]
    floatx4 tr[kWaves][16 * kTrRow / 4]; // per-wave 16 x 16 block transpose buffer (rows of kTrRow floats)
    float s4[64];                 // sum_i dL/dpre4_i  (= db4)
    float dgp[64], dpre3[64], dg[64];
    float vroute[64];             // dL/dpre2 routed to the arg-max node of channel c: dg[c] [g[c] > 0]
    float vred[kWaves][64];
    float vred2[kWaves][64];      // second partial-sum buffer of the global-MLP adjoint
    float vrw[kWaves][64];        // each wave's copy of vroute for its routing pass
    int ired[kWaves][64];
    int argmax[64];
    float dxs[64][3];             // dL/du_hat of the routed arg-max node of each channel
    double dred[kWaves][12];
    int wcnt[kGivenChunks][2][kWaves];   // compaction counts, one set per chunk of a pass
    int wmx[2][kWaves];           // per-wave largest |u_hat| component (float bits), objects present (bits)
    BwdScale bsc;                 // the current item's adjoint scales
    ItemBatch batch;
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Transposed weight fragments for the adjoint layers, in the chain order of
// etac_device.h (K step s, lane group q, element e <-> output chain_k(s, q, e)),
// scaled by 2^s2t and 2^s4t, and W5 scaled by 2^c5t (after stage_net).
__device__ void stage_net_t(BwdLds &S, const float *phi) {
    const int tid = threadIdx.x;
    const float s2 = pow2(uniform(S.net.s2t)), s4 = pow2(uniform(S.net.s4t)), s5 = pow2(uniform(S.net.c5t));
    for (int i = tid; i < 192; i += kWG) S.w5t[i] = phi[kW5 + i] * s5;
    for (int idx = tid; idx < 4 * 2 * 64; idx += kWG) {
        const int lane = idx & 63, s = (idx >> 6) & 1, it = idx >> 7, q = lane >> 4;
        const int in = it * 16 + (lane & 15);
        float a[8], b[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int out = chain_k(s, q, e);
            a[e] = phi[kW2 + out * 64 + in] * s2;
            b[e] = phi[kW4 + out * 128 + in] * s4;
        }
        split8(a, S.w2th[idx], S.w2tl[idx]);
        split8(b, S.w4th[idx], S.w4tl[idx]);
    }
    for (int idx = tid; idx < 3 * 64; idx += kWG) S.w1u[idx >> 6][idx & 63] = phi[kW1 + (idx & 63) * 9 + 6 + (idx >> 6)];
}

// ---------------------------------------------------------------------------
// wave-level tile algebra in two register layouts
//
// T form (the forward's): lane l holds node (l & 15) of a 16-node tile;
// register r of block b holds feature 16 b + 4 (l >> 4) + r.  It is the
// output of W X^T with the tile as the MFMA's B operand, and chains into the
// next layer as B.
// N form: lane l holds feature 16 b + (l & 15) of block b; register r holds
// node 4 (l >> 4) + r.  Feeding the split T-form tile as the A operand instead
// (M = nodes, K = input features) and the same weight fragment as the B
// operand gives X W^T in this layout.  In N form the nodes sit in registers,
// so a weight gradient dW = sum_n a_n (x) b_n per 16 x 16 block takes both
// operands straight from the N-form registers: two v_mfma_f32_16x16x32_f16
// whose K = 32 runs over the tile's 16 nodes twice (hi and lo parts).
// Every accumulator here sees only that one MFMA shape: chaining an
// accumulator from the 16x16x32 shape into the 16x16x16 one gave wrong
// gradients with ROCm 7.2 hipcc for gfx950, so the 16x16x16 shape is not used.
// ---------------------------------------------------------------------------
typedef _Float16 half4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split4(const floatx4 &v, half4 &hi, half4 &lo) {
    uint2t h, l;
    unsigned a, b, c, d;
    split2(v[0], v[1], a, b);
    split2(v[2], v[3], c, d);
    h[0] = a; h[1] = c;
    l[0] = b; l[1] = d;
    hi = __builtin_bit_cast(half4, h);
    lo = __builtin_bit_cast(half4, l);
}



// Input layer (9 -> 64, inputs padded to one K step of 32) in both forms:
// h1T = relu(W1 x + b1), h1N = relu(x W1^T + b1).  The three split passes
// run pass-outermost over the eight independent accumulators, so no MFMA
// waits on the one before it (each accumulator sees the same sequence).
__device__ __forceinline__ void layer1_dual(const NetLds &L, const half8 &xh, const half8 &xl, floatx4 h1T[4],
                                            floatx4 h1N[4]) {
    reload_fence();
    const int lane = lane_id(), gq = lane >> 4, col = lane & 15;
    half8 wh[4], wl[4];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        wh[ob] = L.w1h[ob * 64 + lane];
        wl[ob] = L.w1l[ob * 64 + lane];
        h1T[ob] = *reinterpret_cast<const floatx4 *>(&L.b1s[ob * 16 + 4 * gq]);
        const float bn = L.b1s[ob * 16 + col];
        h1N[ob] = floatx4{bn, bn, bn, bn};
    }
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) { h1T[ob] = mfma16(wh[ob], xh, h1T[ob]); h1N[ob] = mfma16(xh, wh[ob], h1N[ob]); }
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) { h1T[ob] = mfma16(wh[ob], xl, h1T[ob]); h1N[ob] = mfma16(xh, wl[ob], h1N[ob]); }
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        h1T[ob] = relu4(mfma16(wl[ob], xh, h1T[ob]));
        h1N[ob] = relu4(mfma16(xl, wh[ob], h1N[ob]));
    }
}

// A 64 -> 64 layer from a split T-form input (xh, xl: the two K steps):
// yT = W x (+ bias), yN = x W^T (+ bias), each only if requested; relu if
// RELU.  wh / wl: fragments [ob][s][lane] of W (or of a transposed weight).
// Split passes run pass-outermost over the independent accumulators.
template <bool WANT_T, bool WANT_N, bool RELU>
__device__ __forceinline__ void layer64(const half8 *wh, const half8 *wl, const half8 xh[2], const half8 xl[2],
                                        const float *bias, floatx4 yT[4], floatx4 yN[4]) {
    reload_fence();
    const int lane = lane_id(), gq = lane >> 4, col = lane & 15;
    floatx4 aT[4], aN[4];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        aT[ob] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
        aN[ob] = aT[ob];
        if (bias) {
            aT[ob] = *reinterpret_cast<const floatx4 *>(&bias[ob * 16 + 4 * gq]);
            const float bn = bias[ob * 16 + col];
            aN[ob] = floatx4{bn, bn, bn, bn};
        }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        half8 h[4], l[4];
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
            h[ob] = wh[(ob * 2 + s) * 64 + lane];
            l[ob] = wl[(ob * 2 + s) * 64 + lane];
        }
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
            if (WANT_T) aT[ob] = mfma16(h[ob], xh[s], aT[ob]);
            if (WANT_N) aN[ob] = mfma16(xh[s], h[ob], aN[ob]);
        }
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
            if (WANT_T) aT[ob] = mfma16(h[ob], xl[s], aT[ob]);
            if (WANT_N) aN[ob] = mfma16(xh[s], l[ob], aN[ob]);
        }
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
            if (WANT_T) aT[ob] = mfma16(l[ob], xh[s], aT[ob]);
            if (WANT_N) aN[ob] = mfma16(xl[s], h[ob], aN[ob]);
        }
    }
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        if (WANT_T) yT[ob] = RELU ? relu4(aT[ob]) : aT[ob];
        if (WANT_N) yN[ob] = RELU ? relu4(aN[ob]) : aN[ob];
    }
}

// Weight-gradient operands: NB N-form blocks of NT tiles, split and packed as
// K = 32 MFMA operands (lane group q holds k = 8 q .. 8 q + 7; any k order
// contracts correctly as long as both operands use it).
//   NT = 2: h = [hi of tile 0, hi of tile 1], l = the lo parts; the three
//           split products hi*hi, hi*lo, lo*hi take one MFMA each.
//   NT = 1: A operand h = [hi hi], l = [lo 0]; B operand h = [hi lo]; then
//           A.h B.h = hi*hi + hi*lo and A.l B.h = lo*hi.
// Every accumulator sees only the 16x16x32 MFMA shape: chaining an
// accumulator from that shape into the 16x16x16 one gave wrong gradients
// with ROCm 7.2 hipcc for gfx950, so the 16x16x16 shape is not used.
template <int NT, int NB, bool A_ROLE>
struct WOp {
    static_assert(NT == 1 || NT == 2, "one or two tiles");
    half8 h[NB], l[NB];
    __device__ __forceinline__ void set(int u, int j, const floatx4 &v) {
        half4 hi, lo;
        split4(v, hi, lo);
        if constexpr (NT == 2) {
            if (u == 0) { h[j].lo = hi; l[j].lo = lo; }
            else { h[j].hi = hi; l[j].hi = lo; }
        } else if constexpr (A_ROLE) {
            h[j].lo = hi; h[j].hi = hi;
            l[j].lo = lo; l[j].hi = half4{0, 0, 0, 0};
        } else {
            h[j].lo = hi; h[j].hi = lo;
        }
    }
};

// acc[o][i] += sum over the tiles' nodes of A[o] (x) B[i], split passes
// outermost.
template <int NT, int NO, int NI>
__device__ __forceinline__ void wgrad_tiles(const WOp<NT, NO, true> &A, const WOp<NT, NI, false> &B,
                                            floatx4 (&acc)[NO][NI]) {
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int i = 0; i < NI; ++i) acc[o][i] = mfma16(A.h[o], B.h[i], acc[o][i]);
    if constexpr (NT == 2) {
#pragma unroll
        for (int o = 0; o < NO; ++o)
#pragma unroll
            for (int i = 0; i < NI; ++i) acc[o][i] = mfma16(A.h[o], B.l[i], acc[o][i]);
    }
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int i = 0; i < NI; ++i) acc[o][i] = mfma16(A.l[o], B.h[i], acc[o][i]);
}

// acc15[wave][blk0 + o NI + i] += post * sum over the tiles' nodes of
// A[o] (x) B[i] (NO x NI = 4 blocks; post a power of two that brings the
// products to the accumulator's scale, used only if SCALED): products from
// fresh accumulators, then one LDS read-modify-write per block.
template <int NT, int NO, int NI, bool SCALED = false>
__device__ __forceinline__ void acc15_add(floatx4 *acc, int blk0, const WOp<NT, NO, true> &A,
                                          const WOp<NT, NI, false> &B, float post = 1.0f) {
    static_assert(NO * NI == 4, "four blocks");
    const int lane = lane_id();
    floatx4 t[NO][NI];
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int i = 0; i < NI; ++i) t[o][i] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    wgrad_tiles<NT, NO, NI>(A, B, t);
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const int j = blk0 + o * NI + i;
            floatx4 v = acc[j * 64 + lane];
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] += SCALED ? t[o][i][r] * post : t[o][i][r];
            acc[j * 64 + lane] = v;
        }
}

// Network inputs in N form, scaled by xmul: lane l supplies input feature
// (l & 15) of nodes 4 (l >> 4) + r: [p - o_k (3), n (3), U_hat (3)], a
// constant 1 at input 9 (its weight-gradient column is the bias gradient
// db1), zeros above.
__device__ __forceinline__ floatx4 load_xn(const MeshDev &M, int k, int base, const int ln[4], const bool v[4],
                                           const float *uhn, int n_max, float xmul) {
    const int col = lane_id() & 15, N = M.N;
    floatx4 x;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        float val = 0.0f;
        if (v[r]) {
            const int g = base + ln[r];
            if (col < 3) val = M.pos[(size_t)col * N + g] - M.origin[3 * k + col];
            else if (col < 6) val = M.nrm[(size_t)(col - 3) * N + g];
            else if (col < 9) val = uhn[(size_t)(col - 6) * n_max + ln[r]];
            else if (col == 9) val = 1.0f;
        }
        x[r] = val * xmul;
    }
    return x;
}

// This wave's accumulators of the item's parameter gradients.  Blocks are
// 16 x 16 in MFMA output layout: lane l, register r holds row 4 (l >> 4) + r,
// column l & 15 of the block.
// dW1 (row blocks 0-3; columns = 16 padded inputs, column 9 = db1) and dW5
// (column blocks 4-7; rows = the 3 outputs padded to 16) accumulate in the
// wave's own LDS region S.acc15[wave] in the same layout.
struct WGrad {
    floatx4 w4[4][4];    // dW4[:, :64]   [row block][column block]
    floatx4 w2[4][4];    // dW2
    floatx4 b4, b2;      // per-lane partial sums of dpre4 / dpre2 for feature 16 b + (l & 15), b = component
    float b5;            // lanes with (l & 15) < 3: partial db5[l & 15]
};


__device__ __forceinline__ void zero_wgrad(WGrad &G) {
    const floatx4 z = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) { G.w4[a][b] = z; G.w2[a][b] = z; }
    G.b4 = z;
    G.b2 = z;
    G.b5 = 0.0f;
}

// N form of a T-form tile through the wave's LDS buffer, one 16 x 16 block
// at a time: value (feature 4 q + r, node c) of a block is stored at row
// 4 q + r, column c and read back as four consecutive columns of row c.  The
// wave's LDS operations execute in order, so the buffer is reused per block
// with no wait between blocks.
__device__ __forceinline__ void to_n_form(floatx4 *buf, const floatx4 t[4], floatx4 n[4]) {
    float *b = reinterpret_cast<float *>(buf);
    const int lane = lane_id(), gq = lane >> 4, col = lane & 15;
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
#pragma unroll
        for (int r = 0; r < 4; ++r) b[(4 * gq + r) * kTrRow + col] = t[ob][r];
        wave_sync();
        n[ob] = *reinterpret_cast<const floatx4 *>(&b[col * kTrRow + 4 * gq]);
        wave_sync();
    }
}

// T-form layers over NT tiles; each weight fragment is read from LDS once
// for all tiles.  Per tile and block the MFMA sequence is that of layer64:
// per K step hi*hi, hi*lo, lo*hi.  A tile's MFMAs of a K step are issued
// together, so the first tile's output is complete while the next tile's
// MFMAs still run and its ReLU and split overlap them.
template <int NT>
__device__ __forceinline__ void layer1_tiles(const NetLds &L, const half8 (&xh)[NT], const half8 (&xl)[NT],
                                             floatx4 (&h1)[NT][4]) {
    reload_fence();
    const int lane = lane_id(), gq = lane >> 4;
    half8 wh[4], wl[4];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        wh[ob] = L.w1h[ob * 64 + lane];
        wl[ob] = L.w1l[ob * 64 + lane];
        const floatx4 b = *reinterpret_cast<const floatx4 *>(&L.b1s[ob * 16 + 4 * gq]);
#pragma unroll
        for (int u = 0; u < NT; ++u) h1[u][ob] = b;
    }
#pragma unroll
    for (int u = 0; u < NT; ++u) {
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) h1[u][ob] = mfma16(wh[ob], xh[u], h1[u][ob]);
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) h1[u][ob] = mfma16(wh[ob], xl[u], h1[u][ob]);
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) h1[u][ob] = relu4(mfma16(wl[ob], xh[u], h1[u][ob]));
    }
}

// y[u] = W x[u] (+ bias), relu if RELU (T form in and out).
template <int NT, bool RELU>
__device__ __forceinline__ void layer64_tiles(const half8 *wh, const half8 *wl, const half8 (&xh)[NT][2],
                                              const half8 (&xl)[NT][2], const float *bias, floatx4 (&y)[NT][4]) {
    reload_fence();
    const int lane = lane_id(), gq = lane >> 4;
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        const floatx4 b = bias ? *reinterpret_cast<const floatx4 *>(&bias[ob * 16 + 4 * gq])
                               : floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int u = 0; u < NT; ++u) y[u][ob] = b;
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        half8 h[4], l[4];
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
            h[ob] = wh[(ob * 2 + s) * 64 + lane];
            l[ob] = wl[(ob * 2 + s) * 64 + lane];
        }
#pragma unroll
        for (int u = 0; u < NT; ++u) {
#pragma unroll
            for (int ob = 0; ob < 4; ++ob) y[u][ob] = mfma16(h[ob], xh[u][s], y[u][ob]);
#pragma unroll
            for (int ob = 0; ob < 4; ++ob) y[u][ob] = mfma16(h[ob], xl[u][s], y[u][ob]);
#pragma unroll
            for (int ob = 0; ob < 4; ++ob) y[u][ob] = mfma16(l[ob], xh[u][s], y[u][ob]);
        }
    }
    if (RELU)
#pragma unroll
        for (int u = 0; u < NT; ++u)
#pragma unroll
            for (int ob = 0; ob < 4; ++ob) y[u][ob] = relu4(y[u][ob]);
}

// y[u] = x[u] W^T in N form from a split T-form input (no bias, no relu).
template <int NT>
__device__ __forceinline__ void layer64_tiles_n(const half8 *wh, const half8 *wl, const half8 (&xh)[NT][2],
                                                const half8 (&xl)[NT][2], floatx4 (&y)[NT][4]) {
    reload_fence();
    const int lane = lane_id();
#pragma unroll
    for (int ob = 0; ob < 4; ++ob)
#pragma unroll
        for (int u = 0; u < NT; ++u) y[u][ob] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        half8 h[4], l[4];
#pragma unroll
        for (int ob = 0; ob < 4; ++ob) {
            h[ob] = wh[(ob * 2 + s) * 64 + lane];
            l[ob] = wl[(ob * 2 + s) * 64 + lane];
        }
#pragma unroll
        for (int u = 0; u < NT; ++u) {
#pragma unroll
            for (int ob = 0; ob < 4; ++ob) y[u][ob] = mfma16(xh[u][s], h[ob], y[u][ob]);
#pragma unroll
            for (int ob = 0; ob < 4; ++ob) y[u][ob] = mfma16(xh[u][s], l[ob], y[u][ob]);
#pragma unroll
            for (int ob = 0; ob < 4; ++ob) y[u][ob] = mfma16(xl[u][s], h[ob], y[u][ob]);
        }
    }
}

// Adjoint of NT tiles of 16 passive nodes (staged nodes 16 t[u] .. 16 t[u] +
// 15 of the current chunk of cnt): forward recomputation, decoder and encoder
// adjoints, all accumulated into this wave's parameter gradients.  Passive
// nodes have U_hat = 0 and need no dL/du_hat; the stage holds dL/dU (at
// 2^dre) in its third triple.  Every layer runs in T form on MFMA; the N
// forms the weight gradients need are block transposes of the T-form values.
// dW5 (three output rows) accumulates in FP32 on the VALU, so h4 is never
// split.  Accumulator scales: dW5 2^(dre + a4), db5 2^dre, dW4 2^(d4 + af),
// db4 2^d4, dW2 2^(d2 + a1), db2 2^d2, dW1 2^(d1 + ax).
template <int NT>
__device__ void passive_tiles(BwdLds &S, WGrad &G, int cnt, const int (&t)[NT]) {
    const NetLds &L = S.net;
    const StageBuf &xs = S.u.xs;
    const int wave = threadIdx.x >> 6;
    floatx4 *tb = S.tr[wave];
    const int lane = lane_id(), gq = lane >> 4, col = lane & 15;
    // T form: this lane's node; N form: nodes 4 gq + r
    int lj[NT][4];
    bool vr[NT][4];
    floatx4 xn[NT];
    float dr[NT][3];
    half8 xh[NT], xl[NT];
    // N-form network inputs: feature col of nodes lj[r] (U_hat = 0; input 9 =
    // 1).  Reads stay inside the stage (tile rows < kStage) and are masked
    // afterwards, so no lane branches.
    const int fcol = col < 6 ? col : 0;
    const float fsel = col < 6 ? 1.0f : 0.0f, fone = col == 9 ? uniform(S.bsc.fone) : 0.0f;
#pragma unroll
    for (int u = 0; u < NT; ++u) {
        const int li = 16 * t[u] + col;
        const bool valid = li < cnt;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            lj[u][r] = 16 * t[u] + 4 * gq + r;
            vr[u][r] = lj[u][r] < cnt;
            xn[u][r] = vr[u][r] ? xs[fcol][lj[u][r]] * fsel + fone : 0.0f;
        }
        // dL/dr of this lane's node (zero on padding)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float v = xs[6 + c][li];
            dr[u][c] = valid ? v : 0.0f;
        }
        stage_x<true>(xs, li, valid, xh[u], xl[u]);
    }
    // forward recomputation (T form)
    floatx4 h1T[NT][4], fT[NT][4], h4T[NT][4];
    half8 sh[NT][2], sl[NT][2];
    layer1_tiles<NT>(L, xh, xl, h1T);
#pragma unroll
    for (int u = 0; u < NT; ++u) split_chain(h1T[u], sh[u], sl[u]);
    layer64_tiles<NT, true>(L.w2h, L.w2l, sh, sl, L.b2s, fT);
#pragma unroll
    for (int u = 0; u < NT; ++u) split_chain(fT[u], sh[u], sl[u]);
    layer64_tiles<NT, true>(L.w4h, L.w4l, sh, sl, L.c4, h4T);
    // dL/dpre4 = (W5^T dr) [h4 > 0]
    floatx4 d4T[NT][4];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ft = ob * 16 + 4 * gq + r;
            const float w0 = S.w5t[ft], w1 = S.w5t[64 + ft], w2 = S.w5t[128 + ft];
#pragma unroll
            for (int u = 0; u < NT; ++u) {
                const float vt = w0 * dr[u][0] + w1 * dr[u][1] + w2 * dr[u][2];
                d4T[u][ob][r] = h4T[u][ob][r] > 0.0f ? vt : 0.0f;
            }
        }
    // dW5 += dr (x) h4 in FP32: lane l adds, for feature 16 ib + (l & 15),
    // its four nodes 4 gq + r into acc15[4 + ib] (components 0..2; the lane
    // groups are summed when the record is written); db5
    {
        const int ccol = col < 3 ? col : 0;
        floatx4 *a5 = S.acc15[wave] + 4 * 64;
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            floatx4 h4N[4];
            to_n_form(tb, h4T[u], h4N);
            float d[4][3];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float v = xs[6 + c][lj[u][r]];
                    d[r][c] = vr[u][r] ? v : 0.0f;
                }
            G.b5 += col < 3 ? (d[0][ccol] + d[1][ccol]) + (d[2][ccol] + d[3][ccol]) : 0.0f;
#pragma unroll
            for (int ib = 0; ib < 4; ++ib) {
                floatx4 v = a5[ib * 64 + lane];
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    v[c] += (d[0][c] * h4N[ib][0] + d[1][c] * h4N[ib][1]) + (d[2][c] * h4N[ib][2] + d[3][c] * h4N[ib][3]);
                a5[ib * 64 + lane] = v;
            }
        }
    }
    // dW4[:, :64] += dpre4 (x) f, db4; f > 0 kept as bits (4 block + register)
    unsigned fmask[NT];
    {
        WOp<NT, 4, true> A;
        WOp<NT, 4, false> B;
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            floatx4 d4N[4], fN[4];
            to_n_form(tb, d4T[u], d4N);
            to_n_form(tb, fT[u], fN);
            fmask[u] = 0u;
#pragma unroll
            for (int ob = 0; ob < 4; ++ob) {
#pragma unroll
                for (int r = 0; r < 4; ++r) fmask[u] |= (fT[u][ob][r] > 0.0f ? 1u : 0u) << (4 * ob + r);
                B.set(u, ob, fN[ob]);
                G.b4[ob] += (d4N[ob][0] + d4N[ob][1]) + (d4N[ob][2] + d4N[ob][3]);
                A.set(u, ob, d4N[ob]);
            }
        }
        wgrad_tiles<NT, 4, 4>(A, B, G.w4);
    }
    // dL/df = W4[:, :64]^T dpre4
#pragma unroll
    for (int u = 0; u < NT; ++u) split_chain(d4T[u], sh[u], sl[u]);
    floatx4 dfT[NT][4];
    layer64_tiles<NT, false>(S.w4th, S.w4tl, sh, sl, nullptr, dfT);
    // dL/dpre2 = df [f > 0]; dL/dh1 = W2^T dpre2 (N form only: no dL/du_hat here)
    floatx4 d2T[NT][4];
#pragma unroll
    for (int u = 0; u < NT; ++u)
#pragma unroll
        for (int ob = 0; ob < 4; ++ob)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                d2T[u][ob][r] = ((fmask[u] >> (4 * ob + r)) & 1u) ? dfT[u][ob][r] : 0.0f;
#pragma unroll
    for (int u = 0; u < NT; ++u) split_chain(d2T[u], sh[u], sl[u]);
    floatx4 dh1N[NT][4];
    layer64_tiles_n<NT>(S.w2th, S.w2tl, sh, sl, dh1N);
    // dW2 += dpre2 (x) h1, db2; dW1 += dpre1 (x) x (db1 through input 9)
    {
        WOp<NT, 4, true> A2, A1;
        WOp<NT, 4, false> B2;
        WOp<NT, 1, false> B1;
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            floatx4 h1N[4], d2N[4];
            to_n_form(tb, h1T[u], h1N);
            to_n_form(tb, d2T[u], d2N);
#pragma unroll
            for (int ob = 0; ob < 4; ++ob) {
                B2.set(u, ob, h1N[ob]);
                G.b2[ob] += (d2N[ob][0] + d2N[ob][1]) + (d2N[ob][2] + d2N[ob][3]);
                A2.set(u, ob, d2N[ob]);
                floatx4 d1;
#pragma unroll
                for (int r = 0; r < 4; ++r) d1[r] = h1N[ob][r] > 0.0f ? dh1N[u][ob][r] : 0.0f;
                A1.set(u, ob, d1);
            }
            B1.set(u, 0, xn[u]);
        }
        wgrad_tiles<NT, 4, 4>(A2, B2, G.w2);
        acc15_add<NT, 4, 1>(S.acc15[wave], 0, A1, B1);
    }
}

// Max-pool routing for the wave's 16 channels c = 16 wave + j: the
// gradient dL/dpre2 = vroute[c] e_c at the arg-max node of channel c.  Its
// dL/dh1 = W2^T dpre2 is row c of W2 scaled, in both forms; adds the dW2
// rows, dW1 and db1 contributions and leaves dL/du_hat of each channel's
// node in S.dxs (identical in the four lane groups).
// Network inputs of the wave's channels' arg-max nodes, loaded ahead of the
// global-MLP adjoint so that their latency overlaps it: T form (this lane's
// channel 16 wave + (l & 15)) and N form (channels 16 wave + 4 (l >> 4) + r).
struct RouteIn {
    float x[8];
    floatx4 xn;
};

__device__ __forceinline__ void route_inputs(const BwdParams &p, const BwdLds &S, int k, int base, int n,
                                             const float *uhn, float xmul, RouteIn &in) {
    const MeshDev &M = p.mesh;
    const int lane = lane_id(), wave = threadIdx.x >> 6, gq = lane >> 4, col = lane & 15, n_max = p.scr.n_max;
    const int lnT = S.argmax[16 * wave + col];
    const bool vT = lnT < n;
    int lnr[4];
    bool vr[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        lnr[r] = S.argmax[16 * wave + 4 * gq + r];
        vr[r] = lnr[r] < n;
        if (!vr[r]) lnr[r] = 0;
    }
    load_x_raw(M, k, base + (vT ? lnT : 0), vT, uhn, n_max, vT ? lnT : 0, xmul, in.x);
    in.xn = load_xn(M, k, base, lnr, vr, uhn, n_max, xmul);
}

// vroute is unscaled and h1 at 2^a1: 2^d2 brings the routed dL/dpre2 (x) h1
// to dW2's accumulator scale 2^(d2 + a1); the routed dL/dpre1 (unscaled) is
// split at its own scale 2^drt from a bound max |vroute| max |W2|, and its
// dW1 products are brought to the accumulator's scale 2^(d1 + ax) by
// 2^(d1 - drt).
__device__ void routing_tile(const BwdParams &p, BwdLds &S, WGrad &G, int n, const RouteIn &in) {
    const NetLds &L = S.net;
    const int lane = lane_id(), wave = threadIdx.x >> 6, gq = lane >> 4, col = lane & 15;
    const float *vroute = S.vrw[wave];   // this wave's copy (identical in every wave)
    const int drt = uniform(range_exp(wave_max(fabsf(vroute[lane])) * S.net.mw2));   // same in every wave
    const float drt_mul = uniform(pow2(drt)), post = uniform(pow2(uniform(S.bsc.d1) - drt));
    const float d2mul = uniform(pow2(uniform(S.bsc.d2)));
    // T form: channel 16 wave + col; N form: channels 16 wave + 4 gq + r
    const int cT = 16 * wave + col;
    const int lnT = S.argmax[cT];
    const bool vT = lnT < n;
    float vn[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int c = 16 * wave + 4 * gq + r;
        vn[r] = S.argmax[c] < n ? vroute[c] : 0.0f;
    }
    half8 xh, xl;
    {
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = in.x[e];
        split8(v, xh, xl);
    }
    floatx4 h1T[4], h1N[4];
    layer1_dual(L, xh, xl, h1T, h1N);
    // dL/dpre2 is one-hot, vroute[c] e_c, so dL/dh1 = W2^T dpre2 is row c of
    // W2 scaled by vroute[c], in both forms
    const float vt = vT ? vroute[cT] : 0.0f;
    const float *w2 = p.model.phi + kW2;
    floatx4 dh1T[4], dh1N[4];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            dh1T[ob][r] = vt * w2[cT * 64 + ob * 16 + 4 * gq + r];
            dh1N[ob][r] = vn[r] * w2[(16 * wave + 4 * gq + r) * 64 + ob * 16 + col];
        }
    // dL/du_hat of the channel's node: W1[:, 6..8]^T dpre1 in T form
    float du[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ob = 0; ob < 4; ++ob)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int f = ob * 16 + 4 * gq + r;
            const float d1 = h1T[ob][r] > 0.0f ? dh1T[ob][r] : 0.0f;
#pragma unroll
            for (int c = 0; c < 3; ++c) du[c] += S.w1u[c][f] * d1;
        }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        du[c] += __shfl_xor(du[c], 16);
        du[c] += __shfl_xor(du[c], 32);
        S.dxs[cT][c] = du[c];
    }
    // dW2 rows 16 wave + 4 gq + r += vroute h1 (FP32): row block `wave`; the
    // other blocks add exact zeros (no register indexed by the wave number)
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        const bool mine = ob == wave;
#pragma unroll
        for (int ib = 0; ib < 4; ++ib)
#pragma unroll
            for (int r = 0; r < 4; ++r) G.w2[ob][ib][r] += (mine ? vn[r] * d2mul : 0.0f) * h1N[ib][r];
    }
    // dW1 += dpre1 (x) x (db1 through input 9)
    WOp<1, 4, true> A;
    WOp<1, 1, false> B;
    B.set(0, 0, in.xn);
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        floatx4 d1;
#pragma unroll
        for (int r = 0; r < 4; ++r) d1[r] = h1N[ob][r] > 0.0f ? dh1N[ob][r] * drt_mul : 0.0f;
        A.set(0, ob, d1);
    }
    acc15_add<1, 4, 1, true>(S.acc15[wave], 0, A, B, post);
}

// ---------------------------------------------------------------------------
// item-level pieces
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool uses_residual(const BwdParams &p) {
    return p.model.mode != ETAC_DECAY_ONLY;
}

// Stage passive nodes plist[c0 .. c0 + cnt) (position, dL/dU) and, with the
// cutoff on, their block boxes.  Whole workgroup, barriers included.
__device__ __forceinline__ void stage_passive_chunk(const BwdParams &p, DecayStage &st, int base, size_t row,
                                                    const int *plist, int c0, int cnt, bool boxes) {
    const MeshDev &M = p.mesh;
    const int N = M.N;
    const size_t EN = (size_t)p.E * N;
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += kWG) {
        const int i = plist[c0 + t];
        const int gi = base + i;
        st.a[t] = make_float4(M.pos[gi], M.pos[N + gi], M.pos[2 * N + gi], p.grad_u[row + i]);
        st.b[t] = make_float2(p.grad_u[EN + row + i], p.grad_u[2 * EN + row + i]);
    }
    __syncthreads();
    if (boxes) {
        block_boxes(st.a, cnt, st.bb);
        __syncthreads();
    }
}

// Eq. 1 adjoint of one item.  Pairs (active j, passive i) are split over a
// grid of SLOTS active slots x (kWG / SLOTS) passive segments: every thread
// owns A active nodes per pass and one segment of each staged chunk of
// passive nodes (position, g).  Slots are whole waves, so LDS reads stay
// broadcasts.  The segment partials of dL/du_hat_j are combined in segment
// order; the thread's dL/dalpha contribution is returned.
template <int SLOTS, int A>
__device__ double decay_adjoint_grid(const BwdParams &p, DecayStage &st, int e, int k, int base, int m, int np,
                                     const int *alist, const int *plist, const float *uhn, float *gh) {
    const MeshDev &M = p.mesh;
    const int N = M.N, n_max = p.scr.n_max;
    const size_t row = (size_t)e * N + base;
    const float nbeta = (float)(-(double)p.model.alpha[k] * 1.4426950408889634);
    float cut2 = cutoff_d2(p.model.alpha[k]);
    if (!cutoff_useful(M, k, cut2)) cut2 = -1.0f;     // off: no boxes, no tests
    constexpr int nseg = kWG / SLOTS;
    const int slot = threadIdx.x % SLOTS, seg = threadIdx.x / SLOTS;
    // a passive set that fits one chunk is staged once for every pass
    const bool one_chunk = np <= kBChunk;
    if (one_chunk) stage_passive_chunk(p, st, base, row, plist, 0, np, cut2 >= 0.0f);
    double dalpha = 0.0;
    for (int ab = 0; ab < m; ab += A * SLOTS) {
        bool v[A];
        int j[A];
        float px[A], py[A], pz[A], ux[A], uy[A], uz[A];
        double acc[A][3], da[A];
#pragma unroll
        for (int a = 0; a < A; ++a) {
            const int t = ab + slot + a * SLOTS;
            v[a] = t < m;
            j[a] = v[a] ? alist[t] : alist[0];
            const int g = base + j[a];
            px[a] = M.pos[g]; py[a] = M.pos[N + g]; pz[a] = M.pos[2 * N + g];
            ux[a] = uhn[j[a]]; uy[a] = uhn[n_max + j[a]]; uz[a] = uhn[2 * n_max + j[a]];
            acc[a][0] = acc[a][1] = acc[a][2] = 0.0;
            da[a] = 0.0;
        }
        for (int c0 = 0; c0 < np; c0 += kBChunk) {
            const int cnt = min(kBChunk, np - c0);
            if (!one_chunk) stage_passive_chunk(p, st, base, row, plist, c0, cnt, cut2 >= 0.0f);
            const int per = (cnt + nseg - 1) / nseg;
            const int lo = seg * per, hi = min(cnt, lo + per);
            for (int i0 = lo; i0 < hi; i0 += 32) {
                const int i1 = min(hi, i0 + 32);
                if (cut2 >= 0.0f) {   // uniform: the cutoff is on for this item
                    // skip a run no valid active node of the wave reaches within the cutoff
                    // (wave-uniform; the run overlaps boxes b0 and b1)
                    const int b0 = i0 >> 5, b1 = (i1 - 1) >> 5;
                    const float4 lo0 = st.bb[2 * b0], hi0 = st.bb[2 * b0 + 1];
                    const float4 lo1 = st.bb[2 * b1], hi1 = st.bb[2 * b1 + 1];
                    bool need = false;
#pragma unroll
                    for (int a = 0; a < A; ++a)
                        need = need || (v[a] && (box_d2(lo0, hi0, px[a], py[a], pz[a]) < cut2 ||
                                                 box_d2(lo1, hi1, px[a], py[a], pz[a]) < cut2));
                    if (__ballot(need) == 0ull) continue;
                }
                float sx[A], sy[A], sz[A], q[A];
#pragma unroll
                for (int a = 0; a < A; ++a) sx[a] = sy[a] = sz[a] = q[a] = 0.0f;
                // the run's bounds are wave-uniform (segments are whole waves): scalar loop control
                const int ie = uniform(i1);
#pragma unroll 4
                for (int i = uniform(i0); i < ie; ++i) {
                    const float4 pa = st.a[i];
                    const float2 pb = st.b[i];
#pragma unroll
                    for (int a = 0; a < A; ++a) {
                        const float dx = pa.x - px[a], dy = pa.y - py[a], dz = pa.z - pz[a];
                        const float d = __builtin_amdgcn_sqrtf(dx * dx + dy * dy + dz * dz);
                        const float w = __builtin_amdgcn_exp2f(nbeta * d);
                        sx[a] += w * pa.w; sy[a] += w * pb.x; sz[a] += w * pb.y;
                        q[a] += d * w * (pa.w * ux[a] + pb.x * uy[a] + pb.y * uz[a]);
                    }
                }
#pragma unroll
                for (int a = 0; a < A; ++a) {
                    acc[a][0] += sx[a]; acc[a][1] += sy[a]; acc[a][2] += sz[a];
                    da[a] -= q[a];
                }
            }
        }
#pragma unroll
        for (int a = 0; a < A; ++a)
            if (v[a]) dalpha += da[a];
        // combine the segments of each active node in segment order
        if (nseg > 1) {
            __syncthreads();
            double *mine = st.part[threadIdx.x];
#pragma unroll
            for (int a = 0; a < A; ++a) { mine[3 * a] = acc[a][0]; mine[3 * a + 1] = acc[a][1]; mine[3 * a + 2] = acc[a][2]; }
            __syncthreads();
            if (seg == 0)
                for (int q = 1; q < nseg; ++q) {
                    const double *o = st.part[q * SLOTS + slot];
#pragma unroll
                    for (int a = 0; a < A; ++a) { acc[a][0] += o[3 * a]; acc[a][1] += o[3 * a + 1]; acc[a][2] += o[3 * a + 2]; }
                }
        }
        if (seg == 0)
#pragma unroll
            for (int a = 0; a < A; ++a)
                if (v[a]) {
                    gh[j[a]] = (float)((double)gh[j[a]] + acc[a][0]);
                    gh[n_max + j[a]] = (float)((double)gh[n_max + j[a]] + acc[a][1]);
                    gh[2 * n_max + j[a]] = (float)((double)gh[2 * n_max + j[a]] + acc[a][2]);
                }
    }
    __syncthreads();
    return dalpha;
}

// Grid shape for m x np pairs: the (slots, nodes per thread) pair with the
// fewest thread iterations; a nodes per thread cost less than a times one
// (shared LDS reads, independent chains to hide latency).  Returns 0..8
// for (64|128|256) x (1|2|4).
__device__ __forceinline__ int decay_grid_shape(int m, int np) {
    int best = 5;
    float bc = 3.0e38f;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        const int slots = 64 << (c % 3), a = 1 << (c / 3), nseg = kWG / slots;
        const float w = a == 1 ? 1.0f : (a == 2 ? 1.75f : 3.3f);
        const float cost = (float)((m + a * slots - 1) / (a * slots)) * (float)((np + nseg - 1) / nseg) * w;
        if (cost < bc) { bc = cost; best = c; }
    }
    return best;
}

__device__ double decay_adjoint(const BwdParams &p, DecayStage &S, int e, int k, int base, int m, int np,
                                const int *alist, const int *plist, const float *uhn, float *gh) {
    switch (uniform(decay_grid_shape(m, np))) {
        case 0: return decay_adjoint_grid<64, 1>(p, S, e, k, base, m, np, alist, plist, uhn, gh);
        case 1: return decay_adjoint_grid<128, 1>(p, S, e, k, base, m, np, alist, plist, uhn, gh);
        case 2: return decay_adjoint_grid<256, 1>(p, S, e, k, base, m, np, alist, plist, uhn, gh);
        case 3: return decay_adjoint_grid<64, 2>(p, S, e, k, base, m, np, alist, plist, uhn, gh);
        case 4: return decay_adjoint_grid<128, 2>(p, S, e, k, base, m, np, alist, plist, uhn, gh);
        case 5: return decay_adjoint_grid<256, 2>(p, S, e, k, base, m, np, alist, plist, uhn, gh);
        case 6: return decay_adjoint_grid<64, 4>(p, S, e, k, base, m, np, alist, plist, uhn, gh);
        case 7: return decay_adjoint_grid<128, 4>(p, S, e, k, base, m, np, alist, plist, uhn, gh);
        default: return decay_adjoint_grid<256, 4>(p, S, e, k, base, m, np, alist, plist, uhn, gh);
    }
}

// Deterministic workgroup sum of 12 doubles per thread (butterfly within the
// wave, then the waves in order); the result is returned in every thread.
// Blocks that only part of the workgroup executes are whole waves and every
// lane stores the same value, so no single-lane region sits next to a
// barrier (the compiler may otherwise thread the rest of a wave past it).
__device__ void wg_sum12(double (&dred)[kWaves][12], double v[12]) {
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        double x = v[c];
        for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
        v[c] = x;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 12; ++c) dred[wave][c] = v[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        double s = dred[0][c];
        for (int w = 1; w < kWaves; ++w) s += dred[w][c];
        v[c] = s;
    }
    __syncthreads();
}

// Pose partials of one item: for every object, the sum over its active
// nodes.  Objects that win no active node of the item get exact zeros
// without a reduction (usually one object reaches a patch).  known: the
// caller's mask of the objects present among the active nodes (bit o for
// object o), or 0 to find it here.
__device__ void contact_adjoint_item(const BwdParams &p, BwdLds &S, int e, int item, int base, int m,
                                     const int *alist, const int8_t *wobj, const float *gh, unsigned known) {
    const MeshDev &M = p.mesh;
    const int N = M.N, n_max = p.scr.n_max, O = p.scene.O;
    // the item's scene row: its env, or the item itself for a row per item
    const size_t row = p.scene.rows_per_env ? (size_t)item : (size_t)e;
    const int no = min(p.scene.n_obj[row], O);
    float *out = p.bwd.pose_part + (size_t)item * O * 12;
    // objects present among the active nodes (an OR, independent of order)
    unsigned present = known;
    if (present == 0) {
        unsigned mask = 0;
        for (int q = threadIdx.x; q < m; q += kWG) mask |= 1u << wobj[alist[q]];
        mask = wave_or(mask);
        S.ired[threadIdx.x >> 6][lane_id()] = (int)mask;     // identical in every lane of the wave
        __syncthreads();
        for (int w = 0; w < kWaves; ++w) present |= (unsigned)S.ired[w][0];
        present = uniform(present);
        __syncthreads();
    }
    for (int o = 0; o < O; ++o) {
        if (!((present >> o) & 1u) || o >= no) {
            if (threadIdx.x < 64 && lane_id() < 12) out[o * 12 + lane_id()] = 0.0f;
            continue;
        }
        double acc[12];
        for (int c = 0; c < 12; ++c) acc[c] = 0.0;
        const size_t eo = row * O + o;
        const int ty = p.scene.type[eo];
        const float *sh = p.scene.shape + 4 * eo, *R = p.scene.rot + 9 * eo, *t = p.scene.trans + 3 * eo;
        // list positions q and q + kWG per pass: both nodes' loads are issued
        // before either is used (the same nodes, in the same order, as one
        // position per pass)
        for (int q = threadIdx.x; q < m; q += 2 * kWG) {
            const bool two = q + kWG < m;
            const int j0 = alist[q];
            const int j1 = two ? alist[q + kWG] : j0;
            const bool h0 = wobj[j0] == o, h1 = two && wobj[j1] == o;
            const int gj0 = base + j0, gj1 = base + j1;
            const float g0[3] = {gh[j0], gh[n_max + j0], gh[2 * n_max + j0]};
            const float g1[3] = {gh[j1], gh[n_max + j1], gh[2 * n_max + j1]};
            const float x0[3] = {M.pos[gj0], M.pos[N + gj0], M.pos[2 * N + gj0]};
            const float x1[3] = {M.pos[gj1], M.pos[N + gj1], M.pos[2 * N + gj1]};
            if (h0) {
                const double g[3] = {g0[0], g0[1], g0[2]};
                contact_adjoint_node(ty, sh, R, t, x0[0], x0[1], x0[2], g, acc);
            }
            if (h1) {
                const double g[3] = {g1[0], g1[1], g1[2]};
                contact_adjoint_node(ty, sh, R, t, x1[0], x1[1], x1[2], g, acc);
            }
        }
        wg_sum12(S.dred, acc);
        if (threadIdx.x < 12) out[o * 12 + threadIdx.x] = (float)acc[threadIdx.x];
        __syncthreads();
    }
}

// Sum accumulator chunk C over the four waves (in wave order), unscale it
// (blocks 0-3 of the chunk by mul_lo, 4-7 by mul_hi) and store it into the
// item's parameter-gradient partial.
// Record blocks 8 C .. 8 C + 7 of the item: every wave puts its eight
// accumulator blocks in LDS (one 16-byte store per lane and block), then each
// thread sums two (block, lane) entries over the waves in wave order and
// stores them with one 16-byte store each.  Every register is named
// statically, so the accumulators never leave registers.  Chunk 4 (dW1,
// dW5) is summed straight from the waves' LDS accumulators, which are
// complete and published by the barrier after the routing pass.
template <int C>
__device__ __forceinline__ void store_record_chunk(BwdLds &S, const WGrad &G, float *rec, float mul_lo,
                                                   float mul_hi) {
    if constexpr (C < 4) {
        const int wave = threadIdx.x >> 6, lane = lane_id();
        __syncthreads();    // previous users of the buffer are done
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            floatx4 v;
            if (C == 0) v = G.w4[j >> 2][j & 3];
            else if (C == 1) v = G.w4[2 + (j >> 2)][j & 3];
            else if (C == 2) v = G.w2[j >> 2][j & 3];
            else v = G.w2[2 + (j >> 2)][j & 3];
            S.u.red[wave][j][lane] = v;
        }
        __syncthreads();
    }
    // wave w's entry (block j, lane ln) of this chunk
    auto part = [&](int w, int j, int ln) -> floatx4 {
        return C < 4 ? S.u.red[w][j][ln] : S.acc15[w][j * 64 + ln];
    };
    for (int idx = threadIdx.x; idx < 8 * 64; idx += kWG) {
        const int j = idx >> 6, ln = idx & 63;
        floatx4 v = part(0, j, ln);
#pragma unroll
        for (int w = 1; w < kWaves; ++w) {
            const floatx4 x = part(w, j, ln);
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] += x[r];
        }
        if (C == 4 && j >= 4) {
            // dW5: FP32 partials of the four lane groups, summed into the
            // MFMA output layout of the record (output c at lane (l & 15),
            // register c of lane group 0)
            if (ln < 16) {
#pragma unroll
                for (int q = 1; q < 4; ++q)
#pragma unroll
                    for (int w = 0; w < kWaves; ++w) {
                        const floatx4 x = part(w, j, ln + 16 * q);
#pragma unroll
                        for (int r = 0; r < 4; ++r) v[r] += x[r];
                    }
            } else {
                v = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
            }
        }
        const float mul = j < 4 ? mul_lo : mul_hi;
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] *= mul;
        // the record streams to HBM for the reduction kernels: non-temporal
        __builtin_nontemporal_store(v, reinterpret_cast<floatx4 *>(&rec[(8 * C + j) * 256 + 4 * ln]));
    }
}

// Max-pool of the item's encoder features with, per channel, the arg-max
// node (lowest index on ties) recomputed over every node: L.g (unscaled),
// S.argmax.
__device__ void pool_argmax(const BwdParams &p, BwdLds &S, int k, int base, int n, const float *uhn) {
    NetLds &L = S.net;
    const MeshDev &M = p.mesh;
    const int n_max = p.scr.n_max;
    const int lane = lane_id(), wave = threadIdx.x >> 6, gq = lane >> 4;
    floatx4 mx[4];
    int mi[4][4];
    #pragma unroll
    for (int ot = 0; ot < 4; ++ot)
        #pragma unroll
        for (int r = 0; r < 4; ++r) { mx[ot][r] = -1.0f; mi[ot][r] = 0x7fffffff; }
    for (int c0 = 0; c0 < n; c0 += kStage) {
        const int cnt = min(kStage, n - c0);
        __syncthreads();
        const float xmul = uniform(L.isc.xmul);
        stage_nodes(M, k, base, nullptr, c0, cnt, uhn, n_max, 0, xmul, xmul, S.u.xs);
        __syncthreads();
        // two tiles per wave step (t and t + kWaves); the second may be padding
        const int ntl = (cnt + 15) >> 4;
        for (int t = wave; t < ntl; t += 2 * kWaves) {
            int lj[2];
            bool valid[2];
            half8 xh[2], xl[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                lj[u] = (t + u * kWaves) * 16 + (lane & 15);
                valid[u] = lj[u] < cnt;
                stage_x<false>(S.u.xs, valid[u] ? lj[u] : 0, valid[u], xh[u], xl[u]);
            }
            floatx4 f[2][4];
            encoder_tile2(L, xh, xl, f);
            // tile order keeps the lowest node on ties (tile t's nodes precede tile t + kWaves's)
#pragma unroll
            for (int u = 0; u < 2; ++u)
                if (valid[u])
                    #pragma unroll
                    for (int ot = 0; ot < 4; ++ot)
                        #pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (f[u][ot][r] > mx[ot][r]) { mx[ot][r] = f[u][ot][r]; mi[ot][r] = c0 + lj[u]; }
        }
    }
    #pragma unroll
    for (int ot = 0; ot < 4; ++ot)
        #pragma unroll
        for (int r = 0; r < 4; ++r) {
            float v = mx[ot][r];
            int ix = mi[ot][r];
            #pragma unroll
            for (int off = 1; off <= 8; off <<= 1) {
                const float v2 = __shfl_xor(v, off);
                const int i2 = __shfl_xor(ix, off);
                if (v2 > v || (v2 == v && i2 < ix)) { v = v2; ix = i2; }
            }
            mx[ot][r] = v;
            mi[ot][r] = ix;
        }
    // all 16 lanes of a row hold the reduced values: identical stores
        #pragma unroll
        for (int ot = 0; ot < 4; ++ot)
            #pragma unroll
            for (int r = 0; r < 4; ++r) {
                S.vred[wave][ot * 16 + 4 * gq + r] = mx[ot][r];
                S.ired[wave][ot * 16 + 4 * gq + r] = mi[ot][r];
            }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int c = threadIdx.x;
        float v = S.vred[0][c];
        int ix = S.ired[0][c];
        for (int w = 1; w < kWaves; ++w) {
            const float v2 = S.vred[w][c];
            const int i2 = S.ired[w][c];
            if (v2 > v || (v2 == v && i2 < ix)) { v = v2; ix = i2; }
        }
        L.g[c] = v * pow2(-L.isc.af);   // unscaled
        S.argmax[c] = ix;
    }
    __syncthreads();
}

// Residual-network adjoint of one item; writes its parameter-gradient
// partial and adds dL/du_hat of active arg-max nodes into gh.  umax: the
// largest |u_hat| component of the item's nodes; with the largest |dL/dU|
// component of its passive nodes (k_bwd_decay's gmax_st) it sets the range
// scales.
__device__ void residual_adjoint(const BwdParams &p, BwdLds &S, int e, int k, int item, int base, int n, int np,
                                 const int *plist, const float *uhn, const int8_t *wobj, float *gh, float umax) {
    NetLds &L = S.net;
    const MeshDev &M = p.mesh;
    // Opaque per item: keeps the compiler from hoisting the per-lane row
    // addresses of the W4 / W3 loads below out of the item loop, where they
    // would hold 64-bit addresses in ~60 registers (and spill) for the whole
    // kernel instead of being formed where they are used.
    const float *phi = p.model.phi;
    asm volatile("" : "+s"(phi));
    const int N = M.N, n_max = p.scr.n_max;
    const size_t EN = (size_t)p.E * N;
    const size_t row = (size_t)e * N + base;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    float *rec = p.bwd.phi_part + (size_t)item * kRecWords;
    item_biases(L, item_scale(L, item_xbound(M, k, umax)));   // published by the next barrier

    // (a) max-pool with arg-max (lowest node on ties): from the forward's
    //     record, else an encoder pass over every node of the item
    GmlpW gw;
    if (p.saved) {
        gw = load_gmlp(phi);   // issued before the record's loads, used after the barrier
        if (threadIdx.x < 64) {
            const uint32_t *rec = p.saved + (size_t)item * kSavedWords;
            L.g[threadIdx.x] = __uint_as_float(rec[threadIdx.x]);
            // a node outside the patch (a record not written for this item)
            // becomes "no node": wrong gradients, never an access outside it
            const int a = (int)rec[64 + threadIdx.x];
            S.argmax[threadIdx.x] = (a >= 0 && a < n) ? a : n;
        }
        __syncthreads();
    } else {
        pool_argmax(p, S, k, base, n, uhn);
        gw = load_gmlp(phi);
    }
    global_mlp(L, gw, item_scale_lds(L));
    // gradient scales: dL/dU staged at 2^dre, dre from gmax (see BwdScale)
    if (threadIdx.x < 64) {   // wave 0, identical values; published by the stage barrier
        BwdScale bs;
        bs.fone = L.isc.xmul;
        bs.dre = range_exp(p.bwd.gmax_st[item]);
        bs.d4 = bs.dre + L.c5t;
        bs.d2 = bs.d4 + L.s4t;
        bs.d1 = bs.d2 + L.s2t;
        S.bsc = bs;
    }

    // (b) decoder and encoder adjoints over the passive nodes, tile t on wave t % 4
    WGrad G;
    zero_wgrad(G);
    for (int j = 0; j < 8; ++j) S.acc15[wave][j * 64 + lane] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int c0 = 0; c0 < np; c0 += kStage) {
        const int cnt = min(kStage, np - c0);
        __syncthreads();
        stage_nodes(M, k, base, plist, c0, cnt, p.grad_u, EN, row, uniform(L.isc.xmul),
                    pow2(uniform(S.bsc.dre)), S.u.xs);
        __syncthreads();
        // pairs of tiles (t, t + 4) per wave while every wave gets a pair,
        // then single tiles
        const int ptl = (cnt + 15) >> 4;
        int t0 = 0;
        for (; ptl - t0 >= 2 * kWaves; t0 += 2 * kWaves) {
            const int tt[2] = {t0 + wave, t0 + kWaves + wave};
            passive_tiles<2>(S, G, cnt, tt);
        }
        for (int t = t0 + wave; t < ptl; t += kWaves) {
            const int tt[1] = {t};
            passive_tiles<1>(S, G, cnt, tt);
        }
    }

    // (c) db4 = s4 = sum_i dpre4_i; global MLP adjoint: dg' = W4[:, 64:]^T s4,
    //     dpre3 = dg' [g' > 0], dg = W3^T dpre3.  The wave's 16 rows of
    //     W4[:, 64:] and of W3, and the routing pass's node inputs, are
    //     loaded ahead of the reductions they feed, so their latency overlaps
    //     the barriers.
    RouteIn rin;
    route_inputs(p, S, k, base, n, uhn, uniform(L.isc.xmul), rin);
    float w4g[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) w4g[q] = phi[kW4 + (16 * wave + q) * 128 + 64 + lane];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        float v = G.b4[ob];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        S.vred[wave][ob * 16 + (lane & 15)] = v;     // identical in the 4 lane groups
    }
    __syncthreads();
    {
        // Each wave sums 16 of the 64 terms of a product, the partials are
        // added in wave order.  A wave forms the sums its own next product
        // needs (its 16 rows; all 64 for the routing pass) from the four
        // partials itself, so only the partials cross waves: one barrier per
        // product, with two partial buffers in turn.
        const int c = lane, o = 16 * wave + (lane & 15);   // o: identical in the 4 lane groups
        {
            float t = S.vred[0][o];
            for (int w = 1; w < kWaves; ++w) t += S.vred[w][o];
            S.s4[o] = t * pow2(-S.bsc.d4);     // unscaled from here on
        }
        wave_sync();
        float s = 0.0f;
#pragma unroll
        for (int q = 0; q < 16; ++q) s += w4g[q] * S.s4[16 * wave + q];
        S.vred2[wave][c] = s;
        float w3r[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) w3r[q] = phi[kW3 + (16 * wave + q) * 64 + c];
        __syncthreads();
        {
            float t = S.vred2[0][o];
            for (int w = 1; w < kWaves; ++w) t += S.vred2[w][o];
            S.dgp[o] = t;
            S.dpre3[o] = L.gp[o] > 0.0f ? t : 0.0f;
        }
        wave_sync();
        s = 0.0f;
#pragma unroll
        for (int q = 0; q < 16; ++q) s += w3r[q] * S.dpre3[16 * wave + q];
        S.vred[wave][c] = s;     // every wave read vred before the barrier above
        __syncthreads();
        {
            float t = S.vred[0][c];
            for (int w = 1; w < kWaves; ++w) t += S.vred[w][c];
            // f = relu(pre2) >= 0 and f at the arg-max node is g, so its gate is g > 0
            const float vr = L.g[c] > 0.0f ? t : 0.0f;
            S.vrw[wave][c] = vr;
            if (wave == 0) {
                S.dg[c] = t;
                S.vroute[c] = vr;
            }
        }
        wave_sync();
    }

    // (d) max-pool routing: wave w takes channels 16 w .. 16 w + 15
    routing_tile(p, S, G, n, rin);
    __syncthreads();
    // Routed dL/du_hat of active arg-max nodes: channel c owns its node if c
    // is the lowest channel routed there; the owner adds the node's channels
    // (c and the higher ones routed there) to gh once.  Wave w scans channels
    // 16 w .. 16 w + 15 for every c (lane c); wave 0 adds the four partial
    // sums in wave order.  The per-wave transpose buffers are free here.
    {
        const int c = lane;
        const int ln = S.argmax[c];
        const float x0 = S.dxs[c][0], x1 = S.dxs[c][1], x2 = S.dxs[c][2];
        bool lower = false;
        float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
        const int cb = uniform(16 * wave);
#pragma unroll 4
        for (int c2 = cb; c2 < cb + 16; ++c2) {   // channel c2's node and values, read from its lane
            const int l2 = __builtin_amdgcn_readlane(ln, c2);
            const float y0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x0), c2));
            const float y1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x1), c2));
            const float y2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x2), c2));
            const bool same = l2 == ln;
            lower = lower || (same && c2 < c);
            if (same && c2 >= c) { s0 += y0; s1 += y1; s2 += y2; }
        }
        *reinterpret_cast<floatx4 *>(reinterpret_cast<float *>(&S.tr[wave][0]) + 4 * c) =
            floatx4{s0, s1, s2, lower ? 1.0f : 0.0f};
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int c = threadIdx.x;
        const int ln = S.argmax[c];
        bool owner = ln < n;
        float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
        for (int w = 0; w < kWaves; ++w) {
            const floatx4 q = *reinterpret_cast<const floatx4 *>(reinterpret_cast<const float *>(&S.tr[w][0]) + 4 * c);
            s0 += q[0]; s1 += q[1]; s2 += q[2];
            owner = owner && q[3] == 0.0f;
        }
        if (owner && wobj[ln] >= 0) {
            gh[ln] += s0;
            gh[n_max + ln] += s1;
            gh[2 * n_max + ln] += s2;
        }
    }

    // (e) the item's record of the parameter gradients: the four waves'
    //     accumulators summed in wave order, eight blocks per pass
    const ItemScale isc = item_scale_lds(L);
    const int dre = uniform(S.bsc.dre), d4 = uniform(S.bsc.d4), d2 = uniform(S.bsc.d2), d1 = uniform(S.bsc.d1);
    const float m4 = pow2(-(d4 + isc.af)), m2 = pow2(-(d2 + isc.a1));
    store_record_chunk<0>(S, G, rec, m4, m4);
    store_record_chunk<1>(S, G, rec, m4, m4);
    store_record_chunk<2>(S, G, rec, m2, m2);
    store_record_chunk<3>(S, G, rec, m2, m2);
    store_record_chunk<4>(S, G, rec, pow2(-(d1 + isc.ax)), pow2(-(dre + isc.a4)));
    // db2 (passive sums plus the routed one-hots) and db5
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
        float v = G.b2[ob];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        S.vred[wave][ob * 16 + (lane & 15)] = v;
    }
    {
        float v = G.b5;
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        S.ired[wave][lane & 15] = __float_as_int(v);      // lanes (l & 15) < 3 carry db5
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int c = threadIdx.x;
        float t = S.vred[0][c];
        for (int w = 1; w < kWaves; ++w) t += S.vred[w][c];
        rec[kRecB2 + c] = t * pow2(-d2) + S.vroute[c];
        rec[kRecB4 + c] = S.s4[c];
        rec[kRecB3 + c] = S.dpre3[c];
        rec[kRecGp + c] = L.gp[c];     // dW4[:, 64:] = s4 (x) g'
        rec[kRecG + c] = L.g[c];       // dW3 = dpre3 (x) g
        if (c < 4) {
            float b = 0.0f;
            if (c < 3) {
                b = __int_as_float(S.ired[0][c]);
                for (int w = 1; w < kWaves; ++w) b += __int_as_float(S.ired[w][c]);
            }
            rec[kRecB5 + c] = b * pow2(-dre);
        }
    }
    __syncthreads();
}

// Zero partials of the batch's items that no object can reach (wave w takes
// items w, w + 4, ...; no barrier needed).
__device__ void zero_fill_batch_bwd(const BwdParams &p, const ItemBatch &B, int b0) {
    const MeshDev &M = p.mesh;
    const int wave = threadIdx.x >> 6, lane = lane_id(), O = p.scene.O;
    const unsigned long long live = batch_mask(B);
    for (int j = wave; j < p.batch; j += kWaves) {
        const int q = b0 + j;
        if (q >= p.n_items || ((live >> j) & 1ull)) continue;
        int e, k;
        queue_item(M, p.E, q, e, k);
        const size_t item = (size_t)e * M.K + k;
        for (int c = lane; c < O * 12; c += 64) p.bwd.pose_part[item * O * 12 + c] = 0.0f;
        p.bwd.alpha_part[item] = 0.0f;
        p.bwd.item_flag[item] = 0;
        p.bwd.m_st[item] = 0;
    }
}

// ---------------------------------------------------------------------------
// k_bwd_decay: contact and the Eq. 1 adjoint of every item
//
// Runs before k_bwd with a small LDS footprint, so several workgroups share
// a CU.  For every item it recomputes (or reads) contact, writes the active
// count, the alpha partial and, for items without contact, every zero
// partial; for contacted items it hands dL/du_hat (own U plus the decay
// adjoint) and, in the step adjoint, the contact results to k_bwd.
// ---------------------------------------------------------------------------
template <int KIND>
__device__ void decay_item_bwd(const BwdParams &p, DecayLds &S, int item, int e, int k, unsigned cand, float *uhn,
                               float *gh, int *alist, int *plist) {
    const MeshDev &M = p.mesh;
    const int N = M.N, n_max = p.scr.n_max, O = p.scene.O;
    const size_t EN = (size_t)p.E * N;
    const int base = M.offset[k];
    const int n = M.offset[k + 1] - base;
    const size_t row = (size_t)e * N + base;
    float umax;
    int touch;
    const int m = contact_and_compact<KIND == BWD_PROP>(M, p.scene, p.E, n_max, p.cobj_in, p.uhat_in,
                                                        KIND == BWD_STEP ? p.bwd.cobj_st : nullptr, S.wcnt, e, k,
                                                        base, n, cand, uhn, alist, plist, nullptr, umax, touch);
    if (threadIdx.x < 64) p.bwd.m_st[item] = m;     // identical stores
    if (m == 0) {
        if (threadIdx.x < 64) {
            p.bwd.alpha_part[item] = 0.0f;
            p.bwd.item_flag[item] = 0;
        }
        if (KIND == BWD_STEP)
            for (int c = threadIdx.x; c < O * 12; c += kWG) p.bwd.pose_part[(size_t)item * O * 12 + c] = 0.0f;
        if (KIND == BWD_PROP)
            for (int i = threadIdx.x; i < n; i += kWG) {
                p.grad_uhat_out[row + i] = 0.0f;
                p.grad_uhat_out[EN + row + i] = 0.0f;
                p.grad_uhat_out[2 * EN + row + i] = 0.0f;
            }
        __syncthreads();
        return;
    }
    // dL/du_hat of active nodes starts from their own U
    for (int q = threadIdx.x; q < m; q += kWG) {
        const int j = alist[q];
        gh[j] = p.grad_u[row + j];
        gh[n_max + j] = p.grad_u[EN + row + j];
        gh[2 * n_max + j] = p.grad_u[2 * EN + row + j];
    }
    __syncthreads();
    double dalpha = 0.0;
    const int np = n - m;
    if (p.model.mode != ETAC_RESIDUAL_ONLY && np > 0)
        dalpha = decay_adjoint(p, S.st, e, k, base, m, np, alist, plist, uhn, gh);
    {
        double v[12];
        v[0] = dalpha;
        for (int c = 1; c < 12; ++c) v[c] = 0.0;
        wg_sum12(S.dred, v);
        if (threadIdx.x < 64) p.bwd.alpha_part[item] = (float)v[0];
    }
    // the largest |dL/dU| component over the passive nodes: the scale of the
    // network adjoint's gradient operands in k_bwd (these values were just
    // read by the decay adjoint, so they come from the cache)
    if (uses_residual(p)) {
        int gbits = 0;   // bits of a non-negative float: integer order is float order
        for (int t = threadIdx.x; t < np; t += kWG) {
            const int i = plist[t];
            const float g0 = p.grad_u[row + i], g1 = p.grad_u[EN + row + i], g2 = p.grad_u[2 * EN + row + i];
            gbits = max(gbits, __float_as_int(fmaxf(fmaxf(fabsf(g0), fabsf(g1)), fabsf(g2))));
        }
        S.gmx[threadIdx.x >> 6] = wave_max_int(gbits);   // identical in every lane of the wave
        __syncthreads();
        if (threadIdx.x < 64) {
            int g = 0;
            for (int w = 0; w < kWaves; ++w) g = max(g, S.gmx[w]);
            p.bwd.gmax_st[item] = __int_as_float(g);
        }
    }
    // hand-over of the active nodes to k_bwd
    for (int q = threadIdx.x; q < m; q += kWG) {
        const int j = alist[q];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            p.bwd.gh_st[c * EN + row + j] = gh[c * n_max + j];
            if (KIND == BWD_STEP) p.bwd.uhat_st[c * EN + row + j] = uhn[c * n_max + j];
        }
    }
    __syncthreads();
}

template <int KIND>
__global__ __launch_bounds__(kWG) void k_bwd_decay(BwdParams p) {
    __shared__ DecayLds S;
    const int wg = blockIdx.x;
    const int n_max = p.scr.n_max;
    float *uhn = p.scr.uhat_node + (size_t)wg * 3 * n_max;
    float *gh = p.bwd.guhat + (size_t)wg * 3 * n_max;
    int *alist = p.scr.alist + (size_t)wg * n_max;
    int *plist = p.scr.plist + (size_t)wg * n_max;
    for (;;) {
        const int b0 = next_batch<KIND == BWD_PROP ? CULL_NONE : CULL_OBJECTS>(p.scr.counter + 2, S.batch, p.mesh,
                                                                              p.scene, p.E, p.n_items, p.batch);
        if (b0 >= p.n_items) break;
        if (KIND != BWD_PROP) zero_fill_batch_bwd(p, S.batch, b0);
        const int nb = uniform(S.batch.n);
        for (int q = 0; q < nb; ++q) {
            const int pos = uniform(S.batch.item[q]);
            int e, k;
            queue_item(p.mesh, p.E, pos, e, k);
            const unsigned cand = KIND == BWD_PROP
                                      ? 0xffffffffu
                                      : item_cand(p.scene, e, k, uniform((unsigned)S.batch.cand[q]));
            decay_item_bwd<KIND>(p, S, e * p.mesh.K + k, e, k, cand, uhn, gh, alist, plist);
        }
    }
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned done = atomicAdd(&p.scr.counter[3], 1u);
        if (done == gridDim.x - 1) {
            atomicExch(&p.scr.counter[2], 0u);
            atomicExch(&p.scr.counter[3], 0u);
        }
    }
}

// ---------------------------------------------------------------------------
// list of the items with contact, in queue order, for k_bwd's work queue
//
// k_live_count counts them per segment of 1024 queue positions; k_live_list
// writes each segment's positions after the counts of the segments before it
// (wave ballots, waves in order) and the last segment writes the total.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool item_live(const BwdParams &p, int q) {
    int e, k;
    queue_item(p.mesh, p.E, q, e, k);
    return p.bwd.m_st[(size_t)e * p.mesh.K + k] > 0;
}

#ifndef ETAC_BWD_NET_ONLY
__global__ __launch_bounds__(256) void k_live_count(BwdParams p) {
    __shared__ int wsum[kWaves];
    const int s = blockIdx.x, wave = threadIdx.x >> 6;
    int cnt = 0;
    for (int j = 0; j < 4; ++j) {
        const int q = s * 1024 + j * 256 + threadIdx.x;
        cnt += (q < p.n_items && item_live(p, q)) ? 1 : 0;
    }
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off);
    wsum[wave] = cnt;   // identical in every lane
    __syncthreads();
    if (threadIdx.x < 64) p.bwd.seg_cnt[s] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

__global__ __launch_bounds__(256) void k_live_list(BwdParams p) {
    __shared__ int wsum[kWaves];
    const int s = blockIdx.x, wave = threadIdx.x >> 6;
    int run = 0;   // identical in every thread
    for (int t = 0; t < s; ++t) run += p.bwd.seg_cnt[t];
    for (int j = 0; j < 4; ++j) {
        const int q = s * 1024 + j * 256 + threadIdx.x;
        const bool f = q < p.n_items && item_live(p, q);
        const unsigned long long bal = __ballot(f);
        __syncthreads();   // the previous round's wsum reads are done
        wsum[wave] = __popcll(bal);
        __syncthreads();
        int off = run, tot = 0;
        for (int w = 0; w < kWaves; ++w) {
            if (w < wave) off += wsum[w];
            tot += wsum[w];
        }
        if (f) p.bwd.live[off + lanes_below(bal)] = q;
        run += uniform(tot);
    }
    if (s == (int)gridDim.x - 1 && threadIdx.x < 64) p.bwd.seg_cnt[gridDim.x] = run;
}

#endif

// ---------------------------------------------------------------------------
// k_bwd: network and contact adjoint
// ---------------------------------------------------------------------------

// The active and passive node lists of one (env, patch) item from given
// contact results (contact_obj and u_hat of a forward or contact pass), as
// contact_and_compact does with FROM_INPUT, but kGivenChunks chunks of kWG
// nodes per pair of barriers: the loads are cheap and their latencies overlap.
// Lists in ascending node order (chunk, then wave, then lane).  Returns m;
// umax: the largest |u_hat| component over the item's nodes; present: the
// objects that win an active node (bit o for object o).  dL/du_hat of the
// active nodes is read from gsrc into gh in the same pass, so its loads
// overlap those of u_hat.
__device__ int compact_given(int E, int N, int n_max, const int8_t *cobj_in, const float *uhat_in,
                             const float *gsrc, int (&wcnt)[kGivenChunks][2][kWaves], int (&wmx)[2][kWaves], int e,
                             int base, int n, float *uhn, float *gh, int *alist, int *plist, int8_t *wobj,
                             float &umax, unsigned &present) {
    constexpr int G = kGivenChunks;
    const size_t EN = (size_t)E * N;
    const int wave = threadIdx.x >> 6;
    int run_a = 0, run_p = 0;
    int ubits = 0;   // bits of a non-negative float: integer order is float order
    unsigned omask = 0;
    for (int g0 = 0; g0 < n; g0 += G * kWG) {
        bool act[G], pas[G];
#pragma unroll
        for (int c = 0; c < G; ++c) {
            const int i = g0 + c * kWG + threadIdx.x;
            const bool valid = i < n;
            int best = -1;
            float u0 = 0.0f, u1 = 0.0f, u2 = 0.0f;
            if (valid) {
                const size_t en = (size_t)e * N + base + i;
                best = cobj_in[en] >= 0 ? (int)cobj_in[en] : -1;
                if (best >= 0) {
                    u0 = uhat_in[en];
                    u1 = uhat_in[EN + en];
                    u2 = uhat_in[2 * EN + en];
                    const float g0v = gsrc[en], g1v = gsrc[EN + en], g2v = gsrc[2 * EN + en];
                    gh[i] = g0v;
                    gh[n_max + i] = g1v;
                    gh[2 * n_max + i] = g2v;
                    ubits = max(ubits, __float_as_int(fmaxf(fmaxf(fabsf(u0), fabsf(u1)), fabsf(u2))));
                    omask |= 1u << (best & 31);
                }
                uhn[i] = u0;
                uhn[n_max + i] = u1;
                uhn[2 * n_max + i] = u2;
                if (wobj) wobj[i] = (int8_t)best;
            }
            act[c] = valid && best >= 0;
            pas[c] = valid && best < 0;
        }
        wmx[0][wave] = wave_max_int(ubits);
        wmx[1][wave] = (int)wave_or(omask);
        unsigned long long ba[G], bp[G];
#pragma unroll
        for (int c = 0; c < G; ++c) {
            ba[c] = __ballot(act[c]);
            bp[c] = __ballot(pas[c]);
            // every lane stores the same wave counts (no single-lane block next to the barrier)
            wcnt[c][0][wave] = __popcll(ba[c]);
            wcnt[c][1][wave] = __popcll(bp[c]);
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < G; ++c) {
            const int i = g0 + c * kWG + threadIdx.x;
            int oa = run_a, op = run_p, ta = 0, tp = 0;
            for (int w = 0; w < kWaves; ++w) {
                if (w < wave) { oa += wcnt[c][0][w]; op += wcnt[c][1][w]; }
                ta += wcnt[c][0][w];
                tp += wcnt[c][1][w];
            }
            if (act[c]) alist[oa + lanes_below(ba[c])] = i;
            if (pas[c]) plist[op + lanes_below(bp[c])] = i;
            run_a += uniform(ta);
            run_p += uniform(tp);
        }
        if (g0 + G * kWG >= n) {   // last pass: the wave maxima cover every node of the item
            int ub = 0;
            unsigned ob = 0;
            for (int w = 0; w < kWaves; ++w) {
                ub = max(ub, wmx[0][w]);
                ob |= (unsigned)wmx[1][w];
            }
            umax = __int_as_float(uniform(ub));
            present = uniform(ob);
        }
        __syncthreads();
    }
    return uniform(run_a);
}

// One item (item = e K + k indexes the partials).  Step / propagate adjoint:
// only items with active nodes reach here; contact comes from the hand-over
// (step) or the caller (propagate), dL/du_hat of active nodes from the decay
// kernel.  Contact adjoint: contact is recomputed (cand: candidate objects)
// and dL/du_hat is the caller's.
template <int KIND>
__device__ void process_item_bwd(const BwdParams &p, BwdLds &S, int item, int e, int k, unsigned cand, float *uhn,
                                 float *gh, int *alist, int *plist, int8_t *wobj) {
    const MeshDev &M = p.mesh;
    const int N = M.N, n_max = p.scr.n_max, O = p.scene.O;
    const size_t EN = (size_t)p.E * N;
    const int base = M.offset[k];
    const int n = M.offset[k + 1] - base;
    const size_t row = (size_t)e * N + base;
    const int8_t *cin = KIND == BWD_STEP ? p.bwd.cobj_st : p.cobj_in;
    const float *uin = KIND == BWD_STEP ? p.bwd.uhat_st : p.uhat_in;
    int m;
    float umax = 0.0f;
    int touch;
    unsigned present = 0;   // found by contact_adjoint_item for the contact adjoint
    if constexpr (KIND == BWD_CONTACT)
        m = contact_and_compact<false>(M, p.scene, p.E, n_max, nullptr, nullptr, nullptr,
                                       *reinterpret_cast<int (*)[3][kWaves]>(&S.wcnt[0][0][0]), e, k, base, n,
                                       cand, uhn, alist, plist, wobj, umax, touch);
    else
        m = compact_given(p.E, N, n_max, cin, uin, p.bwd.gh_st, S.wcnt, S.wmx, e, base, n, uhn, gh, alist, plist,
                          wobj, umax, present);
    if (m == 0) {
        // contact adjoint only: the other kinds never queue items without contact
        if (threadIdx.x < 64) p.bwd.item_flag[item] = 0;
        for (int c = threadIdx.x; c < O * 12; c += kWG) p.bwd.pose_part[(size_t)item * O * 12 + c] = 0.0f;
        __syncthreads();
        return;
    }
    if constexpr (KIND == BWD_CONTACT) {   // the other kinds read dL/du_hat during compaction
        for (int q = threadIdx.x; q < m; q += kWG) {
            const int j = alist[q];
            gh[j] = p.grad_uhat_in[row + j];
            gh[n_max + j] = p.grad_uhat_in[EN + row + j];
            gh[2 * n_max + j] = p.grad_uhat_in[2 * EN + row + j];
        }
        __syncthreads();
    }
    if (KIND != BWD_CONTACT && uses_residual(p))
        residual_adjoint(p, S, e, k, item, base, n, n - m, plist, uhn, wobj, gh, umax);
    if (threadIdx.x < 64) p.bwd.item_flag[item] = (KIND != BWD_CONTACT && uses_residual(p)) ? 1 : 0;
    __syncthreads();
    if (KIND == BWD_PROP) {
        for (int i = threadIdx.x; i < n; i += kWG) {
            const bool act = wobj[i] >= 0;
            p.grad_uhat_out[row + i] = act ? gh[i] : 0.0f;
            p.grad_uhat_out[EN + row + i] = act ? gh[n_max + i] : 0.0f;
            p.grad_uhat_out[2 * EN + row + i] = act ? gh[2 * n_max + i] : 0.0f;
        }
    } else {
        contact_adjoint_item(p, S, e, item, base, m, alist, wobj, gh, present);
    }
    __syncthreads();
}

template <int KIND>
__global__ __launch_bounds__(kWG) void k_bwd(BwdParams p) {
    __shared__ BwdLds S;
    const int wg = blockIdx.x;
    const int n_max = p.scr.n_max;
    float *uhn = p.scr.uhat_node + (size_t)wg * 3 * n_max;
    float *gh = p.bwd.guhat + (size_t)wg * 3 * n_max;
    int *alist = p.scr.alist + (size_t)wg * n_max;
    int *plist = p.scr.plist + (size_t)wg * n_max;
    int8_t *wobj = reinterpret_cast<int8_t *>(p.scr.resid + (size_t)wg * 3 * n_max);
    if (KIND != BWD_CONTACT && uses_residual(p)) {
        stage_net(S.net, p.model.phi);
        stage_net_t(S, p.model.phi);
        __syncthreads();
    }
    // step / propagate adjoint: positions of the list of items with contact;
    // contact adjoint: every queue position, culled by the objects' reach
    const int n_pos = KIND == BWD_CONTACT ? p.n_items : uniform(p.bwd.seg_cnt[p.n_seg]);
    for (;;) {
        const int b0 = KIND == BWD_CONTACT
                           ? next_batch<CULL_OBJECTS>(p.scr.counter + 2, S.batch, p.mesh, p.scene, p.E, n_pos, p.batch)
                           : next_batch<CULL_LIST>(p.scr.counter + 2, S.batch, p.mesh, p.scene, p.E, n_pos,
                                                   p.net_batch, p.bwd.live);
        if (b0 >= n_pos) break;
        if (KIND == BWD_CONTACT) zero_fill_batch_bwd(p, S.batch, b0);
        const int nb = uniform(S.batch.n);
        for (int q = 0; q < nb; ++q) {
            const int pos = uniform(S.batch.item[q]);
            int e, k;
            queue_item(p.mesh, p.E, pos, e, k);
            const unsigned cand = KIND == BWD_CONTACT
                                      ? item_cand(p.scene, e, k, uniform((unsigned)S.batch.cand[q]))
                                      : 0xffffffffu;
            process_item_bwd<KIND>(p, S, e * p.mesh.K + k, e, k, cand, uhn, gh, alist, plist, wobj);
        }
    }
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned done = atomicAdd(&p.scr.counter[3], 1u);
        if (done == gridDim.x - 1) {
            atomicExch(&p.scr.counter[2], 0u);
            atomicExch(&p.scr.counter[3], 0u);
        }
    }
}

// The network-adjoint kernel is built in a translation unit of its own
// (this file with ETAC_BWD_NET_ONLY), with instruction sinking so that its
// loop-invariant per-lane addresses are formed where used instead of held
// across the item loop: one wave per SIMD leaves no room for them.
#ifdef ETAC_BWD_NET_ONLY
hipError_t launch_bwd_net(const BwdParams &p, int kind, int grid, hipStream_t st) {
    if (kind == BWD_STEP) hipLaunchKernelGGL(k_bwd<BWD_STEP>, dim3(grid), dim3(kWG), 0, st, p);
    else if (kind == BWD_PROP) hipLaunchKernelGGL(k_bwd<BWD_PROP>, dim3(grid), dim3(kWG), 0, st, p);
    else hipLaunchKernelGGL(k_bwd<BWD_CONTACT>, dim3(grid), dim3(kWG), 0, st, p);
    return hipGetLastError();
}
#else
hipError_t launch_bwd_net(const BwdParams &p, int kind, int grid, hipStream_t st);

// ---------------------------------------------------------------------------
// fixed-order reductions of the per-item partials
// ---------------------------------------------------------------------------

// Segment sums of the reduction columns (FP64).  Segment s covers items
// [s R, (s + 1) R), R = ceil(n_items / kPhiSegs), and adds the records of
// the items that wrote one (flag set) in ascending item order.  The block
// compacts its segment's flags into an LDS list 1024 items at a time (wave
// ballots, waves in order), then every thread sums its column over the list
// with eight items in flight.  Plain columns read one record word (record
// order, so a wave reads 256 contiguous bytes); rank-one columns multiply two.
__global__ __launch_bounds__(256) void k_phi_segments(const float *part, const int *flag, int n_items,
                                                      double *seg) {
    __shared__ int list[1024];
    __shared__ int wsum[kWaves];
    const int col = blockIdx.x * 256 + threadIdx.x;
    const int s = blockIdx.y;
    const int wave = threadIdx.x >> 6;
    const int per = (n_items + kPhiSegs - 1) / kPhiSegs;
    const int a = min(n_items, s * per), b = min(n_items, a + per);
    // word(s) of this column (uniform per wave: both regions are 64-aligned);
    // the padding words between kRecWords and kRedPlain add nothing
    const bool rank1 = col >= kRedPlain;
    const int k = col - kRedPlain, w = k >> 12, o = (k >> 6) & 63, i = k & 63;
    const int sa = rank1 ? (w ? kRecB3 + o : kRecB4 + o) : (col < kRecWords ? col : 0);
    const int sb = rank1 ? (w ? kRecG + i : kRecGp + i) : sa;
    const bool live_col = col < kRedCols && (rank1 || col < kRecWords);
    double acc = 0.0;
    for (int c0 = a; c0 < b; c0 += 1024) {
        int cnt = 0;   // identical in every thread
        for (int j = 0; j < 4; ++j) {
            const int it = c0 + j * 256 + threadIdx.x;
            const bool f = it < b && flag[it] != 0;
            const unsigned long long bal = __ballot(f);
            __syncthreads();   // the previous round's wsum reads are done
            wsum[wave] = __popcll(bal);
            __syncthreads();
            int off = cnt, tot = 0;
            for (int v = 0; v < kWaves; ++v) {
                if (v < wave) off += wsum[v];
                tot += wsum[v];
            }
            if (f) list[off + lanes_below(bal)] = it;
            cnt += uniform(tot);
        }
        __syncthreads();
        if (live_col) {
            int q = 0;
            if (rank1) {
                for (; q + 8 <= cnt; q += 8) {
                    double v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const float *r = part + (size_t)list[q + u] * kRecWords;
                        v[u] = (double)r[sa] * (double)r[sb];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) acc += v[u];
                }
                for (; q < cnt; ++q) {
                    const float *r = part + (size_t)list[q] * kRecWords;
                    acc += (double)r[sa] * (double)r[sb];
                }
            } else {
                for (; q + 8 <= cnt; q += 8) {
                    float v[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) v[u] = part[(size_t)list[q + u] * kRecWords + sa];
#pragma unroll
                    for (int u = 0; u < 8; ++u) acc += (double)v[u];
                }
                for (; q < cnt; ++q) acc += (double)part[(size_t)list[q] * kRecWords + sa];
            }
        }
        __syncthreads();   // the list is rewritten by the next chunk
    }
    if (col < kRedCols) seg[(size_t)s * kRedCols + col] = acc;
}

// dL/dphi: each parameter's column of the segment sums added in segment order.
__global__ __launch_bounds__(256) void k_phi_final(const double *seg, const int *map, float *grad_phi) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= kPhiN) return;
    const int col = map[c];
    double acc = 0.0;
    for (int s = 0; s < kPhiSegs; ++s) acc += seg[(size_t)s * kRedCols + col];
    grad_phi[c] = (float)acc;
}

__global__ __launch_bounds__(256) void k_zero(float *x, int n) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) x[i] = 0.0f;
}

// dL/dalpha_k: sum over envs of item (e, k) partials, fixed tree.
__global__ __launch_bounds__(256) void k_alpha(const float *part, int E, int K, float *grad_alpha) {
    __shared__ double red[256];
    const int k = blockIdx.x;
    double acc = 0.0;
    for (int e = threadIdx.x; e < E; e += 256) acc += (double)part[(size_t)e * K + k];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad_alpha[k] = (float)red[0];
}

// Pose gradients: sum over the env's patches in patch order.
__global__ __launch_bounds__(256) void k_pose(const float *part, int E, int K, int O, float *grad_rot,
                                              float *grad_trans) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= E * O * 12) return;
    const int c = t % 12, eo = t / 12, o = eo % O, e = eo / O;
    double acc = 0.0;
    for (int k = 0; k < K; ++k) acc += (double)part[(((size_t)e * K + k) * O + o) * 12 + c];
    if (c < 9) grad_rot[(size_t)eo * 9 + c] = (float)acc;
    else grad_trans[(size_t)eo * 3 + (c - 9)] = (float)acc;
}

hipError_t launch_backward(const Plan &pl, const SceneDev *s, const ModelDev &m, int n_envs, const int8_t *cobj_in,
                           const float *uhat_in, const float *grad_u, const uint32_t *saved, float *grad_uhat,
                           float *grad_rot, float *grad_trans, float *grad_alpha, float *grad_phi,
                           hipStream_t st, const SceneDev *world, const LinksDev *links, float *grad_link_rot,
                           float *grad_link_trans) {
    if (n_envs == 0) {
        // sums over no env: zero parameter gradients
        if (grad_alpha) hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, st, grad_alpha, pl.K);
        if (grad_phi) hipLaunchKernelGGL(k_zero, dim3((kPhiN + 255) / 256), dim3(256), 0, st, grad_phi, kPhiN);
        return hipGetLastError();
    }
    BwdParams p;
    p.mesh = pl.mesh;
    p.scene = s ? *s : SceneDev{nullptr, nullptr, nullptr, nullptr, nullptr, 0, 1};
    p.model = m;
    p.scr = pl.scr;
    p.bwd = pl.bwd;
    // the hand's rows hold up to cap candidates: their own pose partials
    if (links) p.bwd.pose_part = pl.hand->pose_part;
    p.E = n_envs;
    p.n_items = n_envs * pl.K;
    p.batch = pl.bwd_batch;
    p.cobj_in = cobj_in;
    p.uhat_in = uhat_in;
    p.grad_u = grad_u;
    p.grad_uhat_in = nullptr;
    p.grad_uhat_out = grad_uhat;
    p.saved = saved;
    p.net_batch = pl.net_batch;
    p.n_seg = (p.n_items + 1023) / 1024;
    // contact and the decay adjoint, several workgroups per CU
    const int grid_d = min(p.n_items, pl.cu_count * pl.decay_wg_per_cu);
    int slot = timer_begin(pl, ETAC_TIMER_BWD_DECAY, st);
    if (s) hipLaunchKernelGGL(k_bwd_decay<BWD_STEP>, dim3(grid_d), dim3(kWG), 0, st, p);
    else hipLaunchKernelGGL(k_bwd_decay<BWD_PROP>, dim3(grid_d), dim3(kWG), 0, st, p);
    hipError_t e = hipGetLastError();
    timer_end(pl, ETAC_TIMER_BWD_DECAY, slot, st);
    if (e != hipSuccess) return e;
    // the items with contact, in queue order
    hipLaunchKernelGGL(k_live_count, dim3(p.n_seg), dim3(256), 0, st, p);
    hipLaunchKernelGGL(k_live_list, dim3(p.n_seg), dim3(256), 0, st, p);
    // network and contact adjoint of the contacted items, one workgroup per CU
    const int grid = min(p.n_items, pl.cu_count);
    slot = timer_begin(pl, ETAC_TIMER_BACKWARD, st);
    e = launch_bwd_net(p, s ? BWD_STEP : BWD_PROP, grid, st);
    timer_end(pl, ETAC_TIMER_BACKWARD, slot, st);
    if (e != hipSuccess) return e;
    slot = timer_begin(pl, ETAC_TIMER_REDUCE, st);
    if (grad_phi) {
        hipLaunchKernelGGL(k_phi_segments, dim3((kRedCols + 255) / 256, kPhiSegs), dim3(256), 0, st, pl.bwd.phi_part,
                           pl.bwd.item_flag, p.n_items, pl.bwd.phi_seg);
        hipLaunchKernelGGL(k_phi_final, dim3((kPhiN + 255) / 256), dim3(256), 0, st, pl.bwd.phi_seg,
                           pl.bwd.rec_map, grad_phi);
    }
    if (grad_alpha) hipLaunchKernelGGL(k_alpha, dim3(pl.K), dim3(256), 0, st, pl.bwd.alpha_part, n_envs, pl.K, grad_alpha);
    e = hipSuccess;
    if (s && links) {
        e = launch_pose_hand(pl, *world, *links, grad_rot, grad_trans, grad_link_rot, grad_link_trans, st);
    } else if (s) {
        const int nt = n_envs * s->O * 12;
        hipLaunchKernelGGL(k_pose, dim3((nt + 255) / 256), dim3(256), 0, st, pl.bwd.pose_part, n_envs, pl.K, s->O,
                           grad_rot, grad_trans);
    }
    if (e == hipSuccess) e = hipGetLastError();
    timer_end(pl, ETAC_TIMER_REDUCE, slot, st);
    return e;
}

hipError_t launch_contact_backward(const Plan &pl, const SceneDev &s, const float *grad_uhat, float *grad_rot,
                                   float *grad_trans, hipStream_t st) {
    if (s.E == 0) return hipSuccess;
    BwdParams p;
    p.mesh = pl.mesh;
    p.scene = s;
    p.model = ModelDev{ETAC_DECAY_ONLY, nullptr, nullptr};
    p.scr = pl.scr;
    p.bwd = pl.bwd;
    p.E = s.E;
    p.n_items = s.E * pl.K;
    p.batch = pl.bwd_batch;
    p.cobj_in = nullptr;
    p.uhat_in = nullptr;
    p.grad_u = nullptr;
    p.grad_uhat_in = grad_uhat;
    p.grad_uhat_out = nullptr;
    p.saved = nullptr;
    p.net_batch = pl.net_batch;
    p.n_seg = (p.n_items + 1023) / 1024;
    const int grid = min(p.n_items, pl.cu_count);
    hipError_t e = launch_bwd_net(p, BWD_CONTACT, grid, st);
    if (e != hipSuccess) return e;
    const int nt = s.E * s.O * 12;
    hipLaunchKernelGGL(k_pose, dim3((nt + 255) / 256), dim3(256), 0, st, pl.bwd.pose_part, s.E, pl.K, s.O, grad_rot,
                       grad_trans);
    return hipGetLastError();
}

hipError_t init_record_map(const Plan &pl) {
    hipLaunchKernelGGL(k_record_map, dim3((kPhiN + 255) / 256), dim3(256), 0, 0, pl.bwd.rec_map);
    return hipGetLastError();
}

#endif  // ETAC_BWD_NET_ONLY

}  // namespace etac

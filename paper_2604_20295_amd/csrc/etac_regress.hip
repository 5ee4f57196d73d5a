// Real-sensor regressor on gfx950: the displacement field of every (env,
// patch) item mapped to the eight taxel outputs of a real sensor by a
// PointNet-style network with a residual layer and attention pooling (the
// regressor of the paper's appendix, "Modeling Real Sensors").
//
//   k_regress      : persistent, one workgroup of eight waves per CU with the
//                    per-node layers' weights resident in LDS; every wave
//                    claims whole items from a device work queue (largest
//                    patches first), runs their 16-node tiles, two at a
//                    time, through the per-node layers on MFMA with an online
//                    softmax over the tiles, and appends the pooled feature
//                    g as a row.
//   k_regress_head : the head on every row, in FP32.
//   k_regress_fill : items without contact have U = 0 on the whole patch, so
//                    their output is the patch's rest output, computed once
//                    per patch (queue positions 0 .. K - 1, ahead of the E K
//                    items) and copied here.
//
// Per node:  x = [p - o_k, U] (6) -> h1 = relu(E1 x + e1) (64)
//            -> h2 = relu(E2 h1 + e2) + h1 (64) -> f = relu(E3 h2 + e3) (256)
//            -> s = a2 . tanh(A1 f + a1) + a0.
// Per item:  w = softmax(s), g = sum w f, y = D2 relu(D1 g + d1) + d2 (8).
//
// Precision: E1, the layer that sees positions and displacements, uses
// split-FP16 operands (hi + lo, FP32-level), so that displacements well
// below the position scale keep their bits; E2, E3 and A1 take FP16
// operands with FP32 accumulation; the pooled features are the FP16
// operands of A1 (f is held once, in 32 registers per tile); softmax
// weights, pooling sums and the head are FP32.  FP16 rounding is relative
// 2^-11 at most.
#include "etac_device.h"

namespace etac {

constexpr int kRegWG = 512;                  // eight waves, two per SIMD
constexpr int kRegWaves = kRegWG / 64;
constexpr int kRegNT = 2;                    // 16-node tiles per wave and pass (one weight read, kRegNT MFMAs)
// packed parameter offsets (FP32 values)
constexpr int kRE1 = 0, kRe1 = 384, kRE2 = 448, kRe2 = 4544, kRE3 = 4608, kRe3 = 20992;
constexpr int kRA1 = 21248, kRa1 = 54016, kRa2 = 54144, kRa0 = 54272, kRD1 = 54276, kRd1 = 87044;
constexpr int kRD2 = 87172, kRd2 = 88196, kRegN = 88204;
static_assert(kRegN == ETAC_REG_SIZE, "regressor parameter layout");
// 2 log2(e): A1 and a1 are stored times this, so that exp2 of the
// pre-activation is e^(2 z) and tanh z = 1 - 2 / (1 + e^(2 z)).
constexpr float kTwoLog2e = 2.8853900817779268f;

struct RegLds {
    half8 e1h[4 * 64], e1l[4 * 64];              // [E1 | e1] split, inputs padded 7 -> 32 (x_6 = 1 carries e1)
    half8 e2[4 * 2 * 64];                        // E2 FP16, [ot][s][lane], chain order
    half8 e3[16 * 2 * 64];                       // E3 FP16, [ot][s][lane], 256 outputs
    half8 a1[8 * 8 * 64];                        // 2 log2(e) A1 in FP16, [ot][s][lane], 128 outputs over 256 inputs
    float be2[64], be3[256], ba1[128], wa2[128]; // e2, e3, 2 log2(e) a1, -2 a2
};

struct RegParams {
    MeshDev mesh;
    const float *reg;         // [ETAC_REG_SIZE]
    const float *u;           // [3][E][N]
    const int32_t *n_active;  // [E][K]
    float *pooled;            // [rows][256] pooled feature g of each processed item
    int *row_item;            // [rows] its item: e K + k, or -1 - k for patch k's rest item
    unsigned *counter;        // [4] work queue, retired workgroups, rows, rows of the last call
    int E, n_pos;             // queue positions: K rest items, then the E K items
};

__device__ void stage_regressor(RegLds &L, const float *R) {
    const int tid = threadIdx.x;
    for (int idx = tid; idx < 4 * 64; idx += kRegWG) {
        const int lane = idx & 63, ot = idx >> 6, q = lane >> 4, o = ot * 16 + (lane & 15);
        float x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int in = 8 * q + e;
            x[e] = in < 6 ? R[kRE1 + o * 6 + in] : in == 6 ? R[kRe1 + o] : 0.0f;
        }
        split8(x, L.e1h[idx], L.e1l[idx]);
    }
    for (int idx = tid; idx < 4 * 2 * 64; idx += kRegWG) {
        const int lane = idx & 63, s = (idx >> 6) & 1, ot = idx >> 7, q = lane >> 4;
        half8 h;
#pragma unroll
        for (int e = 0; e < 8; ++e) h[e] = (_Float16)R[kRE2 + (ot * 16 + (lane & 15)) * 64 + chain_k(s, q, e)];
        L.e2[idx] = h;
    }
    for (int idx = tid; idx < 16 * 2 * 64; idx += kRegWG) {
        const int lane = idx & 63, s = (idx >> 6) & 1, ot = idx >> 7, q = lane >> 4;
        half8 h;
#pragma unroll
        for (int e = 0; e < 8; ++e) h[e] = (_Float16)R[kRE3 + (ot * 16 + (lane & 15)) * 64 + chain_k(s, q, e)];
        L.e3[idx] = h;
    }
    for (int idx = tid; idx < 8 * 8 * 64; idx += kRegWG) {
        const int lane = idx & 63, s = (idx >> 6) & 7, ot = idx >> 9, q = lane >> 4;
        half8 h;
#pragma unroll
        for (int e = 0; e < 8; ++e)
            h[e] = (_Float16)(kTwoLog2e * R[kRA1 + (ot * 16 + (lane & 15)) * 256 + chain_k(s, q, e)]);
        L.a1[idx] = h;
    }
    for (int i = tid; i < 64; i += kRegWG) L.be2[i] = R[kRe2 + i];
    for (int i = tid; i < 256; i += kRegWG) L.be3[i] = R[kRe3 + i];
    for (int i = tid; i < 128; i += kRegWG) {
        L.ba1[i] = kTwoLog2e * R[kRa1 + i];
        L.wa2[i] = -2.0f * R[kRa2 + i];
    }
}

// FP16 B operands of K step s from a D-layout feature tile (no lo part).
__device__ __forceinline__ half8 chain_f16(const floatx4 *x, int s) {
    half8 h;
#pragma unroll
    for (int e = 0; e < 8; ++e) h[e] = (_Float16)x[2 * s + (e >> 2)][e & 3];
    return h;
}

// relu of two values, rounded to FP16 and packed (rounding commutes with relu).
__device__ __forceinline__ unsigned pack_relu(float a, float b) {
    half2t h = {(_Float16)a, (_Float16)b};
    h = __builtin_elementwise_max(h, half2t{(_Float16)0.0f, (_Float16)0.0f});
    return __builtin_bit_cast(unsigned, h);
}

// acc + w * (low or high FP16 half of h), in one mixed-precision FMA.
template <bool HI>
__device__ __forceinline__ float fma_half(float w, unsigned h, float acc) {
    float d;
    if (HI) asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel:[0,1,0] op_sel_hi:[0,1,0]" : "=v"(d) : "v"(w), "v"(h), "v"(acc));
    else asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel_hi:[0,1,0]" : "=v"(d) : "v"(w), "v"(h), "v"(acc));
    return d;
}

// kRegNT 16-node tiles through the per-node layers.  Out: fb[i][s], the
// tile's features f (256) as FP16 B operands of A1 (element e is feature
// chain_k(s, l >> 4, e) of node l & 15), and sc[i], the attention score of
// the lane's node up to a constant (the same in the four lanes of a node).
// Each weight fragment is read from LDS once per pass and used by every
// tile; A1 runs output block by output block so that the tanh of one block
// overlaps the MFMAs of the next.
__device__ __forceinline__ void regress_tiles(const RegLds &L, const half8 (&xh)[kRegNT], const half8 (&xl)[kRegNT],
                                              half8 (&fb)[kRegNT][8], float (&sc)[kRegNT]) {
    constexpr int NT = kRegNT;
    reload_fence();
    const int lane = lane_id(), gq = lane >> 4;
    floatx4 h1[NT][4];
    {
        const floatx4 z = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            const half8 wh = L.e1h[ot * 64 + lane], wl = L.e1l[ot * 64 + lane];
#pragma unroll
            for (int i = 0; i < NT; ++i) h1[i][ot] = relu4(mfma_split(wh, wl, xh[i], xl[i], z));
        }
    }
    half8 b0[NT], b1[NT];   // h2 as FP16 B operands of E3
    {
        half8 c0[NT], c1[NT];   // h1 as FP16 B operands of E2
#pragma unroll
        for (int i = 0; i < NT; ++i) {
            c0[i] = chain_f16(h1[i], 0);
            c1[i] = chain_f16(h1[i], 1);
        }
        floatx4 h2[NT][4];
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            const floatx4 bias = *reinterpret_cast<const floatx4 *>(&L.be2[ot * 16 + 4 * gq]);
            const half8 w0 = L.e2[(ot * 2 + 0) * 64 + lane], w1 = L.e2[(ot * 2 + 1) * 64 + lane];
#pragma unroll
            for (int i = 0; i < NT; ++i) {
                h2[i][ot] = relu4(mfma16(w1, c1[i], mfma16(w0, c0[i], bias)));
#pragma unroll
                for (int r = 0; r < 4; ++r) h2[i][ot][r] += h1[i][ot][r];
            }
        }
#pragma unroll
        for (int i = 0; i < NT; ++i) {
            b0[i] = chain_f16(h2[i], 0);
            b1[i] = chain_f16(h2[i], 1);
        }
    }
    reload_fence();
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        floatx4 f[NT][2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int ot = 2 * s + j;
            const floatx4 bias = *reinterpret_cast<const floatx4 *>(&L.be3[ot * 16 + 4 * gq]);
            const half8 w0 = L.e3[(ot * 2 + 0) * 64 + lane], w1 = L.e3[(ot * 2 + 1) * 64 + lane];
#pragma unroll
            for (int i = 0; i < NT; ++i) f[i][j] = mfma16(w1, b1[i], mfma16(w0, b0[i], bias));
        }
#pragma unroll
        for (int i = 0; i < NT; ++i) {
            uint4t v;
            v[0] = pack_relu(f[i][0][0], f[i][0][1]);
            v[1] = pack_relu(f[i][0][2], f[i][0][3]);
            v[2] = pack_relu(f[i][1][0], f[i][1][1]);
            v[3] = pack_relu(f[i][1][2], f[i][1][3]);
            fb[i][s] = __builtin_bit_cast(half8, v);
        }
    }
    reload_fence();
    // a2 . tanh(z) = sum(a2) - 2 a2 . 1 / (1 + e^(2 z)); the constant sum(a2)
    // (like a0) cancels in the softmax
#pragma unroll
    for (int i = 0; i < NT; ++i) sc[i] = 0.0f;
#pragma unroll
    for (int ot = 0; ot < 8; ++ot) {
        const floatx4 bias = *reinterpret_cast<const floatx4 *>(&L.ba1[ot * 16 + 4 * gq]);
        floatx4 t[NT];
#pragma unroll
        for (int i = 0; i < NT; ++i) t[i] = bias;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const half8 w = L.a1[(ot * 8 + s) * 64 + lane];
#pragma unroll
            for (int i = 0; i < NT; ++i) t[i] = mfma16(w, fb[i][s], t[i]);
        }
        const floatx4 c = *reinterpret_cast<const floatx4 *>(&L.wa2[ot * 16 + 4 * gq]);
#pragma unroll
        for (int i = 0; i < NT; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                sc[i] += c[r] * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(t[i][r]));
    }
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        sc[i] += __shfl_xor(sc[i], 16);
        sc[i] += __shfl_xor(sc[i], 32);
    }
}

// v from the lane n places along in the same row of 16 lanes (DPP row_ror).
template <int n>
__device__ __forceinline__ float row_ror(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x120 + n, 0xf, 0xf, true));
}

// Sum over the 16 nodes of a lane group (one row of 16 lanes); every lane
// gets it, each in its own fixed order (the same in every row).
__device__ __forceinline__ float node_sum(float v) {
    v += row_ror<8>(v);
    v += row_ror<4>(v);
    v += row_ror<2>(v);
    v += row_ror<1>(v);
    return v;
}

__device__ __forceinline__ float node_max(float v) {
    v = fmaxf(v, row_ror<8>(v));
    v = fmaxf(v, row_ror<4>(v));
    v = fmaxf(v, row_ror<2>(v));
    v = fmaxf(v, row_ror<1>(v));
    return v;
}

// One item on one wave: every 16-node tile of patch k through the per-node
// layers, an online softmax over the tiles (running maximum m, per-lane
// running sums of e^(s - m) and e^(s - m) f), then the pooled feature
// g = sum w f / sum w appended as a row of p.pooled.
__device__ void regress_item(const RegParams &p, const RegLds &L, int e, int k, bool rest) {
    const MeshDev &M = p.mesh;
    const int N = M.N, lane = lane_id(), q = lane >> 4;
    const int base = M.offset[k], n = M.offset[k + 1] - base;
    const size_t EN = (size_t)p.E * N;
    const float o0 = M.origin[3 * k], o1 = M.origin[3 * k + 1], o2 = M.origin[3 * k + 2];
    float m_run = -INFINITY, l_run = 0.0f;   // m_run uniform; l_run per lane (its node's weights)
    floatx4 acc[16];
#pragma unroll
    for (int ot = 0; ot < 16; ++ot) acc[ot] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    const int groups = (n + 16 * kRegNT - 1) / (16 * kRegNT);
    for (int tg = 0; tg < groups; ++tg) {
        half8 xh[kRegNT], xl[kRegNT];
        bool valid[kRegNT];
#pragma unroll
        for (int i = 0; i < kRegNT; ++i) {
            const int j = 16 * (kRegNT * tg + i) + (lane & 15);
            valid[i] = j < n;
            float v[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) v[c] = 0.0f;
            if (q == 0) {
                v[6] = 1.0f;   // carries the bias e1
                if (valid[i]) {
                    const int gi = base + j;
                    v[0] = M.pos[gi] - o0;
                    v[1] = M.pos[N + gi] - o1;
                    v[2] = M.pos[2 * N + gi] - o2;
                    if (!rest) {
                        const size_t en = (size_t)e * N + gi;
                        v[3] = p.u[en];
                        v[4] = p.u[EN + en];
                        v[5] = p.u[2 * EN + en];
                    }
                }
            }
            split8(v, xh[i], xl[i]);
        }
        half8 fb[kRegNT][8];
        float s[kRegNT];
        regress_tiles(L, xh, xl, fb, s);
        float mt = -INFINITY;
#pragma unroll
        for (int i = 0; i < kRegNT; ++i) {
            s[i] = valid[i] ? s[i] : -INFINITY;
            mt = fmaxf(mt, s[i]);
        }
        mt = uniform(node_max(mt));   // the same in every lane; finite (node 0 of the first tile is valid)
        if (mt > m_run) {             // rescale the running sums to the new maximum
            const float c = __expf(m_run - mt);   // 0 on the first pass
#pragma unroll
            for (int ot = 0; ot < 16; ++ot)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[ot][r] *= c;
            l_run *= c;
            m_run = mt;
        }
#pragma unroll
        for (int i = 0; i < kRegNT; ++i) {
            const float w = valid[i] ? __expf(s[i] - m_run) : 0.0f;
            l_run += w;
#pragma unroll
            for (int s8 = 0; s8 < 8; ++s8) {
                const uint4t h = __builtin_bit_cast(uint4t, fb[i][s8]);
#pragma unroll
                for (int e2 = 0; e2 < 4; ++e2) {
                    const int ot = 2 * s8 + (e2 >> 1), r = 2 * (e2 & 1);
                    acc[ot][r] = fma_half<false>(w, h[e2], acc[ot][r]);
                    acc[ot][r + 1] = fma_half<true>(w, h[e2], acc[ot][r + 1]);
                }
            }
        }
    }
    // sums over the 16 node lanes: features 16 ot + 4 q + r in every lane of group q
    const float inv = 1.0f / node_sum(l_run);
#pragma unroll
    for (int ot = 0; ot < 16; ++ot)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[ot][r] = node_sum(acc[ot][r]) * inv;
    const unsigned old = atomicAdd(&p.counter[2], lane == 0 ? 1u : 0u);
    const unsigned row = (unsigned)__builtin_amdgcn_readlane((int)old, 0);
    if ((lane & 15) == 0) {
        float *g = p.pooled + (size_t)row * 256 + 4 * q;
#pragma unroll
        for (int ot = 0; ot < 16; ++ot) *reinterpret_cast<floatx4 *>(g + ot * 16) = acc[ot];
    }
    if (lane == 0) p.row_item[row] = rest ? -1 - k : e * M.K + k;
}

// Persistent; every wave claims items on its own (no barrier per item).
__global__ __launch_bounds__(kRegWG) void k_regress(RegParams p) {
    __shared__ RegLds L;
    stage_regressor(L, p.reg);
    __syncthreads();
    const MeshDev &M = p.mesh;
    for (;;) {
        // one atomic for the wave (lane 0 adds 1), executed by every lane so
        // that no lane-dependent branch enters the loop; lane 0's old value
        // is the claimed position
        const unsigned old = atomicAdd(&p.counter[0], lane_id() == 0 ? 1u : 0u);
        const unsigned pos = (unsigned)__builtin_amdgcn_readlane((int)old, 0);
        if (pos >= (unsigned)p.n_pos) break;
        int e = 0, k;
        const bool rest = pos < (unsigned)M.K;   // rest items first, largest patches first
        if (rest) {
            k = M.order[pos];
        } else {
            queue_item(M, p.E, (int)pos - M.K, e, k);
            if (uniform(p.n_active[(size_t)e * M.K + k]) == 0) continue;   // takes the rest output
        }
        regress_item(p, L, e, k, rest);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned done = atomicAdd(&p.counter[1], 1u);
        if (done == gridDim.x - 1) {   // last workgroup: publish the row count, reset the queue
            atomicExch(&p.counter[3], atomicExch(&p.counter[2], 0u));
            atomicExch(&p.counter[0], 0u);
            atomicExch(&p.counter[1], 0u);
        }
    }
}

// Head of every row: y = D2 relu(D1 g + d1) + d2 in FP32, 32 rows per
// block pass; D1 streamed through LDS transposed in 32-column chunks.
constexpr int kHeadRows = 32;

__global__ __launch_bounds__(256) void k_regress_head(const float *reg, const float *pooled, const int *row_item,
                                                      const unsigned *counter, int K, float *taxels, float *rest) {
    __shared__ float G[kHeadRows][256];
    __shared__ float DT[32][129];
    __shared__ float H[kHeadRows][128];
    const int tid = threadIdx.x, o = tid & 127, rh = tid >> 7;
    const unsigned rows = counter[3];
    for (unsigned b0 = blockIdx.x * kHeadRows; b0 < rows; b0 += gridDim.x * kHeadRows) {
        __syncthreads();   // the previous pass is done with G and H
        for (int idx = tid; idx < kHeadRows * 64; idx += 256) {
            const int r = idx >> 6, c4 = idx & 63;
            floatx4 v = {0.0f, 0.0f, 0.0f, 0.0f};
            if (b0 + r < rows) v = *reinterpret_cast<const floatx4 *>(pooled + (size_t)(b0 + r) * 256 + 4 * c4);
            *reinterpret_cast<floatx4 *>(&G[r][4 * c4]) = v;
        }
        float a[16];
        const float bias = reg[kRd1 + o];
#pragma unroll
        for (int r = 0; r < 16; ++r) a[r] = bias;
#pragma unroll 1
        for (int c0 = 0; c0 < 256; c0 += 32) {
            __syncthreads();   // G written; DT free
#pragma unroll 4
            for (int idx = tid; idx < 128 * 32; idx += 256) {
                const int oo = idx >> 5, cc = idx & 31;
                DT[cc][oo] = reg[kRD1 + oo * 256 + c0 + cc];
            }
            __syncthreads();
#pragma unroll 2
            for (int cc = 0; cc < 32; cc += 4) {
                const float w0 = DT[cc][o], w1 = DT[cc + 1][o], w2 = DT[cc + 2][o], w3 = DT[cc + 3][o];
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const floatx4 g = *reinterpret_cast<const floatx4 *>(&G[rh * 16 + r][c0 + cc]);
                    a[r] += w0 * g[0];
                    a[r] += w1 * g[1];
                    a[r] += w2 * g[2];
                    a[r] += w3 * g[3];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) H[rh * 16 + r][o] = relu1(a[r]);
        __syncthreads();
        {
            const int r = tid >> 3, j = tid & 7;
            if (b0 + r < rows) {
                float y = reg[kRd2 + j];
                const float *d2 = reg + kRD2 + j * 128;
#pragma unroll 8
                for (int c = 0; c < 128; ++c) y += d2[c] * H[r][c];
                const int it = row_item[b0 + r];
                if (it >= 0) taxels[(size_t)it * 8 + j] = y;
                else rest[(size_t)(-1 - it) * 8 + j] = y;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_regress_fill(const int32_t *n_active, const float *rest, int E, int K,
                                                      float *taxels) {
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (size_t)E * K * 8) return;
    const size_t item = t >> 3;
    if (n_active[item] == 0) taxels[t] = rest[(item % (size_t)K) * 8 + (t & 7)];
}

hipError_t launch_regress(const Plan &pl, const float *reg, int n_envs, const float *u, const int32_t *n_active,
                          float *taxels, hipStream_t st) {
    if (n_envs == 0) return hipSuccess;
    unsigned *ctr = pl.scr.counter + 4;
    RegParams p{pl.mesh, reg, u, n_active, pl.reg_pooled, pl.reg_row, ctr, n_envs, pl.K + n_envs * pl.K};
    const int grid = min(pl.cu_count, (p.n_pos + kRegWaves - 1) / kRegWaves);
    const int slot = timer_begin(pl, ETAC_TIMER_REGRESS, st);
    hipLaunchKernelGGL(k_regress, dim3(grid), dim3(kRegWG), 0, st, p);
    hipError_t e = hipGetLastError();
    timer_end(pl, ETAC_TIMER_REGRESS, slot, st);
    if (e != hipSuccess) return e;
    const int head_grid = min(pl.cu_count, (p.n_pos + kHeadRows - 1) / kHeadRows);
    hipLaunchKernelGGL(k_regress_head, dim3(head_grid), dim3(256), 0, st, reg, pl.reg_pooled, pl.reg_row, ctr, pl.K,
                       taxels, pl.reg_rest);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t nt = (size_t)n_envs * pl.K * 8;
    hipLaunchKernelGGL(k_regress_fill, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, n_active, pl.reg_rest,
                       n_envs, pl.K, taxels);
    return hipGetLastError();
}

}  // namespace etac

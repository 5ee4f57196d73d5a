// Adjoint of the ETac step on gfx950.
//
// k_bwd is a persistent kernel over (env, patch) items like the forward step.
// For every item it recomputes the contact pass (nothing is kept from the
// forward call), then for L = sum_i g_i . U_i:
//   1. active nodes: dL/du_hat_j = g_j                        (U_j = u_hat_j)
//   2. Eq. 1 adjoint, transposed pair loop over passive nodes i:
//        dL/du_hat_j += sum_i w_ij g_i,
//        dL/dalpha_k += sum_ij (-d_ij w_ij) (g_i . u_hat_j)
//   3. residual-network adjoint on FP32 MFMA (weight gradients are node
//      contractions, fed through per-wave LDS transposes); the max-pool routes
//      its gradient to the arg-max node of each channel (lowest index on
//      ties), which reaches u_hat of active arg-max nodes through W1;
//   4. contact adjoint: dL/d(R, t) of every winning object from dL/du_hat
//      of its active nodes, in FP64.
// Per-item partials (network parameters, alpha, poses) go to plan scratch and
// are summed by the reduction kernels in a fixed order, so results do not
// depend on which workgroup processed which item.
#include "etac_device.h"

namespace etac {

constexpr int kBChunk = 1024;  // passive nodes staged per pass of the decay adjoint
constexpr int kTS = 68;        // row stride (floats) of the per-wave transpose tiles
constexpr int kPhiSegs = 64;   // segments of the parameter-gradient reduction

enum BwdKind { BWD_STEP = 0, BWD_PROP = 1, BWD_CONTACT = 2 };

struct BwdParams {
    MeshDev mesh;
    SceneDev scene;
    ModelDev model;
    Scratch scr;
    BwdScratch bwd;
    int E, n_items;
    const int8_t *cobj_in;        // BWD_PROP
    const float *uhat_in;         // BWD_PROP
    const float *grad_u;          // [3][E][N]   BWD_STEP, BWD_PROP
    const float *grad_uhat_in;    // [3][E][N]   BWD_CONTACT
    float *grad_uhat_out;         // [3][E][N]   BWD_PROP
};

constexpr int kRS = 82;        // row stride (floats) of the 64-feature round tiles
constexpr int kDS = 34;        // row stride of the 16-feature round tiles
// Both strides put rows 8 apart 16 LDS banks apart, so the four lane groups of
// an MFMA operand read (rows 8 q + e) hit different banks.

// One round of the network adjoint: 4 tiles x 16 nodes (one tile per wave),
// stored as rows [node][feature] so that every wave can contract over all 64
// nodes for the weight-gradient slice it owns.
struct RoundBuf {
    float a[64 * kRS];         // phase A: dL/dpre4   | phase B: dL/dpre2
    float b[64 * kRS];         // phase A: f          | phase B: h1
    float c[64 * kRS];         // phase A: h4         | phase B: dL/dpre1
    float d[64 * kDS];         // phase A: dL/dr      | phase B: x (inputs 0..15; 16..31 scratch)
};

struct BwdLds {
    NetLds net;
    half8 w2th[4 * 2 * 64], w2tl[4 * 2 * 64];   // [it][s][lane] split fragments of W2^T
    half8 w4th[4 * 2 * 64], w4tl[4 * 2 * 64];   // [it][s][lane] split fragments of W4[:, :64]^T
    float w1u[3][64];                           // W1[:, 6..8]: the u_hat inputs
    union {
        struct {
            float4 a[kBChunk];    // (px, py, pz, gx) of staged passive nodes
            float2 b[kBChunk];    // (gy, gz)
            double part[kWG][6];  // per-thread partial dL/du_hat of its two active nodes
        } st;
        RoundBuf rb;
    } u;
    float s4[64];                 // sum_i dL/dpre4_i  (= db4)
    float dgp[64], dpre3[64], dg[64];
    float vred[kWaves][64];
    int ired[kWaves][64];
    int argmax[64];
    float dxs[64][3];             // dL/du_hat of the routed arg-max node of each channel
    double dred[kWaves][12];
    int wcnt[2][kWaves];
    int item;
    unsigned cand;
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Transposed weight fragments for the adjoint layers, in the chain order of
// etac_device.h (K step s, lane group q, element e <-> output chain_k(s, q, e)).
__device__ void stage_net_t(BwdLds &S, const float *phi) {
    const int tid = threadIdx.x;
    for (int idx = tid; idx < 4 * 2 * 64; idx += kWG) {
        const int lane = idx & 63, s = (idx >> 6) & 1, it = idx >> 7, q = lane >> 4;
        const int in = it * 16 + (lane & 15);
        float a[8], b[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int out = chain_k(s, q, e);
            a[e] = phi[kW2 + out * 64 + in];
            b[e] = phi[kW4 + out * 128 + in];
        }
        split8(a, S.w2th[idx], S.w2tl[idx]);
        split8(b, S.w4th[idx], S.w4tl[idx]);
    }
    for (int idx = tid; idx < 3 * 64; idx += kWG) S.w1u[idx >> 6][idx & 63] = phi[kW1 + (idx & 63) * 9 + 6 + (idx >> 6)];
}

// ---------------------------------------------------------------------------
// wave-level tile algebra
// ---------------------------------------------------------------------------

// Y^T = W^T X^T for a 16-node tile with X in D layout (the input-gradient
// chain of a 64 -> 64 layer); wth / wtl: split fragments [it][s][lane].
__device__ __forceinline__ void matT_tile(const half8 *wth, const half8 *wtl, const floatx4 x[4], floatx4 y[4]) {
    reload_fence();
    const int lane = lane_id();
    half8 bh[2], bl[2];
    split_chain(x, bh, bl);
#pragma unroll
    for (int it = 0; it < 4; ++it) {
        floatx4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int fi = (it * 2 + s) * 64 + lane;
            acc = mfma_split(wth[fi], wtl[fi], bh[s], bl[s], acc);
        }
        y[it] = acc;
    }
}

// Store a D-layout tile (16 nodes x 64 features) as round rows row0 .. row0 + 15.
__device__ __forceinline__ void store_rows(float *t, int row0, const floatx4 v[4]) {
    const int lane = lane_id(), node = lane & 15, gq = lane >> 4;
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) {
        float *dst = &t[(row0 + node) * kRS + ot * 16 + 4 * gq];
        *reinterpret_cast<float2 *>(dst) = make_float2(v[ot][0], v[ot][1]);
        *reinterpret_cast<float2 *>(dst + 2) = make_float2(v[ot][2], v[ot][3]);
    }
}

// acc[it] += sum over the 64 nodes of a round of A[node][acol + i] B[node][bcol + 16 it + j]
// (i, j = 0..15), with split-FP16 operands: K = nodes, two K steps of 32 in
// which lane group q supplies nodes 32 s + 8 q .. 32 s + 8 q + 7.  Result in
// the MFMA output layout: lane l, register r holds (i = 4 (l >> 4) + r, j = l & 15).
template <int NB>
__device__ __forceinline__ void round_wgrad(const float *A, int sa, int acol, const float *B, int sb, int bcol,
                                            floatx4 (&acc)[NB]) {
    const int lane = lane_id(), col = lane & 15, q = lane >> 4;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int row0 = 32 * s + 8 * q;
        float av[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) av[e] = A[(row0 + e) * sa + acol + col];
        half8 ah, al;
        split8(av, ah, al);
#pragma unroll
        for (int it = 0; it < NB; ++it) {
            float bv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) bv[e] = B[(row0 + e) * sb + bcol + 16 * it + col];
            half8 bh, bl;
            split8(bv, bh, bl);
            acc[it] = mfma_split(ah, al, bh, bl, acc[it]);
        }
    }
}

// Sum over the 64 round nodes of A[node][acol + i]; every lane returns the
// sum for i = lane & 15 (lane groups sum 16 nodes each, then a butterfly).
__device__ __forceinline__ float round_colsum(const float *A, int sa, int acol) {
    const int lane = lane_id(), col = lane & 15, q = lane >> 4;
    float s = 0.0f;
    for (int r = 0; r < 16; ++r) s += A[(q * 16 + r) * sa + acol + col];
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    return s;
}

// This wave's slices of the parameter gradients: output rows 16 wave .. 16 wave + 15.
struct WaveGrads {
    floatx4 w4[4];       // dW4[:, :64]
    floatx4 w2[4];       // dW2
    floatx4 w1[1];       // dW1 (inputs padded to 16)
    floatx4 w5[1];       // dW5 columns 16 wave + j (outputs padded to 16)
    float b4, b2, b1;    // bias sums of output 16 wave + (lane & 15)
    float b5[3];         // db5 partial (lane group 0 only)
};

__device__ __forceinline__ void zero_grads(WaveGrads &G) {
    const floatx4 z = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int a = 0; a < 4; ++a) { G.w4[a] = z; G.w2[a] = z; }
    G.w1[0] = z;
    G.w5[0] = z;
    G.b4 = G.b2 = G.b1 = 0.0f;
    G.b5[0] = G.b5[1] = G.b5[2] = 0.0f;
}

// Decoder adjoint of one round (phase A).  Each wave passes its tile's f, h4
// and dL/dr; returns dL/dpre4 of its tile and accumulates its dW4 / dW5 / db4
// slices over the round.
__device__ void round_decoder_adjoint(BwdLds &S, WaveGrads &G, const floatx4 f[4], const floatx4 h4[4],
                                      const float dr[3], floatx4 dh4[4]) {
    reload_fence();
    const int wave = threadIdx.x >> 6, lane = lane_id(), gq = lane >> 4, node = lane & 15;
    const NetLds &L = S.net;
    RoundBuf &R = S.u.rb;
#pragma unroll
    for (int ot = 0; ot < 4; ++ot)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int feat = ot * 16 + 4 * gq + r;
            const float v = L.w5[feat] * dr[0] + L.w5[64 + feat] * dr[1] + L.w5[128 + feat] * dr[2];
            dh4[ot][r] = h4[ot][r] > 0.0f ? v : 0.0f;
        }
    if (gq == 0) { G.b5[0] += dr[0]; G.b5[1] += dr[1]; G.b5[2] += dr[2]; }
    __syncthreads();                       // previous users of the round buffer are done
    store_rows(R.a, 16 * wave, dh4);
    store_rows(R.b, 16 * wave, f);
    store_rows(R.c, 16 * wave, h4);
#pragma unroll
    for (int c = gq; c < 16; c += 4) R.d[(16 * wave + node) * kDS + c] = c < 3 ? dr[c] : 0.0f;
    __syncthreads();
    round_wgrad<4>(R.a, kRS, 16 * wave, R.b, kRS, 0, G.w4);
    round_wgrad<1>(R.d, kDS, 0, R.c, kRS, 16 * wave, G.w5);
    G.b4 += round_colsum(R.a, kRS, 16 * wave);
}

// Encoder adjoint of one round (phase B) given dL/df of each wave's tile:
// accumulates the dW2 / dW1 / db2 / db1 slices and returns dL/du_hat of the
// tile's nodes (the gradient of inputs 6..8), valid in every lane for node
// (lane & 15).  xf: this lane's 8 network inputs (features 8 (lane >> 4) + e).
__device__ void round_encoder_adjoint(BwdLds &S, WaveGrads &G, const float xf[8], const floatx4 h1[4],
                                      const floatx4 f[4], const floatx4 df[4], float du[3]) {
    reload_fence();
    const int wave = threadIdx.x >> 6, lane = lane_id(), gq = lane >> 4, node = lane & 15;
    RoundBuf &R = S.u.rb;
    floatx4 dpre2[4], dh1[4];
#pragma unroll
    for (int ot = 0; ot < 4; ++ot)
#pragma unroll
        for (int r = 0; r < 4; ++r) dpre2[ot][r] = f[ot][r] > 0.0f ? df[ot][r] : 0.0f;
    matT_tile(S.w2th, S.w2tl, dpre2, dh1);
#pragma unroll
    for (int ot = 0; ot < 4; ++ot)
#pragma unroll
        for (int r = 0; r < 4; ++r) dh1[ot][r] = h1[ot][r] > 0.0f ? dh1[ot][r] : 0.0f;
    // dL/du_hat = W1[:, 6..8]^T dpre1: partial over this lane's 16 features, then the 4 lane groups
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float t = 0.0f;
#pragma unroll
        for (int ot = 0; ot < 4; ++ot)
#pragma unroll
            for (int r = 0; r < 4; ++r) t += S.w1u[c][ot * 16 + 4 * gq + r] * dh1[ot][r];
        t += __shfl_xor(t, 16);
        t += __shfl_xor(t, 32);
        du[c] = t;
    }
    __syncthreads();
    store_rows(R.a, 16 * wave, dpre2);
    store_rows(R.b, 16 * wave, h1);
    store_rows(R.c, 16 * wave, dh1);
    // x rows: groups 0 and 1 hold inputs 0..15; groups 2 and 3 write zeros to the padding
#pragma unroll
    for (int e = 0; e < 8; ++e) R.d[(16 * wave + node) * kDS + 8 * gq + e] = gq < 2 ? xf[e] : 0.0f;
    __syncthreads();
    round_wgrad<4>(R.a, kRS, 16 * wave, R.b, kRS, 0, G.w2);
    round_wgrad<1>(R.c, kRS, 16 * wave, R.d, kDS, 0, G.w1);
    G.b2 += round_colsum(R.a, kRS, 16 * wave);
    G.b1 += round_colsum(R.c, kRS, 16 * wave);
}

// ---------------------------------------------------------------------------
// item-level pieces
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool uses_residual(const BwdParams &p) {
    return p.model.mode != ETAC_DECAY_ONLY;
}

// Eq. 1 adjoint of one item.  Pairs (active j, passive i) are split over
// (active slot, passive segment): every thread owns two active nodes of a
// pass and one segment of each staged chunk of passive nodes (position, g);
// with few active nodes the passive list is cut into 2 or 4 segments so that
// all threads work.  Slots are whole waves, so LDS reads stay broadcasts.  The
// segment partials of dL/du_hat_j are combined in segment order; the thread's
// dL/dalpha contribution is returned.
__device__ double decay_adjoint(const BwdParams &p, BwdLds &S, int e, int k, int base, int m, int np,
                                const int *alist, const int *plist, const float *uhn, float *gh) {
    const MeshDev &M = p.mesh;
    const int N = M.N, n_max = p.scr.n_max;
    const size_t EN = (size_t)p.E * N;
    const size_t row = (size_t)e * N + base;
    const float nbeta = (float)(-(double)p.model.alpha[k] * 1.4426950408889634);
    const int slots = m <= 128 ? 64 : (m <= 256 ? 128 : kWG);     // threads per segment
    const int nseg = kWG / slots;
    const int slot = threadIdx.x % slots, seg = threadIdx.x / slots;
    double dalpha = 0.0;
    for (int ab = 0; ab < m; ab += 2 * slots) {
        const int t0 = ab + slot, t1 = t0 + slots;
        const bool v0 = t0 < m, v1 = t1 < m;
        const int j0 = v0 ? alist[t0] : alist[0], j1 = v1 ? alist[t1] : alist[0];
        const int g0 = base + j0, g1 = base + j1;
        const float px0 = M.pos[g0], py0 = M.pos[N + g0], pz0 = M.pos[2 * N + g0];
        const float px1 = M.pos[g1], py1 = M.pos[N + g1], pz1 = M.pos[2 * N + g1];
        const float ux0 = uhn[j0], uy0 = uhn[n_max + j0], uz0 = uhn[2 * n_max + j0];
        const float ux1 = uhn[j1], uy1 = uhn[n_max + j1], uz1 = uhn[2 * n_max + j1];
        double a0[3] = {0.0, 0.0, 0.0}, a1[3] = {0.0, 0.0, 0.0};
        double da0 = 0.0, da1 = 0.0;
        for (int c0 = 0; c0 < np; c0 += kBChunk) {
            const int cnt = min(kBChunk, np - c0);
            __syncthreads();
            for (int t = threadIdx.x; t < cnt; t += kWG) {
                const int i = plist[c0 + t];
                const int gi = base + i;
                S.u.st.a[t] = make_float4(M.pos[gi], M.pos[N + gi], M.pos[2 * N + gi], p.grad_u[row + i]);
                S.u.st.b[t] = make_float2(p.grad_u[EN + row + i], p.grad_u[2 * EN + row + i]);
            }
            __syncthreads();
            const int per = (cnt + nseg - 1) / nseg;
            const int lo = seg * per, hi = min(cnt, lo + per);
            for (int i0 = lo; i0 < hi; i0 += 32) {
                const int i1 = min(hi, i0 + 32);
                float s0x = 0.f, s0y = 0.f, s0z = 0.f, s1x = 0.f, s1y = 0.f, s1z = 0.f, q0 = 0.f, q1 = 0.f;
                for (int i = i0; i < i1; ++i) {
                    const float4 a = S.u.st.a[i];
                    const float2 b = S.u.st.b[i];
                    const float dx0 = a.x - px0, dy0 = a.y - py0, dz0 = a.z - pz0;
                    const float dx1 = a.x - px1, dy1 = a.y - py1, dz1 = a.z - pz1;
                    const float d0 = __builtin_amdgcn_sqrtf(dx0 * dx0 + dy0 * dy0 + dz0 * dz0);
                    const float d1 = __builtin_amdgcn_sqrtf(dx1 * dx1 + dy1 * dy1 + dz1 * dz1);
                    const float w0 = __builtin_amdgcn_exp2f(nbeta * d0);
                    const float w1 = __builtin_amdgcn_exp2f(nbeta * d1);
                    s0x += w0 * a.w; s0y += w0 * b.x; s0z += w0 * b.y;
                    s1x += w1 * a.w; s1y += w1 * b.x; s1z += w1 * b.y;
                    q0 += d0 * w0 * (a.w * ux0 + b.x * uy0 + b.y * uz0);
                    q1 += d1 * w1 * (a.w * ux1 + b.x * uy1 + b.y * uz1);
                }
                a0[0] += s0x; a0[1] += s0y; a0[2] += s0z;
                a1[0] += s1x; a1[1] += s1y; a1[2] += s1z;
                da0 -= q0;
                da1 -= q1;
            }
        }
        if (v0) dalpha += da0;
        if (v1) dalpha += da1;
        // combine the segments of each active node in segment order
        __syncthreads();
        double *mine = S.u.st.part[threadIdx.x];
        mine[0] = a0[0]; mine[1] = a0[1]; mine[2] = a0[2];
        mine[3] = a1[0]; mine[4] = a1[1]; mine[5] = a1[2];
        __syncthreads();
        if (seg == 0) {
            for (int q = 1; q < nseg; ++q) {
                const double *o = S.u.st.part[q * slots + slot];
                a0[0] += o[0]; a0[1] += o[1]; a0[2] += o[2];
                a1[0] += o[3]; a1[1] += o[4]; a1[2] += o[5];
            }
            if (v0) {
                gh[j0] = (float)((double)gh[j0] + a0[0]);
                gh[n_max + j0] = (float)((double)gh[n_max + j0] + a0[1]);
                gh[2 * n_max + j0] = (float)((double)gh[2 * n_max + j0] + a0[2]);
            }
            if (v1) {
                gh[j1] = (float)((double)gh[j1] + a1[0]);
                gh[n_max + j1] = (float)((double)gh[n_max + j1] + a1[1]);
                gh[2 * n_max + j1] = (float)((double)gh[2 * n_max + j1] + a1[2]);
            }
        }
    }
    __syncthreads();
    return dalpha;
}

// Deterministic workgroup sum of 12 doubles per thread (butterfly within the
// wave, then the waves in order); the result is returned in every thread.
// Blocks that only part of the workgroup executes are whole waves and every
// lane stores the same value, so no single-lane region sits next to a
// barrier (the compiler may otherwise thread the rest of a wave past it).
__device__ void wg_sum12(BwdLds &S, double v[12]) {
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        double x = v[c];
        for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
        v[c] = x;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 12; ++c) S.dred[wave][c] = v[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        double s = S.dred[0][c];
        for (int w = 1; w < kWaves; ++w) s += S.dred[w][c];
        v[c] = s;
    }
    __syncthreads();
}

// dL/d(R, t) contribution of one active node from dL/du_hat = g (FP64).
// The face / clamp choice repeats the forward's operation order.
__device__ void contact_adjoint_node(int type, const float *sh, const float *Rf, const float *tf, float px, float py,
                                     float pz, const double g[3], double acc[12]) {
#pragma clang fp contract(off)
    const double d[3] = {(double)px - (double)tf[0], (double)py - (double)tf[1], (double)pz - (double)tf[2]};
    double R[9];
    for (int c = 0; c < 9; ++c) R[c] = Rf[c];
    if (type == ETAC_SPHERE) {
        const double r = sh[0];
        const double s = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
        if (s == 0.0) return;
        const double l = sqrt(s);
        const double phi = r / l - 1.0, tphip = -r / (l * s);
        const double gd = g[0] * d[0] + g[1] * d[1] + g[2] * d[2];
        #pragma unroll
        for (int a = 0; a < 3; ++a) acc[9 + a] -= phi * g[a] + tphip * gd * d[a];
        return;
    }
    double q[3];
    for (int c = 0; c < 3; ++c) q[c] = (R[0 * 3 + c] * d[0] + R[1 * 3 + c] * d[1]) + R[2 * 3 + c] * d[2];
    if (type == ETAC_BOX) {
        double best = (double)sh[0] - fabs(q[0]);
        int cs = 0;
        for (int c = 1; c < 3; ++c) {
            const double sl = (double)sh[c] - fabs(q[c]);
            if (sl < best) { best = sl; cs = c; }
        }
        const double sg = q[cs] >= 0.0 ? 1.0 : -1.0;
        const double rc[3] = {R[cs], R[3 + cs], R[6 + cs]};
        const double grc = g[0] * rc[0] + g[1] * rc[1] + g[2] * rc[2];
        const double coef = sg * (double)sh[cs] - q[cs];
        #pragma unroll
        for (int a = 0; a < 3; ++a) {
            acc[9 + a] += grc * rc[a];
            acc[a * 3 + cs] += coef * g[a] - grc * d[a];
        }
        return;
    }
    const double r = sh[0], L = sh[1];
    double z = q[2];
    bool clamped = false;
    if (z < -L) { z = -L; clamped = true; }
    else if (z > L) { z = L; clamped = true; }
    const double v[3] = {q[0], q[1], q[2] - z};
    const double s = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
    if (s == 0.0) return;
    const double l = sqrt(s);
    const double phi = r / l - 1.0, tphip = -r / (l * s);
    double Rv[3], RTg[3];
    #pragma unroll
    for (int a = 0; a < 3; ++a) Rv[a] = R[a * 3] * v[0] + R[a * 3 + 1] * v[1] + R[a * 3 + 2] * v[2];
    for (int c = 0; c < 3; ++c) RTg[c] = R[c] * g[0] + R[3 + c] * g[1] + R[6 + c] * g[2];
    const double gRv = g[0] * Rv[0] + g[1] * Rv[1] + g[2] * Rv[2];
    double av[3];
    for (int c = 0; c < 3; ++c) av[c] = tphip * gRv * v[c] + phi * RTg[c];
    if (!clamped) av[2] = tphip * gRv * v[2];
    #pragma unroll
    for (int a = 0; a < 3; ++a) {
        for (int c = 0; c < 3; ++c) acc[a * 3 + c] += d[a] * av[c] + phi * g[a] * v[c];
        acc[9 + a] -= R[a * 3] * av[0] + R[a * 3 + 1] * av[1] + R[a * 3 + 2] * av[2];
    }
}

// Pose partials of one item: for every object, the sum over its active nodes.
__device__ void contact_adjoint_item(const BwdParams &p, BwdLds &S, int e, int item, int base, int m,
                                     const int *alist, const int8_t *wobj, const float *gh) {
    const MeshDev &M = p.mesh;
    const int N = M.N, n_max = p.scr.n_max, O = p.scene.O;
    const int no = min(p.scene.n_obj[e], O);
    float *out = p.bwd.pose_part + (size_t)item * O * 12;
    for (int o = 0; o < O; ++o) {
        double acc[12];
        for (int c = 0; c < 12; ++c) acc[c] = 0.0;
        if (o < no) {
            const size_t eo = (size_t)e * O + o;
            const int ty = p.scene.type[eo];
            const float *sh = p.scene.shape + 4 * eo, *R = p.scene.rot + 9 * eo, *t = p.scene.trans + 3 * eo;
            for (int q = threadIdx.x; q < m; q += kWG) {
                const int j = alist[q];
                if (wobj[j] != o) continue;
                const int gj = base + j;
                const double g[3] = {gh[j], gh[n_max + j], gh[2 * n_max + j]};
                contact_adjoint_node(ty, sh, R, t, M.pos[gj], M.pos[N + gj], M.pos[2 * N + gj], g, acc);
            }
        }
        wg_sum12(S, acc);
        if (threadIdx.x < 12) out[o * 12 + threadIdx.x] = (float)acc[threadIdx.x];
        __syncthreads();
    }
}

// Residual-network adjoint of one item; writes its parameter-gradient
// partial and adds dL/du_hat of active arg-max nodes into gh.
__device__ void residual_adjoint(const BwdParams &p, BwdLds &S, int e, int k, int item, int base, int n,
                                 const float *uhn, const int8_t *wobj, float *gh) {
    NetLds &L = S.net;
    const MeshDev &M = p.mesh;
    const float *phi = p.model.phi;
    const int N = M.N, n_max = p.scr.n_max;
    const size_t EN = (size_t)p.E * N;
    const size_t row = (size_t)e * N + base;
    const int lane = lane_id(), wave = threadIdx.x >> 6, gq = lane >> 4;
    const int ntiles = (n + 15) >> 4;
    float *out = p.bwd.phi_part + (size_t)item * kPhiN;

    // (a) encoder pass: max-pool with arg-max (lowest node on ties)
    floatx4 mx[4];
    int mi[4][4];
    #pragma unroll
    for (int ot = 0; ot < 4; ++ot)
        #pragma unroll
        for (int r = 0; r < 4; ++r) { mx[ot][r] = -1.0f; mi[ot][r] = 0x7fffffff; }
    for (int t = wave; t < ntiles; t += kWaves) {
        const int ln = t * 16 + (lane & 15);
        const bool valid = ln < n;
        half8 xh, xl;
        load_x(M, k, base + ln, valid, uhn, n_max, ln, xh, xl);
        floatx4 h1[4], f[4];
        encoder_tile(L, xh, xl, h1, f);
        if (valid)
            #pragma unroll
            for (int ot = 0; ot < 4; ++ot)
                #pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (f[ot][r] > mx[ot][r]) { mx[ot][r] = f[ot][r]; mi[ot][r] = ln; }
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
        L.g[c] = v;
        S.argmax[c] = ix;
    }
    __syncthreads();
    global_mlp(L, phi);

    // (b) rounds of four tiles: decoder adjoint (phase A), then encoder
    //     adjoint (phase B) of every tile's passive nodes
    WaveGrads G;
    zero_grads(G);
    for (int t0 = 0; t0 < ntiles; t0 += kWaves) {
        const int ln = (t0 + wave) * 16 + (lane & 15);
        const bool valid = ln < n;
        const bool passive = valid && wobj[ln] < 0;
        half8 xh, xl;
        float xf[8];
        load_x(M, k, base + (valid ? ln : 0), valid, uhn, n_max, valid ? ln : 0, xh, xl, xf);
        floatx4 h1[4], f[4], h4[4];
        encoder_tile(L, xh, xl, h1, f);
        float r_unused[3];
        decoder_tile(L, f, h4, r_unused);
        float dr[3] = {0.0f, 0.0f, 0.0f};
        if (passive) {
            dr[0] = p.grad_u[row + ln];
            dr[1] = p.grad_u[EN + row + ln];
            dr[2] = p.grad_u[2 * EN + row + ln];
        }
        floatx4 dh4[4], df[4];
        float du[3];
        round_decoder_adjoint(S, G, f, h4, dr, dh4);
        matT_tile(S.w4th, S.w4tl, dh4, df);
        round_encoder_adjoint(S, G, xf, h1, f, df, du);
    }
    __syncthreads();
    S.s4[16 * wave + (lane & 15)] = G.b4;    // identical values in the 4 lane groups
    __syncthreads();

    // (c) global MLP adjoint: dg' = W4[:, 64:]^T s4, dpre3 = dg' gated by
    //     g' > 0, dg = W3^T dpre3
    {
        // each wave sums 16 of the 64 terms, the partials are added in wave order
        const int c = lane;
        float s = 0.0f;
#pragma unroll 4
        for (int o = 16 * wave; o < 16 * wave + 16; ++o) s += phi[kW4 + o * 128 + 64 + c] * S.s4[o];
        S.vred[wave][c] = s;
        __syncthreads();
        if (threadIdx.x < 64) {
            float t = S.vred[0][c];
            for (int w = 1; w < kWaves; ++w) t += S.vred[w][c];
            S.dgp[c] = t;
            S.dpre3[c] = L.gp[c] > 0.0f ? t : 0.0f;
        }
        __syncthreads();
        s = 0.0f;
#pragma unroll 4
        for (int o = 16 * wave; o < 16 * wave + 16; ++o) s += phi[kW3 + o * 64 + c] * S.dpre3[o];
        S.vred[wave][c] = s;
        __syncthreads();
        if (threadIdx.x < 64) {
            float t = S.vred[0][c];
            for (int w = 1; w < kWaves; ++w) t += S.vred[w][c];
            S.dg[c] = t;
        }
        __syncthreads();
    }

    // (d) max-pool routing round: slot c carries dL/df = dg[c] e_c at the
    //     arg-max node of channel c; wave w holds slots 16 w .. 16 w + 15
    {
        const int slot = wave * 16 + (lane & 15);
        const int ln = S.argmax[slot];
        const bool valid = ln < n;
        half8 xh, xl;
        float xf[8];
        load_x(M, k, base + (valid ? ln : 0), valid, uhn, n_max, valid ? ln : 0, xh, xl, xf);
        floatx4 h1[4], f[4], df[4];
        encoder_tile(L, xh, xl, h1, f);
#pragma unroll
        for (int ot = 0; ot < 4; ++ot)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int feat = ot * 16 + 4 * gq + r;
                df[ot][r] = (valid && feat == slot) ? S.dg[slot] : 0.0f;
            }
        float du[3];
        round_encoder_adjoint(S, G, xf, h1, f, df, du);
#pragma unroll
        for (int c = 0; c < 3; ++c) S.dxs[slot][c] = du[c];   // identical in the 4 lane groups
    }
    __syncthreads();
    // Wave 0 adds the routed dL/du_hat in slot order; all its lanes do the same update.
    if (threadIdx.x < 64)
        for (int c = 0; c < 64; ++c) {
            const int ln = S.argmax[c];
            if (ln < n && wobj[ln] >= 0) {
                gh[ln] += S.dxs[c][0];
                gh[n_max + ln] += S.dxs[c][1];
                gh[2 * n_max + ln] += S.dxs[c][2];
            }
        }

    // (e) item partial of every parameter gradient; each wave writes its slices
    {
        const int col = lane & 15, o16 = 16 * wave;
#pragma unroll
        for (int it = 0; it < 4; ++it)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = o16 + 4 * gq + r, i = 16 * it + col;
                out[kW4 + o * 128 + i] = G.w4[it][r];
                out[kW2 + o * 64 + i] = G.w2[it][r];
            }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = o16 + 4 * gq + r;
            if (col < 9) out[kW1 + o * 9 + col] = G.w1[0][r];
            const int o5 = 4 * gq + r;
            if (o5 < 3) out[kW5 + o5 * 64 + o16 + col] = G.w5[0][r];
        }
        out[kB4 + o16 + col] = G.b4;
        out[kB2 + o16 + col] = G.b2;
        out[kB1 + o16 + col] = G.b1;
    }
    for (int idx = threadIdx.x; idx < 64 * 64; idx += kWG) {
        const int o = idx >> 6, c = idx & 63;
        out[kW4 + o * 128 + 64 + c] = S.s4[o] * L.gp[c];     // dW4[:, 64:] = s4 (x) g'
        out[kW3 + o * 64 + c] = S.dpre3[o] * L.g[c];          // dW3 = dpre3 (x) g
    }
    if (threadIdx.x < 64) out[kB3 + threadIdx.x] = S.dpre3[threadIdx.x];
    // db5: wave sums (only lane group 0 accumulated), then the waves in order
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float x = G.b5[c];
        for (int off = 1; off <= 32; off <<= 1) x += __shfl_xor(x, off);
        G.b5[c] = x;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) S.vred[wave][c] = G.b5[c];
    __syncthreads();
    if (threadIdx.x < 64)
        for (int c = 0; c < 3; ++c) {
            float s = S.vred[0][c];
            for (int w = 1; w < kWaves; ++w) s += S.vred[w][c];
            out[kB5 + c] = s;
        }
    __syncthreads();
}

template <int KIND>
__device__ void process_item_bwd(const BwdParams &p, BwdLds &S, int item, int e, int k, float *uhn, float *gh,
                                 int *alist, int *plist, int8_t *wobj) {
    const MeshDev &M = p.mesh;
    const int N = M.N, n_max = p.scr.n_max, O = p.scene.O;
    const size_t EN = (size_t)p.E * N;
    const int base = M.offset[k];
    const int n = M.offset[k + 1] - base;
    const size_t row = (size_t)e * N + base;
    unsigned cand = 0xffu;
    int m = 0;
    bool has = true;
    if (KIND != BWD_PROP) {
        if (threadIdx.x < 64) S.cand = cull_objects(p.scene, M, e, k);
        __syncthreads();
        cand = uniform(S.cand);
        __syncthreads();
        has = cand != 0u;
    }
    if (has)
        m = contact_and_compact<KIND == BWD_PROP>(M, p.scene, p.E, n_max, p.cobj_in, p.uhat_in, nullptr, S.wcnt, e, k,
                                                  base, n, cand, uhn, alist, plist, wobj);
    if (m == 0) {
        if (threadIdx.x < 64) {
            p.bwd.alpha_part[item] = 0.0f;
            p.bwd.item_flag[item] = 0;
        }
        if (KIND != BWD_PROP)
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
    // dL/du_hat of active nodes starts from their own U (or the given gradient)
    const float *g0 = KIND == BWD_CONTACT ? p.grad_uhat_in : p.grad_u;
    for (int q = threadIdx.x; q < m; q += kWG) {
        const int j = alist[q];
        gh[j] = g0[row + j];
        gh[n_max + j] = g0[EN + row + j];
        gh[2 * n_max + j] = g0[2 * EN + row + j];
    }
    __syncthreads();
    double dalpha = 0.0;
    if (KIND != BWD_CONTACT) {
        const int np = n - m;
        if (p.model.mode != ETAC_RESIDUAL_ONLY && np > 0)
            dalpha = decay_adjoint(p, S, e, k, base, m, np, alist, plist, uhn, gh);
        if (uses_residual(p)) residual_adjoint(p, S, e, k, item, base, n, uhn, wobj, gh);
    }
    // dL/dalpha partial of the item
    {
        double v[12];
        v[0] = dalpha;
        for (int c = 1; c < 12; ++c) v[c] = 0.0;
        wg_sum12(S, v);
        if (threadIdx.x < 64) {
            p.bwd.alpha_part[item] = (float)v[0];
            p.bwd.item_flag[item] = (KIND != BWD_CONTACT && uses_residual(p)) ? 1 : 0;
        }
    }
    __syncthreads();
    if (KIND == BWD_PROP) {
        for (int i = threadIdx.x; i < n; i += kWG) {
            const bool act = wobj[i] >= 0;
            p.grad_uhat_out[row + i] = act ? gh[i] : 0.0f;
            p.grad_uhat_out[EN + row + i] = act ? gh[n_max + i] : 0.0f;
            p.grad_uhat_out[2 * EN + row + i] = act ? gh[2 * n_max + i] : 0.0f;
        }
    } else {
        contact_adjoint_item(p, S, e, item, base, m, alist, wobj, gh);
    }
    __syncthreads();
}

__device__ __forceinline__ int next_item_bwd(unsigned *counter, BwdLds &S) {
    if (threadIdx.x < 64) {
        const unsigned old = atomicAdd(&counter[2], lane_id() == 0 ? 1u : 0u);
        S.item = __shfl((int)old, 0);
    }
    __syncthreads();
    const int it = uniform(S.item);
    __syncthreads();
    return it;
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
    for (;;) {
        const int item = next_item_bwd(p.scr.counter, S);
        if (item >= p.n_items) break;
        const int e = item / p.mesh.K, k = item - e * p.mesh.K;
        process_item_bwd<KIND>(p, S, item, e, k, uhn, gh, alist, plist, wobj);
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
// fixed-order reductions of the per-item partials
// ---------------------------------------------------------------------------

// Ascending list of items that wrote a parameter-gradient partial.
__global__ __launch_bounds__(1024) void k_list_items(const int *flag, int n_items, int *list, int *n_list) {
    __shared__ int wsum[16];
    const int wave = threadIdx.x >> 6;
    int run = 0;   // identical in every thread
    for (int i0 = 0; i0 < n_items; i0 += 1024) {
        const int i = i0 + threadIdx.x;
        const bool f = i < n_items && flag[i] != 0;
        const unsigned long long b = __ballot(f);
        wsum[wave] = __popcll(b);
        __syncthreads();
        int off = run;
        int tot = 0;
        for (int w = 0; w < 16; ++w) {
            if (w < wave) off += wsum[w];
            tot += wsum[w];
        }
        if (f) list[off + lanes_below(b)] = i;
        run += uniform(tot);
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_list = run;
}

// Segment sums of the parameter partials in list order (FP64).
__global__ __launch_bounds__(256) void k_phi_segments(const float *part, const int *list, const int *n_list,
                                                      double *seg) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int s = blockIdx.y;
    const int nl = *n_list;
    const int per = (nl + kPhiSegs - 1) / kPhiSegs;
    const int a = s * per, b = min(nl, a + per);
    if (c >= kPhiN) return;
    double acc = 0.0;
    for (int q = a; q < b; ++q) acc += (double)part[(size_t)list[q] * kPhiN + c];
    seg[(size_t)s * kPhiN + c] = acc;
}

__global__ __launch_bounds__(256) void k_phi_final(const double *seg, float *grad_phi) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= kPhiN) return;
    double acc = 0.0;
    for (int s = 0; s < kPhiSegs; ++s) acc += seg[(size_t)s * kPhiN + c];
    grad_phi[c] = (float)acc;
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
                           const float *uhat_in, const float *grad_u, float *grad_uhat, float *grad_rot,
                           float *grad_trans, float *grad_alpha, float *grad_phi, hipStream_t st) {
    if (n_envs == 0) return hipSuccess;
    BwdParams p;
    p.mesh = pl.mesh;
    p.scene = s ? *s : SceneDev{nullptr, nullptr, nullptr, nullptr, nullptr, 0, 1};
    p.model = m;
    p.scr = pl.scr;
    p.bwd = pl.bwd;
    p.E = n_envs;
    p.n_items = n_envs * pl.K;
    p.cobj_in = cobj_in;
    p.uhat_in = uhat_in;
    p.grad_u = grad_u;
    p.grad_uhat_in = nullptr;
    p.grad_uhat_out = grad_uhat;
    const int grid = min(p.n_items, pl.cu_count);
    int slot = timer_begin(pl, ETAC_TIMER_BACKWARD, st);
    if (s) hipLaunchKernelGGL(k_bwd<BWD_STEP>, dim3(grid), dim3(kWG), 0, st, p);
    else hipLaunchKernelGGL(k_bwd<BWD_PROP>, dim3(grid), dim3(kWG), 0, st, p);
    hipError_t e = hipGetLastError();
    timer_end(pl, ETAC_TIMER_BACKWARD, slot, st);
    if (e != hipSuccess) return e;
    slot = timer_begin(pl, ETAC_TIMER_REDUCE, st);
    if (grad_phi) {
        hipLaunchKernelGGL(k_list_items, dim3(1), dim3(1024), 0, st, pl.bwd.item_flag, p.n_items, pl.bwd.item_list,
                           pl.bwd.n_list);
        hipLaunchKernelGGL(k_phi_segments, dim3((kPhiN + 255) / 256, kPhiSegs), dim3(256), 0, st, pl.bwd.phi_part,
                           pl.bwd.item_list, pl.bwd.n_list, pl.bwd.phi_seg);
        hipLaunchKernelGGL(k_phi_final, dim3((kPhiN + 255) / 256), dim3(256), 0, st, pl.bwd.phi_seg, grad_phi);
    }
    if (grad_alpha) hipLaunchKernelGGL(k_alpha, dim3(pl.K), dim3(256), 0, st, pl.bwd.alpha_part, n_envs, pl.K, grad_alpha);
    if (s) {
        const int nt = n_envs * s->O * 12;
        hipLaunchKernelGGL(k_pose, dim3((nt + 255) / 256), dim3(256), 0, st, pl.bwd.pose_part, n_envs, pl.K, s->O,
                           grad_rot, grad_trans);
    }
    e = hipGetLastError();
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
    p.cobj_in = nullptr;
    p.uhat_in = nullptr;
    p.grad_u = nullptr;
    p.grad_uhat_in = grad_uhat;
    p.grad_uhat_out = nullptr;
    const int grid = min(p.n_items, pl.cu_count);
    hipLaunchKernelGGL(k_bwd<BWD_CONTACT>, dim3(grid), dim3(kWG), 0, st, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nt = s.E * s.O * 12;
    hipLaunchKernelGGL(k_pose, dim3((nt + 255) / 256), dim3(256), 0, st, pl.bwd.pose_part, s.E, pl.K, s.O, grad_rot,
                       grad_trans);
    return hipGetLastError();
}

}  // namespace etac

// Forward kernels of the ETac step on gfx950:
//   k_contact : contact pass alone, one workgroup per env (HBM-write bound)
//   k_step    : persistent fused contact + propagation, one (env, patch) item
//               at a time per workgroup, items taken from a device work queue
//               in longest-patch-first order.  The same kernel, templated,
//               propagates given contact results (etac_propagate).
#include <mutex>

#include "etac_device.h"

namespace etac {

constexpr int kChunk = 1024;      // active nodes staged in LDS per pass of the decay loop

// ---------------------------------------------------------------------------
// contact pass alone
// ---------------------------------------------------------------------------
struct ContactParams {
    MeshDev mesh;
    SceneDev scene;
    int8_t *cobj;      // [E][N]
    float *uhat;       // [3][E][N] or null
    int32_t *n_active; // [E][K]
    int32_t *n_touch;  // [E][K] active nodes won by external objects, or null
};

// One workgroup per env.  The patches' candidate objects are culled first
// (one mask per patch in LDS), so nodes of patches no object reaches only
// store their empty result; the others are tested one node per thread,
// consecutive threads on consecutive nodes.  ROWS: the hand's candidate rows
// (ids mapped through src, object-won nodes counted).
template <bool ROWS>
__global__ __launch_bounds__(kWG) void k_contact(ContactParams p) {
    __shared__ int cnt[kMaxPatches];
    __shared__ int tcnt[ROWS ? kMaxPatches : 1];
    __shared__ unsigned cand[kMaxPatches];
    const int e = blockIdx.x;
    const MeshDev &M = p.mesh;
    const SceneDev &S = p.scene;
    const int N = M.N, K = M.K;
    const size_t EN = (size_t)S.E * N;
    for (int k = threadIdx.x; k < K; k += kWG) {
        cnt[k] = 0;
        if (ROWS) tcnt[k] = 0;
        cand[k] = ROWS ? cull_objects(S, M, e, k) : cull_objects(S, M, e, k, (size_t)e);
    }
    __syncthreads();
    const size_t row = (size_t)e * N;
    for (int i = threadIdx.x; i < N; i += kWG) {
        int best = -1;
        float u0 = 0.0f, u1 = 0.0f, u2 = 0.0f;
        const int k = M.node_patch[i];
        const unsigned c = cand[k];
        int8_t id = -1;
        if (c) {
            const size_t srow = ROWS ? scene_row(S, e, k) : (size_t)e;
            best = contact_node(S, srow, c, M.pos[i], M.pos[N + i], M.pos[2 * N + i], M.nrm[i], M.nrm[N + i],
                                M.nrm[2 * N + i], u0, u1, u2);
            if (best >= 0) {
                atomicAdd(&cnt[k], 1);
                id = (int8_t)best;
                if (ROWS) {
                    if (S.n_ext && best < S.n_ext[srow]) atomicAdd(&tcnt[k], 1);
                    if (S.src) id = S.src[srow * S.O + best];
                }
            }
        }
        // results stream out: non-temporal stores keep them from displacing cached inputs
        __builtin_nontemporal_store(id, p.cobj + row + i);
        if (p.uhat) {
            __builtin_nontemporal_store(u0, p.uhat + row + i);
            __builtin_nontemporal_store(u1, p.uhat + EN + row + i);
            __builtin_nontemporal_store(u2, p.uhat + 2 * EN + row + i);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += kWG) {
        p.n_active[(size_t)e * K + k] = cnt[k];
        if (ROWS && p.n_touch) p.n_touch[(size_t)e * K + k] = tcnt[k];
    }
}

hipError_t launch_contact(const Plan &p, const SceneDev &s, int8_t *cobj, float *uhat, int32_t *n_active,
                          hipStream_t st) {
    return launch_contact_rows(p, s, cobj, uhat, n_active, nullptr, st);
}

hipError_t launch_contact_rows(const Plan &p, const SceneDev &s, int8_t *cobj, float *uhat, int32_t *n_active,
                               int32_t *n_touch, hipStream_t st) {
    if (s.E == 0) return hipSuccess;
    ContactParams cp{p.mesh, s, cobj, uhat, n_active, n_touch};
    const int slot = timer_begin(p, ETAC_TIMER_CONTACT, st);
    if (s.rows_per_env) hipLaunchKernelGGL(k_contact<true>, dim3(s.E), dim3(kWG), 0, st, cp);
    else hipLaunchKernelGGL(k_contact<false>, dim3(s.E), dim3(kWG), 0, st, cp);
    const hipError_t e = hipGetLastError();
    timer_end(p, ETAC_TIMER_CONTACT, slot, st);
    return e;
}

// ---------------------------------------------------------------------------
// persistent fused step
// ---------------------------------------------------------------------------
struct StepParams {
    MeshDev mesh;
    SceneDev scene;
    ModelDev model;
    Scratch scr;
    int E;
    int n_items;
    int batch;               // queue positions claimed per atomic
    const int8_t *cobj_in;   // propagate-only: given contact results
    const float *uhat_in;
    float *u;                // [3][E][N]
    int8_t *cobj_out;        // [E][N] (fused step)
    int32_t *n_active;       // [E][K] (fused step)
    int32_t *n_touch;        // [E][K] active nodes won by external objects (hand), or null
    uint32_t *saved;         // [E K][kSavedWords] pooling record for the adjoint, or null
};

struct StepLds {
    NetLds net;
    union {
        struct {
            float4 act_a[kChunk];    // (px, py, pz, ux) of staged active nodes
            float2 act_b[kChunk];    // (uy, uz)
            double part[kWG][6];     // per-thread partial sums of its passive nodes (segment combine)
        };
        StageBuf xs;                 // node inputs of the network passes (before the decay)
    };
    int wcnt[3][kWaves];
    ItemBatch batch;
};

// Work queue: counter[0] hands out batches of kBatch items in queue order
// (patches by size, largest first; envs within a patch), counter[1] counts
// finished workgroups; the last workgroup resets both so the next launch (or
// graph replay) starts from zero without a host-side clear.
//
// Every block that only part of the workgroup executes is a whole wave (wave
// 0, storing identical values), and every item ends at a barrier: a block
// taken by single lanes next to a barrier lets the compiler thread the other
// lanes of the wave past it into the barrier, which deadlocks the queue.
__device__ __forceinline__ void retire(unsigned *counter) {
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned done = atomicAdd(&counter[1], 1u);
        if (done == gridDim.x - 1) {
            atomicExch(&counter[0], 0u);
            atomicExch(&counter[1], 0u);
        }
    }
}

// Zero deformation for a patch without contact (whole workgroup).
__device__ __forceinline__ void write_zero_item(const StepParams &p, int e, int base, int n, bool write_cobj) {
    const size_t EN = (size_t)p.E * p.mesh.N;
    const size_t row = (size_t)e * p.mesh.N + base;
    for (int i = threadIdx.x; i < n; i += kWG) {
        __builtin_nontemporal_store(0.0f, p.u + row + i);
        __builtin_nontemporal_store(0.0f, p.u + EN + row + i);
        __builtin_nontemporal_store(0.0f, p.u + 2 * EN + row + i);
        if (write_cobj) __builtin_nontemporal_store((int8_t)-1, p.cobj_out + row + i);
    }
}

// Outputs of the batch's items that no object can reach: U = 0, no contact,
// m = 0.  Wave w takes items w, w + 4, ...; no barrier is needed.
__device__ void zero_fill_batch(const StepParams &p, const ItemBatch &B, int b0) {
    const int batch = p.batch;
    const MeshDev &M = p.mesh;
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const unsigned long long live = batch_mask(B);
    const size_t EN = (size_t)p.E * M.N;
    for (int j = wave; j < batch; j += kWaves) {
        const int item = b0 + j;
        if (item >= p.n_items || ((live >> j) & 1ull)) continue;
        int e, k;
        queue_item(M, p.E, item, e, k);
        const int base = M.offset[k], n = M.offset[k + 1] - base;
        const size_t row = (size_t)e * M.N + base;
        for (int i = lane; i < n; i += 64) {
            __builtin_nontemporal_store(0.0f, p.u + row + i);
            __builtin_nontemporal_store(0.0f, p.u + EN + row + i);
            __builtin_nontemporal_store(0.0f, p.u + 2 * EN + row + i);
            __builtin_nontemporal_store((int8_t)-1, p.cobj_out + row + i);
        }
        p.n_active[(size_t)e * M.K + k] = 0;
        if (p.n_touch) p.n_touch[(size_t)e * M.K + k] = 0;
    }
}

// Residual network over the whole patch: max-pool pass over every node,
// global MLP, then the decoder pass writing r into `resid` ([3][n_max]) for
// the passive nodes (plist[0 .. np)), the only ones whose residual is used.
// The encoder is recomputed in the decoder pass instead of keeping n x 64
// features.  umax: the largest |u_hat| component of the item's nodes (with
// the patch's geometry it bounds the network inputs: the range scaling).
__device__ void residual_item(const StepParams &p, StepLds &S, const GmlpW &gw, int item, int k, int base, int n,
                              const float *uhn, const int *plist, int np, float *resid, float umax) {
    NetLds &L = S.net;
    const int lane = lane_id(), wave = threadIdx.x >> 6, gq = lane >> 4;
    const int n_max = p.scr.n_max;
    const ItemScale sc = item_scale(L, item_xbound(p.mesh, k, umax));
    item_biases(L, sc);    // published by the first stage barrier
    // max-pool with arg-max (lowest node on ties); f >= 0 beats the initial -1
    floatx4 mx[4];
    int mi[4][4];
    #pragma unroll
    for (int ot = 0; ot < 4; ++ot)
        #pragma unroll
        for (int r = 0; r < 4; ++r) { mx[ot][r] = -1.0f; mi[ot][r] = 0x7fffffff; }
    for (int c0 = 0; c0 < n; c0 += kStage) {
        const int cnt = min(kStage, n - c0);
        __syncthreads();
        stage_nodes(p.mesh, k, base, nullptr, c0, cnt, uhn, n_max, 0, sc.xmul, sc.xmul, S.xs);
        __syncthreads();
        // two tiles per wave step (t and t + kWaves); the second may be padding
        const int ntl = (cnt + 15) >> 4;
        for (int t = wave; t < ntl; t += 2 * kWaves) {
            bool valid[2];
            half8 xh[2], xl[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int lj = (t + u * kWaves) * 16 + (lane & 15);
                valid[u] = lj < cnt;
                stage_x<false>(S.xs, valid[u] ? lj : 0, valid[u], xh[u], xl[u]);
            }
            floatx4 f[2][4];
            encoder_tile2(L, xh, xl, f);
            // a lane meets its nodes in increasing order (tile t before t + kWaves)
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int node = c0 + (t + u * kWaves) * 16 + (lane & 15);
                if (valid[u])
                    #pragma unroll
                    for (int ot = 0; ot < 4; ++ot)
                        #pragma unroll
                        for (int r = 0; r < 4; ++r)
                            if (f[u][ot][r] > mx[ot][r]) { mx[ot][r] = f[u][ot][r]; mi[ot][r] = node; }
            }
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
    // the per-wave arg-maxes go to the node stage, free once every wave is done with it
    __syncthreads();
    int (*ipart)[64] = reinterpret_cast<int (*)[64]>(&S.xs[0][0]);
    // after the row reduction all 16 lanes of a row hold the same values (identical stores)
        #pragma unroll
        for (int ot = 0; ot < 4; ++ot)
            #pragma unroll
            for (int r = 0; r < 4; ++r) {
                L.part[wave][ot * 16 + 4 * gq + r] = mx[ot][r];
                ipart[wave][ot * 16 + 4 * gq + r] = mi[ot][r];
            }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int c = threadIdx.x;
        float v = L.part[0][c];
        int ix = ipart[0][c];
        for (int w = 1; w < kWaves; ++w) {
            const float v2 = L.part[w][c];
            const int i2 = ipart[w][c];
            if (v2 > v || (v2 == v && i2 < ix)) { v = v2; ix = i2; }
        }
        v *= pow2(-sc.af);    // the pooled feature, unscaled
        L.g[c] = v;
        if (p.saved) {
            uint32_t *rec = p.saved + (size_t)item * kSavedWords;
            rec[c] = __float_as_uint(v);
            rec[64 + c] = (uint32_t)ix;
        }
    }
    __syncthreads();
    global_mlp(L, gw, sc);
    const float r_mul = pow2(-sc.a4);
    for (int c0 = 0; c0 < np; c0 += kStage) {
        const int cnt = min(kStage, np - c0);
        __syncthreads();
        stage_nodes(p.mesh, k, base, plist, c0, cnt, nullptr, 0, 0, sc.xmul, 0.0f, S.xs);   // passive: U_hat = 0
        __syncthreads();
        // pairs of tiles (t, t + 4) per wave while every wave gets a pair,
        // then single tiles (the same residuals either way)
        const int ptl = (cnt + 15) >> 4;
        int t0 = 0;
        for (; ptl - t0 >= 2 * kWaves; t0 += 2 * kWaves) {
            int lj[2];
            bool valid[2];
            half8 xh[2], xl[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                lj[u] = (t0 + u * kWaves + wave) * 16 + (lane & 15);
                valid[u] = lj[u] < cnt;     // the chunk's last tile may be ragged
                stage_x<true>(S.xs, lj[u], valid[u], xh[u], xl[u]);
            }
            floatx4 f[2][4];
            encoder_tile2(L, xh, xl, f);
            float r[2][3];
            decoder_tile2(L, f, r_mul, r);
#pragma unroll
            for (int u = 0; u < 2; ++u)
                if (valid[u] && gq < 3) resid[gq * n_max + plist[c0 + lj[u]]] = r[u][gq];
        }
        for (int t = t0 + wave; t < ptl; t += kWaves) {
            const int lj = t * 16 + (lane & 15);
            const bool valid = lj < cnt;
            half8 xh, xl;
            stage_x<true>(S.xs, lj, valid, xh, xl);
            floatx4 h1[4], f[4], h4[4];
            encoder_tile(L, xh, xl, h1, f);
            float r[3];
            decoder_tile(L, f, r_mul, h4, r);
            if (valid && gq < 3) resid[gq * n_max + plist[c0 + lj]] = r[gq];
        }
    }
    __syncthreads();
}

// Stage active nodes [c0, c0 + cnt) of the item into LDS, positions times
// sc (|alpha| log2(e): distances then come out in units of the decay's
// exponent, see decay_range).
__device__ __forceinline__ void stage_active(const StepParams &p, StepLds &S, int base, const int *alist,
                                             const float *uhn, int c0, int cnt, float sc) {
    const MeshDev &M = p.mesh;
    const int N = M.N, n_max = p.scr.n_max;
    for (int t = threadIdx.x; t < cnt; t += kWG) {
        const int j = alist[c0 + t];
        const int gj = base + j;
        S.act_a[t] = make_float4(M.pos[gj] * sc, M.pos[N + gj] * sc, M.pos[2 * N + gj] * sc, uhn[j]);
        S.act_b[t] = make_float2(uhn[n_max + j], uhn[2 * n_max + j]);
    }
}

// Eq. 1 over staged active nodes [lo, hi) for P passive nodes per thread.
// Positions come scaled by |alpha| log2(e), so a pair's scaled distance d
// gives its weight exp(-alpha |p_j - p_i|) as 2^-d (2^d for alpha < 0: GROW).
// FP32 terms are summed in blocks of 32 and the block sums are accumulated
// in FP64.
// Runs of 32 staged actives that no valid passive node of the wave can reach
// within the cutoff are skipped (a run overlaps at most two boxes); cut2 < 0
// turns the cutoff off.
template <int P, bool GROW>
__device__ __forceinline__ void decay_range(const StepLds &S, const float4 *bb, float cut2, int lo, int hi,
                                            const bool (&v)[P], const float (&px)[P],
                                            const float (&py)[P], const float (&pz)[P], double (&acc)[P][3]) {
    for (int j0 = lo; j0 < hi; j0 += 32) {
        const int j1 = min(hi, j0 + 32);
        if (cut2 >= 0.0f) {   // uniform: the cutoff is on for this item
            // [j0, j1) overlaps boxes b0 and b1 (equal when aligned)
            const int b0 = j0 >> 5, b1 = (j1 - 1) >> 5;
            const float4 lo0 = bb[2 * b0], hi0 = bb[2 * b0 + 1], lo1 = bb[2 * b1], hi1 = bb[2 * b1 + 1];
            bool need = false;
#pragma unroll
            for (int a = 0; a < P; ++a)
                need = need || (v[a] && (box_d2(lo0, hi0, px[a], py[a], pz[a]) < cut2 ||
                                         box_d2(lo1, hi1, px[a], py[a], pz[a]) < cut2));
            if (__ballot(need) == 0ull) continue;   // wave-uniform
        }
        float sx[P], sy[P], sz[P];
#pragma unroll
        for (int a = 0; a < P; ++a) sx[a] = sy[a] = sz[a] = 0.0f;
        // the run's bounds are wave-uniform (segments are whole waves): scalar loop control
        const int je = uniform(j1);
#pragma unroll 4
        for (int j = uniform(j0); j < je; ++j) {
            const float4 pa = S.act_a[j];
            const float2 pb = S.act_b[j];
#pragma unroll
            for (int a = 0; a < P; ++a) {
                const float dx = pa.x - px[a], dy = pa.y - py[a], dz = pa.z - pz[a];
                const float d = __builtin_amdgcn_sqrtf(dx * dx + dy * dy + dz * dz);
                const float w = __builtin_amdgcn_exp2f(GROW ? d : -d);
                sx[a] += w * pa.w; sy[a] += w * pb.x; sz[a] += w * pb.y;
            }
        }
#pragma unroll
        for (int a = 0; a < P; ++a) { acc[a][0] += sx[a]; acc[a][1] += sy[a]; acc[a][2] += sz[a]; }
    }
}

// Passive nodes of one item: U = Omega U_a (Eq. 1) + residual.  Pairs are
// split over a grid of SLOTS passive slots x (kWG / SLOTS) active segments:
// every thread owns P passive nodes per pass and one segment of each staged
// chunk of active nodes; segment partials are combined in segment order.
// Active nodes are already staged when the item has one chunk.
template <int SLOTS, int P>
__device__ void decay_item(const StepParams &p, StepLds &S, int base, int m, int np, const int *alist,
                           const int *plist, const float *uhn, const float *resid, bool use_dec, bool use_res,
                           float sc, bool grow, float cut2, size_t row) {
    const MeshDev &M = p.mesh;
    const int N = M.N, n_max = p.scr.n_max;
    const size_t EN = (size_t)p.E * N;
    constexpr int nseg = kWG / SLOTS;
    const int slot = threadIdx.x % SLOTS, seg = threadIdx.x / SLOTS;
    const bool one_chunk = m <= kChunk;
    const float4 *bb = reinterpret_cast<const float4 *>(&S.net.part[0][0]);   // block boxes (free during the decay)
    for (int pb = 0; pb < np; pb += P * SLOTS) {
        bool v[P];
        int ii[P];
        float px[P], py[P], pz[P];
        double acc[P][3];
#pragma unroll
        for (int a = 0; a < P; ++a) {
            const int t = pb + slot + a * SLOTS;
            v[a] = t < np;
            ii[a] = v[a] ? plist[t] : 0;
            const int g = base + ii[a];
            px[a] = M.pos[g] * sc; py[a] = M.pos[N + g] * sc; pz[a] = M.pos[2 * N + g] * sc;
            acc[a][0] = acc[a][1] = acc[a][2] = 0.0;
        }
        if (use_dec) {
            if (one_chunk) {
                const int per = (m + nseg - 1) / nseg, lo = seg * per;
                if (grow) decay_range<P, true>(S, bb, cut2, lo, min(m, lo + per), v, px, py, pz, acc);
                else decay_range<P, false>(S, bb, cut2, lo, min(m, lo + per), v, px, py, pz, acc);
            } else {
                for (int c0 = 0; c0 < m; c0 += kChunk) {
                    const int cnt = min(kChunk, m - c0);
                    __syncthreads();
                    stage_active(p, S, base, alist, uhn, c0, cnt, sc);
                    __syncthreads();
                    if (cut2 >= 0.0f) {
                        block_boxes(S.act_a, cnt, reinterpret_cast<float4 *>(&S.net.part[0][0]));
                        __syncthreads();
                    }
                    const int per = (cnt + nseg - 1) / nseg, lo = seg * per;
                    if (grow) decay_range<P, true>(S, bb, cut2, lo, min(cnt, lo + per), v, px, py, pz, acc);
                    else decay_range<P, false>(S, bb, cut2, lo, min(cnt, lo + per), v, px, py, pz, acc);
                }
            }
            if (nseg > 1) {
                __syncthreads();
                double *mine = S.part[threadIdx.x];
#pragma unroll
                for (int a = 0; a < P; ++a) { mine[3 * a] = acc[a][0]; mine[3 * a + 1] = acc[a][1]; mine[3 * a + 2] = acc[a][2]; }
                __syncthreads();
                if (seg == 0)
                    for (int q = 1; q < nseg; ++q) {
                        const double *o = S.part[q * SLOTS + slot];
#pragma unroll
                        for (int a = 0; a < P; ++a) { acc[a][0] += o[3 * a]; acc[a][1] += o[3 * a + 1]; acc[a][2] += o[3 * a + 2]; }
                    }
            }
        }
        if (seg == 0)
#pragma unroll
            for (int a = 0; a < P; ++a)
                if (v[a]) {
                    const int i = ii[a];
                    if (use_res)
                        for (int c = 0; c < 3; ++c) acc[a][c] += (double)resid[c * n_max + i];
                    __builtin_nontemporal_store((float)acc[a][0], p.u + row + i);
                    __builtin_nontemporal_store((float)acc[a][1], p.u + EN + row + i);
                    __builtin_nontemporal_store((float)acc[a][2], p.u + 2 * EN + row + i);
                }
    }
}

// Same shape choice as the adjoint: fewest thread iterations over the
// np x m pairs, two nodes per thread weighted 1.75.  0..5 = (64|128|256) x (1|2).
__device__ __forceinline__ int decay_grid_shape(int np, int m) {
    int best = 5;
    float bc = 3.0e38f;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const int slots = 64 << (c % 3), a = 1 + c / 3, nseg = kWG / slots;
        const float cost = (float)((np + a * slots - 1) / (a * slots)) * (float)((m + nseg - 1) / nseg) *
                           (a == 2 ? 1.75f : 1.0f);
        if (cost < bc) { bc = cost; best = c; }
    }
    return best;
}

// One item with at least one candidate object (cand: objects that may reach
// the patch; all bits set when contact results are given).
template <bool FROM_INPUT>
__device__ void process_item(const StepParams &p, StepLds &S, const GmlpW &gw, int e, int k, unsigned cand, float *uhn,
                             float *resid, int *alist, int *plist) {
    const MeshDev &M = p.mesh;
    const int N = M.N, n_max = p.scr.n_max;
    const size_t EN = (size_t)p.E * N;
    const int base = M.offset[k];
    const int n = M.offset[k + 1] - base;
    const int mode = p.model.mode;
    float umax;
    int touch;
    const int m = contact_and_compact<FROM_INPUT, true>(M, p.scene, p.E, p.scr.n_max, p.cobj_in, p.uhat_in, p.cobj_out,
                                                  S.wcnt, e, k, base, n, cand, uhn, alist, plist, nullptr, umax,
                                                  touch);
    if (!FROM_INPUT && threadIdx.x < 64) {
        p.n_active[(size_t)e * M.K + k] = m;
        if (p.n_touch) p.n_touch[(size_t)e * M.K + k] = touch;
    }
    if (m == 0) {
        write_zero_item(p, e, base, n, false);
        __syncthreads();
        return;
    }
    const size_t row = (size_t)e * N + base;
    // active nodes keep their contact displacement
    for (int t = threadIdx.x; t < m; t += kWG) {
        const int i = alist[t];
        __builtin_nontemporal_store(uhn[i], p.u + row + i);
        __builtin_nontemporal_store(uhn[n_max + i], p.u + EN + row + i);
        __builtin_nontemporal_store(uhn[2 * n_max + i], p.u + 2 * EN + row + i);
    }
    const bool use_res = mode != ETAC_DECAY_ONLY, use_dec = mode != ETAC_RESIDUAL_ONLY;
    const int np = n - m;
    if (use_res) residual_item(p, S, gw, e * M.K + k, k, base, n, uhn, plist, np, resid, umax);
    // exp(-alpha d) = 2^-(alpha log2(e) d): positions are scaled by
    // sc = |alpha| log2(e), the cutoff D by the same factor (sc D = kCutLog2)
    const float alpha = p.model.alpha[k];
    const float sc = (float)(fabs((double)alpha) * 1.4426950408889634);
    const bool grow = alpha < 0.0f;
    const float cut2 = cutoff_useful(M, k, cutoff_d2(alpha)) ? kCut2Scaled : -1.0f;   // off: no boxes, no tests
    if (use_dec && m <= kChunk) {
        stage_active(p, S, base, alist, uhn, 0, m, sc);
        __syncthreads();
        if (cut2 >= 0.0f) {
            block_boxes(S.act_a, m, reinterpret_cast<float4 *>(&S.net.part[0][0]));
            __syncthreads();
        }
    }
    // with the decay off (residual only) every shape does the same work
    const int shape = use_dec ? uniform(decay_grid_shape(np, m)) : 5;
    switch (shape) {
        case 0: decay_item<64, 1>(p, S, base, m, np, alist, plist, uhn, resid, use_dec, use_res, sc, grow, cut2, row); break;
        case 1: decay_item<128, 1>(p, S, base, m, np, alist, plist, uhn, resid, use_dec, use_res, sc, grow, cut2, row); break;
        case 2: decay_item<256, 1>(p, S, base, m, np, alist, plist, uhn, resid, use_dec, use_res, sc, grow, cut2, row); break;
        case 3: decay_item<64, 2>(p, S, base, m, np, alist, plist, uhn, resid, use_dec, use_res, sc, grow, cut2, row); break;
        case 4: decay_item<128, 2>(p, S, base, m, np, alist, plist, uhn, resid, use_dec, use_res, sc, grow, cut2, row); break;
        default: decay_item<256, 2>(p, S, base, m, np, alist, plist, uhn, resid, use_dec, use_res, sc, grow, cut2, row); break;
    }
    __syncthreads();
}

template <bool FROM_INPUT>
__global__ __launch_bounds__(kWG) void k_step(StepParams p) {
    __shared__ StepLds S;
    const int wg = blockIdx.x;
    const int n_max = p.scr.n_max;
    float *uhn = p.scr.uhat_node + (size_t)wg * 3 * n_max;
    float *resid = p.scr.resid + (size_t)wg * 3 * n_max;
    int *alist = p.scr.alist + (size_t)wg * n_max;
    int *plist = p.scr.plist + (size_t)wg * n_max;
    GmlpW gw{};   // the global MLP's weights, held in registers across the items
    if (p.model.mode != ETAC_DECAY_ONLY) {
        stage_net(S.net, p.model.phi);
        gw = load_gmlp(p.model.phi);
        __syncthreads();
    }
    for (;;) {
        const int b0 = next_batch<FROM_INPUT ? CULL_NONE : CULL_OBJECTS>(p.scr.counter, S.batch, p.mesh, p.scene, p.E,
                                                                        p.n_items, p.batch);
        if (b0 >= p.n_items) break;
        if (!FROM_INPUT) zero_fill_batch(p, S.batch, b0);
        const int nb = uniform(S.batch.n);
        for (int q = 0; q < nb; ++q) {
            const int item = uniform(S.batch.item[q]);
            int e, k;
            queue_item(p.mesh, p.E, item, e, k);
            const unsigned cand = FROM_INPUT ? 0xffffffffu
                                             : item_cand(p.scene, e, k, uniform((unsigned)S.batch.cand[q]));
            process_item<FROM_INPUT>(p, S, gw, e, k, cand, uhn, resid, alist, plist);
        }
    }
    retire(p.scr.counter);
}

hipError_t launch_step(const Plan &pl, const SceneDev *s, const ModelDev &m, int n_envs,
                       const int8_t *cobj_in, const float *uhat_in, float *u, int8_t *cobj_out,
                       int32_t *n_active, uint32_t *saved, hipStream_t st, int32_t *n_touch) {
    if (n_envs == 0) return hipSuccess;
    StepParams p;
    p.mesh = pl.mesh;
    if (s) p.scene = *s;
    else p.scene = SceneDev{nullptr, nullptr, nullptr, nullptr, nullptr, 0, 1};
    p.model = m;
    p.scr = pl.scr;
    p.E = n_envs;
    p.n_items = n_envs * pl.K;
    p.batch = pl.batch;
    p.cobj_in = cobj_in;
    p.uhat_in = uhat_in;
    p.u = u;
    p.cobj_out = cobj_out;
    p.n_active = n_active;
    p.n_touch = n_touch;
    p.saved = saved;
    const int grid = p.n_items < pl.grid ? p.n_items : pl.grid;
    const int slot = timer_begin(pl, ETAC_TIMER_STEP, st);
    if (s) hipLaunchKernelGGL(k_step<false>, dim3(grid), dim3(kWG), 0, st, p);
    else hipLaunchKernelGGL(k_step<true>, dim3(grid), dim3(kWG), 0, st, p);
    const hipError_t e = hipGetLastError();
    timer_end(pl, ETAC_TIMER_STEP, slot, st);
    return e;
}

// ---------------------------------------------------------------------------
// the fused step with its scratch in a file-scope device array
//
// For callers that cannot allocate (code under stream capture, serving
// loops): the per-workgroup slices of the fused step (u_hat, residuals and
// node lists of the current item) and the work-queue counters live in
// `scratch`, which every device the library runs on holds until the process
// ends.  Host code uses only the array's device address, looked up once per
// device by static_scratch_init (at plan creation, with that device
// current); the array's name is never used as an address on the host.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_static_mu;
static void *g_static_ptr[kMaxDevices];

hipError_t static_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e == hipSuccess) g_static_ptr[device] = ptr;
    if (cur != device) {
        const hipError_t e2 = hipSetDevice(cur);
        if (e == hipSuccess) e = e2;
    }
    return e;
}

// Bytes of the array one persistent workgroup's slice needs: u_hat and
// residuals [3][n_max] floats, active and passive lists [n_max] ints.
size_t static_scratch_per_wg(int n_max) { return ((size_t)32 * (size_t)n_max + 255) / 256 * 256; }

// The work-queue counters start at zero (a fill kernel, not a memset, so that
// a captured graph replays it reliably).
__global__ __launch_bounds__(64) void k_clear_counters(unsigned *c) {
    if (threadIdx.x < 4) c[threadIdx.x] = 0u;
}

hipError_t launch_step_static(const Plan &pl, const SceneDev &s, const ModelDev &m, float *u, int8_t *cobj_out,
                              int32_t *n_active, uint32_t *saved, hipStream_t st) {
    void *base = nullptr;
    if (pl.device >= 0 && pl.device < kMaxDevices) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        base = g_static_ptr[pl.device];
    }
    if (!base) return hipErrorNotInitialized;
    if (s.E == 0) return hipSuccess;
    const size_t per_wg = static_scratch_per_wg(pl.n_max);
    const int n_items = s.E * pl.K;
    int grid = (int)std::min<size_t>((size_t)pl.grid, (kStaticScratchBytes - 256) / per_wg);
    grid = std::min(grid, n_items);
    if (grid < 1) return hipErrorInvalidValue;      // the caller checks the size first
    const size_t nm = (size_t)pl.n_max, g = (size_t)grid;
    char *b = static_cast<char *>(base);
    Scratch scr;
    scr.counter = reinterpret_cast<unsigned *>(b);
    scr.uhat_node = reinterpret_cast<float *>(b + 256);
    scr.resid = scr.uhat_node + g * 3 * nm;
    scr.alist = reinterpret_cast<int *>(scr.resid + g * 3 * nm);
    scr.plist = scr.alist + g * nm;
    scr.n_max = pl.n_max;
    StepParams p;
    p.mesh = pl.mesh;
    p.scene = s;
    p.model = m;
    p.scr = scr;
    p.E = s.E;
    p.n_items = n_items;
    p.batch = pl.batch;
    p.cobj_in = nullptr;
    p.uhat_in = nullptr;
    p.u = u;
    p.cobj_out = cobj_out;
    p.n_active = n_active;
    p.n_touch = nullptr;
    p.saved = saved;
    hipLaunchKernelGGL(k_clear_counters, dim3(1), dim3(64), 0, st, scr.counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int slot = timer_begin(pl, ETAC_TIMER_STEP, st);
    hipLaunchKernelGGL(k_step<false>, dim3(grid), dim3(kWG), 0, st, p);
    e = hipGetLastError();
    timer_end(pl, ETAC_TIMER_STEP, slot, st);
    return e;
}

}  // namespace etac

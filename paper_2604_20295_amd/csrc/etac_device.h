// Device building blocks of the ETac step on gfx950: the pinned FP64 contact
// predicate, the per-item active/passive compaction and the FP32-MFMA
// residual network tiles.
#pragma once

#include "etac_internal.h"

namespace etac {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Offsets of the packed network parameters (layout documented in etac.h).
constexpr int kW1 = 0, kB1 = 576, kW2 = 640, kB2 = 4736, kW3 = 4800, kB3 = 8896;
constexpr int kW4 = 8960, kB4 = 17152, kW5 = 17216, kB5 = 17408, kPhiN = 17411;

// ---------------------------------------------------------------------------
// contact (Sec. III-A: SDF contact of nodes with rigid objects)
// ---------------------------------------------------------------------------

struct Pen {
    bool inside;
    double depth, u0, u1, u2;
};

// Penetration of a node into one primitive.  FP64, every operation in the
// order written and rounded to nearest-even, no contraction into FMA:
//   d = p - t;  q_c = (R[0][c] d_0 + R[1][c] d_1) + R[2][c] d_2
//   sphere  : s = (d_0^2 + d_1^2) + d_2^2 < r^2,  depth = r - sqrt(s),
//             u = (depth / sqrt(s)) d
//   box     : |q_c| < h_c for all c; face = first argmin (h_c - |q_c|);
//             u = (sign(q_face) depth) R[:, face]  (sign(0) = +1)
//   capsule : z = clamp(q_2, -L, L), v = (q_0, q_1, q_2 - z), s = v.v < r^2,
//             u = (depth / sqrt(s)) R v
// A node on the centre point / axis segment gets depth r and u = -r n.
// Inside tests are sqrt-free; depth uses the correctly rounded FP64 sqrt, so
// the inside set and the deepest-object choice are reproducible bit for bit.
__device__ __forceinline__ Pen penetrate(int type, const float *sh, const float *R, const float *t,
                                         float px, float py, float pz, float nx, float ny, float nz) {
#pragma clang fp contract(off)
    Pen h;
    h.inside = false;
    h.depth = 0.0;
    h.u0 = h.u1 = h.u2 = 0.0;
    const double d0 = (double)px - (double)t[0];
    const double d1 = (double)py - (double)t[1];
    const double d2 = (double)pz - (double)t[2];
    if (type == ETAC_SPHERE) {
        const double r = (double)sh[0];
        const double s = (d0 * d0 + d1 * d1) + d2 * d2;
        if (!(s < r * r)) return h;
        h.inside = true;
        if (s == 0.0) {
            h.depth = r;
            h.u0 = -r * (double)nx; h.u1 = -r * (double)ny; h.u2 = -r * (double)nz;
            return h;
        }
        const double l = sqrt(s);
        h.depth = r - l;
        const double sc = h.depth / l;
        h.u0 = sc * d0; h.u1 = sc * d1; h.u2 = sc * d2;
        return h;
    }
    const double r00 = R[0], r01 = R[1], r02 = R[2];
    const double r10 = R[3], r11 = R[4], r12 = R[5];
    const double r20 = R[6], r21 = R[7], r22 = R[8];
    const double q0 = (r00 * d0 + r10 * d1) + r20 * d2;
    const double q1 = (r01 * d0 + r11 * d1) + r21 * d2;
    const double q2 = (r02 * d0 + r12 * d1) + r22 * d2;
    if (type == ETAC_BOX) {
        const double h0 = sh[0], h1 = sh[1], h2 = sh[2];
        if (!(fabs(q0) < h0)) return h;
        if (!(fabs(q1) < h1)) return h;
        if (!(fabs(q2) < h2)) return h;
        h.inside = true;
        double best = h0 - fabs(q0);
        int cs = 0;
        double qs = q0;
        const double s1 = h1 - fabs(q1);
        if (s1 < best) { best = s1; cs = 1; qs = q1; }
        const double s2 = h2 - fabs(q2);
        if (s2 < best) { best = s2; cs = 2; qs = q2; }
        h.depth = best;
        const double a = (qs >= 0.0) ? best : -best;
        const double c0 = cs == 0 ? r00 : (cs == 1 ? r01 : r02);
        const double c1 = cs == 0 ? r10 : (cs == 1 ? r11 : r12);
        const double c2 = cs == 0 ? r20 : (cs == 1 ? r21 : r22);
        h.u0 = a * c0; h.u1 = a * c1; h.u2 = a * c2;
        return h;
    }
    const double r = sh[0], L = sh[1];
    double z = q2;
    if (z < -L) z = -L;
    else if (z > L) z = L;
    const double v0 = q0, v1 = q1, v2 = q2 - z;
    const double s = (v0 * v0 + v1 * v1) + v2 * v2;
    if (!(s < r * r)) return h;
    h.inside = true;
    if (s == 0.0) {
        h.depth = r;
        h.u0 = -r * (double)nx; h.u1 = -r * (double)ny; h.u2 = -r * (double)nz;
        return h;
    }
    const double l = sqrt(s);
    h.depth = r - l;
    const double sc = h.depth / l;
    h.u0 = sc * ((r00 * v0 + r01 * v1) + r02 * v2);
    h.u1 = sc * ((r10 * v0 + r11 * v1) + r12 * v2);
    h.u2 = sc * ((r20 * v0 + r21 * v1) + r22 * v2);
    return h;
}

// Radius of a ball around the object's origin that contains the primitive.
__device__ __forceinline__ float bounding_radius(int type, const float *sh) {
    if (type == ETAC_SPHERE) return sh[0];
    if (type == ETAC_BOX) return sqrtf(sh[0] * sh[0] + sh[1] * sh[1] + sh[2] * sh[2]);
    return sh[0] + sh[1];
}

// Contact of one node with the candidate objects of scene row `row` (bit o
// of `cand`).  A cheap FP32 ball test with a relative margin of 1e-3 (far
// above FP32 rounding) skips objects that cannot contain the node; survivors
// take the exact FP64 test.  Deepest penetration wins, lowest index on ties.
// Returns the winning slot or -1; u is the winner's u_hat rounded to FP32.
__device__ __forceinline__ int contact_node(const SceneDev &S, size_t row, unsigned cand, float px, float py,
                                            float pz, float nx, float ny, float nz, float &u0, float &u1,
                                            float &u2) {
    int best = -1;
    double bd = 0.0, b0 = 0.0, b1 = 0.0, b2 = 0.0;
    const int no = min(S.n_obj[row], S.O);   // device contents are not validated on the host
    for (int o = 0; o < no; ++o) {
        if (!((cand >> o) & 1u)) continue;
        const size_t eo = row * S.O + o;
        const int ty = S.type[eo];
        const float *sh = S.shape + 4 * eo;
        const float *R = S.rot + 9 * eo;
        const float *t = S.trans + 3 * eo;
        const float dx = px - t[0], dy = py - t[1], dz = pz - t[2];
        const float rb = bounding_radius(ty, sh) * 1.001f + 1e-3f;
        if (dx * dx + dy * dy + dz * dz > rb * rb) continue;
        const Pen h = penetrate(ty, sh, R, t, px, py, pz, nx, ny, nz);
        if (h.inside && (best < 0 || h.depth > bd)) {
            best = o;
            bd = h.depth;
            b0 = h.u0; b1 = h.u1; b2 = h.u2;
        }
    }
    u0 = (float)b0; u1 = (float)b1; u2 = (float)b2;
    return best;
}

// dL/d(R, t) contribution of one active node from dL/du_hat = g (FP64),
// added to acc[0..8] (R, row-major) and acc[9..11] (t).
// The face / clamp choice repeats the forward's operation order.
__device__ inline void contact_adjoint_node(int type, const float *sh, const float *Rf, const float *tf, float px, float py,
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

// Conservative test that a primitive's bounding ball (centre t) may reach the
// ball b = (centre, radius): relative margins of 1e-3 and 1e-5, far above
// FP32 rounding.
__device__ __forceinline__ bool ball_reaches(const float4 &b, int type, const float *shape, const float *t) {
    const float dx = b.x - t[0], dy = b.y - t[1], dz = b.z - t[2];
    const float reach = (b.w + bounding_radius(type, shape)) * 1.001f + 1e-3f;
    const float d2 = dx * dx + dy * dy + dz * dz;
    return d2 * (1.0f - 1e-5f) <= reach * reach;
}

// Primitives of item (e, k)'s scene row whose bounding ball may reach patch
// k's bounding sphere (objects of other types, triangle meshes included, are
// ignored).
__device__ __forceinline__ unsigned cull_objects(const SceneDev &S, const MeshDev &M, int e, int k, size_t row) {
    unsigned cand = 0;
    const int no = min(S.n_obj[row], S.O);
    const float4 b = M.bound[k];
    for (int o = 0; o < no; ++o) {
        const size_t eo = row * S.O + o;
        if ((unsigned)S.type[eo] > (unsigned)ETAC_CAPSULE) continue;
        if (ball_reaches(b, S.type[eo], S.shape + 4 * eo, S.trans + 3 * eo)) cand |= 1u << o;
    }
    return cand;
}

__device__ __forceinline__ unsigned cull_objects(const SceneDev &S, const MeshDev &M, int e, int k) {
    return cull_objects(S, M, e, k, scene_row(S, e, k));
}

// ---------------------------------------------------------------------------
// wave helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Values that are equal across the workgroup but come from LDS must be made
// visibly uniform before they steer control flow that contains barriers:
// otherwise the compiler treats the branch as divergent and may split a wave
// around a barrier (e.g. one lane leaving to finish a store while the others
// re-enter the barrier and read stale LDS).
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ unsigned uniform(unsigned v) { return (unsigned)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ float uniform(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ unsigned lanes_below(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Maximum over the wave, returned in every lane.
__device__ __forceinline__ unsigned wave_or(unsigned v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v |= (unsigned)__shfl_xor((int)v, off);
    return v;
}
__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    return v;
}

// ---------------------------------------------------------------------------
// certified cutoff of the Eq. 1 pair sums
//
// Staged points are grouped in blocks of 32 consecutive list entries (node
// order, so spatially compact strips) with a bounding box each.  A wave skips
// a block when none of its own nodes lies within D of the box, where
// exp(-alpha D) = 2^-50: every skipped weight is below 2^-50, so a skipped
// block changes a sum by less than 2^-50 times the sum of its |terms|, far
// below FP32 rounding of the sums themselves.
// ---------------------------------------------------------------------------
constexpr double kCutLog2 = 50.0;
// The cutoff in units of the decay's exponent (positions scaled by
// |alpha| log2(e)): kCutLog2^2, rounded up.
constexpr float kCut2Scaled = (float)(kCutLog2 * kCutLog2 * (1.0 + 1e-6));

// D^2 for the item's alpha, rounded up (no cutoff when alpha <= 0).
__device__ __forceinline__ float cutoff_d2(float alpha) {
    if (!(alpha > 0.0f)) return __builtin_inff();
    const double d = kCutLog2 / ((double)alpha * 1.4426950408889634);
    return (float)(d * d * (1.0 + 1e-6));
}

// Boxes of the blocks of 32 among staged points pts[0 .. cnt): bb[2 b] =
// lower corner, bb[2 b + 1] = upper corner.  Thread t loads point t and each
// aligned group of 32 lanes reduces by shuffles.  The caller brackets it with
// barriers.
__device__ __forceinline__ void block_boxes(const float4 *pts, int cnt, float4 *bb) {
    for (int t0 = 0; t0 < cnt; t0 += kWG) {
        const int t = t0 + threadIdx.x;
        const bool ok = t < cnt;
        const float4 q = pts[ok ? t : 0];
        float lx = ok ? q.x : 3.0e38f, ly = ok ? q.y : 3.0e38f, lz = ok ? q.z : 3.0e38f;
        float hx = ok ? q.x : -3.0e38f, hy = ok ? q.y : -3.0e38f, hz = ok ? q.z : -3.0e38f;
#pragma unroll
        for (int off = 16; off >= 1; off >>= 1) {
            lx = fminf(lx, __shfl_xor(lx, off)); ly = fminf(ly, __shfl_xor(ly, off)); lz = fminf(lz, __shfl_xor(lz, off));
            hx = fmaxf(hx, __shfl_xor(hx, off)); hy = fmaxf(hy, __shfl_xor(hy, off)); hz = fmaxf(hz, __shfl_xor(hz, off));
        }
        if ((t & 31) == 0 && ok) {
            bb[2 * (t >> 5)] = make_float4(lx, ly, lz, 0.0f);
            bb[2 * (t >> 5) + 1] = make_float4(hx, hy, hz, 0.0f);
        }
    }
}

// Whether the cutoff can skip anything in patch k: only if the patch is wider
// than D (its bounding sphere's diameter exceeds the cutoff radius).
__device__ __forceinline__ bool cutoff_useful(const MeshDev &M, int k, float cut2) {
    const float d = 2.0f * M.bound[k].w;
    return d * d > cut2;
}

// Squared distance from (x, y, z) to the box [lo, hi].
__device__ __forceinline__ float box_d2(const float4 &lo, const float4 &hi, float x, float y, float z) {
    const float dx = fmaxf(fmaxf(lo.x - x, x - hi.x), 0.0f);
    const float dy = fmaxf(fmaxf(lo.y - y, y - hi.y), 0.0f);
    const float dz = fmaxf(fmaxf(lo.z - z, z - hi.z), 0.0f);
    return dx * dx + dy * dy + dz * dz;
}

// ---------------------------------------------------------------------------
// batched work queue
//
// The persistent kernels claim `batch` (1 .. kBatch) consecutive queue
// positions per atomic.
// Queue position q maps to patch order[q / E] (patches by node count, largest
// first) and env q % E.  Wave 0 culls the whole batch at once, one item per
// lane; only items that some object may reach are processed one by one, the
// rest only need their zero outputs.
// ---------------------------------------------------------------------------
constexpr int kBatch = 64;

struct ItemBatch {
    int item[kBatch];          // queue positions of the live items, ascending
    uint8_t cand[kBatch];      // their candidate-object masks
    unsigned mask_lo, mask_hi; // live items as a bit mask over the batch
    int n;                     // number of live items
    int b0;                    // first queue position of the batch
};

__device__ __forceinline__ void queue_item(const MeshDev &M, int E, int q, int &e, int &k) {
    const int kk = q / E;
    e = q - kk * E;
    k = M.order[kk];
}

__device__ __forceinline__ unsigned long long batch_mask(const ItemBatch &B) {
    return ((unsigned long long)uniform(B.mask_hi) << 32) | (unsigned long long)uniform(B.mask_lo);
}

// How a claimed batch is culled.
enum CullMode {
    CULL_NONE = 0,      // every item is live (contact results are given)
    CULL_OBJECTS = 1,   // live if some object's bounding ball may reach the patch
    CULL_LIST = 2       // positions index a list of live queue positions (live[q])
};

// Claim the next batch and cull it.  Returns the batch's first position
// (>= n_items when the queue is empty); B.item holds the live items' queue
// positions.
template <int CULL>
__device__ int next_batch(unsigned *counter, ItemBatch &B, const MeshDev &M, const SceneDev &Sc, int E,
                          int n_items, int batch, const int *list = nullptr) {
    __syncthreads();   // every wave is done with the previous batch
    if (threadIdx.x < 64) {
        const int lane = lane_id();
        // one atomic for the wave (lane 0 adds `batch`), every lane learns the result
        const unsigned old = atomicAdd(&counter[0], lane == 0 ? (unsigned)batch : 0u);
        const int b0 = __shfl((int)old, 0);
        const int q = b0 + lane;
        unsigned cand = 0;
        if (lane < batch && q < n_items) {
            if (CULL == CULL_OBJECTS) {
                int e, k;
                queue_item(M, E, q, e, k);
                cand = cull_objects(Sc, M, e, k);
            } else {
                cand = 0xffu;
            }
        }
        const unsigned long long live = __ballot(cand != 0u);
        if (cand != 0u) {
            const int slot = (int)lanes_below(live);
            B.item[slot] = CULL == CULL_LIST ? list[q] : q;
            // a row scene's mask may use all 32 bits: the item recomputes it (item_cand)
            B.cand[slot] = (uint8_t)(Sc.rows_per_env ? 1u : cand);
        }
        // identical values from every lane
        B.mask_lo = (unsigned)live;
        B.mask_hi = (unsigned)(live >> 32);
        B.n = __popcll(live);
        B.b0 = b0;
    }
    __syncthreads();
    return uniform(B.b0);
}

// Candidate mask of an item taken from a batch: the batch keeps 8 bits per
// item, enough for env rows (at most ETAC_MAX_OBJ objects).  An item row of
// the hand holds only candidates that passed the same ball test when the row
// was filled, so its mask is every slot of the row.
__device__ __forceinline__ unsigned item_cand(const SceneDev &S, int e, int k, unsigned stored) {
    if (!S.rows_per_env) return stored;
    const int n = min(S.n_obj[scene_row(S, e, k)], S.O);
    return uniform(n >= 32 ? ~0u : (1u << n) - 1u);
}

// Contact (or given contact results) for every node of one (env, patch)
// item, then the active and passive node lists in ascending node order
// (wave ballots, prefix over waves).  Writes u_hat of every node into `uhn`
// ([3][n_max], 0 on passive nodes), the winner's slot into `wobj` when
// given, and contact_obj into `cobj_out` when computing contact (the
// winner's source id for a row scene with `src`).  Returns m; `touch`
// counts the active nodes won by external objects (slots below the row's
// n_ext; 0 without n_ext).  IDS = false (the adjoint's hand-over) skips the
// id mapping and the touch count.
template <bool FROM_INPUT, bool IDS = false>
__device__ int contact_and_compact(const MeshDev &M, const SceneDev &Sc, int E, int n_max, const int8_t *cobj_in,
                                   const float *uhat_in, int8_t *cobj_out, int (&wcnt)[3][kWaves], int e, int k,
                                   int base, int n, unsigned cand, float *uhn, int *alist, int *plist,
                                   int8_t *wobj, float &umax, int &touch) {
    const int N = M.N;
    const size_t EN = (size_t)E * N;
    const int wave = threadIdx.x >> 6;
    const size_t srow = FROM_INPUT ? 0 : scene_row(Sc, e, k);
    const int n_ext = (IDS && !FROM_INPUT && Sc.n_ext) ? uniform(Sc.n_ext[srow]) : 0;
    int run_a = 0, run_p = 0, run_t = 0;
    int ubits = 0;   // largest |u_hat| component of this thread's nodes (bits of a non-negative float)
    for (int i0 = 0; i0 < n; i0 += kWG) {
        const int i = i0 + threadIdx.x;
        const bool valid = i < n;
        int best = -1;
        float u0 = 0.0f, u1 = 0.0f, u2 = 0.0f;
        if (valid) {
            const int gi = base + i;
            const size_t en = (size_t)e * N + gi;
            if (FROM_INPUT) {
                best = cobj_in[en] >= 0 ? (int)cobj_in[en] : -1;
                if (best >= 0) {
                    u0 = uhat_in[en];
                    u1 = uhat_in[EN + en];
                    u2 = uhat_in[2 * EN + en];
                }
            } else {
                best = contact_node(Sc, srow, cand, M.pos[gi], M.pos[N + gi], M.pos[2 * N + gi], M.nrm[gi],
                                    M.nrm[N + gi], M.nrm[2 * N + gi], u0, u1, u2);
                if (cobj_out)
                    cobj_out[en] = (IDS && best >= 0 && Sc.src) ? Sc.src[srow * Sc.O + best] : (int8_t)best;
            }
            uhn[i] = u0;
            uhn[n_max + i] = u1;
            uhn[2 * n_max + i] = u2;
            if (wobj) wobj[i] = (int8_t)best;
            ubits = max(ubits, __float_as_int(fmaxf(fmaxf(fabsf(u0), fabsf(u1)), fabsf(u2))));
        }
        const bool act = valid && best >= 0, pas = valid && best < 0;
        const unsigned long long ba = __ballot(act), bp = __ballot(pas), bt = IDS ? __ballot(act && best < n_ext) : 0ull;
        // every lane stores the same wave counts (no single-lane block next to
        // the barrier); external-object touches ride in the upper half-word
        wcnt[0][wave] = __popcll(ba) | (__popcll(bt) << 16);
        wcnt[1][wave] = __popcll(bp);
        wcnt[2][wave] = wave_max_int(ubits);
        __syncthreads();
        int oa = run_a, op = run_p, ta = 0, tp = 0, tt = 0;
        for (int w = 0; w < kWaves; ++w) {
            const int ca = wcnt[0][w] & 0xffff;
            if (w < wave) { oa += ca; op += wcnt[1][w]; }
            ta += ca;
            tp += wcnt[1][w];
            tt += wcnt[0][w] >> 16;
        }
        if (act) alist[oa + lanes_below(ba)] = i;
        if (pas) plist[op + lanes_below(bp)] = i;
        run_a += uniform(ta);
        run_p += uniform(tp);
        run_t += uniform(tt);
        if (i0 + kWG >= n) {   // last chunk: the wave maxima cover every node of the item
            int ub = 0;
            for (int w = 0; w < kWaves; ++w) ub = max(ub, wcnt[2][w]);
            umax = __int_as_float(uniform(ub));
        }
        __syncthreads();
    }
    touch = run_t;
    return uniform(run_a);
}

// ---------------------------------------------------------------------------
// residual network Phi on MFMA with split-FP16 operands
//
// Every FP32 operand x is split as x = hi + lo with hi = fp16(x) and
// lo = fp16(x - hi) (22 significant bits together), and a product is taken as
// hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_f16 with FP32 accumulation.
// The dropped lo*lo term is ~2^-22 relative, so a layer keeps FP32-level
// accuracy at the FP16 matrix rate (about 5x the FP32 matrix rate).
//
// Range.  The pair keeps 22 bits only while |x| lies in [2^-3, 2^15]: above
// 65504 hi overflows, below 2^-3 lo is subnormal (absolute floor 2^-25).  So
// every split operand carries a power-of-two scale that keeps it below 2^15
// (T) with its bound within a factor two of T; a block's small elements then
// lose relative precision only below 2^-40 of that bound.  The node inputs
// are scaled per item (2^ax from X, the largest |component| of the item's
// inputs, at least 1).  The weights are scaled per launch by constants
// chosen from their infinity norms (largest row sum of |w|, or column sum
// for a transposed use) so that the products land below T without a
// rescale: |h1| <= (||W1|| + 2 max|b1|) T 2^s1 < T for inputs below T, and so
// on through the layers.  The biases follow the item's scales.  Powers of
// two are exact: the scaling changes no value beyond the rounding of the
// splits.  (A weight block whose scaled maximum falls below 2^-3 keeps
// 2^-25 absolute accuracy, about 2^-19 of its largest element at worst.)
//
// A 16-node tile is processed by one wave in transposed form, Y^T = W X^T:
// the MFMA's M dimension is the layer's output features, N the 16 nodes, K the
// input features.  Lane l holds node (l & 15).  After a layer it holds output
// features 16 ot + 4 (l >> 4) + r (r = 0..3) of out-tile ot in register r of
// accumulator ot.  The next layer's K dimension is ordered so that these same
// registers are its B operand: in K step s, lane group q = l >> 4 supplies
// inputs 16 (2 s + (e >> 2)) + 4 q + (e & 3) for e = 0..7.  Weight fragments
// are pre-arranged in LDS in that order (hi and lo halves), so every A
// operand is one 16-byte LDS read.
// ---------------------------------------------------------------------------
typedef _Float16 half8 __attribute__((ext_vector_type(8)));

constexpr int kTopExp = 15;   // scaled operand bounds lie in [2^14, 2^15): T = 2^15
constexpr float kTop = 32768.0f;

// Exponent s of the scale 2^s that puts `bound` in [2^(kTopExp-1), 2^kTopExp);
// 0 for a zero or non-finite bound; clamped to [-100, 100].
__device__ __forceinline__ int range_exp(float bound) {
    if (!(bound > 0.0f) || !(bound <= 3.0e38f)) return 0;
    int e;
    (void)frexpf(bound, &e);   // bound = m 2^e, m in [0.5, 1)
    return max(-100, min(100, kTopExp - e));
}

// 2^s, exact for -149 <= s <= 127 (subnormal below -126).
__device__ __forceinline__ float pow2(int s) { return ldexpf(1.0f, s); }

// Scales of one item's activations (uniform; every thread computes the same
// values).  X bounds every component of the item's node inputs.
// Scales of one item's activations: x at 2^ax, h1 at 2^a1 = 2^(s1 + ax),
// f at 2^af = 2^(s2 + a1), h4 at 2^a4 = 2^(s4 + af).
struct ItemScale {
    int ax, a1, af, a4;
    float xmul;          // 2^ax
};

struct NetLds {
    half8 w1h[4 * 64], w1l[4 * 64];          // [ot][lane]    W1 2^s1, inputs padded 9 -> 32 (one K step)
    half8 w2h[4 * 2 * 64], w2l[4 * 2 * 64];  // [ot2][s][lane] W2 2^s2
    half8 w4h[4 * 2 * 64], w4l[4 * 2 * 64];  // [ot2][s][lane] W4 columns 0..63 (per-node part) 2^s4
    float b1[64], b2[64];
    float b1s[64], b2s[64];                  // per item: b1 2^a1, b2 2^af
    float c4[64];                            // per item: (W4[:, 64:] g' + b4) 2^a4
    float w5[3 * 64];
    float b5[4];
    float g[64], gp[64];                     // pooled feature and global MLP output (unscaled)
    float part[kWaves][64];                  // per-wave partials
    // per launch: scale exponents of the staged weights (W1 2^s1, W2 2^s2,
    // W4[:, :64] 2^s4) and of the adjoint's transposed uses (W5^T 2^c5t,
    // W4[:, :64]^T 2^s4t, W2^T 2^s2t)
    int s1, s2, s4, c5t, s4t, s2t;
    float mw2;               // max |W2|
    ItemScale isc;           // per item: the activation scales (a copy for readers that re-read them)
};

typedef _Float16 half2t __attribute__((ext_vector_type(2)));
typedef unsigned uint2t __attribute__((ext_vector_type(2)));
typedef unsigned uint4t __attribute__((ext_vector_type(4)));

// x - (float)h exactly, for h the FP16 value in the low (HI_HALF false) or
// high half of a packed register: one v_fma_mix_f32 (-h * 1.0 + x with the
// FP16 operand converted inside the instruction).
template <bool HI_HALF>
__device__ __forceinline__ float sub_f16(float x, unsigned h2) {
    float r;
    if (HI_HALF) asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(h2), "v"(x));
    else asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(h2), "v"(x));
    return r;
}

// Split two floats: hi = fp16(a), fp16(b) packed; lo = fp16 of the exact
// remainders.  Four instructions per pair.
__device__ __forceinline__ void split2(float a, float b, unsigned &hi, unsigned &lo) {
    const half2t h = {(_Float16)a, (_Float16)b};
    hi = __builtin_bit_cast(unsigned, h);
    const half2t l = {(_Float16)sub_f16<false>(a, hi), (_Float16)sub_f16<true>(b, hi)};
    lo = __builtin_bit_cast(unsigned, l);
}

__device__ __forceinline__ void split8(const float v[8], half8 &hi, half8 &lo) {
    uint4t h, l;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        unsigned a, b;
        split2(v[2 * e], v[2 * e + 1], a, b);
        h[e] = a;
        l[e] = b;
    }
    hi = __builtin_bit_cast(half8, h);
    lo = __builtin_bit_cast(half8, l);
}

// Input feature of K step s, lane group q, element e of a 64 -> 64 layer.
__device__ __forceinline__ int chain_k(int s, int q, int e) { return 16 * (2 * s + (e >> 2)) + 4 * q + (e & 3); }

// Per-launch quantities of the range scaling (whole workgroup; the caller
// brackets it with barriers).  Wave w takes rows (or columns) 16 w + (l & 15);
// lane group q = l >> 4 sums a quarter of each, the quarters are added with
// two shuffles and the wave's largest sum goes to L.part.
__device__ void net_norms(NetLds &L, const float *phi) {
    const int lane = lane_id(), wave = threadIdx.x >> 6, q = lane >> 4;
    const int r = 16 * wave + (lane & 15);
    float s1 = 0.0f, s2 = 0.0f, s4 = 0.0f, t2 = 0.0f, t4 = 0.0f, t5 = 0.0f;
    float m2 = 0.0f, m4 = 0.0f, mb1 = 0.0f, mb2 = 0.0f;
    for (int c = 16 * q; c < 16 * q + 16; ++c) {
        const float a = fabsf(phi[kW2 + r * 64 + c]), b = fabsf(phi[kW4 + r * 128 + c]);
        s2 += a; s4 += b;
        m2 = fmaxf(m2, a); m4 = fmaxf(m4, b);
        t2 += fabsf(phi[kW2 + c * 64 + r]);
        t4 += fabsf(phi[kW4 + c * 128 + r]);
    }
    if (q == 0) {
        for (int c = 0; c < 9; ++c) s1 += fabsf(phi[kW1 + r * 9 + c]);
        for (int c = 0; c < 3; ++c) t5 += fabsf(phi[kW5 + c * 64 + r]);
        mb1 = fabsf(phi[kB1 + r]);
        mb2 = fabsf(phi[kB2 + r]);
    }
    float v[10] = {s1, s2, s4, t2, t4, t5, m2, m4, mb1, mb2};
#pragma unroll
    for (int j = 0; j < 6; ++j) {   // sums over the four quarters
        v[j] += __shfl_xor(v[j], 16);
        v[j] += __shfl_xor(v[j], 32);
    }
#pragma unroll
    for (int j = 0; j < 10; ++j) {
        v[j] = wave_max(v[j]);
        L.part[wave][j] = v[j];      // identical in every lane
    }
}

// Stage the network into LDS in fragment order (whole workgroup), each
// weight matrix scaled by its per-launch power of two, and set the scale
// exponents.  With inputs x 2^ax below T (X at least 1, so 2^ax <= 2T):
//   h1 = W1 2^s1 x + b1 2^a1:  |h1| <= (||W1|| + 2 max|b1|) T 2^s1 < T,
//   f  = W2 2^s2 h1 + b2 2^af: |f| <= (||W2|| T + 2 max|b2| T 2^s1) 2^s2 < T,
//   h4 = W4 2^s4 f + c4 2^a4 with s4 from max |W4[:, :64]| (h4 is never split).
// Adjoint, with dL/dU 2^dre below T: W5^T 2^c5t, W4[:, :64]^T 2^s4t and W2^T
// 2^s2t by their column norms keep dL/dpre4, dL/dpre2 and dL/dpre1 below T.
// Ends with a barrier.
__device__ void stage_net(NetLds &L, const float *phi) {
    const int tid = threadIdx.x;
    net_norms(L, phi);
    __syncthreads();
    float v[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) {
        v[j] = L.part[0][j];
        for (int w = 1; w < kWaves; ++w) v[j] = fmaxf(v[j], L.part[w][j]);
    }
    const float n1 = v[0], n2 = v[1], n4t = v[4], n2t = v[3], n5t = v[5];
    const float mw2 = v[6], mw4 = v[7], mb1 = v[8], mb2 = v[9];
    const int s1 = range_exp((n1 + 2.0f * mb1) * kTop);
    const int s2 = range_exp((n2 * kTop + 2.0f * mb2 * kTop * pow2(s1)));
    const int s4 = range_exp(mw4);
    const float e1 = pow2(s1), e2 = pow2(s2), e4 = pow2(s4);
    for (int idx = tid; idx < 4 * 64; idx += kWG) {
        const int lane = idx & 63, ot = idx >> 6, q = lane >> 4;
        float x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int in = 8 * q + e;
            x[e] = in < 9 ? phi[kW1 + (ot * 16 + (lane & 15)) * 9 + in] * e1 : 0.0f;
        }
        split8(x, L.w1h[idx], L.w1l[idx]);
    }
    for (int idx = tid; idx < 4 * 2 * 64; idx += kWG) {
        const int lane = idx & 63, s = (idx >> 6) & 1, ot2 = idx >> 7, q = lane >> 4;
        const int out = ot2 * 16 + (lane & 15);
        float a[8], b[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int in = chain_k(s, q, e);
            a[e] = phi[kW2 + out * 64 + in] * e2;
            b[e] = phi[kW4 + out * 128 + in] * e4;
        }
        split8(a, L.w2h[idx], L.w2l[idx]);
        split8(b, L.w4h[idx], L.w4l[idx]);
    }
    for (int i = tid; i < 64; i += kWG) {
        L.b1[i] = phi[kB1 + i];
        L.b2[i] = phi[kB2 + i];
    }
    for (int i = tid; i < 192; i += kWG) L.w5[i] = phi[kW5 + i];
    for (int i = tid; i < 4; i += kWG) L.b5[i] = i < 3 ? phi[kB5 + i] : 0.0f;
    if (tid < 64) {   // wave 0, identical values
        L.s1 = s1; L.s2 = s2; L.s4 = s4;
        L.c5t = range_exp(n5t * kTop);
        L.s4t = range_exp(n4t * kTop);
        L.s2t = range_exp(n2t * kTop);
        L.mw2 = mw2;
    }
    __syncthreads();
}

// Scales of the activations of an item whose inputs are bounded by X
// (uniform; every thread computes the same values, kept in scalar registers).
__device__ __forceinline__ ItemScale item_scale(const NetLds &L, float X) {
    ItemScale s;
    s.ax = uniform(range_exp(fmaxf(X, 1.0f)));
    s.a1 = uniform(L.s1) + s.ax;
    s.af = uniform(L.s2) + s.a1;
    s.a4 = uniform(L.s4) + s.af;
    s.xmul = uniform(pow2(s.ax));
    return s;
}

// Scaled biases of the item's encoder layers and a copy of the scales in
// L.isc (threads < 64; the caller's next barrier publishes them).
__device__ __forceinline__ void item_biases(NetLds &L, const ItemScale &s) {
    if (threadIdx.x < 64) {
        const int i = threadIdx.x;
        L.b1s[i] = L.b1[i] * pow2(s.a1);
        L.b2s[i] = L.b2[i] * pow2(s.af);
        L.isc = s;   // identical values from every lane
    }
}

// The item's scales as published by item_biases, in scalar registers.
__device__ __forceinline__ ItemScale item_scale_lds(const NetLds &L) {
    ItemScale s;
    s.ax = uniform(L.isc.ax);
    s.a1 = uniform(L.isc.a1);
    s.af = uniform(L.isc.af);
    s.a4 = uniform(L.isc.a4);
    s.xmul = uniform(L.isc.xmul);
    return s;
}

// Input bound of item (patch k) given the largest |u_hat| component of its nodes.
__device__ __forceinline__ float item_xbound(const MeshDev &M, int k, float umax) {
    return fmaxf(M.xbound[k], umax);
}

// Keeps the compiler from hoisting the (loop-invariant) LDS weight-fragment
// loads of a tile out of the node loops: hoisted, they would need ~280 extra
// registers per lane and spill.  Emits no instruction.
__device__ __forceinline__ void reload_fence() { asm volatile("" ::: "memory"); }

__device__ __forceinline__ floatx4 mfma16(const half8 &a, const half8 &b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// acc += A B with split operands (hi*hi + hi*lo + lo*hi)
__device__ __forceinline__ floatx4 mfma_split(const half8 &ah, const half8 &al, const half8 &bh, const half8 &bl,
                                              floatx4 acc) {
    acc = mfma16(ah, bh, acc);
    acc = mfma16(ah, bl, acc);
    return mfma16(al, bh, acc);
}

// max(x, 0) as a signed-integer max of the bits: negative floats (and -0)
// have negative bit patterns; one instruction, no NaN canonicalisation.
__device__ __forceinline__ float relu1(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

__device__ __forceinline__ floatx4 relu4(floatx4 v) {
    floatx4 o;
#pragma unroll
    for (int r = 0; r < 4; ++r) o[r] = relu1(v[r]);
    return o;
}

// Split a D-layout 64-feature tile into the B operands of the two K steps of
// the next 64 -> 64 layer.
__device__ __forceinline__ void split_chain(const floatx4 x[4], half8 bh[2], half8 bl[2]) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = x[2 * s + (e >> 2)][e & 3];
        split8(v, bh[s], bl[s]);
    }
}

// Network input of this lane's node, scaled by xmul: lane group q = lane >> 4
// supplies input features 8 q .. 8 q + 7 of [p - o_k (3), n (3), U_hat (3)],
// zero padded to 32.
__device__ __forceinline__ void load_x_raw(const MeshDev &M, int k, int gnode, bool valid, const float *uhn,
                                           int n_max, int lnode, float xmul, float (&v)[8]) {
    const int q = lane_id() >> 4;
    const int N = M.N;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = 0.0f;
    if (valid && q == 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            v[a] = (M.pos[(size_t)a * N + gnode] - M.origin[3 * k + a]) * xmul;
            v[3 + a] = M.nrm[(size_t)a * N + gnode] * xmul;
        }
        v[6] = uhn[lnode] * xmul;
        v[7] = uhn[(size_t)n_max + lnode] * xmul;
    } else if (valid && q == 1) {
        v[0] = uhn[(size_t)2 * n_max + lnode] * xmul;
    }
}

// y = W x + acc over the two K steps of a 64 -> 64 layer in T form; the three
// split passes run pass-outermost over the four output blocks, so no MFMA
// waits on the one before it (each block sees hi*hi, hi*lo, lo*hi per step).
__device__ __forceinline__ void layer64_t(const half8 *wh, const half8 *wl, const half8 bh[2], const half8 bl[2],
                                          floatx4 acc[4]) {
    const int lane = lane_id();
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        half8 h[4], l[4];
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            h[ot] = wh[(ot * 2 + s) * 64 + lane];
            l[ot] = wl[(ot * 2 + s) * 64 + lane];
        }
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) acc[ot] = mfma16(h[ot], bh[s], acc[ot]);
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) acc[ot] = mfma16(h[ot], bl[s], acc[ot]);
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) acc[ot] = mfma16(l[ot], bh[s], acc[ot]);
    }
}

// ---------------------------------------------------------------------------
// node inputs staged in LDS for the network passes
//
// xs[f][j], f = 0..8: [p - o_k (3), n (3), a third triple] of staged node j.
// The third triple is U_hat (network input) or, in the adjoint's pass over
// passive nodes, dL/dU (U_hat is 0 there).  One parallel gather per chunk of
// kStage nodes replaces dependent global loads per 16-node tile.
// ---------------------------------------------------------------------------
constexpr int kStage = 1024;
typedef float StageBuf[9][kStage];

// Stage nodes c0 + j (list == nullptr) or list[c0 + j], j < cnt; the
// geometric features are multiplied by xmul, the third triple
// third[c * stride + off + node] by tmul (zeros when third is null).
// Whole workgroup; the caller brackets it with barriers.
__device__ __forceinline__ void stage_nodes(const MeshDev &M, int k, int base, const int *list, int c0, int cnt,
                                            const float *third, size_t stride, size_t off, float xmul, float tmul,
                                            StageBuf &xs) {
    const int N = M.N;
    const float o0 = M.origin[3 * k], o1 = M.origin[3 * k + 1], o2 = M.origin[3 * k + 2];
    for (int j = threadIdx.x; j < cnt; j += kWG) {
        const int i = list ? list[c0 + j] : c0 + j;
        const int g = base + i;
        xs[0][j] = (M.pos[g] - o0) * xmul;
        xs[1][j] = (M.pos[N + g] - o1) * xmul;
        xs[2][j] = (M.pos[2 * N + g] - o2) * xmul;
        xs[3][j] = M.nrm[g] * xmul;
        xs[4][j] = M.nrm[N + g] * xmul;
        xs[5][j] = M.nrm[2 * N + g] * xmul;
        xs[6][j] = third ? third[off + i] * tmul : 0.0f;
        xs[7][j] = third ? third[stride + off + i] * tmul : 0.0f;
        xs[8][j] = third ? third[2 * stride + off + i] * tmul : 0.0f;
    }
}

// T-form network input of staged node j (lane group q supplies features
// 8 q .. 8 q + 7, zero padded to 32); with ZERO_U the U_hat features are 0.
template <bool ZERO_U>
__device__ __forceinline__ void stage_x(const StageBuf &xs, int j, bool valid, half8 &xh, half8 &xl) {
    const int q = lane_id() >> 4;
    // every lane reads inside the stage (j < kStage) and masks: no branches
    const bool g0 = valid && q == 0, g1 = valid && q == 1 && !ZERO_U;
    float v[8];
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const float x = xs[e][j];
        v[e] = g0 ? x : 0.0f;
    }
    const float u0 = xs[6][j], u1 = xs[7][j], u2 = xs[8][j];
    v[6] = (g0 && !ZERO_U) ? u0 : 0.0f;
    v[7] = (g0 && !ZERO_U) ? u1 : 0.0f;
    v[0] = g1 ? u2 : v[0];
    split8(v, xh, xl);
}

// Encoder: h1 = relu(W1 x + b1), f = relu(W2 h1 + b2) for a 16-node tile of
// scaled inputs (2^ax x); h1 and f come out at the item's scales 2^a1, 2^af.
__device__ __forceinline__ void encoder_tile(const NetLds &L, const half8 &xh, const half8 &xl, floatx4 h1[4],
                                             floatx4 f[4]) {
    reload_fence();
    const int lane = lane_id(), gq = lane >> 4;
    half8 wh[4], wl[4];
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) {
        wh[ot] = L.w1h[ot * 64 + lane];
        wl[ot] = L.w1l[ot * 64 + lane];
        h1[ot] = *reinterpret_cast<const floatx4 *>(&L.b1s[ot * 16 + 4 * gq]);
    }
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) h1[ot] = mfma16(wh[ot], xh, h1[ot]);
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) h1[ot] = mfma16(wh[ot], xl, h1[ot]);
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) h1[ot] = relu4(mfma16(wl[ot], xh, h1[ot]));
    half8 bh[2], bl[2];
    split_chain(h1, bh, bl);
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) f[ot] = *reinterpret_cast<const floatx4 *>(&L.b2s[ot * 16 + 4 * gq]);
    layer64_t(L.w2h, L.w2l, bh, bl, f);
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) f[ot] = relu4(f[ot]);
}

// Encoder of two independent 16-node tiles at once: the weight fragments are
// read once for both.  Each tile's MFMAs of a K step are issued together, so
// the first tile's ReLU and split overlap the second tile's MFMAs.
__device__ __forceinline__ void encoder_tile2(const NetLds &L, const half8 (&xh)[2], const half8 (&xl)[2],
                                              floatx4 (&f)[2][4]) {
    reload_fence();
    const int lane = lane_id(), gq = lane >> 4;
    floatx4 h1[2][4];
    {
        half8 wh[4], wl[4];
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            wh[ot] = L.w1h[ot * 64 + lane];
            wl[ot] = L.w1l[ot * 64 + lane];
            const floatx4 b = *reinterpret_cast<const floatx4 *>(&L.b1s[ot * 16 + 4 * gq]);
            h1[0][ot] = b;
            h1[1][ot] = b;
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
#pragma unroll
            for (int ot = 0; ot < 4; ++ot) h1[u][ot] = mfma16(wh[ot], xh[u], h1[u][ot]);
#pragma unroll
            for (int ot = 0; ot < 4; ++ot) h1[u][ot] = mfma16(wh[ot], xl[u], h1[u][ot]);
#pragma unroll
            for (int ot = 0; ot < 4; ++ot) h1[u][ot] = relu4(mfma16(wl[ot], xh[u], h1[u][ot]));
        }
    }
    half8 bh[2][2], bl[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u) split_chain(h1[u], bh[u], bl[u]);
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) {
        const floatx4 b = *reinterpret_cast<const floatx4 *>(&L.b2s[ot * 16 + 4 * gq]);
        f[0][ot] = b;
        f[1][ot] = b;
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        half8 h[4], l[4];
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            h[ot] = L.w2h[(ot * 2 + s) * 64 + lane];
            l[ot] = L.w2l[(ot * 2 + s) * 64 + lane];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
#pragma unroll
            for (int ot = 0; ot < 4; ++ot) f[u][ot] = mfma16(h[ot], bh[u][s], f[u][ot]);
#pragma unroll
            for (int ot = 0; ot < 4; ++ot) f[u][ot] = mfma16(h[ot], bl[u][s], f[u][ot]);
#pragma unroll
            for (int ot = 0; ot < 4; ++ot) f[u][ot] = mfma16(l[ot], bh[u][s], f[u][ot]);
        }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) f[u][ot] = relu4(f[u][ot]);
}

// Decoder: h4 = relu(W4 [f; g'] + b4) with the g' part folded into c4, then
// r = W5 h4 + b5.  h4 comes out at 2^a4 and r_mul = 2^-a4 unscales the W5
// sum.  Every lane returns r of its node (lane & 15).
__device__ __forceinline__ void decoder_tile(const NetLds &L, const floatx4 f[4], float r_mul, floatx4 h4[4],
                                             float r_out[3]) {
    reload_fence();
    const int lane = lane_id(), gq = lane >> 4;
    half8 bh[2], bl[2];
    split_chain(f, bh, bl);
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) h4[ot] = *reinterpret_cast<const floatx4 *>(&L.c4[ot * 16 + 4 * gq]);
    layer64_t(L.w4h, L.w4l, bh, bl, h4);
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) h4[ot] = relu4(h4[ot]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float s = 0.0f;
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            const floatx4 w = *reinterpret_cast<const floatx4 *>(&L.w5[c * 64 + ot * 16 + 4 * gq]);
            s += w[0] * h4[ot][0] + w[1] * h4[ot][1] + w[2] * h4[ot][2] + w[3] * h4[ot][3];
        }
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        r_out[c] = s * r_mul + L.b5[c];
    }
}

// Decoder of two independent tiles at once (each tile's results identical to
// decoder_tile's): the W4 fragments are read once for both, and each tile's
// MFMAs of a K step are issued together.
__device__ __forceinline__ void decoder_tile2(const NetLds &L, const floatx4 (&f)[2][4], float r_mul,
                                              float (&r_out)[2][3]) {
    reload_fence();
    const int lane = lane_id(), gq = lane >> 4;
    half8 bh[2][2], bl[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u) split_chain(f[u], bh[u], bl[u]);
    floatx4 h4[2][4];
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) {
        const floatx4 b = *reinterpret_cast<const floatx4 *>(&L.c4[ot * 16 + 4 * gq]);
        h4[0][ot] = b;
        h4[1][ot] = b;
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        half8 h[4], l[4];
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) {
            h[ot] = L.w4h[(ot * 2 + s) * 64 + lane];
            l[ot] = L.w4l[(ot * 2 + s) * 64 + lane];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
#pragma unroll
            for (int ot = 0; ot < 4; ++ot) h4[u][ot] = mfma16(h[ot], bh[u][s], h4[u][ot]);
#pragma unroll
            for (int ot = 0; ot < 4; ++ot) h4[u][ot] = mfma16(h[ot], bl[u][s], h4[u][ot]);
#pragma unroll
            for (int ot = 0; ot < 4; ++ot) h4[u][ot] = mfma16(l[ot], bh[u][s], h4[u][ot]);
        }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
        for (int ot = 0; ot < 4; ++ot) h4[u][ot] = relu4(h4[u][ot]);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float s = 0.0f;
#pragma unroll
            for (int ot = 0; ot < 4; ++ot) {
                const floatx4 w = *reinterpret_cast<const floatx4 *>(&L.w5[c * 64 + ot * 16 + 4 * gq]);
                s += w[0] * h4[u][ot][0] + w[1] * h4[u][ot][1] + w[2] * h4[u][ot][2] + w[3] * h4[u][ot][3];
            }
            s += __shfl_xor(s, 16);
            s += __shfl_xor(s, 32);
            r_out[u][c] = s * r_mul + L.b5[c];
        }
    }
}

// The global MLP's weights this thread uses (row tid & 63, input features
// 16 (tid >> 6) .. + 15 of W3 and of W4[:, 64:], and the row's biases): the
// persistent forward loads them once and keeps them in registers across its
// items instead of reading them for every item.
struct GmlpW {
    float w3[16], w4[16], b3, b4;
};

__device__ __forceinline__ GmlpW load_gmlp(const float *phi) {
    const int tid = threadIdx.x, o = tid & 63, w = tid >> 6;
    GmlpW g;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        g.w3[c] = phi[kW3 + o * 64 + 16 * w + c];
        g.w4[c] = phi[kW4 + o * 128 + 64 + 16 * w + c];
    }
    g.b3 = phi[kB3 + o];
    g.b4 = phi[kB4 + o];
    return g;
}

// Global MLP of one item from the (unscaled) pooled feature in L.g:
// g' = relu(W3 g + b3) and c4 = W4[:, 64:] g' + b4, stored at h4's scale
// 2^a4.  Whole workgroup; each wave sums 16 input features and the four
// partials are added in wave order.
__device__ void global_mlp(NetLds &L, const GmlpW &gw, const ItemScale &sc) {
    const int tid = threadIdx.x, o = tid & 63, w = tid >> 6;
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < 16; ++c) acc += gw.w3[c] * L.g[16 * w + c];
    L.part[w][o] = acc;
    __syncthreads();
    if (tid < 64) {
        float s = gw.b3;
        for (int q = 0; q < kWaves; ++q) s += L.part[q][o];
        L.gp[o] = fmaxf(s, 0.0f);
    }
    __syncthreads();
    acc = 0.0f;
#pragma unroll
    for (int c = 0; c < 16; ++c) acc += gw.w4[c] * L.gp[16 * w + c];
    L.part[w][o] = acc;
    __syncthreads();
    if (tid < 64) {
        float s = gw.b4;
        for (int q = 0; q < kWaves; ++q) s += L.part[q][o];
        L.c4[o] = s * pow2(sc.a4);
    }
    __syncthreads();
}

// The same, its weights read for this item.
__device__ __forceinline__ void global_mlp(NetLds &L, const float *phi, const ItemScale &sc) {
    global_mlp(L, load_gmlp(phi), sc);
}

}  // namespace etac

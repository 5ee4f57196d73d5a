// Contact with rigid objects given as closed triangle meshes (ETac, Sec. III-A
// contact detection against object SDFs; the objects of Sec. IV are meshes).
//
//   host : etac_meshset_create validates the meshes, computes the FP64
//          angle-weighted pseudo-normals (Baerentzen and Aanaes, IEEE TVCG
//          2005) of every face, edge and vertex, splits each mesh into
//          clusters of 32 triangles by recursive splits of the triangle
//          centroids, builds a conservative occupancy grid per mesh, and
//          uploads it all.
//   k_contact_mesh : one workgroup per env, as the primitive contact pass.
//          Primitives are tested one node per lane.  For a mesh object the
//          nodes inside its bounding ball and not in a cell of the grid that
//          is certainly outside are queried one at a time by the whole wave:
//          lanes take the clusters' lower bounds, then the triangles of the
//          two nearest unvisited clusters (one cluster per half-wave, one
//          triangle per lane), with DPP wave reductions for the minimum;
//          clusters whose lower bound exceeds the best distance so far are
//          never opened.
//
// The closest point of a triangle follows the Voronoi-region classification
// of Ericson ("Real-Time Collision Detection", 2005, Sec. 5.1.5).  All of it
// runs in FP64 in a fixed operation order without contraction into FMA, the
// divisions and square roots correctly rounded, so the inside set and the
// deepest-object choice are reproducible bit for bit.  Cluster skipping
// never changes the result: a cluster's oriented bounding box carries a
// margin of 1e-6 mm on every half extent, far above the rounding of the
// distances compared, so a skipped cluster's triangles are strictly farther
// than the best one.
#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <thread>
#include <utility>
#include <vector>

#include "etac_device.h"

namespace etac {

// ---------------------------------------------------------------------------
// device
// ---------------------------------------------------------------------------

// Triangles per cluster: one half-wave each.  Cluster c of a mesh holds
// its triangles kCluster (c - first cluster) onwards, in cluster order.
constexpr int kCluster = 32;

// Features of a triangle holding its closest point.
enum { FEAT_FACE = 0, FEAT_AB = 1, FEAT_BC = 2, FEAT_CA = 3, FEAT_A = 4, FEAT_B = 5, FEAT_C = 6 };

struct TriCorners {
    double a0, a1, a2, b0, b1, b2, c0, c1, c2;
};

__device__ __forceinline__ TriCorners load_tri(const MeshSetDev &ms, int t) {
    const size_t T = (size_t)ms.T;
    const float *c = ms.corner + t;
    return TriCorners{c[0], c[T], c[2 * T], c[3 * T], c[4 * T], c[5 * T], c[6 * T], c[7 * T], c[8 * T]};
}

// Closest point (x0, x1, x2) of the triangle to q, its feature, and the
// squared distance.  Dot products are (x0 y0 + x1 y1) + x2 y2.
__host__ __device__ __forceinline__ double closest_tri(double q0, double q1, double q2, const TriCorners &t,
                                                       double &x0, double &x1, double &x2, int &feat) {
#pragma clang fp contract(off)
    const double ab0 = t.b0 - t.a0, ab1 = t.b1 - t.a1, ab2 = t.b2 - t.a2;
    const double ac0 = t.c0 - t.a0, ac1 = t.c1 - t.a1, ac2 = t.c2 - t.a2;
    const double ap0 = q0 - t.a0, ap1 = q1 - t.a1, ap2 = q2 - t.a2;
    const double d1 = (ab0 * ap0 + ab1 * ap1) + ab2 * ap2;
    const double d2 = (ac0 * ap0 + ac1 * ap1) + ac2 * ap2;
    const double bp0 = q0 - t.b0, bp1 = q1 - t.b1, bp2 = q2 - t.b2;
    const double d3 = (ab0 * bp0 + ab1 * bp1) + ab2 * bp2;
    const double d4 = (ac0 * bp0 + ac1 * bp1) + ac2 * bp2;
    const double cq0 = q0 - t.c0, cq1 = q1 - t.c1, cq2 = q2 - t.c2;
    const double d5 = (ab0 * cq0 + ab1 * cq1) + ab2 * cq2;
    const double d6 = (ac0 * cq0 + ac1 * cq1) + ac2 * cq2;
    const double vc = d1 * d4 - d3 * d2;
    const double vb = d5 * d2 - d1 * d6;
    const double va = d3 * d6 - d5 * d4;
    const double e4 = d4 - d3, e5 = d5 - d6;
    if (d1 <= 0.0 && d2 <= 0.0) {
        feat = FEAT_A;
        x0 = t.a0; x1 = t.a1; x2 = t.a2;
    } else if (d3 >= 0.0 && d4 <= d3) {
        feat = FEAT_B;
        x0 = t.b0; x1 = t.b1; x2 = t.b2;
    } else if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
        const double v = d1 / (d1 - d3);
        feat = FEAT_AB;
        x0 = t.a0 + v * ab0; x1 = t.a1 + v * ab1; x2 = t.a2 + v * ab2;
    } else if (d6 >= 0.0 && d5 <= d6) {
        feat = FEAT_C;
        x0 = t.c0; x1 = t.c1; x2 = t.c2;
    } else if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
        const double w = d2 / (d2 - d6);
        feat = FEAT_CA;
        x0 = t.a0 + w * ac0; x1 = t.a1 + w * ac1; x2 = t.a2 + w * ac2;
    } else if (va <= 0.0 && e4 >= 0.0 && e5 >= 0.0) {
        const double w = e4 / (e4 + e5);
        feat = FEAT_BC;
        x0 = t.b0 + w * (t.c0 - t.b0); x1 = t.b1 + w * (t.c1 - t.b1); x2 = t.b2 + w * (t.c2 - t.b2);
    } else {
        const double den = (va + vb) + vc;
        const double v = vb / den, w = vc / den;
        feat = FEAT_FACE;
        x0 = (t.a0 + v * ab0) + w * ac0;
        x1 = (t.a1 + v * ab1) + w * ac1;
        x2 = (t.a2 + v * ab2) + w * ac2;
    }
    const double w0 = q0 - x0, w1 = q1 - x1, w2 = q2 - x2;
    return (w0 * w0 + w1 * w1) + w2 * w2;
}

// Wave-wide minima through DPP row permutes (xor 1, xor 2, half-row and
// row mirrors: every lane ends with its row's minimum), then the four row
// minima read lane by lane.  Every lane of the wave must be active; every
// lane gets the result.
template <int CTRL>
__device__ __forceinline__ int dpp(int v) {
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
}

template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    const int lo = dpp<CTRL>(__double2loint(v)), hi = dpp<CTRL>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

__device__ __forceinline__ double wave_min(double v) {
    v = fmin(v, dpp<0xb1>(v));    // quad_perm [1, 0, 3, 2]
    v = fmin(v, dpp<0x4e>(v));    // quad_perm [2, 3, 0, 1]
    v = fmin(v, dpp<0x141>(v));   // row_half_mirror
    v = fmin(v, dpp<0x140>(v));   // row_mirror
    return fmin(fmin(read_lane(v, 0), read_lane(v, 16)), fmin(read_lane(v, 32), read_lane(v, 48)));
}

__device__ __forceinline__ int wave_min(int v) {
    v = min(v, dpp<0xb1>(v));
    v = min(v, dpp<0x4e>(v));
    v = min(v, dpp<0x141>(v));
    v = min(v, dpp<0x140>(v));
    return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// Wave-wide sum in a fixed order (pairwise within rows, then the four row
// sums), the same value in every lane.
__device__ __forceinline__ double wave_sum(double v) {
    v = v + dpp<0xb1>(v);
    v = v + dpp<0x4e>(v);
    v = v + dpp<0x141>(v);
    v = v + dpp<0x140>(v);
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Signed-distance query of one point q (object frame, the same value in
// every lane of the wave) against mesh `mesh`; the whole wave takes part.
// Returns the same result in every lane.
__device__ Pen mesh_query(const MeshSetDev &ms, int mesh, double q0, double q1, double q2, const float *R,
                          int &tri) {
#pragma clang fp contract(off)
    const int lane = lane_id();
    const int4 mr = ms.mesh[mesh];
    const double kInf = __builtin_inf();
    double best_s = kInf;
    int best_o = 0x7fffffff, best_t = -1, best_f = 0;
    double bx0 = 0.0, bx1 = 0.0, bx2 = 0.0;   // the winning closest point, read from its lane
    const int half = lane >> 5;
    for (int cb = mr.z; cb < mr.w; cb += 64) {
        const int c = cb + lane;
        double lb = kInf;   // squared distance to cluster c's box: a lower bound for its triangles
        if (c < mr.w) {
            const double *b = ms.box + 16 * (size_t)c;
            const double dx = q0 - b[0], dy = q1 - b[1], dz = q2 - b[2];
            double e0 = fabs((dx * b[3] + dy * b[4]) + dz * b[5]) - b[12];
            double e1 = fabs((dx * b[6] + dy * b[7]) + dz * b[8]) - b[13];
            double e2 = fabs((dx * b[9] + dy * b[10]) + dz * b[11]) - b[14];
            e0 = e0 > 0.0 ? e0 : 0.0;
            e1 = e1 > 0.0 ? e1 : 0.0;
            e2 = e2 > 0.0 ? e2 : 0.0;
            lb = (e0 * e0 + e1 * e1) + e2 * e2;
        }
        // first the two clusters of least bound, then, two at a time, every
        // cluster whose bound does not exceed the best distance so far
        // (re-checked after each pass); each half-wave takes one cluster
        const double m1 = wave_min(lb);
        // every cluster of this pass strictly farther; a non-finite bound
        // (non-finite pose) gives no result
        if (!(m1 < kInf) || !(m1 <= best_s)) continue;
        const int a0 = __ffsll((unsigned long long)__ballot(lb == m1)) - 1;
        const double m2 = wave_min(lane == a0 ? kInf : lb);
        int ca = a0, cbb = -1;
        if (m2 < kInf && m2 <= best_s) cbb = __ffsll((unsigned long long)__ballot(lane != a0 && lb == m2)) - 1;
        while (ca >= 0) {
            if (lane == ca || lane == cbb) lb = kInf;
            const int mine = half ? cbb : ca;
            int t = -1;
            double s = kInf;
            int o = 0x7fffffff;
            if (mine >= 0) {   // clusters hold kCluster triangles, the mesh's last one possibly fewer
                const int tt = mr.x + kCluster * (cb + mine - mr.z) + (lane & 31);
                if (tt < mr.y) t = tt;
            }
            double x0 = 0.0, x1 = 0.0, x2 = 0.0;
            int f = 0;
            if (t >= 0) {
                s = closest_tri(q0, q1, q2, load_tri(ms, t), x0, x1, x2, f);
                o = ms.orig[t];
            }
            const double sm = wave_min(s);
            unsigned long long at = __ballot(s == sm);
            int om;
            if (__popcll(at) == 1) {
                om = __builtin_amdgcn_readlane(o, __ffsll(at) - 1);
            } else {   // equal distances: the lowest triangle index
                om = wave_min(s == sm ? o : 0x7fffffff);
                at = __ballot(s == sm && o == om);
            }
            if (sm < best_s || (sm == best_s && om < best_o)) {
                const int wl = __ffsll(at) - 1;
                best_s = sm;
                best_o = om;
                best_t = __builtin_amdgcn_readlane(t, wl);
                best_f = __builtin_amdgcn_readlane(f, wl);
                bx0 = read_lane(x0, wl);
                bx1 = read_lane(x1, wl);
                bx2 = read_lane(x2, wl);
            }
            unsigned long long todo = __ballot(lb <= best_s && lb < kInf);
            ca = __ffsll(todo) - 1;
            todo &= todo - 1;
            cbb = __ffsll(todo) - 1;
        }
    }
    Pen h;
    h.inside = false;
    h.depth = 0.0;
    h.u0 = h.u1 = h.u2 = 0.0;
    tri = best_t;
    if (best_t < 0) return h;
    const double x0 = bx0, x1 = bx1, x2 = bx2;
    const int f = best_f;
    const double *n = ms.pn + ((size_t)best_t * 7 + f) * 3;
    const double w0 = q0 - x0, w1 = q1 - x1, w2 = q2 - x2;
    if (!((w0 * n[0] + w1 * n[1]) + w2 * n[2] < 0.0)) return h;
    h.inside = true;
    h.depth = sqrt(best_s);
    const double v0 = x0 - q0, v1 = x1 - q1, v2 = x2 - q2;
    h.u0 = ((double)R[0] * v0 + (double)R[1] * v1) + (double)R[2] * v2;
    h.u1 = ((double)R[3] * v0 + (double)R[4] * v1) + (double)R[5] * v2;
    h.u2 = ((double)R[6] * v0 + (double)R[7] * v1) + (double)R[8] * v2;
    return h;
}

// dL/d(R, t) of one node won by a mesh object (triangle `tri`), from
// dL/du_hat = g, added to acc[0..8] (R) and acc[9..11] (t).  With the
// closest point c(q) on the triangle's winning feature held fixed,
// w = c - q, u_hat = R w and dw/dq = J (face: -n n^T; edge with direction
// e: e e^T / |e|^2 - I; vertex: -I; J symmetric): for h = J R^T g,
// dL/dR = g w^T + d h^T and dL/dt = -R h.
__device__ void mesh_adjoint_node(const MeshSetDev &ms, int tri, const float *Rf, const float *tf, float px,
                                  float py, float pz, const double g[3], double acc[12]) {
#pragma clang fp contract(off)
    const double d0 = (double)px - (double)tf[0], d1 = (double)py - (double)tf[1], d2 = (double)pz - (double)tf[2];
    double R[9];
    for (int c = 0; c < 9; ++c) R[c] = Rf[c];
    const double q0 = (R[0] * d0 + R[3] * d1) + R[6] * d2;
    const double q1 = (R[1] * d0 + R[4] * d1) + R[7] * d2;
    const double q2 = (R[2] * d0 + R[5] * d1) + R[8] * d2;
    const TriCorners T = load_tri(ms, tri);
    double x0, x1, x2;
    int f;
    closest_tri(q0, q1, q2, T, x0, x1, x2, f);
    const double rg0 = (R[0] * g[0] + R[3] * g[1]) + R[6] * g[2];
    const double rg1 = (R[1] * g[0] + R[4] * g[1]) + R[7] * g[2];
    const double rg2 = (R[2] * g[0] + R[5] * g[1]) + R[8] * g[2];
    double h0, h1, h2;
    if (f == FEAT_FACE) {
        const double *n = ms.pn + (size_t)tri * 21;
        const double nd = (n[0] * rg0 + n[1] * rg1) + n[2] * rg2;
        h0 = -n[0] * nd; h1 = -n[1] * nd; h2 = -n[2] * nd;
    } else if (f == FEAT_AB || f == FEAT_BC || f == FEAT_CA) {
        const double s0 = f == FEAT_AB ? T.a0 : (f == FEAT_BC ? T.b0 : T.c0);
        const double s1 = f == FEAT_AB ? T.a1 : (f == FEAT_BC ? T.b1 : T.c1);
        const double s2 = f == FEAT_AB ? T.a2 : (f == FEAT_BC ? T.b2 : T.c2);
        const double e0 = (f == FEAT_AB ? T.b0 : (f == FEAT_BC ? T.c0 : T.a0)) - s0;
        const double e1 = (f == FEAT_AB ? T.b1 : (f == FEAT_BC ? T.c1 : T.a1)) - s1;
        const double e2 = (f == FEAT_AB ? T.b2 : (f == FEAT_BC ? T.c2 : T.a2)) - s2;
        const double k = ((e0 * rg0 + e1 * rg1) + e2 * rg2) / ((e0 * e0 + e1 * e1) + e2 * e2);
        h0 = e0 * k - rg0; h1 = e1 * k - rg1; h2 = e2 * k - rg2;
    } else {
        h0 = -rg0; h1 = -rg1; h2 = -rg2;
    }
    const double w0 = x0 - q0, w1 = x1 - q1, w2 = x2 - q2;
    const double d[3] = {d0, d1, d2}, w[3] = {w0, w1, w2}, h[3] = {h0, h1, h2};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int b = 0; b < 3; ++b) acc[a * 3 + b] += g[a] * w[b] + d[a] * h[b];
        acc[9 + a] -= (R[a * 3] * h0 + R[a * 3 + 1] * h1) + R[a * 3 + 2] * h2;
    }
}

// Mesh index named by a mesh object's shape[0], or -1.
__device__ __forceinline__ int mesh_of(const float *sh, int M) {
    const float x = sh[0];
    return (x >= 0.0f && x < (float)M && x == floorf(x)) ? (int)x : -1;
}

struct MeshContactParams {
    MeshDev mesh;
    SceneDev scene;
    MeshSetDev ms;
    int8_t *cobj;      // [E][N]
    float *uhat;       // [3][E][N] or null
    int32_t *n_active; // [E][K]
    int32_t *hit;            // [E][N] or null: winning triangle (cluster order) of mesh-won nodes, else -1
    // adjoint
    const float *grad_uhat;  // [3][E][N]
    float *grad_rot;         // [E][O][9]
    float *grad_trans;       // [E][O][3]
    const int8_t *cobj_in;   // [E][N] and
    const int32_t *hit_in;   // [E][N]: the forward's records, or null (contact recomputed)
};

// Candidate objects (primitives and valid meshes) of env e whose bounding
// ball may reach patch k's bounding sphere.
__device__ __forceinline__ unsigned cull_mesh_objects(const MeshContactParams &p, int e, int k) {
    const SceneDev &S = p.scene;
    unsigned cand = 0;
    const int no = min(S.n_obj[e], S.O);
    const float4 b = p.mesh.bound[k];
    for (int o = 0; o < no; ++o) {
        const size_t eo = (size_t)e * S.O + o;
        const int ty = S.type[eo];
        float rad;
        if (ty >= ETAC_SPHERE && ty <= ETAC_CAPSULE) {
            rad = bounding_radius(ty, S.shape + 4 * eo);
        } else if (ty == ETAC_MESH) {
            const int m = mesh_of(S.shape + 4 * eo, p.ms.M);
            if (m < 0) continue;
            rad = p.ms.radius[m];
        } else {
            continue;
        }
        const float *t = S.trans + 3 * eo;
        const float dx = b.x - t[0], dy = b.y - t[1], dz = b.z - t[2];
        const float reach = (b.w + rad) * 1.001f + 1e-3f;
        if ((dx * dx + dy * dy + dz * dz) * (1.0f - 1e-5f) <= reach * reach) cand |= 1u << o;
    }
    return cand;
}

// Four waves per SIMD (at most 128 registers): the queries are latency-bound.
// ADJ: the adjoint (every node's pose gradient added to its winning object's
// sums: per wave in a fixed order, then over the waves in wave order, so
// results do not depend on timing), with contact recomputed or, REC, read
// from the forward's records.
template <bool ADJ, bool REC>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_contact_mesh(MeshContactParams p) {
    __shared__ int cnt[kMaxPatches];
    __shared__ uint8_t cand[kMaxPatches];
    __shared__ double sacc[ADJ ? kWaves : 1][ADJ ? ETAC_MAX_OBJ : 1][12];
    const int e = blockIdx.x;
    const MeshDev &M = p.mesh;
    const SceneDev &S = p.scene;
    const int N = M.N, K = M.K;
    const size_t EN = (size_t)S.E * N;
    for (int k = threadIdx.x; k < K; k += kWG) {
        cnt[k] = 0;
        cand[k] = (uint8_t)cull_mesh_objects(p, e, k);
    }
    if (ADJ)
        for (int c = threadIdx.x; c < kWaves * ETAC_MAX_OBJ * 12; c += kWG) (&sacc[0][0][0])[c] = 0.0;
    __syncthreads();
    const int lane = lane_id();
    const int no = min(S.n_obj[e], S.O);
    const size_t row = (size_t)e * N;
    // whole waves step through the nodes: every lane reaches the wave-wide queries
    for (int i0 = threadIdx.x - lane; i0 < N; i0 += kWG) {
        const int i = i0 + lane;
        const bool valid = i < N;
        const int k = valid ? M.node_patch[i] : 0;
        const unsigned c = valid ? cand[k] : 0u;
        const float px = valid ? M.pos[i] : 0.0f, py = valid ? M.pos[N + i] : 0.0f;
        const float pz = valid ? M.pos[2 * N + i] : 0.0f;
        int best = -1, btri = -1;   // btri: winning triangle when a mesh wins
        double bd = 0.0, b0 = 0.0, b1 = 0.0, b2 = 0.0;
        if (REC) {
            // the forward's records; values that cannot come from it are skipped
            if (valid && c != 0u) {
                const int o = p.cobj_in[row + i];
                if (o >= 0 && o < no) {
                    const size_t eo = (size_t)e * S.O + o;
                    const int ty = S.type[eo];
                    const int h = p.hit_in[row + i];
                    if (ty >= ETAC_SPHERE && ty <= ETAC_CAPSULE) {
                        best = o;
                    } else if (ty == ETAC_MESH) {
                        const int m = mesh_of(S.shape + 4 * eo, p.ms.M);
                        if (m >= 0 && h >= p.ms.mesh[m].x && h < p.ms.mesh[m].y) {
                            best = o;
                            btri = h;
                        }
                    }
                }
            }
        } else if (__ballot(c != 0u)) {
            for (int o = 0; o < no; ++o) {
                const size_t eo = (size_t)e * S.O + o;
                const int ty = S.type[eo];
                const float *sh = S.shape + 4 * eo;
                const float *R = S.rot + 9 * eo;
                const float *t = S.trans + 3 * eo;
                const bool take = (c >> o) & 1u;
                const float dx = px - t[0], dy = py - t[1], dz = pz - t[2];
                const float d2 = dx * dx + dy * dy + dz * dz;
                if (ty >= ETAC_SPHERE && ty <= ETAC_CAPSULE) {
                    const float rb = bounding_radius(ty, sh) * 1.001f + 1e-3f;
                    if (!take || d2 > rb * rb) continue;
                    const Pen h = penetrate(ty, sh, R, t, px, py, pz, M.nrm[i], M.nrm[N + i], M.nrm[2 * N + i]);
                    if (h.inside && (best < 0 || h.depth > bd)) {
                        best = o;
                        btri = -1;
                        bd = h.depth;
                        b0 = h.u0; b1 = h.u1; b2 = h.u2;
                    }
                } else if (ty == ETAC_MESH) {
                    const int m = mesh_of(sh, p.ms.M);
                    if (m < 0) continue;
                    const float rb = p.ms.radius[m] * 1.001f + 1e-3f;
                    bool near = take && d2 <= rb * rb;
                    if (near) {   // the occupancy grid rules out nodes certainly outside
                        const float4 g = p.ms.grid_lo[m];
                        const int4 gd = p.ms.grid_dim[m];
                        const float qx = (R[0] * dx + R[3] * dy) + R[6] * dz;
                        const float qy = (R[1] * dx + R[4] * dy) + R[7] * dz;
                        const float qz = (R[2] * dx + R[5] * dy) + R[8] * dz;
                        const float gx = (qx - g.x) * g.w, gy = (qy - g.y) * g.w, gz = (qz - g.z) * g.w;
                        near = gx >= 0.0f && gy >= 0.0f && gz >= 0.0f && gx < (float)gd.x && gy < (float)gd.y &&
                               gz < (float)gd.z;
                        if (near) {
                            const int ix = min((int)gx, gd.x - 1), iy = min((int)gy, gd.y - 1);
                            const int iz = min((int)gz, gd.z - 1);
                            const unsigned bit = (unsigned)gd.w + (unsigned)((iz * gd.y + iy) * gd.x + ix);
                            near = (p.ms.grid_bits[bit >> 5] >> (bit & 31u)) & 1u;
                        }
                    }
                    unsigned long long todo = __ballot(near);
                    const double t0 = t[0], t1 = t[1], t2 = t[2];
                    const double r00 = R[0], r01 = R[1], r02 = R[2];
                    const double r10 = R[3], r11 = R[4], r12 = R[5];
                    const double r20 = R[6], r21 = R[7], r22 = R[8];
                    while (todo) {
                        const int src = __ffsll(todo) - 1;
                        todo &= todo - 1;
                        // the node of lane src, the same value in every lane
                        const double d0 = (double)__shfl(px, src) - t0;
                        const double d1 = (double)__shfl(py, src) - t1;
                        const double e2 = (double)__shfl(pz, src) - t2;
                        double q0, q1, q2;
                        {
#pragma clang fp contract(off)
                            q0 = (r00 * d0 + r10 * d1) + r20 * e2;
                            q1 = (r01 * d0 + r11 * d1) + r21 * e2;
                            q2 = (r02 * d0 + r12 * d1) + r22 * e2;
                        }
                        int tri;
                        const Pen h = mesh_query(p.ms, m, q0, q1, q2, R, tri);
                        if (lane == src && h.inside && (best < 0 || h.depth > bd)) {
                            best = o;
                            btri = tri;
                            bd = h.depth;
                            b0 = h.u0; b1 = h.u1; b2 = h.u2;
                        }
                    }
                }
            }
        }
        if (ADJ) {
            if (__ballot(best >= 0)) {
                double acc[12];
#pragma unroll
                for (int q = 0; q < 12; ++q) acc[q] = 0.0;
                if (best >= 0) {
                    const size_t eo = (size_t)e * S.O + best;
                    const double g[3] = {p.grad_uhat[row + i], p.grad_uhat[EN + row + i],
                                         p.grad_uhat[2 * EN + row + i]};
                    if (btri >= 0)
                        mesh_adjoint_node(p.ms, btri, S.rot + 9 * eo, S.trans + 3 * eo, px, py, pz, g, acc);
                    else
                        contact_adjoint_node(S.type[eo], S.shape + 4 * eo, S.rot + 9 * eo, S.trans + 3 * eo, px, py,
                                             pz, g, acc);
                }
                const int wave = threadIdx.x >> 6;
                for (int o = 0; o < no; ++o) {
                    if (!__ballot(best == o)) continue;
#pragma unroll
                    for (int q = 0; q < 12; ++q) {
                        const double v = wave_sum(best == o ? acc[q] : 0.0);
                        if (lane == 0) sacc[wave][o][q] += v;   // one writer per wave, chunks in order
                    }
                }
            }
        } else if (valid) {
            p.cobj[row + i] = (int8_t)best;
            if (p.hit) p.hit[row + i] = best >= 0 ? btri : -1;
            if (p.uhat) {
                p.uhat[row + i] = (float)b0;
                p.uhat[EN + row + i] = (float)b1;
                p.uhat[2 * EN + row + i] = (float)b2;
            }
            if (best >= 0) atomicAdd(&cnt[k], 1);
        }
    }
    __syncthreads();
    if (ADJ) {
        for (int c = threadIdx.x; c < S.O * 12; c += kWG) {
            const int o = c / 12, q = c % 12;
            double v = 0.0;
            for (int w = 0; w < kWaves; ++w) v += sacc[w][o][q];
            const size_t eo = (size_t)e * S.O + o;
            if (q < 9) p.grad_rot[eo * 9 + q] = (float)v;
            else p.grad_trans[eo * 3 + q - 9] = (float)v;
        }
    } else {
        for (int k = threadIdx.x; k < K; k += kWG) p.n_active[(size_t)e * K + k] = cnt[k];
    }
}

hipError_t launch_contact_mesh(const Plan &p, const MeshSetDev &ms, const SceneDev &s, int8_t *cobj, float *uhat,
                               int32_t *n_active, int32_t *hit, hipStream_t st) {
    if (s.E == 0) return hipSuccess;
    MeshContactParams cp{p.mesh, s, ms, cobj, uhat, n_active, hit, nullptr, nullptr, nullptr, nullptr, nullptr};
    hipLaunchKernelGGL((k_contact_mesh<false, false>), dim3(s.E), dim3(kWG), 0, st, cp);
    return hipGetLastError();
}

hipError_t launch_contact_mesh_backward(const Plan &p, const MeshSetDev &ms, const SceneDev &s,
                                        const float *grad_uhat, const int8_t *cobj, const int32_t *hit,
                                        float *grad_rot, float *grad_trans, hipStream_t st) {
    if (s.E == 0) return hipSuccess;
    MeshContactParams cp{p.mesh, s, ms, nullptr, nullptr, nullptr, nullptr, grad_uhat, grad_rot, grad_trans,
                         hit ? cobj : nullptr, cobj ? hit : nullptr};
    if (cp.hit_in) hipLaunchKernelGGL((k_contact_mesh<true, true>), dim3(s.E), dim3(kWG), 0, st, cp);
    else hipLaunchKernelGGL((k_contact_mesh<true, false>), dim3(s.E), dim3(kWG), 0, st, cp);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// host: mesh-set construction
// ---------------------------------------------------------------------------
namespace {

struct V3 {
    double x, y, z;
};

#pragma clang fp contract(off)
inline V3 sub(const V3 &a, const V3 &b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
inline double dot(const V3 &a, const V3 &b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }

// Unit normal of triangle (a, b, c); false for zero area.
bool face_normal(const V3 &a, const V3 &b, const V3 &c, V3 &n) {
    const V3 ab = sub(b, a), ac = sub(c, a);
    const V3 x{ab.y * ac.z - ab.z * ac.y, ab.z * ac.x - ab.x * ac.z, ab.x * ac.y - ab.y * ac.x};
    const double len = std::sqrt(dot(x, x));
    if (!(len > 0.0) || !std::isfinite(len)) return false;
    n = V3{x.x / len, x.y / len, x.z / len};
    return true;
}

// Interior angle at p0 of the triangle (p0, p1, p2).
double corner_angle(const V3 &p0, const V3 &p1, const V3 &p2) {
    const V3 e1 = sub(p1, p0), e2 = sub(p2, p0);
    double cs = dot(e1, e2) / (std::sqrt(dot(e1, e1)) * std::sqrt(dot(e2, e2)));
    cs = std::min(1.0, std::max(-1.0, cs));
    return std::acos(cs);
}

struct BuiltMesh {
    std::vector<int> order;              // triangles (index within the mesh) in cluster order
    std::vector<std::pair<int, int>> clusters;   // ranges into `order`
};

// Recursive split of the triangle centroids along the longest axis of their
// bounding box, down to clusters of kCluster triangles (the last one of a
// mesh may hold fewer): the lower side takes kCluster times half the number
// of clusters needed, rounded up.
void split(std::vector<int> &ids, int lo, int hi, const std::vector<V3> &cen, BuiltMesh &out) {
    if (hi - lo <= kCluster) {
        out.clusters.push_back({lo, hi});
        return;
    }
    V3 mn = cen[ids[lo]], mx = mn;
    for (int i = lo; i < hi; ++i) {
        const V3 &c = cen[ids[i]];
        mn = V3{std::min(mn.x, c.x), std::min(mn.y, c.y), std::min(mn.z, c.z)};
        mx = V3{std::max(mx.x, c.x), std::max(mx.y, c.y), std::max(mx.z, c.z)};
    }
    const double ex = mx.x - mn.x, ey = mx.y - mn.y, ez = mx.z - mn.z;
    const int axis = (ex >= ey && ex >= ez) ? 0 : (ey >= ez ? 1 : 2);
    auto coord = [&](int t) { return axis == 0 ? cen[t].x : (axis == 1 ? cen[t].y : cen[t].z); };
    const int mid = lo + kCluster * (((hi - lo + kCluster - 1) / kCluster + 1) / 2);
    std::nth_element(ids.begin() + lo, ids.begin() + mid, ids.begin() + hi, [&](int a, int b) {
        const double ca = coord(a), cb = coord(b);
        return ca < cb || (ca == cb && a < b);
    });
    split(ids, lo, mid, cen, out);
    split(ids, mid, hi, cen, out);
}

// Signed distance of x to one mesh (negative inside), for the occupancy
// grid only: the same closest-point rule, clusters visited by ascending
// lower bound.
struct HostMesh {
    const int32_t *tv;                   // vertex indices of the mesh's triangles, as given
    const float *verts;
    const std::vector<int> *order;       // cluster order -> triangle
    const std::vector<std::pair<int, int>> *clusters;
    const double4 *ball;                 // this mesh's cluster balls
    const double *pn;                    // [nt][21] pseudo-normals, as given
};

double host_sdf(const HostMesh &hm, double x0, double x1, double x2) {
    const int nc = (int)hm.clusters->size();
    std::vector<std::pair<double, int>> lb(nc);
    for (int c = 0; c < nc; ++c) {
        const double4 b = hm.ball[c];
        const double dx = x0 - b.x, dy = x1 - b.y, dz = x2 - b.z;
        const double l = std::sqrt((dx * dx + dy * dy) + dz * dz) - b.w;
        lb[c] = {l > 0.0 ? l * l : 0.0, c};
    }
    std::sort(lb.begin(), lb.end());
    double best = INFINITY, c0 = 0.0, c1 = 0.0, c2 = 0.0;
    int bf = -1, bfeat = 0;
    for (auto [l, c] : lb) {
        if (l > best) break;
        for (int i = (*hm.clusters)[c].first; i < (*hm.clusters)[c].second; ++i) {
            const int f = (*hm.order)[i];
            const float *a = hm.verts + 3 * (size_t)hm.tv[3 * f], *b = hm.verts + 3 * (size_t)hm.tv[3 * f + 1];
            const float *cc = hm.verts + 3 * (size_t)hm.tv[3 * f + 2];
            const TriCorners t{a[0], a[1], a[2], b[0], b[1], b[2], cc[0], cc[1], cc[2]};
            double y0, y1, y2;
            int ft;
            const double sq = closest_tri(x0, x1, x2, t, y0, y1, y2, ft);
            if (sq < best || (sq == best && f < bf)) {
                best = sq; bf = f; bfeat = ft;
                c0 = y0; c1 = y1; c2 = y2;
            }
        }
    }
    const double *n = hm.pn + (size_t)21 * bf + 3 * bfeat;
    const double d = std::sqrt(best);
    return ((x0 - c0) * n[0] + (x1 - c1) * n[1]) + (x2 - c2) * n[2] < 0.0 ? -d : d;
}

// Occupancy grid of one mesh: cubic cells, about kGridCells along the longest
// side of the bounding box (padded by 0.01 mm).  A cell's bit is cleared when
// its centre is outside by more than the half diagonal plus 0.01 mm: the
// signed distance changes no faster than the distance moved, so every point
// of the cell (and up to 0.01 mm beyond it) is outside.
constexpr int kGridCells = 40;

void build_grid(const HostMesh &hm, V3 lo, V3 hi, float4 &glo, int4 &gdim, std::vector<unsigned> &bits) {
    const double pad = 0.01;
    lo = V3{lo.x - pad, lo.y - pad, lo.z - pad};
    hi = V3{hi.x + pad, hi.y + pad, hi.z + pad};
    const double h = std::max({hi.x - lo.x, hi.y - lo.y, hi.z - lo.z}) / kGridCells;
    const int nx = std::max(1, (int)std::ceil((hi.x - lo.x) / h)), ny = std::max(1, (int)std::ceil((hi.y - lo.y) / h));
    const int nz = std::max(1, (int)std::ceil((hi.z - lo.z) / h));
    const size_t ncell = (size_t)nx * ny * nz, base = bits.size() * 32;
    bits.resize((base + ncell + 31) / 32, 0u);
    std::vector<uint8_t> maybe(ncell, 1);
    const double reach = h * std::sqrt(3.0) / 2.0 + 0.01;
    const int nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (int w = 0; w < nth; ++w)
        pool.emplace_back([&, w]() {
            for (size_t c = w; c < ncell; c += nth) {
                const int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((size_t)nx * ny));
                const double sd = host_sdf(hm, lo.x + (i + 0.5) * h, lo.y + (j + 0.5) * h, lo.z + (k + 0.5) * h);
                maybe[c] = !(sd > reach);
            }
        });
    for (auto &t : pool) t.join();
    for (size_t c = 0; c < ncell; ++c)
        if (maybe[c]) bits[(base + c) / 32] |= 1u << ((base + c) % 32);
    glo = make_float4((float)lo.x, (float)lo.y, (float)lo.z, (float)(1.0 / h));
    gdim = make_int4(nx, ny, nz, (int)base);
}

}  // namespace
}  // namespace etac

extern "C" {

static etac_status meshset_create(int32_t n_meshes, const int32_t *tri_offset, int32_t n_verts, const float *verts,
                                  const int32_t *tris, etac_meshset **out) {
    using namespace etac;
    if (!tri_offset || !verts || !tris || !out) return ETAC_ERR_NULL;
    // at most 4096 meshes: their occupancy grids (at most 41^3 cells each) keep 32-bit bit offsets
    if (n_meshes < 1 || n_meshes > 4096 || n_verts < 3) return ETAC_ERR_SHAPE;
    if (tri_offset[0] != 0) return ETAC_ERR_SHAPE;
    for (int m = 0; m < n_meshes; ++m)
        if (tri_offset[m + 1] - tri_offset[m] < 4) return ETAC_ERR_SHAPE;
    const int T = tri_offset[n_meshes];
    if (T > (1 << 24)) return ETAC_ERR_SHAPE;
    for (size_t i = 0; i < (size_t)n_verts * 3; ++i)
        if (!std::isfinite(verts[i])) return ETAC_ERR_VALUE;
    for (size_t i = 0; i < (size_t)T * 3; ++i)
        if (tris[i] < 0 || tris[i] >= n_verts) return ETAC_ERR_VALUE;
    auto vtx = [&](int v) { return V3{verts[3 * (size_t)v], verts[3 * (size_t)v + 1], verts[3 * (size_t)v + 2]}; };

    std::vector<float> corner((size_t)9 * T);
    std::vector<int> orig(T);
    std::vector<double> pn((size_t)21 * T);
    std::vector<double4> ball;   // cluster balls, for the host-side grid classification
    std::vector<double> box;     // [C][16] cluster boxes: centre, three axes, half extents (with margin)
    std::vector<int4> mesh(n_meshes);
    std::vector<float> radius(n_meshes);
    std::vector<float4> grid_lo(n_meshes);
    std::vector<int4> grid_dim(n_meshes);
    std::vector<unsigned> grid_bits;
    for (int m = 0; m < n_meshes; ++m) {
        const int t0 = tri_offset[m], nt = tri_offset[m + 1] - t0;
        const int32_t *tv = tris + 3 * (size_t)t0;
        // closed and consistently oriented: every directed edge once, its reverse once
        std::map<std::pair<int, int>, int> edge;   // directed edge -> triangle
        for (int f = 0; f < nt; ++f)
            for (int k = 0; k < 3; ++k) {
                const std::pair<int, int> key{tv[3 * f + k], tv[3 * f + (k + 1) % 3]};
                if (key.first == key.second || !edge.emplace(key, f).second) return ETAC_ERR_VALUE;
            }
        std::vector<V3> fn(nt), cen(nt);
        for (int f = 0; f < nt; ++f) {
            const V3 a = vtx(tv[3 * f]), b = vtx(tv[3 * f + 1]), c = vtx(tv[3 * f + 2]);
            if (!face_normal(a, b, c, fn[f])) return ETAC_ERR_VALUE;
            cen[f] = V3{(a.x + b.x + c.x) / 3.0, (a.y + b.y + c.y) / 3.0, (a.z + b.z + c.z) / 3.0};
        }
        // per-triangle pseudo-normals in the order given
        std::vector<double> mpn((size_t)21 * nt);
        std::map<int, V3> vsum;   // vertex -> angle-weighted normal sum, faces in ascending order
        for (int f = 0; f < nt; ++f)
            for (int k = 0; k < 3; ++k) {
                const int v = tv[3 * f + k];
                const double th = corner_angle(vtx(v), vtx(tv[3 * f + (k + 1) % 3]), vtx(tv[3 * f + (k + 2) % 3]));
                V3 &acc = vsum.emplace(v, V3{0.0, 0.0, 0.0}).first->second;
                acc = V3{acc.x + th * fn[f].x, acc.y + th * fn[f].y, acc.z + th * fn[f].z};
            }
        for (int f = 0; f < nt; ++f) {
            double *o = mpn.data() + (size_t)21 * f;
            o[0] = fn[f].x; o[1] = fn[f].y; o[2] = fn[f].z;
            for (int k = 0; k < 3; ++k) {   // edges ab, bc, ca
                auto it = edge.find({tv[3 * f + (k + 1) % 3], tv[3 * f + k]});
                if (it == edge.end()) return ETAC_ERR_VALUE;   // open mesh
                const V3 &g = fn[it->second];
                o[3 + 3 * k] = fn[f].x + g.x;
                o[4 + 3 * k] = fn[f].y + g.y;
                o[5 + 3 * k] = fn[f].z + g.z;
            }
            for (int k = 0; k < 3; ++k) {   // vertices a, b, c
                const V3 &s = vsum[tv[3 * f + k]];
                o[12 + 3 * k] = s.x; o[13 + 3 * k] = s.y; o[14 + 3 * k] = s.z;
            }
        }
        // clusters
        BuiltMesh bm;
        bm.order.resize(nt);
        std::iota(bm.order.begin(), bm.order.end(), 0);
        split(bm.order, 0, nt, cen, bm);
        const int c_first = (int)ball.size();
        double rmax = 0.0;
        for (size_t ci = 0; ci < bm.clusters.size(); ++ci)   // the kernel derives the ranges
            if (bm.clusters[ci].first != kCluster * (int)ci ||
                bm.clusters[ci].second != std::min(nt, kCluster * (int)ci + kCluster))
                return ETAC_ERR_VALUE;
        for (auto [lo, hi] : bm.clusters) {
            V3 mn{INFINITY, INFINITY, INFINITY}, mx{-INFINITY, -INFINITY, -INFINITY};
            for (int i = lo; i < hi; ++i)
                for (int k = 0; k < 3; ++k) {
                    const V3 p = vtx(tv[3 * bm.order[i] + k]);
                    mn = V3{std::min(mn.x, p.x), std::min(mn.y, p.y), std::min(mn.z, p.z)};
                    mx = V3{std::max(mx.x, p.x), std::max(mx.y, p.y), std::max(mx.z, p.z)};
                }
            const V3 cc{(mn.x + mx.x) / 2.0, (mn.y + mx.y) / 2.0, (mn.z + mx.z) / 2.0};
            double r = 0.0;
            for (int i = lo; i < hi; ++i)
                for (int k = 0; k < 3; ++k) {
                    const V3 d = sub(vtx(tv[3 * bm.order[i] + k]), cc);
                    r = std::max(r, std::sqrt(dot(d, d)));
                    const V3 p = vtx(tv[3 * bm.order[i] + k]);
                    rmax = std::max(rmax, std::sqrt(dot(p, p)));
                }
            const double scale = std::sqrt(dot(cc, cc)) + r;
            ball.push_back(make_double4(cc.x, cc.y, cc.z, r + 1e-6 + 1e-12 * scale));
            // oriented box: one axis along the area-weighted mean normal (thin
            // for a surface patch), one towards the farthest vertex in the
            // plane across it, the third their cross product
            V3 nsum{0.0, 0.0, 0.0};
            for (int i = lo; i < hi; ++i) {
                const int f = bm.order[i];
                const V3 a = vtx(tv[3 * f]), b = vtx(tv[3 * f + 1]), c = vtx(tv[3 * f + 2]);
                const V3 ab = sub(b, a), ac = sub(c, a);
                nsum = V3{nsum.x + (ab.y * ac.z - ab.z * ac.y), nsum.y + (ab.z * ac.x - ab.x * ac.z),
                          nsum.z + (ab.x * ac.y - ab.y * ac.x)};
            }
            auto unit = [](V3 v, V3 fallback) {
                const double l = std::sqrt(dot(v, v));
                return l > 1e-12 ? V3{v.x / l, v.y / l, v.z / l} : fallback;
            };
            const V3 ax0 = unit(nsum, V3{0.0, 0.0, 1.0});
            V3 far{0.0, 0.0, 0.0};
            double fl = -1.0;
            for (int i = lo; i < hi; ++i)
                for (int k = 0; k < 3; ++k) {
                    const V3 d = sub(vtx(tv[3 * bm.order[i] + k]), cc);
                    const double dn = dot(d, ax0);
                    const V3 u{d.x - dn * ax0.x, d.y - dn * ax0.y, d.z - dn * ax0.z};
                    if (dot(u, u) > fl) { fl = dot(u, u); far = u; }
                }
            const V3 any = std::fabs(ax0.x) < 0.9 ? V3{1.0, 0.0, 0.0} : V3{0.0, 1.0, 0.0};
            const V3 anyp{any.y * ax0.z - any.z * ax0.y, any.z * ax0.x - any.x * ax0.z, any.x * ax0.y - any.y * ax0.x};
            V3 ax1 = unit(far, unit(anyp, V3{0.0, 1.0, 0.0}));
            const double p1 = dot(ax1, ax0);   // re-orthogonalise against rounding
            ax1 = unit(V3{ax1.x - p1 * ax0.x, ax1.y - p1 * ax0.y, ax1.z - p1 * ax0.z}, ax1);
            const V3 ax2 = unit(V3{ax0.y * ax1.z - ax0.z * ax1.y, ax0.z * ax1.x - ax0.x * ax1.z,
                                   ax0.x * ax1.y - ax0.y * ax1.x}, V3{0.0, 0.0, 1.0});
            const V3 ax[3] = {ax0, ax1, ax2};
            double lo_k[3] = {INFINITY, INFINITY, INFINITY}, hi_k[3] = {-INFINITY, -INFINITY, -INFINITY};
            for (int i = lo; i < hi; ++i)
                for (int k = 0; k < 3; ++k) {
                    const V3 d = sub(vtx(tv[3 * bm.order[i] + k]), cc);
                    for (int j = 0; j < 3; ++j) {
                        lo_k[j] = std::min(lo_k[j], dot(d, ax[j]));
                        hi_k[j] = std::max(hi_k[j], dot(d, ax[j]));
                    }
                }
            V3 bc = cc;
            for (int j = 0; j < 3; ++j) {
                const double mid = (lo_k[j] + hi_k[j]) / 2.0;
                bc = V3{bc.x + mid * ax[j].x, bc.y + mid * ax[j].y, bc.z + mid * ax[j].z};
            }
            double half[3] = {0.0, 0.0, 0.0};
            for (int i = lo; i < hi; ++i)
                for (int k = 0; k < 3; ++k) {
                    const V3 d = sub(vtx(tv[3 * bm.order[i] + k]), bc);
                    for (int j = 0; j < 3; ++j) half[j] = std::max(half[j], std::fabs(dot(d, ax[j])));
                }
            const double bx[16] = {bc.x, bc.y, bc.z, ax0.x, ax0.y, ax0.z, ax1.x, ax1.y, ax1.z, ax2.x, ax2.y, ax2.z,
                                   half[0] + 1e-6 + 1e-12 * scale, half[1] + 1e-6 + 1e-12 * scale,
                                   half[2] + 1e-6 + 1e-12 * scale, 0.0};
            box.insert(box.end(), bx, bx + 16);
        }
        for (int i = 0; i < nt; ++i) {
            const int f = bm.order[i], slot = t0 + i;
            for (int k = 0; k < 3; ++k) {
                const V3 p = vtx(tv[3 * f + k]);
                corner[(size_t)(3 * k) * T + slot] = (float)p.x;
                corner[(size_t)(3 * k + 1) * T + slot] = (float)p.y;
                corner[(size_t)(3 * k + 2) * T + slot] = (float)p.z;
            }
            orig[slot] = f;
            std::copy(mpn.begin() + (size_t)21 * f, mpn.begin() + (size_t)21 * (f + 1), pn.begin() + (size_t)21 * slot);
        }
        mesh[m] = make_int4(t0, t0 + nt, c_first, (int)ball.size());
        {
            V3 lo{INFINITY, INFINITY, INFINITY}, hi{-INFINITY, -INFINITY, -INFINITY};
            for (int f = 0; f < nt; ++f)
                for (int k = 0; k < 3; ++k) {
                    const V3 p = vtx(tv[3 * f + k]);
                    lo = V3{std::min(lo.x, p.x), std::min(lo.y, p.y), std::min(lo.z, p.z)};
                    hi = V3{std::max(hi.x, p.x), std::max(hi.y, p.y), std::max(hi.z, p.z)};
                }
            const HostMesh hm{tv, verts, &bm.order, &bm.clusters, ball.data() + c_first, mpn.data()};
            build_grid(hm, lo, hi, grid_lo[m], grid_dim[m], grid_bits);
        }
        float rf = (float)rmax;
        if ((double)rf < rmax) rf = std::nextafter(rf, INFINITY);
        radius[m] = rf;
    }

    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(nullptr, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return ETAC_ERR_CAPTURE;
    etac_meshset *ms = new (std::nothrow) etac_meshset();
    if (!ms) return ETAC_ERR_HIP;
    ms->n_allocs = 0;
    if (hipGetDevice(&ms->device) != hipSuccess) {
        delete ms;
        return ETAC_ERR_HIP;
    }
    auto upload = [&](const void *src, size_t bytes, void **dst) -> hipError_t {
        void *d = nullptr;
        if (ms->n_allocs >= (int)(sizeof(ms->allocs) / sizeof(ms->allocs[0]))) return hipErrorOutOfMemory;
        hipError_t e = hipMalloc(&d, bytes ? bytes : 1);
        if (e != hipSuccess) return e;
        ms->allocs[ms->n_allocs++] = d;
        *dst = d;
        return bytes ? hipMemcpy(d, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
    };
    void *p[9];
    hipError_t e = hipSuccess;
    const void *src[9] = {mesh.data(), radius.data(), corner.data(), orig.data(), pn.data(), box.data(),
                          grid_lo.data(), grid_dim.data(), grid_bits.data()};
    const size_t bytes[9] = {mesh.size() * sizeof(int4), radius.size() * sizeof(float),
                             corner.size() * sizeof(float), orig.size() * sizeof(int), pn.size() * sizeof(double),
                             box.size() * sizeof(double), grid_lo.size() * sizeof(float4),
                             grid_dim.size() * sizeof(int4), grid_bits.size() * sizeof(unsigned)};
    for (int i = 0; i < 9 && e == hipSuccess; ++i) e = upload(src[i], bytes[i], &p[i]);
    if (e != hipSuccess) {
        etac_meshset_destroy(ms);
        return ETAC_ERR_HIP;
    }
    ms->d = MeshSetDev{(const int4 *)p[0], (const float *)p[1], (const float *)p[2], (const int *)p[3],
                       (const double *)p[4], (const double *)p[5], (const float4 *)p[6], (const int4 *)p[7],
                       (const unsigned *)p[8], n_meshes, T, (int)ball.size()};
    *out = ms;
    return ETAC_OK;
}

etac_status etac_meshset_create(int32_t n_meshes, const int32_t *tri_offset, int32_t n_verts, const float *verts,
                                const int32_t *tris, etac_meshset **out) {
    try {   // host containers and worker threads may throw; no exception crosses the C ABI
        return meshset_create(n_meshes, tri_offset, n_verts, verts, tris, out);
    } catch (...) {
        return ETAC_ERR_HIP;
    }
}

etac_status etac_meshset_destroy(etac_meshset *ms) {
    if (!ms) return ETAC_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(ms->device);
    (void)hipDeviceSynchronize();
    for (int i = 0; i < ms->n_allocs; ++i) (void)hipFree(ms->allocs[i]);
    (void)hipSetDevice(cur);
    delete ms;
    return ETAC_OK;
}

}  // extern "C"

// Articulated hand on gfx950: every patch rides on one link of the hand, its
// nodes, normals, origin, u_hat and U given in that link's frame.  Contact
// of a patch covers the env's objects and the collision primitives of the
// other links it may touch (self-contact, Sec. III-A contact detection),
// all expressed in the patch's link frame; the contact reward of Sec. IV-B
// (contact-reward equation) comes from per-item counts the contact pass
// already produces.
//
//   k_hand_scene  : one thread per (env, patch) item, fills the item's row of
//                   candidates (relative poses, FP64 then rounded to FP32,
//                   culled against the patch's bounding sphere);
//   k_hand_reward : one thread per env, n_a, touched links and r_contact;
//   k_pose_hand   : one thread per (env, object or link), the chain rule
//                   from the rows' relative-pose gradients to object and
//                   link poses, summed in item and slot order in FP64.
// The fused step, the contact pass and the adjoint kernels run unchanged on
// the rows (SceneDev with one row per item).
#include "etac_device.h"

namespace etac {

// Relative pose of a world pose (Rw, tw) in the frame (Rl, tl):
//   R' = Rl^T Rw,  t' = Rl^T (tw - tl),
// every entry a sum of three products taken as (x0 y0 + x1 y1) + x2 y2 in
// FP64, no fused multiply-add, then rounded to FP32 (the values the contact
// test reads).
__device__ __forceinline__ void relative_pose(const double Rl[9], const double tl[3], const double Rw[9],
                                              const double tw[3], float Rr[9], float tr[3]) {
#pragma clang fp contract(off)
    const double d[3] = {tw[0] - tl[0], tw[1] - tl[1], tw[2] - tl[2]};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            Rr[a * 3 + c] = (float)((Rl[0 * 3 + a] * Rw[0 * 3 + c] + Rl[1 * 3 + a] * Rw[1 * 3 + c]) +
                                    Rl[2 * 3 + a] * Rw[2 * 3 + c]);
#pragma unroll
    for (int c = 0; c < 3; ++c)
        tr[c] = (float)((Rl[0 * 3 + c] * d[0] + Rl[1 * 3 + c] * d[1]) + Rl[2 * 3 + c] * d[2]);
}

// World pose of link j's collision primitive: Rw = Rj C_R, tw = Rj C_t + tj
// (same summation order).
__device__ __forceinline__ void primitive_world(const double Rj[9], const double tj[3], const float *CR,
                                                const float *Ct, double Rw[9], double tw[3]) {
#pragma clang fp contract(off)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            Rw[a * 3 + c] = (Rj[a * 3 + 0] * (double)CR[0 * 3 + c] + Rj[a * 3 + 1] * (double)CR[1 * 3 + c]) +
                            Rj[a * 3 + 2] * (double)CR[2 * 3 + c];
        tw[a] = ((Rj[a * 3 + 0] * (double)Ct[0] + Rj[a * 3 + 1] * (double)Ct[1]) + Rj[a * 3 + 2] * (double)Ct[2]) +
                tj[a];
    }
}

__device__ __forceinline__ void load_pose(const float *R, const float *t, double Rd[9], double td[3]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) Rd[i] = R[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) td[i] = t[i];
}

struct HandSceneParams {
    MeshDev mesh;
    SceneDev world;
    LinksDev links;
    HandDev hand;
    int n_items;
};

// Append one candidate to the item's row when its bounding ball may reach the
// patch (the test cull_objects repeats on the row, on the same FP32 values).
__device__ __forceinline__ void put_candidate(const HandSceneParams &p, size_t row, const float4 &b, int &n,
                                              int8_t id, int type, const float *shape, const float Rr[9],
                                              const float tr[3]) {
    if (!ball_reaches(b, type, shape, tr)) return;
    const size_t s = row * p.hand.cap + n;
    p.hand.type[s] = type;
    p.hand.src[s] = id;
#pragma unroll
    for (int i = 0; i < 4; ++i) p.hand.shape[4 * s + i] = shape[i];
#pragma unroll
    for (int i = 0; i < 9; ++i) p.hand.rot[9 * s + i] = Rr[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) p.hand.trans[3 * s + i] = tr[i];
    ++n;
}

__global__ __launch_bounds__(256) void k_hand_scene(HandSceneParams p) {
    const int item = blockIdx.x * 256 + threadIdx.x;
    if (item >= p.n_items) return;
    const MeshDev &M = p.mesh;
    const HandDev &H = p.hand;
    const int K = M.K, L = H.L, O = p.world.O;
    const int e = item / K, k = item - e * K;
    const int l = H.patch_link[k];
    double Rl[9], tl[3];
    load_pose(p.links.rot + ((size_t)e * L + l) * 9, p.links.trans + ((size_t)e * L + l) * 3, Rl, tl);
    const float4 b = M.bound[k];
    const size_t row = (size_t)item;
    int n = 0;
    // the env's objects (ids 0 .. O-1), then the other links' primitives (O + j)
    const int no = min(p.world.n_obj[e], O);
    for (int o = 0; o < no; ++o) {
        const size_t eo = (size_t)e * O + o;
        const int ty = p.world.type[eo];
        if ((unsigned)ty > (unsigned)ETAC_CAPSULE) continue;
        double Rw[9], tw[3];
        load_pose(p.world.rot + 9 * eo, p.world.trans + 3 * eo, Rw, tw);
        float Rr[9], tr[3];
        relative_pose(Rl, tl, Rw, tw, Rr, tr);
        put_candidate(p, row, b, n, (int8_t)o, ty, p.world.shape + 4 * eo, Rr, tr);
    }
    const int n_ext = n;
    const unsigned pairs = H.collide[l] & ~(1u << l);
    for (int j = 0; j < L; ++j) {
        if (!((pairs >> j) & 1u) || (unsigned)H.ptype[j] > (unsigned)ETAC_CAPSULE) continue;
        double Rj[9], tj[3], Rw[9], tw[3];
        load_pose(p.links.rot + ((size_t)e * L + j) * 9, p.links.trans + ((size_t)e * L + j) * 3, Rj, tj);
        primitive_world(Rj, tj, H.prot + 9 * j, H.ptrans + 3 * j, Rw, tw);
        float Rr[9], tr[3];
        relative_pose(Rl, tl, Rw, tw, Rr, tr);
        put_candidate(p, row, b, n, (int8_t)(O + j), H.ptype[j], H.pshape + 4 * j, Rr, tr);
    }
    H.n_obj[row] = n;
    H.n_ext[row] = n_ext;
}

hipError_t launch_hand_scene(const Plan &pl, const SceneDev &world, const LinksDev &links, SceneDev *rows,
                             hipStream_t st) {
    const HandDev &H = *pl.hand;
    HandSceneParams p{pl.mesh, world, links, H, world.E * pl.K};
    *rows = SceneDev{H.n_obj, H.type, H.shape, H.rot, H.trans, world.E, H.cap};
    rows->rows_per_env = pl.K;
    rows->src = H.src;
    rows->n_ext = H.n_ext;
    if (p.n_items == 0) return hipSuccess;
    hipLaunchKernelGGL(k_hand_scene, dim3((p.n_items + 255) / 256), dim3(256), 0, st, p);
    return hipGetLastError();
}

// r_contact = (links touched by an object) / L + omega_a (n_a / N if n_a > 0,
// else -0.1), n_a the nodes won by objects over the hand.
__global__ __launch_bounds__(256) void k_hand_reward(int E, int K, int L, int N, const int *patch_link,
                                                     const int32_t *n_touch, float omega_a, int32_t *n_a,
                                                     uint32_t *link_mask, float *r_contact) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= E) return;
    long long s = 0;
    unsigned mask = 0;
    for (int k = 0; k < K; ++k) {
        const int t = n_touch[(size_t)e * K + k];
        s += t;
        if (t > 0) mask |= 1u << patch_link[k];
    }
    if (n_a) n_a[e] = (int32_t)s;
    if (link_mask) link_mask[e] = mask;
    if (r_contact) {
        const double ra = s > 0 ? (double)s / (double)N : -0.1;
        r_contact[e] = (float)((double)__popc(mask) / (double)L + (double)omega_a * ra);
    }
}

hipError_t launch_hand_reward(const Plan &pl, int n_envs, const int32_t *n_touch, float omega_a, int32_t *n_a,
                              uint32_t *link_mask, float *r_contact, hipStream_t st) {
    if (n_envs == 0 || (!n_a && !link_mask && !r_contact)) return hipSuccess;
    hipLaunchKernelGGL(k_hand_reward, dim3((n_envs + 255) / 256), dim3(256), 0, st, n_envs, pl.K, pl.hand->L, pl.N,
                       pl.hand->patch_link, n_touch, omega_a, n_a, link_mask, r_contact);
    return hipGetLastError();
}

// Chain rule of the hand's pose adjoint.  A row slot of item (e, k) on link
// l holds G' = dL/dR', g' = dL/dt' of its candidate's relative pose.  With the
// candidate's world pose (Rw, tw):
//   source : dL/dRw = Rl G',  dL/dtw = Rl g'
//            (link j's primitive: dL/dRj += dL/dRw C_R^T + dL/dtw C_t^T,
//             dL/dtj += dL/dtw);
//   frame  : dL/dRl += Rw G'^T + (tw - tl) g'^T,  dL/dtl -= Rl g'.
// One thread per (env, target), target an object (t < O) or link t - O;
// contributions are added in item and slot order in FP64.
struct PoseHandParams {
    SceneDev world;
    LinksDev links;
    HandDev hand;
    const float *part;       // [E K][cap][12]
    int E, K;
    float *grad_rot, *grad_trans, *grad_link_rot, *grad_link_trans;
};

__global__ __launch_bounds__(256) void k_pose_hand(PoseHandParams p) {
    const HandDev &H = p.hand;
    const int O = p.world.O, L = H.L, T = O + L;
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= p.E * T) return;
    const int e = idx / T, target = idx - e * T;
    const bool is_link = target >= O;
    const int tl_link = target - O;
    double G[9], g[3];
#pragma unroll
    for (int i = 0; i < 9; ++i) G[i] = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) g[i] = 0.0;
    for (int k = 0; k < p.K; ++k) {
        const size_t row = (size_t)e * p.K + k;
        const int l = H.patch_link[k];
        const bool frame = is_link && l == tl_link;
        const int n = min(H.n_obj[row], H.cap);
        double Rl[9], tl[3];
        bool have_l = false;
        for (int s = 0; s < n; ++s) {
            const int src = H.src[row * H.cap + s];
            if (!frame && src != target) continue;
            if (!have_l) {
                load_pose(p.links.rot + ((size_t)e * L + l) * 9, p.links.trans + ((size_t)e * L + l) * 3, Rl, tl);
                have_l = true;
            }
            const float *gp = p.part + (row * H.cap + s) * 12;
            double Gp[9], tp[3];
#pragma unroll
            for (int i = 0; i < 9; ++i) Gp[i] = gp[i];
#pragma unroll
            for (int i = 0; i < 3; ++i) tp[i] = gp[9 + i];
            double GRw[9], gtw[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    GRw[a * 3 + c] = Rl[a * 3 + 0] * Gp[0 * 3 + c] + Rl[a * 3 + 1] * Gp[1 * 3 + c] +
                                     Rl[a * 3 + 2] * Gp[2 * 3 + c];
                gtw[a] = Rl[a * 3 + 0] * tp[0] + Rl[a * 3 + 1] * tp[1] + Rl[a * 3 + 2] * tp[2];
            }
            double Rw[9], tw[3];
            if (src < O) {
                load_pose(p.world.rot + ((size_t)e * O + src) * 9, p.world.trans + ((size_t)e * O + src) * 3, Rw, tw);
            } else {
                const int j = src - O;
                double Rj[9], tj[3];
                load_pose(p.links.rot + ((size_t)e * L + j) * 9, p.links.trans + ((size_t)e * L + j) * 3, Rj, tj);
                primitive_world(Rj, tj, H.prot + 9 * j, H.ptrans + 3 * j, Rw, tw);
            }
            if (frame) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
#pragma unroll
                    for (int b = 0; b < 3; ++b)
                        G[a * 3 + b] += (Rw[a * 3 + 0] * Gp[b * 3 + 0] + Rw[a * 3 + 1] * Gp[b * 3 + 1] +
                                         Rw[a * 3 + 2] * Gp[b * 3 + 2]) +
                                        (tw[a] - tl[a]) * tp[b];
                    g[a] -= gtw[a];
                }
            } else if (src < O) {
#pragma unroll
                for (int i = 0; i < 9; ++i) G[i] += GRw[i];
#pragma unroll
                for (int i = 0; i < 3; ++i) g[i] += gtw[i];
            } else {
                const float *CR = H.prot + 9 * (src - O), *Ct = H.ptrans + 3 * (src - O);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
#pragma unroll
                    for (int b = 0; b < 3; ++b)
                        G[a * 3 + b] += GRw[a * 3 + 0] * (double)CR[b * 3 + 0] + GRw[a * 3 + 1] * (double)CR[b * 3 + 1] +
                                        GRw[a * 3 + 2] * (double)CR[b * 3 + 2] + gtw[a] * (double)Ct[b];
                    g[a] += gtw[a];
                }
            }
        }
    }
    float *gr = is_link ? p.grad_link_rot + ((size_t)e * L + tl_link) * 9 : p.grad_rot + ((size_t)e * O + target) * 9;
    float *gt = is_link ? p.grad_link_trans + ((size_t)e * L + tl_link) * 3
                        : p.grad_trans + ((size_t)e * O + target) * 3;
#pragma unroll
    for (int i = 0; i < 9; ++i) gr[i] = (float)G[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) gt[i] = (float)g[i];
}

hipError_t launch_pose_hand(const Plan &pl, const SceneDev &world, const LinksDev &links, float *grad_rot,
                            float *grad_trans, float *grad_link_rot, float *grad_link_trans, hipStream_t st) {
    if (world.E == 0) return hipSuccess;
    PoseHandParams p{world, links, *pl.hand, pl.hand->pose_part, world.E, pl.K,
                     grad_rot, grad_trans, grad_link_rot, grad_link_trans};
    const int nt = world.E * (world.O + pl.hand->L);
    hipLaunchKernelGGL(k_pose_hand, dim3((nt + 255) / 256), dim3(256), 0, st, p);
    return hipGetLastError();
}

}  // namespace etac

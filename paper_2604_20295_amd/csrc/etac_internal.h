// Internal declarations shared by the host API and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/etac.h"

namespace etac {

constexpr int kWG = 256;           // threads per workgroup: 4 waves of 64
constexpr int kWaves = kWG / 64;
constexpr int kSavedWords = ETAC_SAVED_WORDS;   // pooling record per (env, patch) item
constexpr int kRecWords = 10564;                  // parameter-gradient record per item with contact
constexpr int kRedColsMax = 10624 + 8192;         // columns of the parameter reduction
constexpr int kMaxPatches = 1024;  // per-patch counters of the contact kernel live in LDS
constexpr int kDefaultWgPerCu = 2;
constexpr int kDefaultBatch = 4;   // work-queue positions claimed per atomic
constexpr int kDefaultDecayWgPerCu = 3;
constexpr int kDefaultNetBatch = 2;   // workgroups per CU of the decay-adjoint kernel

// Device view of the plan's mesh copy.
struct MeshDev {
    const float *pos;      // [3][N]
    const float *nrm;      // [3][N]
    const float *origin;   // [K][3]
    const int *offset;     // [K+1]
    const float4 *bound;   // [K] conservative bounding sphere (cx, cy, cz, radius)
    const int16_t *node_patch;  // [N] patch of each node
    const int *order;      // [K] patches sorted by node count, largest first
    const float *xbound;   // [K] largest |component| of p - o_k and of n over the patch's nodes (rounded up)
    int K, N, n_max;
};

// Objects the contact test sees, in rows of O candidates: one row per env
// (rows_per_env = 0), or one row per (env, patch) item (rows_per_env = K:
// the articulated hand, whose rows hold each patch's candidates in its link
// frame).  With `src`, contact_obj reports src[row][winner] instead of the
// winner's slot; with `n_ext`, slots below n_ext[row] are external objects
// (their nodes count towards the contact reward).
struct SceneDev {
    const int *n_obj;      // [rows]
    const int *type;       // [rows][O]
    const float *shape;    // [rows][O][4]
    const float *rot;      // [rows][O][9]
    const float *trans;    // [rows][O][3]
    int E, O;
    int rows_per_env = 0;
    const int8_t *src = nullptr;   // [rows][O]
    const int *n_ext = nullptr;    // [rows]
};

__host__ __device__ inline size_t scene_row(const SceneDev &S, int e, int k) {
    return S.rows_per_env ? (size_t)e * S.rows_per_env + k : (size_t)e;
}

// Articulated hand (etac_plan_set_hand): the link description on the device
// and the per-item candidate table its pre-pass fills.
constexpr int kMaxLinks = 24;
constexpr int kMaxRowObj = 32;     // candidates per item row (one bit each in a 32-bit mask)

struct HandDev {
    int L;
    int cap;                       // row capacity: plan max_obj + largest self-contact set
    const int *patch_link;         // [K]
    const unsigned *collide;       // [L]
    const int *ptype;              // [L] primitive type or -1
    const float *pshape;           // [L][4]
    const float *prot;             // [L][9] primitive pose in its link frame
    const float *ptrans;           // [L][3]
    // candidate table, one row per (env, patch) item
    int *n_obj;                    // [E K]
    int *n_ext;                    // [E K]
    int *type;                     // [E K][cap]
    float *shape;                  // [E K][cap][4]
    float *rot;                    // [E K][cap][9]
    float *trans;                  // [E K][cap][3]
    int8_t *src;                   // [E K][cap]
    float *pose_part;              // [E K][cap][12] relative-pose gradient partials (backward)
    int *n_touch;                  // [E K] reward counts when the caller passes none
};

// Per-step inputs of the hand: link poses.
struct LinksDev {
    const float *rot;              // [E][L][9]
    const float *trans;            // [E][L][3]
};

struct ModelDev {
    int mode;
    const float *alpha;    // [K]
    const float *phi;      // [17411] or null in decay-only mode
};

// Per-workgroup scratch of the persistent kernels (device memory).
struct Scratch {
    float *uhat_node;      // [G][3][n_max] u_hat of every node of the current item (0 passive)
    float *resid;          // [G][3][n_max] residual-network output
    int *alist;            // [G][n_max]    active node indices (patch-local, ascending)
    int *plist;            // [G][n_max]    passive node indices (patch-local, ascending)
    unsigned *counter;     // [8]           work-queue counters (self-resetting)
    int n_max;
};

// Backward scratch (plan flag ETAC_PLAN_BACKWARD).
struct BwdScratch {
    float *guhat;          // [G][3][n_max]    dL/du_hat per node of the current item
    float *phi_part;       // [E*K][kRecWords] per-item parameter-gradient records
    int *rec_map;          // [17411]          reduction column of every parameter
    float *alpha_part;     // [E*K]            per-item dL/dalpha partials
    float *pose_part;      // [E*K][O][12]     per-item pose-gradient partials
    int *item_flag;        // [E*K]            1 if the item wrote partials
    double *phi_seg;       // [64][kRedColsMax] segment sums of the parameter reduction
    // hand-over from the decay kernel to the network / contact kernel
    int8_t *cobj_st;       // [E][N]    contact winners of every candidate item (step adjoint)
    float *uhat_st;        // [3][E][N] u_hat of active nodes (step adjoint)
    float *gh_st;          // [3][E][N] dL/du_hat of active nodes after the decay adjoint
    int *m_st;             // [E*K]     active-node count of every item
    float *gmax_st;        // [E*K]     largest |dL/dU| component over each contacted item's passive nodes
    int *live;             // [E*K]     queue positions of the items with contact, in queue order
    int *seg_cnt;          // [n_seg + 1] items with contact per 1024 queue positions; [n_seg] = total
};

// Event pairs bracketing kernel launches (etac_plan_set_timing).
struct Timers {
    bool on;
    hipEvent_t ev[ETAC_TIMER_COUNT][ETAC_TIMER_SLOTS][2];
    int n[ETAC_TIMER_COUNT];
};

struct Plan {
    int device;
    int cu_count;
    int wg_per_cu;
    int grid;              // persistent workgroups
    int batch;             // forward work-queue positions claimed per atomic (1 .. 64)
    int bwd_batch;         // adjoint work-queue positions claimed per atomic (1 .. 64)
    int decay_wg_per_cu;   // workgroups per CU of the decay-adjoint kernel (1 .. 8)
    int net_batch;         // list positions per claim of the network-adjoint kernel (1 .. 64)
    int n_envs, max_obj, K, N, n_max;
    uint32_t flags;
    MeshDev mesh;
    Scratch scr;
    BwdScratch bwd;
    bool has_bwd;
    // device allocations owned by the plan
    void *allocs[48];
    int n_allocs;
    int64_t scratch_bytes;
    Timers *timers;        // null until timing is first turned on
    HandDev *hand;         // null until etac_plan_set_hand (host copy of the device view)
    void *hand_mem;        // the hand's device block (one allocation)
    float *reg_rest;       // [K][8] regressor outputs of the patches at U = 0
    float *reg_pooled;     // [E K + K][256] regressor pooled features, one row per processed item
    int *reg_row;          // [E K + K] the item of each row
};

// Open a timed span of timer k on stream st; returns the slot, or -1 when
// timing is off or the stream is being captured.
inline int timer_begin(const Plan &p, int k, hipStream_t st) {
    Timers *t = p.timers;
    if (!t || !t->on) return -1;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return -1;
    const int slot = t->n[k] % ETAC_TIMER_SLOTS;
    return hipEventRecord(t->ev[k][slot][0], st) == hipSuccess ? slot : -1;
}

inline void timer_end(const Plan &p, int k, int slot, hipStream_t st) {
    if (slot < 0) return;
    if (hipEventRecord(p.timers->ev[k][slot][1], st) == hipSuccess) p.timers->n[k]++;
}

// Launchers (return hipError_t of the launch).
// Real-sensor regressor: taxels [E][K][8] from u [3][E][N] (n_envs = E).
hipError_t launch_regress(const Plan &p, const float *reg, int n_envs, const float *u, const int32_t *n_active,
                          float *taxels, hipStream_t st);
hipError_t launch_contact(const Plan &p, const SceneDev &s, int8_t *cobj, float *uhat, int32_t *n_active,
                          hipStream_t st);
hipError_t launch_contact_rows(const Plan &p, const SceneDev &s, int8_t *cobj, float *uhat, int32_t *n_active,
                               int32_t *n_touch, hipStream_t st);
hipError_t launch_step(const Plan &p, const SceneDev *s, const ModelDev &m, int n_envs,
                       const int8_t *cobj_in, const float *uhat_in, float *u, int8_t *cobj_out,
                       int32_t *n_active, uint32_t *saved, hipStream_t st, int32_t *n_touch = nullptr);
// hand: with `links`, pose partials are relative-pose gradients of the hand's
// candidate rows, chained to object and link poses (grad_link_rot/trans).
hipError_t launch_backward(const Plan &p, const SceneDev *s, const ModelDev &m, int n_envs,
                           const int8_t *cobj_in, const float *uhat_in, const float *grad_u,
                           const uint32_t *saved, float *grad_uhat, float *grad_rot, float *grad_trans,
                           float *grad_alpha, float *grad_phi, hipStream_t st, const SceneDev *world = nullptr,
                           const LinksDev *links = nullptr, float *grad_link_rot = nullptr,
                           float *grad_link_trans = nullptr);
// hand pre-pass: fills the candidate rows of every (env, patch) item from the
// world scene and the link poses; returns the row view in *rows.
hipError_t launch_hand_scene(const Plan &p, const SceneDev &world, const LinksDev &links, SceneDev *rows,
                             hipStream_t st);
hipError_t launch_hand_reward(const Plan &p, int n_envs, const int32_t *n_touch, float omega_a, int32_t *n_a,
                              uint32_t *link_mask, float *r_contact, hipStream_t st);
hipError_t launch_pose_hand(const Plan &p, const SceneDev &world, const LinksDev &links, float *grad_rot,
                            float *grad_trans, float *grad_link_rot, float *grad_link_trans, hipStream_t st);
hipError_t init_record_map(const Plan &p);

// The fused step with its scratch in the library's file-scope device array
// (etac_step_static): size of the array, the slice one persistent workgroup
// needs, the once-per-device lookup of the array's address, and the launch.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
size_t static_scratch_per_wg(int n_max);
hipError_t static_scratch_init(int device);
hipError_t launch_step_static(const Plan &p, const SceneDev &s, const ModelDev &m, float *u, int8_t *cobj,
                              int32_t *n_active, uint32_t *saved, hipStream_t st);
hipError_t launch_contact_backward(const Plan &p, const SceneDev &s, const float *grad_uhat,
                                   float *grad_rot, float *grad_trans, hipStream_t st);

// Triangle meshes of rigid objects on the device (one etac_meshset).  The
// triangles of each mesh are stored in cluster order (clusters of at most 64
// spatially close triangles); `orig` keeps each triangle's index within its
// mesh as given, which breaks distance ties.
struct MeshSetDev {
    const int4 *mesh;        // [M] first triangle, end triangle, first cluster, end cluster
    const float *radius;     // [M] ball about the object origin holding the mesh (rounded up)
    const float *corner;     // [9][T] a.x a.y a.z b.x b.y b.z c.x c.y c.z per triangle
    const int *orig;         // [T] index of the triangle within its mesh, as given
    const double *pn;        // [T][7][3] pseudo-normals: face, edges ab bc ca, vertices a b c
    const double *box;       // [C][16] cluster bounding box: centre, three unit axes, half extents (with margin)
    // occupancy grid per mesh over its bounding box: bit (i, j, k) is clear
    // when every point of that cell is certainly outside the mesh
    const float4 *grid_lo;   // [M] box corner (object frame), 1 / cell size
    const int4 *grid_dim;    // [M] cells along x, y, z; first bit in grid_bits
    const unsigned *grid_bits;
    int M, T, C;
};

hipError_t launch_contact_mesh(const Plan &p, const MeshSetDev &ms, const SceneDev &s, int8_t *cobj, float *uhat,
                               int32_t *n_active, int32_t *hit, hipStream_t st);
hipError_t launch_contact_mesh_backward(const Plan &p, const MeshSetDev &ms, const SceneDev &s,
                                        const float *grad_uhat, const int8_t *cobj, const int32_t *hit,
                                        float *grad_rot, float *grad_trans, hipStream_t st);

}  // namespace etac

struct etac_meshset {
    int device;
    etac::MeshSetDev d;
    void *allocs[16];
    int n_allocs;
};

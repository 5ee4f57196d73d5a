/*
 * etac.h -- C ABI of the MI355X ETac tactile step library (libetac.so).
 *
 * What the library computes (ETac, Sec. III-A):
 *   contact   : surface nodes of an elastomer patch lying strictly inside a
 *               rigid primitive are active; each gets the displacement u_hat
 *               that moves it to the closest point of the primitive surface
 *               (the local penalty-style contact displacement, Sec. III-A
 *               "Overview"); the deepest object wins, lowest index on ties.
 *   propagate : passive nodes get U_p = Omega U_a + Phi_p(P, U_hat, N)
 *               (Eq. 2) with Omega[i,j] = exp(-alpha ||p_j - p_i||) (Eq. 1)
 *               and Phi the PointNet residual network of Sec. III-A
 *               "Residual Displacement Correction"; active nodes keep u_hat;
 *               a patch with no active node has U = 0.
 *   backward  : the adjoint of L = sum_i g_i . U_i with respect to object
 *               poses (R, t), alpha and the network parameters (ETac is
 *               differentiable, Table 1; Sec. III-A fits alpha and Phi by
 *               gradient descent).
 *
 * Units: mm and 1/mm.  All float arrays are IEEE FP32.
 *
 * Layouts (row-major, "SoA" = component-major):
 *   node arrays          [3][N]       x for all nodes, then y, then z
 *   per-env node arrays  [3][E][N]    component, env, node
 *   contact_obj          [E][N]       int8: -1 passive, else winning object
 *   n_active             [E][K]       int32 active-node count per patch
 *   object arrays        [E][O][...]  type int32; shape float[4]; rot float[9]
 *                                     row-major R (world x = R q + t);
 *                                     trans float[3]
 *   primitive shapes     sphere (r); box (hx, hy, hz half extents);
 *                        capsule (r, half segment length L along object z)
 *   phi                  packed FP32 network parameters, ETAC_PHI_SIZE floats:
 *                        W1[64][9] b1[64] W2[64][64] b2[64] W3[64][64] b3[64]
 *                        W4[64][128] b4[64] W5[3][64] b5[3]
 *                        network input x_i = [p_i - o_k, n_i, U_hat_i]
 *                        (U_hat_i = 0 on passive nodes); h1 = relu(W1 x + b1);
 *                        f = relu(W2 h1 + b2); g = max over the patch's nodes;
 *                        g' = relu(W3 g + b3); h4 = relu(W4 [f; g'] + b4);
 *                        r = W5 h4 + b5.
 *
 * Memory: every pointer marked DEVICE is a device pointer on the plan's
 * device; HOST pointers are read during the call only.  The caller owns all
 * inputs and outputs; outputs are overwritten, never accumulated.  The plan
 * owns its copy of the mesh and all scratch memory; no call other than
 * etac_plan_create / etac_plan_destroy, etac_plan_autotune and the two
 * kernel-timing calls allocates, frees or synchronises, so every compute
 * call may be captured in a HIP graph.
 *
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  Every call
 * only enqueues work on it.  A plan is used by one stream at a time.
 *
 * Errors: arguments are validated on the host before anything is enqueued;
 * on error nothing is enqueued and an ETAC_ERR_* code is returned.  A failed
 * kernel launch returns ETAC_ERR_HIP; etac_last_hip_error() gives the HIP
 * code.  No C++ exception crosses this interface.
 */
#ifndef ETAC_H
#define ETAC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t etac_status;

#define ETAC_OK             0
#define ETAC_ERR_NULL      -1   /* a required pointer is NULL                  */
#define ETAC_ERR_SHAPE     -2   /* sizes negative, inconsistent or too large   */
#define ETAC_ERR_VALUE     -3   /* bad mode / flags / primitive type           */
#define ETAC_ERR_WORKSPACE -4   /* plan was created without what this call needs */
#define ETAC_ERR_HIP       -5   /* HIP runtime error                           */
#define ETAC_ERR_CAPTURE   -6   /* plan creation or autotuning during stream capture */

#define ETAC_SPHERE  0
#define ETAC_BOX     1
#define ETAC_CAPSULE 2
#define ETAC_MESH    3          /* closed triangle mesh of an etac_meshset;
                                   shape[0] = mesh index (an integer value);
                                   only etac_contact_mesh tests these, every
                                   other call ignores such objects          */

#define ETAC_FULL          0    /* Eq. 2: decay + residual (Table 2, full)     */
#define ETAC_DECAY_ONLY    1    /* Eq. 1 only (Table 2, linear decay only)     */
#define ETAC_RESIDUAL_ONLY 2    /* Phi only (Table 2, residual network only)   */

#define ETAC_PHI_SIZE 17411
#define ETAC_MAX_OBJ  8         /* objects per env                             */
#define ETAC_MAX_PATCH_NODES 65536

/* plan flags */
#define ETAC_PLAN_BACKWARD 1u   /* reserve the scratch the backward calls need */

typedef struct etac_plan etac_plan;

/* Elastomer surfaces, shared by all envs (node positions P and normals N,
 * Sec. III-A).  All pointers HOST; the plan keeps its own device copy. */
typedef struct {
    int32_t n_patches;            /* K >= 1                                    */
    int32_t n_nodes;              /* N = patch_offset[K]                        */
    const int32_t *patch_offset;  /* [K+1] ascending, [0] = 0, patch k owns
                                     nodes patch_offset[k] .. patch_offset[k+1]-1,
                                     every patch 1..ETAC_MAX_PATCH_NODES nodes  */
    const float *pos;             /* [3][N] undeformed node positions, mm       */
    const float *nrm;             /* [3][N] unit outward normals                */
    const float *origin;          /* [K][3] per-patch origin o_k (network input)*/
} etac_mesh;

/* Rigid primitives of every env.  Array pointers DEVICE.  Objects
 * o >= n_obj[e] are ignored.  n_envs may be smaller than the plan's. */
typedef struct {
    int32_t n_envs;               /* E, 0 <= E <= plan n_envs                  */
    int32_t max_obj;              /* O, 1 <= O <= plan max_obj                 */
    const int32_t *n_obj;         /* [E] values 0..O                           */
    const int32_t *type;          /* [E][O] ETAC_SPHERE / BOX / CAPSULE        */
    const float *shape;           /* [E][O][4]                                  */
    const float *rot;             /* [E][O][9]                                  */
    const float *trans;           /* [E][O][3]                                  */
} etac_scene;

/* Propagation model (Eqs. 1-2).  Pointers DEVICE. */
typedef struct {
    int32_t mode;                 /* ETAC_FULL / DECAY_ONLY / RESIDUAL_ONLY    */
    const float *alpha;           /* [K] decay rate per patch, 1/mm            */
    const float *phi;             /* [ETAC_PHI_SIZE]; may be NULL iff mode ==
                                     ETAC_DECAY_ONLY                            */
} etac_model;

/* Create a plan for `mesh` and up to n_envs envs with up to max_obj objects.
 * Validates the mesh, uploads it, computes per-patch bounding spheres and the
 * longest-first item order, and allocates scratch (more with
 * ETAC_PLAN_BACKWARD).  Synchronous; must not be called during stream
 * capture (ETAC_ERR_CAPTURE). *out is set only on success. */
etac_status etac_plan_create(const etac_mesh *mesh, int32_t n_envs, int32_t max_obj,
                             uint32_t flags, etac_plan **out);

/* Free a plan and its device memory (synchronises the device). NULL is OK. */
etac_status etac_plan_destroy(etac_plan *plan);

/* Contact pass only (Sec. III-A contact detection and local displacement).
 * Outputs DEVICE: contact_obj [E][N], uhat [3][E][N] (0 on passive nodes),
 * n_active [E][K].  uhat may be NULL to skip it. */
etac_status etac_contact(etac_plan *plan, const etac_scene *scene, int8_t *contact_obj,
                         float *uhat, int32_t *n_active, void *stream);

/* Pooling record of a forward call, for the adjoint (optional).  The
 * residual network (Eq. 2) max-pools its per-node encoder features over the
 * patch; the adjoint needs the pooled features and, per channel, the node
 * that attains the maximum.  A forward call given `saved` writes, for every
 * (env e, patch k) item with at least one active node and a model that uses
 * the residual, ETAC_SAVED_WORDS 32-bit words at word offset
 * (e K + k) ETAC_SAVED_WORDS: words 0..63 the pooled features (float),
 * words 64..127 the arg-max node of each channel (int32, index within the
 * patch, lowest index on ties).  Other items are not written.  An adjoint
 * call given the same buffer reads these records instead of repeating the
 * encoder pass over every node of the contacted patches; it must come from
 * the forward call on the same inputs (same scene or contact results, same
 * model, same n_envs), which nothing can check.  With saved = NULL the
 * adjoint recomputes them; both give identical results.  Size:
 * n_envs K ETAC_SAVED_WORDS 4 bytes. */
#define ETAC_SAVED_WORDS 128

/* Propagation of given contact results (Eqs. 1-2).  Inputs DEVICE:
 * contact_obj [E][N] (any value >= 0 marks an active node), uhat [3][E][N]
 * (read on active nodes only).  Output DEVICE: u [3][E][N].  E = n_envs.
 * saved (DEVICE, may be NULL): the pooling record for the adjoint. */
etac_status etac_propagate(etac_plan *plan, const etac_model *model, int32_t n_envs,
                           const int8_t *contact_obj, const float *uhat, float *u, void *saved,
                           void *stream);

/* Whole step, contact + propagation, as one persistent fused launch.
 * Outputs DEVICE: u [3][E][N], contact_obj [E][N], n_active [E][K].
 * saved (DEVICE, may be NULL): the pooling record for the adjoint, see
 * ETAC_SAVED_WORDS. */
etac_status etac_step(etac_plan *plan, const etac_scene *scene, const etac_model *model,
                      float *u, int8_t *contact_obj, int32_t *n_active, void *saved, void *stream);

/* The fused step for callers that cannot allocate device memory or may not
 * call hipMalloc (code under stream capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, outputs and errors as etac_step,
 * identical results; it allocates and frees nothing.  The per-workgroup
 * scratch of its kernel (u_hat, residuals and node lists of the current
 * item, work-queue counters) is a library-owned 64 MiB device array, which
 * every device the library runs on holds until the process ends, instead of
 * the plan's scratch.  All calls on one device share that array: calls that
 * could run at the same time on one device (different streams without
 * ordering between them) race and must not be made.  A workgroup needs
 * 32 n_max bytes of it (n_max: the plan's largest patch); when the plan's
 * persistent grid needs more than the array holds, fewer workgroups run.
 * ETAC_ERR_SHAPE if one workgroup's slice does not fit; ETAC_ERR_WORKSPACE if
 * the array's address on the plan's device is not known (it is looked up
 * when a plan is created on that device). */
etac_status etac_step_static(etac_plan *plan, const etac_scene *scene, const etac_model *model, float *u,
                             int8_t *contact_obj, int32_t *n_active, void *saved, void *stream);

/* Rigid objects given as closed triangle meshes (the paper's objects are
 * meshes whose signed distance fields drive contact, Sec. III-A contact
 * detection and Sec. IV).  A mesh set holds several meshes: mesh m owns
 * triangles tri_offset[m] .. tri_offset[m+1]-1 of `tris` [T][3] (vertex
 * indices into `verts` [n_verts][3], object-frame positions in mm, FP32),
 * counter-clockwise seen from outside.  Every mesh must be closed and
 * consistently oriented (each directed edge used once, its reverse once by
 * another triangle), with no zero-area triangle: otherwise ETAC_ERR_VALUE.
 * Limits: 1 <= n_meshes <= 4096, 4 <= triangles per mesh, T <= 2^24.
 * All pointers HOST, read during the call.  The set computes the
 * angle-weighted pseudo-normals of every face, edge and vertex in FP64,
 * groups each mesh's triangles into clusters of 32 with oriented bounding
 * boxes, classifies the cells of a grid over each mesh as certainly outside
 * or not, and uploads everything to the current device (synchronous; not
 * during stream capture: ETAC_ERR_CAPTURE).  *out is set only on success. */
typedef struct etac_meshset etac_meshset;
etac_status etac_meshset_create(int32_t n_meshes, const int32_t *tri_offset, int32_t n_verts,
                                const float *verts, const int32_t *tris, etac_meshset **out);

/* Free a mesh set and its device memory (synchronises the device). NULL is OK. */
etac_status etac_meshset_destroy(etac_meshset *ms);

/* Contact pass with primitives and triangle meshes (Sec. III-A contact
 * detection and local displacement).  Objects of type ETAC_MESH name a mesh
 * of `ms` by shape[0]; a value that is not an integer in [0, n_meshes) makes
 * the object ignored.  A node is inside a mesh when (q - c) . n < 0 for its
 * closest surface point c (minimum point-triangle distance, lowest triangle
 * index on ties) and the pseudo-normal n of the face, edge or vertex holding
 * c; its depth is |q - c| and u_hat = R (c - q).  The deepest object wins
 * over primitives and meshes alike, lowest index on ties.  Same outputs and
 * layouts as etac_contact (uhat may be NULL); the results feed
 * etac_propagate.  hit (DEVICE [E][N] int32, may be NULL): a record for the
 * adjoint, the winning triangle of each node a mesh object wins (an index
 * into `ms`'s own triangle order), -1 for every other node.  `ms` must live
 * on the plan's device (ETAC_ERR_VALUE otherwise); etac_contact_mesh_backward
 * is its adjoint. */
etac_status etac_contact_mesh(etac_plan *plan, const etac_meshset *ms, const etac_scene *scene,
                              int8_t *contact_obj, float *uhat, int32_t *n_active, int32_t *hit, void *stream);

/* Adjoint of etac_contact_mesh with respect to the object poses (ETac is
 * differentiable, Table 1): given dL/du_hat [3][E][N] (DEVICE; read on the
 * active nodes), writes dL/dR [E][O][9] and dL/dt [E][O][3] (DEVICE) for
 * primitives and meshes alike.  For a mesh node the
 * winning triangle and the feature holding its closest point are held
 * fixed: with w = c - q, u_hat = R w and dw/dq = J (face: -n n^T; edge of
 * direction e: e e^T / |e|^2 - I; vertex: -I), and h = J R^T g,
 * dL/dR = g w^T + d h^T (R's nine entries as free inputs, d = p - t) and
 * dL/dt = -R h.  Objects that win no node get zeros.  Sums run in a fixed
 * order: results do not depend on scheduling.  No plan scratch is used.
 * contact_obj and hit (DEVICE, both or neither): the records of the
 * etac_contact_mesh call on the same scene and mesh set; given them, the
 * call reads each node's winner and triangle instead of repeating the
 * distance search (identical results, at a fraction of the cost); entries
 * that cannot come from that call (an object index out of range, a
 * triangle outside the object's mesh) are skipped.  Both NULL: contact is
 * recomputed.  Only one of them NULL: ETAC_ERR_NULL. */
etac_status etac_contact_mesh_backward(etac_plan *plan, const etac_meshset *ms, const etac_scene *scene,
                                       const float *grad_uhat, const int8_t *contact_obj, const int32_t *hit,
                                       float *grad_rot, float *grad_trans, void *stream);

/* Adjoint of the contact pass: given dL/du_hat [3][E][N] (DEVICE; read on
 * active nodes only) returns dL/dR [E][O][9] and dL/dt [E][O][3] (DEVICE,
 * overwritten, zero for absent objects).  dL/dR treats the nine entries of R
 * as free inputs of the displacement formula.  Recomputes the contact pass.
 * Needs a plan created with ETAC_PLAN_BACKWARD (its per-item pose partials
 * live in the backward scratch). */
etac_status etac_contact_backward(etac_plan *plan, const etac_scene *scene, const float *grad_uhat,
                                  float *grad_rot, float *grad_trans, void *stream);

/* Adjoint of the propagation: given contact_obj, uhat and dL/du [3][E][N]
 * returns dL/du_hat [3][E][N] (0 on passive nodes), dL/dalpha [K] and
 * dL/dphi [ETAC_PHI_SIZE] (all DEVICE, overwritten; grad_alpha / grad_phi may
 * be NULL to skip).  saved: NULL, or the pooling record written by
 * etac_propagate on the same inputs.  Needs a plan created with
 * ETAC_PLAN_BACKWARD. */
etac_status etac_propagate_backward(etac_plan *plan, const etac_model *model, int32_t n_envs,
                                    const int8_t *contact_obj, const float *uhat,
                                    const float *grad_u, const void *saved, float *grad_uhat,
                                    float *grad_alpha, float *grad_phi, void *stream);

/* Adjoint of the whole step.  It recomputes the contact pass; the only thing
 * it can take from the forward call is the optional pooling record `saved`
 * (NULL, or written by etac_step on the same inputs).  Outputs as above.
 * Needs ETAC_PLAN_BACKWARD. */
etac_status etac_step_backward(etac_plan *plan, const etac_scene *scene, const etac_model *model,
                               const float *grad_u, const void *saved, float *grad_rot,
                               float *grad_trans, float *grad_alpha, float *grad_phi, void *stream);

/* Human-readable text of a status code (static storage). */
const char *etac_status_string(etac_status status);

/* HIP error code of the most recent ETAC_ERR_HIP in this thread (0 if none). */
int32_t etac_last_hip_error(void);

/* Plan introspection: number of (env, patch) items, persistent grid size,
 * scratch bytes.  Any output pointer may be NULL. */
etac_status etac_plan_info(const etac_plan *plan, int32_t *n_items, int32_t *grid,
                           int64_t *scratch_bytes);

/* Launch-shape override for the autotuner: persistent workgroups per CU for
 * the fused kernels (0 = built-in default). */
etac_status etac_plan_set_occupancy(etac_plan *plan, int32_t wg_per_cu);

/* Work-queue granularity for the autotuner: (env, patch) items claimed per
 * queue atomic by the persistent kernels, 1 .. 64 (0 = built-in default).
 * Results do not depend on it.  ETAC_ERR_VALUE outside 0 .. 64. */
etac_status etac_plan_set_batch(etac_plan *plan, int32_t items);

/* Launch shape of the persistent kernels (autotuner knobs; 0 keeps the
 * current value): forward workgroups per CU (1 .. 8), forward work-queue
 * batch (1 .. 64), work-queue batch of the decay-adjoint kernel (1 .. 64),
 * workgroups per CU of the decay-adjoint kernel (1 .. 8), and items claimed
 * at a time by the network-adjoint kernel from its list of items with
 * contact (1 .. 64).  Results do not depend on them.  ETAC_ERR_VALUE outside
 * those ranges. */
etac_status etac_plan_set_launch(etac_plan *plan, int32_t fwd_wg_per_cu, int32_t fwd_batch,
                                 int32_t bwd_batch, int32_t decay_wg_per_cu, int32_t net_batch);

/* The current launch shape, in the order of etac_plan_set_launch (HOST int32[5]). */
etac_status etac_plan_get_launch(const etac_plan *plan, int32_t *shape);

/* Autotuner.  Times every candidate launch shape of the persistent kernels
 * on the caller's inputs (as for etac_step and etac_step_backward; all
 * DEVICE pointers, outputs overwritten; `saved` may be NULL and is passed to
 * both calls) with HIP events over `reps` calls
 * (1 .. 1000) after a warm-up call, and keeps the fastest: forward
 * workgroups per CU in {1, 2} x batch in {1, 2, 4, 8, 16}; with grad_u
 * non-NULL also decay-kernel workgroups per CU in {2, 3, 4} x its batch in
 * {2, 4, 8, 16}, then the network-adjoint claim in {1, 2, 4}.  Every
 * candidate gives identical results.  `best` (HOST int32[5], may be NULL)
 * receives the chosen shape as in etac_plan_get_launch.  Blocks the host and creates two HIP events, so it
 * must not be called during stream capture (ETAC_ERR_CAPTURE). */
etac_status etac_plan_autotune(etac_plan *plan, const etac_scene *scene, const etac_model *model,
                               const float *grad_u, float *u, int8_t *contact_obj, int32_t *n_active,
                               void *saved, float *grad_rot, float *grad_trans, float *grad_alpha,
                               float *grad_phi, int32_t reps, int32_t *best, void *stream);

/* Kernel timing (diagnostics, not part of the method).  With timing on, every
 * launch of a timed kernel made outside stream capture is bracketed by a pair
 * of HIP events recorded on the stream the kernel is launched on, so the
 * measured span is that kernel's own execution on the device.  The plan keeps
 * the most recent ETAC_TIMER_SLOTS pairs per timer. */
#define ETAC_TIMER_SLOTS 256
typedef enum {
    ETAC_TIMER_CONTACT = 0,   /* k_contact: contact only (etac_contact)                  */
    ETAC_TIMER_STEP = 1,      /* k_step: the fused persistent forward                    */
    ETAC_TIMER_BACKWARD = 2,  /* k_bwd: network and contact adjoint of contacted items   */
    ETAC_TIMER_REDUCE = 3,    /* the fixed-order reductions that follow k_bwd, as one span */
    ETAC_TIMER_BWD_DECAY = 4, /* k_bwd_decay: contact and Eq. 1 adjoint, before k_bwd     */
    ETAC_TIMER_REGRESS = 5,   /* k_regress: the real-sensor regressor (etac_regress)      */
    ETAC_TIMER_COUNT = 6
} etac_timer;

/* Turn timing on (enable != 0) or off.  The first call that turns it on
 * creates the plan's events (host-side objects, freed by etac_plan_destroy);
 * turning it on resets every timer.  ETAC_ERR_HIP if event creation fails. */
etac_status etac_plan_set_timing(etac_plan *plan, int32_t enable);

/* Waits for the recorded launches of `timer` (blocks the host), writes how
 * many were recorded (at most ETAC_TIMER_SLOTS, the latest ones) and their
 * summed device time in ms, and resets that timer.  Both outputs are HOST
 * pointers.  ETAC_ERR_VALUE for an unknown timer; zero launches if timing was
 * never turned on. */
etac_status etac_plan_kernel_time(etac_plan *plan, int32_t timer, int32_t *launches, double *total_ms);

/* ------------------------------------------------------------------------
 * Articulated hand and self-contact.  The paper's contact detection covers
 * the hand's own links besides the external objects (Sec. III-A, contact
 * detection), and its contact reward counts active nodes and touched links
 * (Sec. IV-B, contact-reward equation).  Here every patch rides on one link
 * of the hand: the plan's mesh gives patch k's node positions, normals and
 * origin in the frame of link patch_link[k], and the hand calls return u_hat
 * and U in that frame.  Contact of patch k on link l is evaluated in link
 * l's frame against
 *   - the env's objects (contact_obj ids 0 .. O-1, O = scene max_obj), and
 *   - the collision primitive of every link j with bit j of collide[l] set,
 *     j != l (id O + j),
 * each at its relative pose R' = R_l^T R_w, t' = R_l^T (t_w - t_l), formed in
 * FP64 (every entry (a0 b0 + a1 b1) + a2 b2, no fused multiply-add) and
 * rounded to FP32; link j's primitive has world pose R_w = R_j C_R,
 * t_w = R_j C_t + t_j for its pose (C_R, C_t) in link j's frame.  Candidates
 * are ordered objects first, then links by index; the deepest penetration
 * wins, the first candidate on ties.  Triangle-mesh objects are ignored by
 * the hand calls.
 * ------------------------------------------------------------------------ */
#define ETAC_MAX_LINKS 24

/* The hand's links.  All pointers HOST; etac_plan_set_hand copies them. */
typedef struct {
    int32_t n_links;              /* L, 1 .. ETAC_MAX_LINKS                     */
    const int32_t *patch_link;    /* [K] link carrying each patch, 0 .. L-1     */
    const uint32_t *collide;      /* [L] bit j: link j's primitive is tested
                                     against the patches on this link (bit of
                                     the link itself ignored)                   */
    const int32_t *prim_type;     /* [L] ETAC_SPHERE / BOX / CAPSULE, or -1 for
                                     a link without a collision primitive       */
    const float *prim_shape;      /* [L][4] as etac_scene shapes                 */
    const float *prim_rot;        /* [L][9] primitive pose in its link frame     */
    const float *prim_trans;      /* [L][3]                                      */
} etac_hand;

/* Link poses of every env (world x = R q + t for a link-frame point q).
 * DEVICE [E][L][9] and [E][L][3]. */
typedef struct {
    const float *rot;
    const float *trans;
} etac_links;

/* Contact-reward outputs (DEVICE; each pointer may be NULL to skip it).
 * n_touch[e][k]: nodes of patch k won by an object (not by a link);
 * n_a[e] = sum over k of n_touch; link_mask[e] bit l: some patch on link l
 * has n_touch > 0 (the paper's S_cr); r_contact[e] = popcount(link_mask) / L
 * + omega_a (n_a / N if n_a > 0, else -0.1), N the plan's node count. */
typedef struct {
    float omega_a;
    int32_t *n_touch;             /* [E][K] */
    int32_t *n_a;                 /* [E]    */
    uint32_t *link_mask;          /* [E]    */
    float *r_contact;             /* [E]    */
} etac_reward;

/* Attach a hand to a plan (replaces a previous one).  Validates it (every
 * patch_link in range, primitive types, positive shapes; the largest
 * candidate set max_obj + popcount(collide[l]) at most 32: ETAC_ERR_SHAPE
 * beyond), uploads it and allocates the per-item candidate table (and the
 * adjoint's partials with ETAC_PLAN_BACKWARD).  Synchronous; not during
 * stream capture (ETAC_ERR_CAPTURE). */
etac_status etac_plan_set_hand(etac_plan *plan, const etac_hand *hand);

/* Contact pass of the hand: contact_obj [E][N] (ids as above, -1 passive),
 * uhat [3][E][N] (link frames; may be NULL), n_active [E][K], and the reward
 * outputs (reward may be NULL).  ETAC_ERR_WORKSPACE without a hand. */
etac_status etac_hand_contact(etac_plan *plan, const etac_scene *scene, const etac_links *links,
                              int8_t *contact_obj, float *uhat, int32_t *n_active, const etac_reward *reward,
                              void *stream);

/* Fused step of the hand (contact as above, then Eqs. 1-2 in the link
 * frames): u [3][E][N], contact_obj, n_active, reward (may be NULL), saved
 * (may be NULL: the pooling record, see ETAC_SAVED_WORDS). */
etac_status etac_hand_step(etac_plan *plan, const etac_scene *scene, const etac_links *links,
                           const etac_model *model, float *u, int8_t *contact_obj, int32_t *n_active,
                           const etac_reward *reward, void *saved, void *stream);

/* Adjoint of L = sum g . U of the hand step: dL/dR [E][O][9], dL/dt [E][O][3]
 * of the objects, dL/dR [E][L][9], dL/dt [E][L][3] of the links (rotation
 * entries as free inputs), dL/dalpha, dL/dphi (may be NULL).  Recomputes
 * contact; saved as for etac_step_backward.  Needs ETAC_PLAN_BACKWARD. */
etac_status etac_hand_step_backward(etac_plan *plan, const etac_scene *scene, const etac_links *links,
                                    const etac_model *model, const float *grad_u, const void *saved,
                                    float *grad_rot, float *grad_trans, float *grad_link_rot,
                                    float *grad_link_trans, float *grad_alpha, float *grad_phi, void *stream);

/* ------------------------------------------------------------------------
 * Real-sensor regressor (appendix, "Modeling Real Sensors"): the displacement
 * field of each (env, patch) item is mapped to the eight pressure-taxel
 * outputs of a real sensor by a PointNet-style network with a residual layer
 * whose per-node features are pooled with attention (an MLP [256, 128, 1]
 * with tanh, normalised by a softmax over the item's nodes).  Per node i of
 * patch k:
 *   x_i  = [p_i - o_k, U_i]                  (6)
 *   h1_i = relu(E1 x_i + e1)                 (64)
 *   h2_i = relu(E2 h1_i + e2) + h1_i         (64, residual)
 *   f_i  = relu(E3 h2_i + e3)                (256)
 *   s_i  = a2 . tanh(A1 f_i + a1) + a0       (scalar score)
 * per item: w = softmax(s), g = sum_i w_i f_i, y = D2 relu(D1 g + d1) + d2.
 * reg: packed FP32, ETAC_REG_SIZE floats: E1[64][6] e1[64] E2[64][64] e2[64]
 * E3[256][64] e3[256] A1[128][256] a1[128] a2[128] a0[4] (a0[0] used; the
 * softmax does not depend on it) D1[128][256] d1[128] D2[8][128] d2[8].
 * Arithmetic: E1 at FP32 level (split FP16 operands); E2, E3 and A1 on FP16
 * operands with FP32 accumulation, the pooled features as those FP16 values;
 * softmax weights, pooling sums and the head in FP32.
 * ------------------------------------------------------------------------ */
#define ETAC_REG_SIZE 88204
#define ETAC_TAXELS 8

/* taxels [E][K][8] (DEVICE, overwritten) from u [3][E][N] and n_active [E][K]
 * (DEVICE, as written by a step call with the same n_envs = E; items with
 * n_active 0 must have U = 0 on their patch, as every step leaves them: they
 * take the patch's output at U = 0, evaluated once per call).  reg DEVICE
 * [ETAC_REG_SIZE].  0 <= n_envs <= the plan's n_envs (ETAC_ERR_SHAPE).  Uses
 * the plan's own scratch (a [K][8] table and a work counter), so calls on one
 * plan must not overlap; non-finite parameters propagate to the outputs. */
etac_status etac_regress(etac_plan *plan, const float *reg, int32_t n_envs, const float *u,
                         const int32_t *n_active, float *taxels, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ETAC_H */

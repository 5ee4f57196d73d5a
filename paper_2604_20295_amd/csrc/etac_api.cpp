// Host side of the C ABI declared in include/etac.h: plan creation (mesh
// validation and upload, conservative per-patch bounding spheres, the
// longest-patch-first item order, scratch allocation) and argument validation
// for every call.  Nothing here computes the method; all arithmetic of the
// step runs in the kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <new>
#include <vector>

#include "etac_internal.h"

struct etac_plan {
    etac::Plan p;
};

namespace {

thread_local int32_t g_last_hip = 0;

etac_status hip_fail(hipError_t e) {
    g_last_hip = (int32_t)e;
    return ETAC_ERR_HIP;
}

template <typename T>
hipError_t plan_alloc(etac::Plan &p, T **ptr, size_t count) {
    *ptr = nullptr;
    if (count == 0) count = 1;
    if (p.n_allocs >= (int)(sizeof(p.allocs) / sizeof(p.allocs[0]))) return hipErrorOutOfMemory;
    void *v = nullptr;
    hipError_t e = hipMalloc(&v, count * sizeof(T));
    if (e != hipSuccess) return e;
    p.allocs[p.n_allocs++] = v;
    p.scratch_bytes += (int64_t)(count * sizeof(T));
    *ptr = static_cast<T *>(v);
    return hipSuccess;
}

void plan_free_all(etac::Plan &p) {
    for (int i = 0; i < p.n_allocs; ++i) (void)hipFree(p.allocs[i]);
    p.n_allocs = 0;
    if (p.hand_mem) (void)hipFree(p.hand_mem);
    p.hand_mem = nullptr;
    delete p.hand;
    p.hand = nullptr;
    if (p.timers) {
        for (int k = 0; k < ETAC_TIMER_COUNT; ++k)
            for (int i = 0; i < ETAC_TIMER_SLOTS; ++i)
                for (int j = 0; j < 2; ++j)
                    if (p.timers->ev[k][i][j]) (void)hipEventDestroy(p.timers->ev[k][i][j]);
        delete p.timers;
        p.timers = nullptr;
    }
}

// Round a non-negative double up to the next float at or above it.
float round_up_float(double v) {
    float f = (float)v;
    if ((double)f < v) f = std::nextafter(f, std::numeric_limits<float>::infinity());
    return f;
}

etac_status check_scene(const etac::Plan &p, const etac_scene *s) {
    if (!s) return ETAC_ERR_NULL;
    if (s->n_envs < 0 || s->n_envs > p.n_envs) return ETAC_ERR_SHAPE;
    if (s->max_obj < 1 || s->max_obj > p.max_obj) return ETAC_ERR_SHAPE;
    if (s->n_envs > 0 && (!s->n_obj || !s->type || !s->shape || !s->rot || !s->trans)) return ETAC_ERR_NULL;
    return ETAC_OK;
}

etac_status check_model(const etac_model *m) {
    if (!m) return ETAC_ERR_NULL;
    if (m->mode != ETAC_FULL && m->mode != ETAC_DECAY_ONLY && m->mode != ETAC_RESIDUAL_ONLY) return ETAC_ERR_VALUE;
    if (!m->alpha) return ETAC_ERR_NULL;
    if (!m->phi && m->mode != ETAC_DECAY_ONLY) return ETAC_ERR_VALUE;
    return ETAC_OK;
}

etac::SceneDev scene_dev(const etac_scene *s) {
    return etac::SceneDev{s->n_obj, s->type, s->shape, s->rot, s->trans, s->n_envs, s->max_obj};
}

etac::ModelDev model_dev(const etac_model *m) { return etac::ModelDev{m->mode, m->alpha, m->phi}; }

etac_status check_hand_call(const etac::Plan &p, const etac_scene *scene, const etac_links *links) {
    etac_status st = check_scene(p, scene);
    if (st != ETAC_OK) return st;
    if (!links) return ETAC_ERR_NULL;
    if (scene->n_envs > 0 && (!links->rot || !links->trans)) return ETAC_ERR_NULL;
    if (!p.hand) return ETAC_ERR_WORKSPACE;
    return ETAC_OK;
}

int32_t *touch_buffer(const etac::Plan &p, const etac_reward *r) {
    return (r && r->n_touch) ? r->n_touch : p.hand->n_touch;
}

hipError_t hand_reward(const etac::Plan &p, int E, const int32_t *touch, const etac_reward *r, hipStream_t st) {
    if (!r) return hipSuccess;
    return etac::launch_hand_reward(p, E, touch, r->omega_a, r->n_a, r->link_mask, r->r_contact, st);
}


}  // namespace

extern "C" {

const char *etac_status_string(etac_status s) {
    switch (s) {
        case ETAC_OK: return "ok";
        case ETAC_ERR_NULL: return "required pointer is NULL";
        case ETAC_ERR_SHAPE: return "sizes negative, inconsistent with the plan, or too large";
        case ETAC_ERR_VALUE: return "invalid mode, flags or value";
        case ETAC_ERR_WORKSPACE: return "plan lacks the scratch this call needs (create it with ETAC_PLAN_BACKWARD)";
        case ETAC_ERR_HIP: return "HIP runtime error (see etac_last_hip_error)";
        case ETAC_ERR_CAPTURE: return "plan creation or autotuning is not allowed during stream capture";
        default: return "unknown status";
    }
}

int32_t etac_last_hip_error(void) { return g_last_hip; }

etac_status etac_plan_create(const etac_mesh *mesh, int32_t n_envs, int32_t max_obj, uint32_t flags,
                             etac_plan **out) {
    if (!mesh || !out) return ETAC_ERR_NULL;
    if (!mesh->patch_offset || !mesh->pos || !mesh->nrm || !mesh->origin) return ETAC_ERR_NULL;
    const int K = mesh->n_patches, N = mesh->n_nodes;
    if (K < 1 || K > etac::kMaxPatches || N < 1) return ETAC_ERR_SHAPE;
    if (n_envs < 1 || max_obj < 1 || max_obj > ETAC_MAX_OBJ) return ETAC_ERR_SHAPE;
    if (flags & ~ETAC_PLAN_BACKWARD) return ETAC_ERR_VALUE;
    if (mesh->patch_offset[0] != 0 || mesh->patch_offset[K] != N) return ETAC_ERR_SHAPE;
    int n_max = 0;
    for (int k = 0; k < K; ++k) {
        const int64_t n = (int64_t)mesh->patch_offset[k + 1] - mesh->patch_offset[k];
        if (n < 1 || n > ETAC_MAX_PATCH_NODES) return ETAC_ERR_SHAPE;
        n_max = std::max(n_max, (int)n);
    }
    if ((int64_t)n_envs * K > std::numeric_limits<int32_t>::max()) return ETAC_ERR_SHAPE;
    if ((int64_t)n_envs * N > (std::numeric_limits<int64_t>::max() / 16)) return ETAC_ERR_SHAPE;
    for (int64_t i = 0; i < 3 * (int64_t)N; ++i)
        if (!std::isfinite(mesh->pos[i]) || !std::isfinite(mesh->nrm[i])) return ETAC_ERR_VALUE;
    for (int i = 0; i < 3 * K; ++i)
        if (!std::isfinite(mesh->origin[i])) return ETAC_ERR_VALUE;

    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(nullptr, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return ETAC_ERR_CAPTURE;

    etac_plan *h = new (std::nothrow) etac_plan();
    if (!h) return ETAC_ERR_SHAPE;
    etac::Plan &p = h->p;
    std::memset(&p, 0, sizeof(p));
    p.flags = flags;
    p.n_envs = n_envs;
    p.max_obj = max_obj;
    p.K = K;
    p.N = N;
    p.n_max = n_max;
    p.wg_per_cu = etac::kDefaultWgPerCu;
    p.batch = etac::kDefaultBatch;
    p.bwd_batch = etac::kDefaultBatch;
    p.decay_wg_per_cu = etac::kDefaultDecayWgPerCu;
    p.net_batch = etac::kDefaultNetBatch;
    hipError_t e = hipGetDevice(&p.device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&p.cu_count, hipDeviceAttributeMultiprocessorCount, p.device);
    // the device address of the static scratch of etac_step_static, once per device
    if (e == hipSuccess) e = etac::static_scratch_init(p.device);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e);
    }
    p.grid = p.cu_count * p.wg_per_cu;

    // host-side tables
    std::vector<float4> bound(K);
    std::vector<int16_t> node_patch(N);
    std::vector<int> order(K);
    std::vector<float> xbound(K);
    for (int k = 0; k < K; ++k) {
        const int o0 = mesh->patch_offset[k], o1 = mesh->patch_offset[k + 1];
        double lo[3], hi[3];
        for (int a = 0; a < 3; ++a) { lo[a] = 1e300; hi[a] = -1e300; }
        for (int i = o0; i < o1; ++i)
            for (int a = 0; a < 3; ++a) {
                const double v = mesh->pos[(size_t)a * N + i];
                lo[a] = std::min(lo[a], v);
                hi[a] = std::max(hi[a], v);
            }
        double c[3];
        for (int a = 0; a < 3; ++a) c[a] = 0.5 * (lo[a] + hi[a]);
        float cf[3];
        for (int a = 0; a < 3; ++a) cf[a] = (float)c[a];
        double rad = 0.0;
        for (int i = o0; i < o1; ++i) {
            double d2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double d = (double)mesh->pos[(size_t)a * N + i] - (double)cf[a];
                d2 += d * d;
            }
            rad = std::max(rad, std::sqrt(d2));
            node_patch[i] = (int16_t)k;
        }
        bound[k] = make_float4(cf[0], cf[1], cf[2], round_up_float(rad * (1.0 + 1e-6) + 1e-4));
        // bound of the geometric network inputs of the patch (the scale of its split operands)
        double xb = 0.0;
        for (int i = o0; i < o1; ++i)
            for (int a = 0; a < 3; ++a) {
                xb = std::max(xb, std::fabs((double)mesh->pos[(size_t)a * N + i] - (double)mesh->origin[3 * k + a]));
                xb = std::max(xb, std::fabs((double)mesh->nrm[(size_t)a * N + i]));
            }
        xbound[k] = round_up_float(xb * (1.0 + 1e-6));
        order[k] = k;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (mesh->patch_offset[a + 1] - mesh->patch_offset[a]) > (mesh->patch_offset[b + 1] - mesh->patch_offset[b]);
    });

    float *pos = nullptr, *nrm = nullptr, *origin = nullptr;
    int *offset = nullptr, *ord = nullptr;
    float4 *bnd = nullptr;
    float *xbd = nullptr;
    int16_t *np = nullptr;
    e = plan_alloc(p, &pos, 3 * (size_t)N);
    if (e == hipSuccess) e = plan_alloc(p, &nrm, 3 * (size_t)N);
    if (e == hipSuccess) e = plan_alloc(p, &origin, 3 * (size_t)K);
    if (e == hipSuccess) e = plan_alloc(p, &offset, (size_t)K + 1);
    if (e == hipSuccess) e = plan_alloc(p, &ord, (size_t)K);
    if (e == hipSuccess) e = plan_alloc(p, &bnd, (size_t)K);
    if (e == hipSuccess) e = plan_alloc(p, &np, (size_t)N);
    if (e == hipSuccess) e = plan_alloc(p, &xbd, (size_t)K);
    if (e == hipSuccess) e = hipMemcpy(pos, mesh->pos, 3 * (size_t)N * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(nrm, mesh->nrm, 3 * (size_t)N * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(origin, mesh->origin, 3 * (size_t)K * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(offset, mesh->patch_offset, ((size_t)K + 1) * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ord, order.data(), (size_t)K * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(bnd, bound.data(), (size_t)K * sizeof(float4), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(np, node_patch.data(), (size_t)N * sizeof(int16_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(xbd, xbound.data(), (size_t)K * sizeof(float), hipMemcpyHostToDevice);
    p.mesh = etac::MeshDev{pos, nrm, origin, offset, bnd, np, ord, xbd, K, N, n_max};

    // forward scratch, one slice per persistent workgroup
    const size_t G = (size_t)p.cu_count * 8;  // enough for any occupancy override
    p.scr.n_max = n_max;
    if (e == hipSuccess) e = plan_alloc(p, &p.scr.uhat_node, G * 3 * n_max);
    if (e == hipSuccess) e = plan_alloc(p, &p.scr.resid, G * 3 * n_max);
    if (e == hipSuccess) e = plan_alloc(p, &p.scr.alist, G * n_max);
    if (e == hipSuccess) e = plan_alloc(p, &p.scr.plist, G * n_max);
    // work counters: [0..1] forward, [2..3] adjoint, [4..5] regressor
    if (e == hipSuccess) e = plan_alloc(p, &p.scr.counter, 8);
    if (e == hipSuccess) e = hipMemset(p.scr.counter, 0, 8 * sizeof(unsigned));
    // regressor: rest outputs, and a pooled-feature row per item it may process
    if (e == hipSuccess) e = plan_alloc(p, &p.reg_rest, 8 * (size_t)K);
    if (e == hipSuccess) e = plan_alloc(p, &p.reg_pooled, ((size_t)n_envs * K + K) * 256);
    if (e == hipSuccess) e = plan_alloc(p, &p.reg_row, (size_t)n_envs * K + K);

    if (e == hipSuccess && (flags & ETAC_PLAN_BACKWARD)) {
        const size_t items = (size_t)n_envs * K;
        etac::BwdScratch &b = p.bwd;
        e = plan_alloc(p, &b.guhat, G * 3 * (size_t)n_max);
        if (e == hipSuccess) e = plan_alloc(p, &b.phi_part, items * etac::kRecWords);
        if (e == hipSuccess) e = plan_alloc(p, &b.rec_map, ETAC_PHI_SIZE);
        if (e == hipSuccess) e = plan_alloc(p, &b.alpha_part, items);
        if (e == hipSuccess) e = plan_alloc(p, &b.pose_part, items * (size_t)max_obj * 12);
        if (e == hipSuccess) e = plan_alloc(p, &b.item_flag, items);
        if (e == hipSuccess) e = plan_alloc(p, &b.phi_seg, (size_t)64 * etac::kRedColsMax);
        const size_t EN = (size_t)n_envs * N;
        if (e == hipSuccess) e = plan_alloc(p, &b.cobj_st, EN);
        if (e == hipSuccess) e = plan_alloc(p, &b.uhat_st, 3 * EN);
        if (e == hipSuccess) e = plan_alloc(p, &b.gh_st, 3 * EN);
        if (e == hipSuccess) e = plan_alloc(p, &b.m_st, items);
        if (e == hipSuccess) e = plan_alloc(p, &b.gmax_st, items);
        if (e == hipSuccess) e = plan_alloc(p, &b.live, items);
        if (e == hipSuccess) e = plan_alloc(p, &b.seg_cnt, (items + 1023) / 1024 + 1);
        if (e == hipSuccess) e = etac::init_record_map(p);
        p.has_bwd = (e == hipSuccess);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        const etac_status st = (e == hipErrorStreamCaptureUnsupported || e == hipErrorStreamCaptureImplicit)
                                   ? ETAC_ERR_CAPTURE : hip_fail(e);
        plan_free_all(p);
        delete h;
        return st;
    }
    *out = h;
    return ETAC_OK;
}

etac_status etac_plan_destroy(etac_plan *plan) {
    if (!plan) return ETAC_OK;
    (void)hipDeviceSynchronize();
    plan_free_all(plan->p);
    delete plan;
    return ETAC_OK;
}

etac_status etac_plan_info(const etac_plan *plan, int32_t *n_items, int32_t *grid, int64_t *scratch_bytes) {
    if (!plan) return ETAC_ERR_NULL;
    if (n_items) *n_items = plan->p.n_envs * plan->p.K;
    if (grid) *grid = plan->p.grid;
    if (scratch_bytes) *scratch_bytes = plan->p.scratch_bytes;
    return ETAC_OK;
}

etac_status etac_plan_set_occupancy(etac_plan *plan, int32_t wg_per_cu) {
    if (!plan) return ETAC_ERR_NULL;
    if (wg_per_cu < 0 || wg_per_cu > 8) return ETAC_ERR_VALUE;
    plan->p.wg_per_cu = wg_per_cu == 0 ? etac::kDefaultWgPerCu : wg_per_cu;
    plan->p.grid = plan->p.cu_count * plan->p.wg_per_cu;
    return ETAC_OK;
}

etac_status etac_plan_set_batch(etac_plan *plan, int32_t items) {
    if (!plan) return ETAC_ERR_NULL;
    if (items < 0 || items > 64) return ETAC_ERR_VALUE;
    plan->p.batch = plan->p.bwd_batch = items == 0 ? etac::kDefaultBatch : items;
    return ETAC_OK;
}

etac_status etac_plan_set_launch(etac_plan *plan, int32_t fwd_wg_per_cu, int32_t fwd_batch, int32_t bwd_batch,
                                 int32_t decay_wg_per_cu, int32_t net_batch) {
    if (!plan) return ETAC_ERR_NULL;
    if (fwd_wg_per_cu < 0 || fwd_wg_per_cu > 8 || fwd_batch < 0 || fwd_batch > 64 || bwd_batch < 0 ||
        bwd_batch > 64 || decay_wg_per_cu < 0 || decay_wg_per_cu > 8 || net_batch < 0 || net_batch > 64)
        return ETAC_ERR_VALUE;
    etac::Plan &p = plan->p;
    if (fwd_wg_per_cu) {
        p.wg_per_cu = fwd_wg_per_cu;
        p.grid = p.cu_count * p.wg_per_cu;
    }
    if (fwd_batch) p.batch = fwd_batch;
    if (bwd_batch) p.bwd_batch = bwd_batch;
    if (decay_wg_per_cu) p.decay_wg_per_cu = decay_wg_per_cu;
    if (net_batch) p.net_batch = net_batch;
    return ETAC_OK;
}

etac_status etac_plan_get_launch(const etac_plan *plan, int32_t *shape) {
    if (!plan || !shape) return ETAC_ERR_NULL;
    shape[0] = plan->p.wg_per_cu;
    shape[1] = plan->p.batch;
    shape[2] = plan->p.bwd_batch;
    shape[3] = plan->p.decay_wg_per_cu;
    shape[4] = plan->p.net_batch;
    return ETAC_OK;
}

etac_status etac_plan_set_timing(etac_plan *plan, int32_t enable) {
    if (!plan) return ETAC_ERR_NULL;
    etac::Plan &p = plan->p;
    if (!enable) {
        if (p.timers) p.timers->on = false;
        return ETAC_OK;
    }
    if (!p.timers) {
        etac::Timers *t = new (std::nothrow) etac::Timers();
        if (!t) return ETAC_ERR_SHAPE;
        std::memset(t, 0, sizeof(*t));
        p.timers = t;
        for (int k = 0; k < ETAC_TIMER_COUNT; ++k)
            for (int i = 0; i < ETAC_TIMER_SLOTS; ++i)
                for (int j = 0; j < 2; ++j) {
                    hipError_t e = hipEventCreate(&t->ev[k][i][j]);
                    if (e != hipSuccess) {
                        t->ev[k][i][j] = nullptr;
                        return hip_fail(e);
                    }
                }
    }
    for (int k = 0; k < ETAC_TIMER_COUNT; ++k) p.timers->n[k] = 0;
    p.timers->on = true;
    return ETAC_OK;
}

etac_status etac_plan_kernel_time(etac_plan *plan, int32_t timer, int32_t *launches, double *total_ms) {
    if (!plan || !launches || !total_ms) return ETAC_ERR_NULL;
    if (timer < 0 || timer >= ETAC_TIMER_COUNT) return ETAC_ERR_VALUE;
    *launches = 0;
    *total_ms = 0.0;
    etac::Timers *t = plan->p.timers;
    if (!t) return ETAC_OK;
    const int n = std::min(t->n[timer], ETAC_TIMER_SLOTS);
    double sum = 0.0;
    for (int i = 0; i < n; ++i) {
        hipError_t e = hipEventSynchronize(t->ev[timer][i][1]);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t->ev[timer][i][0], t->ev[timer][i][1]);
        if (e != hipSuccess) return hip_fail(e);
        sum += ms;
    }
    t->n[timer] = 0;
    *launches = n;
    *total_ms = sum;
    return ETAC_OK;
}

etac_status etac_contact(etac_plan *plan, const etac_scene *scene, int8_t *contact_obj, float *uhat,
                         int32_t *n_active, void *stream) {
    if (!plan) return ETAC_ERR_NULL;
    etac_status st = check_scene(plan->p, scene);
    if (st != ETAC_OK) return st;
    if (scene->n_envs > 0 && (!contact_obj || !n_active)) return ETAC_ERR_NULL;
    hipError_t e = etac::launch_contact(plan->p, scene_dev(scene), contact_obj, uhat, n_active, (hipStream_t)stream);
    return e == hipSuccess ? ETAC_OK : hip_fail(e);
}

etac_status etac_contact_mesh(etac_plan *plan, const etac_meshset *ms, const etac_scene *scene, int8_t *contact_obj,
                              float *uhat, int32_t *n_active, int32_t *hit, void *stream) {
    if (!plan || !ms) return ETAC_ERR_NULL;
    etac_status st = check_scene(plan->p, scene);
    if (st != ETAC_OK) return st;
    if (ms->device != plan->p.device) return ETAC_ERR_VALUE;
    if (scene->n_envs > 0 && (!contact_obj || !n_active)) return ETAC_ERR_NULL;
    hipError_t e = etac::launch_contact_mesh(plan->p, ms->d, scene_dev(scene), contact_obj, uhat, n_active, hit,
                                             (hipStream_t)stream);
    return e == hipSuccess ? ETAC_OK : hip_fail(e);
}

etac_status etac_contact_mesh_backward(etac_plan *plan, const etac_meshset *ms, const etac_scene *scene,
                                       const float *grad_uhat, const int8_t *contact_obj, const int32_t *hit,
                                       float *grad_rot, float *grad_trans, void *stream) {
    if (!plan || !ms) return ETAC_ERR_NULL;
    etac_status st = check_scene(plan->p, scene);
    if (st != ETAC_OK) return st;
    if (ms->device != plan->p.device) return ETAC_ERR_VALUE;
    if (scene->n_envs > 0 && (!grad_uhat || !grad_rot || !grad_trans)) return ETAC_ERR_NULL;
    if ((contact_obj == nullptr) != (hit == nullptr)) return ETAC_ERR_NULL;   // both records or neither
    hipError_t e = etac::launch_contact_mesh_backward(plan->p, ms->d, scene_dev(scene), grad_uhat, contact_obj, hit,
                                                      grad_rot, grad_trans, (hipStream_t)stream);
    return e == hipSuccess ? ETAC_OK : hip_fail(e);
}

etac_status etac_propagate(etac_plan *plan, const etac_model *model, int32_t n_envs, const int8_t *contact_obj,
                           const float *uhat, float *u, void *saved, void *stream) {
    if (!plan) return ETAC_ERR_NULL;
    etac_status st = check_model(model);
    if (st != ETAC_OK) return st;
    if (n_envs < 0 || n_envs > plan->p.n_envs) return ETAC_ERR_SHAPE;
    if (n_envs > 0 && (!contact_obj || !uhat || !u)) return ETAC_ERR_NULL;
    hipError_t e = etac::launch_step(plan->p, nullptr, model_dev(model), n_envs, contact_obj, uhat, u, nullptr,
                                     nullptr, static_cast<uint32_t *>(saved), (hipStream_t)stream);
    return e == hipSuccess ? ETAC_OK : hip_fail(e);
}

etac_status etac_step(etac_plan *plan, const etac_scene *scene, const etac_model *model, float *u,
                      int8_t *contact_obj, int32_t *n_active, void *saved, void *stream) {
    if (!plan) return ETAC_ERR_NULL;
    etac_status st = check_scene(plan->p, scene);
    if (st != ETAC_OK) return st;
    st = check_model(model);
    if (st != ETAC_OK) return st;
    if (scene->n_envs > 0 && (!u || !contact_obj || !n_active)) return ETAC_ERR_NULL;
    const etac::SceneDev sd = scene_dev(scene);
    hipError_t e = etac::launch_step(plan->p, &sd, model_dev(model), scene->n_envs, nullptr, nullptr, u,
                                     contact_obj, n_active, static_cast<uint32_t *>(saved), (hipStream_t)stream);
    return e == hipSuccess ? ETAC_OK : hip_fail(e);
}

etac_status etac_step_static(etac_plan *plan, const etac_scene *scene, const etac_model *model, float *u,
                             int8_t *contact_obj, int32_t *n_active, void *saved, void *stream) {
    if (!plan) return ETAC_ERR_NULL;
    etac_status st = check_scene(plan->p, scene);
    if (st != ETAC_OK) return st;
    st = check_model(model);
    if (st != ETAC_OK) return st;
    if (scene->n_envs > 0 && (!u || !contact_obj || !n_active)) return ETAC_ERR_NULL;
    // one workgroup's slice plus the counters must fit the array
    if (etac::static_scratch_per_wg(plan->p.n_max) + 256 > etac::kStaticScratchBytes) return ETAC_ERR_SHAPE;
    const etac::SceneDev sd = scene_dev(scene);
    const hipError_t e = etac::launch_step_static(plan->p, sd, model_dev(model), u, contact_obj, n_active,
                                                  static_cast<uint32_t *>(saved), (hipStream_t)stream);
    if (e == hipErrorNotInitialized) return ETAC_ERR_WORKSPACE;
    return e == hipSuccess ? ETAC_OK : hip_fail(e);
}

etac_status etac_contact_backward(etac_plan *plan, const etac_scene *scene, const float *grad_uhat,
                                  float *grad_rot, float *grad_trans, void *stream) {
    if (!plan) return ETAC_ERR_NULL;
    etac_status st = check_scene(plan->p, scene);
    if (st != ETAC_OK) return st;
    if (scene->n_envs > 0 && (!grad_uhat || !grad_rot || !grad_trans)) return ETAC_ERR_NULL;
    if (!plan->p.has_bwd) return ETAC_ERR_WORKSPACE;
    hipError_t e = etac::launch_contact_backward(plan->p, scene_dev(scene), grad_uhat, grad_rot, grad_trans,
                                                 (hipStream_t)stream);
    return e == hipSuccess ? ETAC_OK : hip_fail(e);
}

etac_status etac_propagate_backward(etac_plan *plan, const etac_model *model, int32_t n_envs,
                                    const int8_t *contact_obj, const float *uhat, const float *grad_u,
                                    const void *saved, float *grad_uhat, float *grad_alpha, float *grad_phi,
                                    void *stream) {
    if (!plan) return ETAC_ERR_NULL;
    etac_status st = check_model(model);
    if (st != ETAC_OK) return st;
    if (n_envs < 0 || n_envs > plan->p.n_envs) return ETAC_ERR_SHAPE;
    if (n_envs > 0 && (!contact_obj || !uhat || !grad_u || !grad_uhat)) return ETAC_ERR_NULL;
    if (!plan->p.has_bwd) return ETAC_ERR_WORKSPACE;
    hipError_t e = etac::launch_backward(plan->p, nullptr, model_dev(model), n_envs, contact_obj, uhat, grad_u,
                                         static_cast<const uint32_t *>(saved), grad_uhat, nullptr, nullptr,
                                         grad_alpha, grad_phi, (hipStream_t)stream);
    return e == hipSuccess ? ETAC_OK : hip_fail(e);
}

etac_status etac_step_backward(etac_plan *plan, const etac_scene *scene, const etac_model *model,
                               const float *grad_u, const void *saved, float *grad_rot, float *grad_trans,
                               float *grad_alpha, float *grad_phi, void *stream) {
    if (!plan) return ETAC_ERR_NULL;
    etac_status st = check_scene(plan->p, scene);
    if (st != ETAC_OK) return st;
    st = check_model(model);
    if (st != ETAC_OK) return st;
    if (scene->n_envs > 0 && (!grad_u || !grad_rot || !grad_trans)) return ETAC_ERR_NULL;
    if (!plan->p.has_bwd) return ETAC_ERR_WORKSPACE;
    const etac::SceneDev sd = scene_dev(scene);
    hipError_t e = etac::launch_backward(plan->p, &sd, model_dev(model), scene->n_envs, nullptr, nullptr, grad_u,
                                         static_cast<const uint32_t *>(saved), nullptr, grad_rot, grad_trans,
                                         grad_alpha, grad_phi, (hipStream_t)stream);
    return e == hipSuccess ? ETAC_OK : hip_fail(e);
}

etac_status etac_plan_autotune(etac_plan *plan, const etac_scene *scene, const etac_model *model,
                               const float *grad_u, float *u, int8_t *contact_obj, int32_t *n_active,
                               void *saved, float *grad_rot, float *grad_trans, float *grad_alpha,
                               float *grad_phi, int32_t reps, int32_t *best, void *stream) {
    if (!plan) return ETAC_ERR_NULL;
    if (reps < 1 || reps > 1000) return ETAC_ERR_VALUE;
    etac::Plan &p = plan->p;
    const hipStream_t st = (hipStream_t)stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return ETAC_ERR_CAPTURE;
    // one validated call of each before any timing (argument errors come back here)
    etac_status s = etac_step(plan, scene, model, u, contact_obj, n_active, saved, stream);
    if (s != ETAC_OK) return s;
    if (grad_u) {
        s = etac_step_backward(plan, scene, model, grad_u, saved, grad_rot, grad_trans, grad_alpha, grad_phi,
                               stream);
        if (s != ETAC_OK) return s;
    }
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    // time `reps` calls after one warm-up call of the current shape
    auto timed = [&](bool fwd, float &ms) -> etac_status {
        for (int r = 0; r <= reps; ++r) {
            if (r == 1 && hipEventRecord(ev[0], st) != hipSuccess) return ETAC_ERR_HIP;
            const etac_status q = fwd ? etac_step(plan, scene, model, u, contact_obj, n_active, saved, stream)
                                      : etac_step_backward(plan, scene, model, grad_u, saved, grad_rot,
                                                           grad_trans, grad_alpha, grad_phi, stream);
            if (q != ETAC_OK) return q;
        }
        hipError_t h = hipEventRecord(ev[1], st);
        if (h == hipSuccess) h = hipEventSynchronize(ev[1]);
        if (h == hipSuccess) h = hipEventElapsedTime(&ms, ev[0], ev[1]);
        return h == hipSuccess ? ETAC_OK : hip_fail(h);
    };
    etac_status out = e == hipSuccess ? ETAC_OK : hip_fail(e);
    // forward: workgroups per CU x work-queue batch
    int bf_occ = p.wg_per_cu, bf_batch = p.batch;
    float bf_ms = 3.0e38f;
    static const int kOcc[] = {1, 2};
    static const int kBatch[] = {1, 2, 4, 8, 16};
    for (int oi = 0; out == ETAC_OK && oi < 2; ++oi)
        for (int bi = 0; out == ETAC_OK && bi < 5; ++bi) {
            p.wg_per_cu = kOcc[oi];
            p.grid = p.cu_count * p.wg_per_cu;
            p.batch = kBatch[bi];
            float ms = 0.0f;
            out = timed(true, ms);
            if (out == ETAC_OK && ms < bf_ms) { bf_ms = ms; bf_occ = p.wg_per_cu; bf_batch = p.batch; }
        }
    p.wg_per_cu = bf_occ;
    p.grid = p.cu_count * p.wg_per_cu;
    p.batch = bf_batch;
    // adjoint: decay-kernel workgroups per CU x its work-queue batch, then
    // the network kernel's claim size
    if (grad_u) {
        int bb_dec = p.decay_wg_per_cu, bb_batch = p.bwd_batch;
        float bb_ms = 3.0e38f;
        static const int kDec[] = {2, 3, 4};
        for (int di = 0; out == ETAC_OK && di < 3; ++di)
            for (int bi = 1; out == ETAC_OK && bi < 5; ++bi) {
                p.decay_wg_per_cu = kDec[di];
                p.bwd_batch = kBatch[bi];
                float ms = 0.0f;
                out = timed(false, ms);
                if (out == ETAC_OK && ms < bb_ms) { bb_ms = ms; bb_dec = p.decay_wg_per_cu; bb_batch = p.bwd_batch; }
            }
        p.decay_wg_per_cu = bb_dec;
        p.bwd_batch = bb_batch;
        int bn = p.net_batch;
        float bn_ms = 3.0e38f;
        for (int ni = 0; out == ETAC_OK && ni < 3; ++ni) {
            p.net_batch = kBatch[ni];
            float ms = 0.0f;
            out = timed(false, ms);
            if (out == ETAC_OK && ms < bn_ms) { bn_ms = ms; bn = p.net_batch; }
        }
        p.net_batch = bn;
    }
    for (int i = 0; i < 2; ++i)
        if (ev[i]) (void)hipEventDestroy(ev[i]);
    if (best) {
        best[0] = p.wg_per_cu;
        best[1] = p.batch;
        best[2] = p.bwd_batch;
        best[3] = p.decay_wg_per_cu;
        best[4] = p.net_batch;
    }
    return out;
}


// ---------------------------------------------------------------------------
// articulated hand
// ---------------------------------------------------------------------------
etac_status etac_plan_set_hand(etac_plan *plan, const etac_hand *hand) {
    if (!plan || !hand) return ETAC_ERR_NULL;
    if (!hand->patch_link || !hand->collide || !hand->prim_type || !hand->prim_shape || !hand->prim_rot ||
        !hand->prim_trans)
        return ETAC_ERR_NULL;
    etac::Plan &p = plan->p;
    const int L = hand->n_links, K = p.K;
    if (L < 1 || L > ETAC_MAX_LINKS) return ETAC_ERR_SHAPE;
    for (int k = 0; k < K; ++k)
        if (hand->patch_link[k] < 0 || hand->patch_link[k] >= L) return ETAC_ERR_VALUE;
    unsigned with_prim = 0;
    for (int l = 0; l < L; ++l) {
        const int ty = hand->prim_type[l];
        if (ty < -1 || ty > ETAC_CAPSULE) return ETAC_ERR_VALUE;
        for (int i = 0; i < 4; ++i)
            if (!std::isfinite(hand->prim_shape[4 * l + i])) return ETAC_ERR_VALUE;
        for (int i = 0; i < 9; ++i)
            if (!std::isfinite(hand->prim_rot[9 * l + i])) return ETAC_ERR_VALUE;
        for (int i = 0; i < 3; ++i)
            if (!std::isfinite(hand->prim_trans[3 * l + i])) return ETAC_ERR_VALUE;
        if (ty < 0) continue;
        const float *sh = hand->prim_shape + 4 * l;
        if (!(sh[0] > 0.0f)) return ETAC_ERR_VALUE;
        if (ty == ETAC_BOX && !(sh[1] > 0.0f && sh[2] > 0.0f)) return ETAC_ERR_VALUE;
        if (ty == ETAC_CAPSULE && !(sh[1] >= 0.0f)) return ETAC_ERR_VALUE;
        with_prim |= 1u << l;
    }
    int most = 0;
    for (int l = 0; l < L; ++l)
        most = std::max(most, __builtin_popcount(hand->collide[l] & ~(1u << l) & with_prim));
    const int cap = std::max(1, p.max_obj + most);
    if (cap > etac::kMaxRowObj) return ETAC_ERR_SHAPE;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(nullptr, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return ETAC_ERR_CAPTURE;

    // one device block, carved at 256-byte boundaries
    const size_t rows = (size_t)p.n_envs * K, rc = rows * (size_t)cap;
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off += (bytes + 255) / 256 * 256; return o; };
    const size_t o_pl = take(K * sizeof(int)), o_co = take(L * sizeof(unsigned)), o_pt = take(L * sizeof(int));
    const size_t o_ps = take(4 * L * sizeof(float)), o_pr = take(9 * L * sizeof(float)), o_pp = take(3 * L * sizeof(float));
    const size_t o_no = take(rows * sizeof(int)), o_ne = take(rows * sizeof(int)), o_ty = take(rc * sizeof(int));
    const size_t o_sh = take(4 * rc * sizeof(float)), o_ro = take(9 * rc * sizeof(float));
    const size_t o_tr = take(3 * rc * sizeof(float)), o_sr = take(rc), o_nt = take(rows * sizeof(int));
    const size_t o_pa = p.has_bwd ? take(12 * rc * sizeof(float)) : 0;
    void *mem = nullptr;
    hipError_t e = hipMalloc(&mem, off);
    if (e != hipSuccess) return hip_fail(e);
    char *b = static_cast<char *>(mem);
    etac::HandDev *h = new (std::nothrow) etac::HandDev();
    if (!h) {
        (void)hipFree(mem);
        return ETAC_ERR_SHAPE;
    }
    h->L = L;
    h->cap = cap;
    h->patch_link = reinterpret_cast<int *>(b + o_pl);
    h->collide = reinterpret_cast<unsigned *>(b + o_co);
    h->ptype = reinterpret_cast<int *>(b + o_pt);
    h->pshape = reinterpret_cast<float *>(b + o_ps);
    h->prot = reinterpret_cast<float *>(b + o_pr);
    h->ptrans = reinterpret_cast<float *>(b + o_pp);
    h->n_obj = reinterpret_cast<int *>(b + o_no);
    h->n_ext = reinterpret_cast<int *>(b + o_ne);
    h->type = reinterpret_cast<int *>(b + o_ty);
    h->shape = reinterpret_cast<float *>(b + o_sh);
    h->rot = reinterpret_cast<float *>(b + o_ro);
    h->trans = reinterpret_cast<float *>(b + o_tr);
    h->src = reinterpret_cast<int8_t *>(b + o_sr);
    h->n_touch = reinterpret_cast<int *>(b + o_nt);
    h->pose_part = p.has_bwd ? reinterpret_cast<float *>(b + o_pa) : nullptr;
    std::vector<unsigned> collide(L);
    for (int l = 0; l < L; ++l) collide[l] = hand->collide[l] & ~(1u << l) & with_prim & (L < 32 ? (1u << L) - 1u : ~0u);
    e = hipMemcpy(b + o_pl, hand->patch_link, K * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b + o_co, collide.data(), L * sizeof(unsigned), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b + o_pt, hand->prim_type, L * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b + o_ps, hand->prim_shape, 4 * L * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b + o_pr, hand->prim_rot, 9 * L * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b + o_pp, hand->prim_trans, 3 * L * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(b + o_no, 0, rows * sizeof(int));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        delete h;
        (void)hipFree(mem);
        return hip_fail(e);
    }
    (void)hipDeviceSynchronize();
    if (p.hand_mem) (void)hipFree(p.hand_mem);
    delete p.hand;
    p.hand = h;
    p.hand_mem = mem;
    return ETAC_OK;
}

etac_status etac_hand_contact(etac_plan *plan, const etac_scene *scene, const etac_links *links,
                              int8_t *contact_obj, float *uhat, int32_t *n_active, const etac_reward *reward,
                              void *stream) {
    if (!plan) return ETAC_ERR_NULL;
    const etac::Plan &p = plan->p;
    etac_status st = check_hand_call(p, scene, links);
    if (st != ETAC_OK) return st;
    if (scene->n_envs > 0 && (!contact_obj || !n_active)) return ETAC_ERR_NULL;
    if (scene->n_envs == 0) return ETAC_OK;
    const hipStream_t s = (hipStream_t)stream;
    const etac::LinksDev lk{links->rot, links->trans};
    etac::SceneDev rows;
    hipError_t e = etac::launch_hand_scene(p, scene_dev(scene), lk, &rows, s);
    int32_t *touch = touch_buffer(p, reward);
    if (e == hipSuccess) e = etac::launch_contact_rows(p, rows, contact_obj, uhat, n_active, touch, s);
    if (e == hipSuccess) e = hand_reward(p, scene->n_envs, touch, reward, s);
    return e == hipSuccess ? ETAC_OK : hip_fail(e);
}

etac_status etac_hand_step(etac_plan *plan, const etac_scene *scene, const etac_links *links,
                           const etac_model *model, float *u, int8_t *contact_obj, int32_t *n_active,
                           const etac_reward *reward, void *saved, void *stream) {
    if (!plan) return ETAC_ERR_NULL;
    const etac::Plan &p = plan->p;
    etac_status st = check_hand_call(p, scene, links);
    if (st != ETAC_OK) return st;
    st = check_model(model);
    if (st != ETAC_OK) return st;
    if (scene->n_envs > 0 && (!u || !contact_obj || !n_active)) return ETAC_ERR_NULL;
    if (scene->n_envs == 0) return ETAC_OK;
    const hipStream_t s = (hipStream_t)stream;
    const etac::LinksDev lk{links->rot, links->trans};
    etac::SceneDev rows;
    hipError_t e = etac::launch_hand_scene(p, scene_dev(scene), lk, &rows, s);
    int32_t *touch = touch_buffer(p, reward);
    if (e == hipSuccess)
        e = etac::launch_step(p, &rows, model_dev(model), scene->n_envs, nullptr, nullptr, u, contact_obj, n_active,
                              static_cast<uint32_t *>(saved), s, touch);
    if (e == hipSuccess) e = hand_reward(p, scene->n_envs, touch, reward, s);
    return e == hipSuccess ? ETAC_OK : hip_fail(e);
}

etac_status etac_hand_step_backward(etac_plan *plan, const etac_scene *scene, const etac_links *links,
                                    const etac_model *model, const float *grad_u, const void *saved,
                                    float *grad_rot, float *grad_trans, float *grad_link_rot,
                                    float *grad_link_trans, float *grad_alpha, float *grad_phi, void *stream) {
    if (!plan) return ETAC_ERR_NULL;
    const etac::Plan &p = plan->p;
    etac_status st = check_hand_call(p, scene, links);
    if (st != ETAC_OK) return st;
    st = check_model(model);
    if (st != ETAC_OK) return st;
    if (!p.has_bwd) return ETAC_ERR_WORKSPACE;
    if (scene->n_envs > 0 && (!grad_u || !grad_rot || !grad_trans || !grad_link_rot || !grad_link_trans))
        return ETAC_ERR_NULL;
    const hipStream_t s = (hipStream_t)stream;
    const etac::SceneDev world = scene_dev(scene);
    const etac::LinksDev lk{links->rot, links->trans};
    etac::SceneDev rows;
    hipError_t e = etac::launch_hand_scene(p, world, lk, &rows, s);
    // the adjoint hands winners over as row slots: no id mapping, no reward counts
    rows.src = nullptr;
    rows.n_ext = nullptr;
    if (e == hipSuccess)
        e = etac::launch_backward(p, &rows, model_dev(model), scene->n_envs, nullptr, nullptr, grad_u,
                                  static_cast<const uint32_t *>(saved), nullptr, grad_rot, grad_trans, grad_alpha,
                                  grad_phi, s, &world, &lk, grad_link_rot, grad_link_trans);
    return e == hipSuccess ? ETAC_OK : hip_fail(e);
}

etac_status etac_regress(etac_plan *plan, const float *reg, int32_t n_envs, const float *u,
                         const int32_t *n_active, float *taxels, void *stream) {
    if (!plan) return ETAC_ERR_NULL;
    const etac::Plan &p = plan->p;
    if (n_envs < 0 || n_envs > p.n_envs) return ETAC_ERR_SHAPE;
    if (n_envs > 0 && (!reg || !u || !n_active || !taxels)) return ETAC_ERR_NULL;
    const hipError_t e = etac::launch_regress(p, reg, n_envs, u, n_active, taxels, (hipStream_t)stream);
    return e == hipSuccess ? ETAC_OK : hip_fail(e);
}

}  // extern "C"

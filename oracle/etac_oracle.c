/*
 * etac_oracle.c -- plain FP64 CPU oracle of the ETac tactile step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * What it computes (ETac, Sec. III-A, "Lightweight Tactile Simulation
 * Framework"):
 *   1. contact: nodes of an elastomer patch that lie strictly inside a rigid
 *      object are "active"; each gets the displacement that moves it to the
 *      closest point of the object surface (the penalty-style local contact
 *      displacement u_hat, Sec. III-A "Overview");
 *   2. decay-based linear propagation (Eq. 1): a passive node i receives
 *      sum_j exp(-alpha ||p_j - p_i||) u_hat_j over the active nodes j of its
 *      patch, i.e. Omega U_a with Omega[i,j] = exp(-alpha ||p_j - p_i||);
 *   3. residual correction Phi (Sec. III-A "Residual Displacement
 *      Correction"): PointNet encoder on [P, N, U_hat] (n x 9) -> shared MLP ->
 *      64-d per-node features, max-pool -> 64-d global feature, global MLP,
 *      broadcast-concatenate -> n x 128, shared-MLP decoder -> n x 3, masked to
 *      passive nodes;
 *   4. Eq. 2: U_p = Omega U_a + Phi_p; active nodes keep u_hat.
 * and the reverse-mode adjoint of all of it with respect to object poses
 * (R, t), alpha and the network parameters.  Objects are primitives
 * (sphere, box, capsule) or closed triangle meshes (1b below: the exact
 * triangle SDF with pseudo-normal signs, and its pose adjoint).
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   - contact displacement = closest-point penetration vector; strict inside;
 *     deepest object wins, lowest index on ties;
 *   - FP64 predicate evaluated in the fixed order written below, no FMA
 *     (build with -ffp-contract=off), so masks are reproducible bit for bit;
 *   - Omega and the max-pool act per patch; alpha is one value per patch;
 *   - a patch with no active node has U = 0;
 *   - network widths 9-64-64 | 64 | 64 + [f;g'] 128-64-3, ReLU, linear
 *     output; input position is p - o_k (o_k: per-patch origin).
 *
 * Inputs are FP64 (the Python side promotes the FP32 arrays exactly).
 * Layouts: pos/nrm [3][N]; uhat/U/grad_u [3][E][N]; contact_obj [E][N];
 * n_active [E][K]; object arrays [E][O][...]; phi packed as
 * W1(64x9) b1 W2(64x64) b2 W3(64x64) b3 W4(64x128) b4 W5(3x64) b5.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NF 64        /* per-node / global feature width */
#define NIN 9        /* [p - o, n, u_hat] */
#define PHI_N 17411

enum { O_SPHERE = 0, O_BOX = 1, O_CAPSULE = 2, O_MESH = 3 };
enum { O_FULL = 0, O_DECAY_ONLY = 1, O_RESIDUAL_ONLY = 2 };

/* ------------------------------------------------------------------------ */
/* packed network parameters                                                */
/* ------------------------------------------------------------------------ */
typedef struct {
    const double *W1, *b1, *W2, *b2, *W3, *b3, *W4, *b4, *W5, *b5;
} net_t;

static net_t net_view(const double *phi) {
    net_t n;
    n.W1 = phi;            n.b1 = n.W1 + 64 * 9;
    n.W2 = n.b1 + 64;      n.b2 = n.W2 + 64 * 64;
    n.W3 = n.b2 + 64;      n.b3 = n.W3 + 64 * 64;
    n.W4 = n.b3 + 64;      n.b4 = n.W4 + 64 * 128;
    n.W5 = n.b4 + 64;      n.b5 = n.W5 + 3 * 64;
    return n;
}

/* gradient views share the same packing */
typedef struct {
    double *W1, *b1, *W2, *b2, *W3, *b3, *W4, *b4, *W5, *b5;
} dnet_t;

static dnet_t dnet_view(double *g) {
    dnet_t n;
    n.W1 = g;              n.b1 = n.W1 + 64 * 9;
    n.W2 = n.b1 + 64;      n.b2 = n.W2 + 64 * 64;
    n.W3 = n.b2 + 64;      n.b3 = n.W3 + 64 * 64;
    n.W4 = n.b3 + 64;      n.b4 = n.W4 + 64 * 128;
    n.W5 = n.b4 + 64;      n.b5 = n.W5 + 3 * 64;
    return n;
}

/* ------------------------------------------------------------------------ */
/* 64-bit FNV-1a fingerprint of discrete decisions (for the FD harness)     */
/* ------------------------------------------------------------------------ */
static uint64_t fnv(uint64_t h, int64_t v) {
    for (int b = 0; b < 8; ++b) {
        h ^= (uint64_t)((v >> (8 * b)) & 0xff);
        h *= 1099511628211ULL;
    }
    return h;
}

/* ------------------------------------------------------------------------ */
/* 1. contact: point vs rigid primitive                                     */
/* ------------------------------------------------------------------------ */
/* Discrete outcome of one node-object test. */
typedef struct {
    int inside;
    double depth;     /* penetration depth (distance to the surface) */
    double u[3];      /* displacement to the closest surface point */
    int face;         /* box: face axis; capsule: 1 if the axial clamp is active */
    int sign;         /* box: +1/-1 side of the face */
    int degenerate;   /* sphere/capsule: node on the centre point/axis */
} hit_t;

/*
 * Penetration of point p (normal nrm) into one object.  The frame transform
 * and the inside tests use this exact operation order in FP64 with
 * round-to-nearest-even and no fused multiply-add:
 *   d_c = p_c - t_c
 *   q_c = (R[0][c] d_0 + R[1][c] d_1) + R[2][c] d_2          (q = R^T d)
 *   sphere : s = (d_0 d_0 + d_1 d_1) + d_2 d_2,   inside <=> s < r r
 *   box    : inside <=> |q_c| < h_c for c = 0,1,2
 *   capsule: z = clamp(q_2, -L, L), v = (q_0, q_1, q_2 - z),
 *            s = (v_0 v_0 + v_1 v_1) + v_2 v_2,   inside <=> s < r r
 * The closest surface point then gives u_hat:
 *   sphere : depth = r - sqrt(s), u = (depth / sqrt(s)) d
 *   box    : face c* = argmin_c (h_c - |q_c|) (lowest c on ties),
 *            sign = +1 if q_c* >= 0 else -1, depth = h_c* - |q_c*|,
 *            u = (sign depth) R[:, c*]
 *   capsule: depth = r - sqrt(s), u = (depth / sqrt(s)) (R v)
 * A node exactly on the centre point (sphere) or on the axis segment
 * (capsule) has no unique closest point; it takes depth r and u = -r n.
 */
static hit_t penetrate(int type, const double *shape, const double *R, const double *t,
                       const double p[3], const double nrm[3]) {
    hit_t h;
    memset(&h, 0, sizeof h);
    double d0 = p[0] - t[0], d1 = p[1] - t[1], d2 = p[2] - t[2];
    if (type == O_SPHERE) {
        double r = shape[0];
        double s = (d0 * d0 + d1 * d1) + d2 * d2;
        if (!(s < r * r)) return h;
        h.inside = 1;
        if (s == 0.0) {
            h.degenerate = 1;
            h.depth = r;
            for (int a = 0; a < 3; ++a) h.u[a] = -r * nrm[a];
            return h;
        }
        double l = sqrt(s);
        h.depth = r - l;
        double sc = h.depth / l;
        h.u[0] = sc * d0; h.u[1] = sc * d1; h.u[2] = sc * d2;
        return h;
    }
    double q[3];
    for (int c = 0; c < 3; ++c) q[c] = (R[0 * 3 + c] * d0 + R[1 * 3 + c] * d1) + R[2 * 3 + c] * d2;
    if (type == O_BOX) {
        for (int c = 0; c < 3; ++c)
            if (!(fabs(q[c]) < shape[c])) return h;
        h.inside = 1;
        int cs = 0;
        double best = shape[0] - fabs(q[0]);
        for (int c = 1; c < 3; ++c) {
            double sl = shape[c] - fabs(q[c]);
            if (sl < best) { best = sl; cs = c; }
        }
        h.face = cs;
        h.sign = (q[cs] >= 0.0) ? 1 : -1;
        h.depth = best;
        double a = (double)h.sign * best;
        for (int r = 0; r < 3; ++r) h.u[r] = a * R[r * 3 + cs];
        return h;
    }
    /* capsule: radius shape[0], half segment length shape[1] along object z */
    double r = shape[0], L = shape[1];
    double z = q[2];
    int clamped = 0;
    if (z < -L) { z = -L; clamped = 1; }
    else if (z > L) { z = L; clamped = 1; }
    double v0 = q[0], v1 = q[1], v2 = q[2] - z;
    double s = (v0 * v0 + v1 * v1) + v2 * v2;
    if (!(s < r * r)) return h;
    h.inside = 1;
    h.face = clamped;
    if (s == 0.0) {
        h.degenerate = 1;
        h.depth = r;
        for (int a = 0; a < 3; ++a) h.u[a] = -r * nrm[a];
        return h;
    }
    double l = sqrt(s);
    h.depth = r - l;
    double sc = h.depth / l;
    for (int a = 0; a < 3; ++a) {
        double w = (R[a * 3 + 0] * v0 + R[a * 3 + 1] * v1) + R[a * 3 + 2] * v2;
        h.u[a] = sc * w;
    }
    return h;
}

typedef struct {
    int K, N;
    const int32_t *offset;
    const double *pos, *nrm, *origin;
    int E, O;
    const int32_t *n_obj, *type;
    const double *shape, *rot, *trans;
} problem_t;

/* Contact for every node of env e.  Several objects: the deepest penetration
 * wins (union of the objects' signed distance fields), ties to the lowest
 * object index.  Passive nodes get contact_obj = -1 and u_hat = 0. */
static void contact_env(const problem_t *P, int e, int8_t *cobj, double *uhat, int32_t *n_active,
                        uint64_t *sig) {
    const int N = P->N, E = P->E, O = P->O;
    for (int k = 0; k < P->K; ++k) n_active[(size_t)e * P->K + k] = 0;
    for (int k = 0; k < P->K; ++k) {
        for (int i = P->offset[k]; i < P->offset[k + 1]; ++i) {
            double p[3] = {P->pos[i], P->pos[N + i], P->pos[2 * N + i]};
            double n[3] = {P->nrm[i], P->nrm[N + i], P->nrm[2 * N + i]};
            int best = -1;
            hit_t bh;
            memset(&bh, 0, sizeof bh);
            for (int o = 0; o < P->n_obj[e]; ++o) {
                size_t eo = (size_t)e * O + o;
                if (P->type[eo] < O_SPHERE || P->type[eo] > O_CAPSULE) continue; /* meshes: contact_mesh_env */
                hit_t h = penetrate(P->type[eo], P->shape + 4 * eo, P->rot + 9 * eo,
                                    P->trans + 3 * eo, p, n);
                if (h.inside && (best < 0 || h.depth > bh.depth)) { best = o; bh = h; }
            }
            size_t en = (size_t)e * N + i;
            cobj[en] = (int8_t)best;
            for (int a = 0; a < 3; ++a) uhat[(size_t)a * E * N + en] = best >= 0 ? bh.u[a] : 0.0;
            if (best >= 0) n_active[(size_t)e * P->K + k] += 1;
            if (sig) {
                *sig = fnv(*sig, best);
                if (best >= 0) *sig = fnv(fnv(fnv(*sig, bh.face), bh.sign), bh.degenerate);
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* 1b. contact: point vs closed triangle mesh                               */
/* ------------------------------------------------------------------------ */
/*
 * The paper's contact queries the signed distance field of each object's
 * mesh (Sec. III-A, contact detection; the objects of Sec. IV are meshes).
 * Here the SDF is evaluated exactly on the triangles: the distance is the
 * minimum over the triangles of the point-triangle distance, and the sign
 * comes from the angle-weighted pseudo-normal of the closest feature
 * (face, edge or vertex), which is exact for a closed, consistently
 * oriented mesh (Baerentzen and Aanaes, IEEE TVCG 2005).  The closest point
 * on a triangle follows the Voronoi-region classification of Ericson
 * ("Real-Time Collision Detection", 2005, Sec. 5.1.5).  Readings (listed in
 * the design notes): the node is inside iff (q - c) . n < 0 for its closest
 * point c and pseudo-normal n; depth = |q - c|; u_hat = R (c - q); the
 * lowest triangle index wins distance ties; the deepest object (primitive
 * or mesh) wins, lowest object index on ties.
 *
 * FP64 operation order (round to nearest-even, no FMA); dot(x, y) means
 * (x0 y0 + x1 y1) + x2 y2 and vector +, - are componentwise:
 *   q = R^T (p - t) as for the primitives;
 *   ab = b - a, ac = c - a, ap = q - a, d1 = dot(ab, ap), d2 = dot(ac, ap)
 *   d1 <= 0 and d2 <= 0                      -> vertex a
 *   bp = q - b, d3 = dot(ab, bp), d4 = dot(ac, bp)
 *   d3 >= 0 and d4 <= d3                     -> vertex b
 *   vc = d1 d4 - d3 d2
 *   vc <= 0 and d1 >= 0 and d3 <= 0          -> edge ab, v = d1 / (d1 - d3), c = a + v ab
 *   cp = q - c, d5 = dot(ab, cp), d6 = dot(ac, cp)
 *   d6 >= 0 and d5 <= d6                     -> vertex c
 *   vb = d5 d2 - d1 d6
 *   vb <= 0 and d2 >= 0 and d6 <= 0          -> edge ca, w = d2 / (d2 - d6), c = a + w ac
 *   va = d3 d6 - d5 d4, e4 = d4 - d3, e5 = d5 - d6
 *   va <= 0 and e4 >= 0 and e5 >= 0          -> edge bc, w = e4 / (e4 + e5), c = b + w (c - b)
 *   otherwise face: den = (va + vb) + vc, v = vb / den, w = vc / den,
 *                   c = (a + v ab) + w ac
 *   s = dot(q - c, q - c); minimum over triangles with strict <.
 * Pseudo-normals (from the FP32 vertices promoted to FP64):
 *   face   : x = ab x ac = (ab1 ac2 - ab2 ac1, ab2 ac0 - ab0 ac2, ab0 ac1 - ab1 ac0),
 *            n_f = x / sqrt(dot(x, x));
 *   edge   : n_f + n_g, f and g the two faces sharing the edge;
 *   vertex : sum over the faces f containing it, ascending f, of theta_f n_f,
 *            theta = acos(clamp(dot(e1, e2) / (sqrt(dot(e1, e1)) sqrt(dot(e2, e2)), -1, 1)),
 *            e1, e2 the edges leaving the vertex in the order (a: b - a, c - a;
 *            b: c - b, a - b; c: a - c, b - c).
 */
enum { F_FACE = 0, F_EDGE_AB = 1, F_EDGE_BC = 2, F_EDGE_CA = 3, F_VERT_A = 4, F_VERT_B = 5, F_VERT_C = 6 };

static inline double dot3(const double x[3], const double y[3]) {
    return (x[0] * y[0] + x[1] * y[1]) + x[2] * y[2];
}

/* Closest point cp of triangle (a, b, c) to q; returns the squared distance
 * and the feature holding cp. */
static double closest_on_triangle(const double q[3], const double a[3], const double b[3],
                                  const double c[3], double cp[3], int *feature) {
    double ab[3], ac[3], ap[3], bp[3], cq[3], w[3];
    for (int i = 0; i < 3; ++i) { ab[i] = b[i] - a[i]; ac[i] = c[i] - a[i]; ap[i] = q[i] - a[i]; }
    double d1 = dot3(ab, ap), d2 = dot3(ac, ap);
    if (d1 <= 0.0 && d2 <= 0.0) {
        *feature = F_VERT_A;
        for (int i = 0; i < 3; ++i) cp[i] = a[i];
        goto done;
    }
    for (int i = 0; i < 3; ++i) bp[i] = q[i] - b[i];
    double d3 = dot3(ab, bp), d4 = dot3(ac, bp);
    if (d3 >= 0.0 && d4 <= d3) {
        *feature = F_VERT_B;
        for (int i = 0; i < 3; ++i) cp[i] = b[i];
        goto done;
    }
    double vc = d1 * d4 - d3 * d2;
    if (vc <= 0.0 && d1 >= 0.0 && d3 <= 0.0) {
        double v = d1 / (d1 - d3);
        *feature = F_EDGE_AB;
        for (int i = 0; i < 3; ++i) cp[i] = a[i] + v * ab[i];
        goto done;
    }
    for (int i = 0; i < 3; ++i) cq[i] = q[i] - c[i];
    double d5 = dot3(ab, cq), d6 = dot3(ac, cq);
    if (d6 >= 0.0 && d5 <= d6) {
        *feature = F_VERT_C;
        for (int i = 0; i < 3; ++i) cp[i] = c[i];
        goto done;
    }
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) {
        double wv = d2 / (d2 - d6);
        *feature = F_EDGE_CA;
        for (int i = 0; i < 3; ++i) cp[i] = a[i] + wv * ac[i];
        goto done;
    }
    double va = d3 * d6 - d5 * d4;
    double e4 = d4 - d3, e5 = d5 - d6;
    if (va <= 0.0 && e4 >= 0.0 && e5 >= 0.0) {
        double wv = e4 / (e4 + e5);
        *feature = F_EDGE_BC;
        for (int i = 0; i < 3; ++i) cp[i] = b[i] + wv * (c[i] - b[i]);
        goto done;
    }
    {
        double den = (va + vb) + vc;
        double v = vb / den, wv = vc / den;
        *feature = F_FACE;
        for (int i = 0; i < 3; ++i) cp[i] = (a[i] + v * ab[i]) + wv * ac[i];
    }
done:
    for (int i = 0; i < 3; ++i) w[i] = q[i] - cp[i];
    return dot3(w, w);
}

/* One mesh of a mesh set: corners and the seven pseudo-normals per triangle. */
typedef struct {
    int T;
    double *corner; /* [T][3 corners][3] */
    double *pn;     /* [T][7 features][3], feature order F_FACE .. F_VERT_C */
} trimesh_t;

static void trimesh_free(trimesh_t *m) {
    free(m->corner);
    free(m->pn);
    m->corner = m->pn = NULL;
}

/* Build mesh `m` of a set: triangles tri_offset[m] .. tri_offset[m+1]-1 of
 * `tris` (vertex indices into `verts` [V][3]).  Returns 0, or -2 when an
 * edge is not shared by exactly one other triangle in reverse direction
 * (the mesh is not closed and consistently oriented), or -3 for a zero-area
 * triangle or a vertex index out of range. */
static int trimesh_build(trimesh_t *out, int V, const double *verts, const int32_t *tris, int t0, int t1) {
    const int T = t1 - t0;
    out->T = T;
    out->corner = (double *)calloc((size_t)T * 9 + 1, sizeof(double));
    out->pn = (double *)calloc((size_t)T * 21 + 1, sizeof(double));
    double *fn = (double *)calloc((size_t)T * 3 + 1, sizeof(double));
    if (!out->corner || !out->pn || !fn) { free(fn); trimesh_free(out); return -3; }
    int rc = 0;
    for (int f = 0; f < T && rc == 0; ++f) {
        const int32_t *tv = tris + 3 * (size_t)(t0 + f);
        for (int k = 0; k < 3; ++k) {
            if (tv[k] < 0 || tv[k] >= V) { rc = -3; break; }
            for (int i = 0; i < 3; ++i) out->corner[f * 9 + k * 3 + i] = verts[3 * (size_t)tv[k] + i];
        }
        if (rc) break;
        const double *a = out->corner + f * 9, *b = a + 3, *c = a + 6;
        double ab[3], ac[3], x[3];
        for (int i = 0; i < 3; ++i) { ab[i] = b[i] - a[i]; ac[i] = c[i] - a[i]; }
        x[0] = ab[1] * ac[2] - ab[2] * ac[1];
        x[1] = ab[2] * ac[0] - ab[0] * ac[2];
        x[2] = ab[0] * ac[1] - ab[1] * ac[0];
        double len = sqrt(dot3(x, x));
        if (!(len > 0.0)) { rc = -3; break; }
        for (int i = 0; i < 3; ++i) fn[f * 3 + i] = x[i] / len;
    }
    /* edges: the face across directed edge (u -> v) holds (v -> u) */
    for (int f = 0; f < T && rc == 0; ++f) {
        const int32_t *tv = tris + 3 * (size_t)(t0 + f);
        for (int k = 0; k < 3 && rc == 0; ++k) {
            int u = tv[k], v = tv[(k + 1) % 3], other = -1, cnt = 0;
            for (int g = 0; g < T; ++g) {
                const int32_t *gv = tris + 3 * (size_t)(t0 + g);
                for (int l = 0; l < 3; ++l)
                    if (gv[l] == v && gv[(l + 1) % 3] == u) { other = g; ++cnt; }
                for (int l = 0; l < 3; ++l)
                    if (g != f && gv[l] == u && gv[(l + 1) % 3] == v) cnt += 2; /* duplicated direction */
            }
            if (cnt != 1) { rc = -2; break; }
            /* k = 0: edge ab, 1: bc, 2: ca */
            for (int i = 0; i < 3; ++i) out->pn[f * 21 + (1 + k) * 3 + i] = fn[f * 3 + i] + fn[other * 3 + i];
        }
    }
    /* vertices: angle-weighted sums over the incident faces, ascending face */
    for (int f = 0; f < T && rc == 0; ++f) {
        const int32_t *tv = tris + 3 * (size_t)(t0 + f);
        for (int i = 0; i < 3; ++i) out->pn[f * 21 + i] = fn[f * 3 + i];
        for (int k = 0; k < 3; ++k) {
            double acc[3] = {0.0, 0.0, 0.0};
            for (int g = 0; g < T; ++g) {
                const int32_t *gv = tris + 3 * (size_t)(t0 + g);
                for (int l = 0; l < 3; ++l) {
                    if (gv[l] != tv[k]) continue;
                    const double *P0 = out->corner + g * 9 + l * 3;
                    const double *P1 = out->corner + g * 9 + ((l + 1) % 3) * 3;
                    const double *P2 = out->corner + g * 9 + ((l + 2) % 3) * 3;
                    double e1[3], e2[3];
                    for (int i = 0; i < 3; ++i) { e1[i] = P1[i] - P0[i]; e2[i] = P2[i] - P0[i]; }
                    double cs = dot3(e1, e2) / (sqrt(dot3(e1, e1)) * sqrt(dot3(e2, e2)));
                    if (cs < -1.0) cs = -1.0;
                    if (cs > 1.0) cs = 1.0;
                    double th = acos(cs);
                    for (int i = 0; i < 3; ++i) acc[i] = acc[i] + th * fn[g * 3 + i];
                }
            }
            for (int i = 0; i < 3; ++i) out->pn[f * 21 + (4 + k) * 3 + i] = acc[i];
        }
    }
    free(fn);
    if (rc) trimesh_free(out);
    return rc;
}

/* Penetration of point p into mesh object (R, t). */
static hit_t mesh_penetrate(const trimesh_t *m, const double *R, const double *t, const double p[3]) {
    hit_t h;
    memset(&h, 0, sizeof h);
    double d0 = p[0] - t[0], d1 = p[1] - t[1], d2 = p[2] - t[2];
    double q[3];
    for (int c = 0; c < 3; ++c) q[c] = (R[0 * 3 + c] * d0 + R[1 * 3 + c] * d1) + R[2 * 3 + c] * d2;
    int bf = -1, bfeat = 0;
    double bs = 0.0, bcp[3] = {0.0, 0.0, 0.0};
    for (int f = 0; f < m->T; ++f) {
        double cp[3];
        int feat;
        const double *a = m->corner + f * 9;
        double s = closest_on_triangle(q, a, a + 3, a + 6, cp, &feat);
        if (bf < 0 || s < bs) {
            bf = f; bs = s; bfeat = feat;
            for (int i = 0; i < 3; ++i) bcp[i] = cp[i];
        }
    }
    if (bf < 0) return h;
    double w[3] = {q[0] - bcp[0], q[1] - bcp[1], q[2] - bcp[2]};
    if (!(dot3(w, m->pn + bf * 21 + bfeat * 3) < 0.0)) return h;
    h.inside = 1;
    h.face = bf;
    h.sign = bfeat;
    h.depth = sqrt(bs);
    double v[3] = {bcp[0] - q[0], bcp[1] - q[1], bcp[2] - q[2]};
    for (int a = 0; a < 3; ++a) h.u[a] = (R[a * 3 + 0] * v[0] + R[a * 3 + 1] * v[1]) + R[a * 3 + 2] * v[2];
    return h;
}

/*
 * Adjoint of one mesh node with respect to the pose (R, t), the winning
 * triangle f and feature held fixed.  With d = p - t, q = R^T d, c(q) the
 * closest point and w = c - q, u_hat = R w, and dw/dq = J:
 *   vertex : J = -I
 *   edge   : J = e e^T / |e|^2 - I   (e the edge direction)
 *   face   : J = -n n^T              (n the unit face normal)
 * J is symmetric.  For L = g . u_hat, with h = J R^T g:
 *   dL/dR = g w^T + d h^T  (R's nine entries taken as free inputs)
 *   dL/dt = -R h
 */
static void mesh_node_backward(const trimesh_t *m, const double *R, const double *t, const double p[3],
                               const double g[3], double *gR, double *gt) {
    double d[3] = {p[0] - t[0], p[1] - t[1], p[2] - t[2]};
    double q[3];
    for (int c = 0; c < 3; ++c) q[c] = (R[0 * 3 + c] * d[0] + R[1 * 3 + c] * d[1]) + R[2 * 3 + c] * d[2];
    int bf = -1, bfeat = 0;
    double bs = 0.0, bcp[3] = {0.0, 0.0, 0.0};
    for (int f = 0; f < m->T; ++f) {
        double cp[3];
        int feat;
        const double *a = m->corner + f * 9;
        double sq = closest_on_triangle(q, a, a + 3, a + 6, cp, &feat);
        if (bf < 0 || sq < bs) {
            bf = f; bs = sq; bfeat = feat;
            for (int i = 0; i < 3; ++i) bcp[i] = cp[i];
        }
    }
    const double *A = m->corner + bf * 9, *B = A + 3, *C = A + 6;
    double J[9];
    for (int i = 0; i < 9; ++i) J[i] = 0.0;
    if (bfeat == F_FACE) {
        const double *n = m->pn + bf * 21;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) J[i * 3 + j] = -n[i] * n[j];
    } else if (bfeat >= F_EDGE_AB && bfeat <= F_EDGE_CA) {
        const double *e0 = bfeat == F_EDGE_AB ? A : (bfeat == F_EDGE_BC ? B : C);
        const double *e1 = bfeat == F_EDGE_AB ? B : (bfeat == F_EDGE_BC ? C : A);
        double e[3] = {e1[0] - e0[0], e1[1] - e0[1], e1[2] - e0[2]};
        double ee = dot3(e, e);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) J[i * 3 + j] = e[i] * e[j] / ee - (i == j ? 1.0 : 0.0);
    } else {
        for (int i = 0; i < 3; ++i) J[i * 4] = -1.0;
    }
    double RTg[3], h[3], w[3];
    for (int c = 0; c < 3; ++c) RTg[c] = R[0 * 3 + c] * g[0] + R[1 * 3 + c] * g[1] + R[2 * 3 + c] * g[2];
    for (int i = 0; i < 3; ++i) h[i] = J[i * 3 + 0] * RTg[0] + J[i * 3 + 1] * RTg[1] + J[i * 3 + 2] * RTg[2];
    for (int i = 0; i < 3; ++i) w[i] = bcp[i] - q[i];
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b) gR[a * 3 + b] += g[a] * w[b] + d[a] * h[b];
        gt[a] += -(R[a * 3 + 0] * h[0] + R[a * 3 + 1] * h[1] + R[a * 3 + 2] * h[2]);
    }
}

/* Mesh index of an ETAC-mesh object, or -1 when shape[0] is not an integer
 * in [0, n_meshes). */
static int mesh_index(const double *shape, int n_meshes) {
    double x = shape[0];
    if (!(x >= 0.0) || !(x < (double)n_meshes) || x != floor(x)) return -1;
    return (int)x;
}

/* Contact of env e with primitives and meshes: the deepest object wins,
 * lowest object index on ties. */
static void contact_mesh_env(const problem_t *P, const trimesh_t *meshes, int n_meshes, int e, int8_t *cobj,
                             double *uhat, int32_t *n_active) {
    const int N = P->N, E = P->E, O = P->O;
    for (int k = 0; k < P->K; ++k) n_active[(size_t)e * P->K + k] = 0;
    for (int k = 0; k < P->K; ++k) {
        for (int i = P->offset[k]; i < P->offset[k + 1]; ++i) {
            double p[3] = {P->pos[i], P->pos[N + i], P->pos[2 * N + i]};
            double n[3] = {P->nrm[i], P->nrm[N + i], P->nrm[2 * N + i]};
            int best = -1;
            hit_t bh;
            memset(&bh, 0, sizeof bh);
            for (int o = 0; o < P->n_obj[e]; ++o) {
                size_t eo = (size_t)e * O + o;
                hit_t h;
                int ty = P->type[eo];
                if (ty >= O_SPHERE && ty <= O_CAPSULE) {
                    h = penetrate(ty, P->shape + 4 * eo, P->rot + 9 * eo, P->trans + 3 * eo, p, n);
                } else if (ty == O_MESH) {
                    int mi = mesh_index(P->shape + 4 * eo, n_meshes);
                    if (mi < 0) continue;
                    h = mesh_penetrate(meshes + mi, P->rot + 9 * eo, P->trans + 3 * eo, p);
                } else {
                    continue;
                }
                if (h.inside && (best < 0 || h.depth > bh.depth)) { best = o; bh = h; }
            }
            size_t en = (size_t)e * N + i;
            cobj[en] = (int8_t)best;
            for (int a = 0; a < 3; ++a) uhat[(size_t)a * E * N + en] = best >= 0 ? bh.u[a] : 0.0;
            if (best >= 0) n_active[(size_t)e * P->K + k] += 1;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* 2./3./4. propagation for one patch of one env                            */
/* ------------------------------------------------------------------------ */
static inline double relu(double x) { return x > 0.0 ? x : 0.0; }

/* scratch for one patch (sized for the largest patch) */
typedef struct {
    int *act, *pas;
    double *x;          /* [n][9]   */
    double *pre1, *h1;  /* [n][64]  */
    double *pre2, *f;   /* [n][64]  */
    double *df;         /* [n][64]  */
    int *argmax;        /* [64]     */
    double g[NF], pre3[NF], gp[NF];
} scratch_t;

static scratch_t scratch_new(int nmax) {
    scratch_t s;
    s.act = malloc(sizeof(int) * nmax);
    s.pas = malloc(sizeof(int) * nmax);
    s.x = malloc(sizeof(double) * nmax * NIN);
    s.pre1 = malloc(sizeof(double) * nmax * NF);
    s.h1 = malloc(sizeof(double) * nmax * NF);
    s.pre2 = malloc(sizeof(double) * nmax * NF);
    s.f = malloc(sizeof(double) * nmax * NF);
    s.df = malloc(sizeof(double) * nmax * NF);
    s.argmax = malloc(sizeof(int) * NF);
    return s;
}

static void scratch_free(scratch_t *s) {
    free(s->act); free(s->pas); free(s->x); free(s->pre1); free(s->h1);
    free(s->pre2); free(s->f); free(s->df); free(s->argmax);
}

static int max_patch(const problem_t *P) {
    int m = 1;
    for (int k = 0; k < P->K; ++k) {
        int n = P->offset[k + 1] - P->offset[k];
        if (n > m) m = n;
    }
    return m;
}

/* Encoder of the residual network for every node of the patch, then the
 * max-pool over all n nodes (lowest node wins ties) and the global MLP.
 * Network input x_i = [p_i - o_k, n_i, U_hat_i] with U_hat_i = 0 for passive
 * nodes. */
static void phi_encode(const problem_t *P, const net_t *W, int e, int k, const int8_t *cobj,
                       const double *uhat, scratch_t *S, double *margin, uint64_t *sig) {
    const int N = P->N, E = P->E;
    const int o0 = P->offset[k], n = P->offset[k + 1] - o0;
    for (int li = 0; li < n; ++li) {
        int i = o0 + li;
        size_t en = (size_t)e * N + i;
        double *x = S->x + (size_t)li * NIN;
        for (int a = 0; a < 3; ++a) {
            x[a] = P->pos[(size_t)a * N + i] - P->origin[3 * k + a];
            x[3 + a] = P->nrm[(size_t)a * N + i];
            x[6 + a] = cobj[en] >= 0 ? uhat[(size_t)a * E * N + en] : 0.0;
        }
        double *pre1 = S->pre1 + (size_t)li * NF, *h1 = S->h1 + (size_t)li * NF;
        for (int o = 0; o < NF; ++o) {
            double acc = W->b1[o];
            for (int c = 0; c < NIN; ++c) acc += W->W1[o * NIN + c] * x[c];
            pre1[o] = acc;
            h1[o] = relu(acc);
        }
        double *pre2 = S->pre2 + (size_t)li * NF, *f = S->f + (size_t)li * NF;
        for (int o = 0; o < NF; ++o) {
            double acc = W->b2[o];
            for (int c = 0; c < NF; ++c) acc += W->W2[o * NF + c] * h1[c];
            pre2[o] = acc;
            f[o] = relu(acc);
        }
        if (margin)
            for (int o = 0; o < NF; ++o) {
                if (fabs(pre1[o]) < *margin) *margin = fabs(pre1[o]);
                if (fabs(pre2[o]) < *margin) *margin = fabs(pre2[o]);
            }
        if (sig)
            for (int o = 0; o < NF; ++o) *sig = fnv(fnv(*sig, pre1[o] > 0.0), pre2[o] > 0.0);
    }
    /* max-pool over all nodes of the patch */
    for (int c = 0; c < NF; ++c) {
        int am = 0;
        double best = S->f[c];
        for (int li = 1; li < n; ++li)
            if (S->f[(size_t)li * NF + c] > best) { best = S->f[(size_t)li * NF + c]; am = li; }
        S->g[c] = best;
        S->argmax[c] = am;
        if (margin && best > 0.0) {
            /* gap to the runner-up: an FP32 evaluation may pick another node */
            double second = -1.0;
            for (int li = 0; li < n; ++li)
                if (li != am && S->f[(size_t)li * NF + c] > second) second = S->f[(size_t)li * NF + c];
            if (second >= 0.0 && best - second < *margin) *margin = best - second;
        }
        if (sig) *sig = fnv(*sig, am);
    }
    /* global MLP */
    for (int o = 0; o < NF; ++o) {
        double acc = W->b3[o];
        for (int c = 0; c < NF; ++c) acc += W->W3[o * NF + c] * S->g[c];
        S->pre3[o] = acc;
        S->gp[o] = relu(acc);
        if (margin && fabs(acc) < *margin) *margin = fabs(acc);
        if (sig) *sig = fnv(*sig, acc > 0.0);
    }
}

/* Decoder for one node: z = [f_i ; g'] (per-node features first),
 * h4 = ReLU(W4 z + b4), r = W5 h4 + b5. */
static void phi_decode(const net_t *W, const double *f, const double *gp, double *pre4, double *h4,
                       double r[3]) {
    for (int o = 0; o < NF; ++o) {
        double acc = W->b4[o];
        for (int c = 0; c < NF; ++c) acc += W->W4[o * 2 * NF + c] * f[c];
        for (int c = 0; c < NF; ++c) acc += W->W4[o * 2 * NF + NF + c] * gp[c];
        pre4[o] = acc;
        h4[o] = relu(acc);
    }
    for (int a = 0; a < 3; ++a) {
        double acc = W->b5[a];
        for (int c = 0; c < NF; ++c) acc += W->W5[a * NF + c] * h4[c];
        r[a] = acc;
    }
}

/* Eq. 1 weight between two nodes: exp(-alpha ||p_j - p_i||_2). */
static inline double decay_weight(const problem_t *P, double alpha, int i, int j, double *dist) {
    const int N = P->N;
    double dx = P->pos[j] - P->pos[i];
    double dy = P->pos[N + j] - P->pos[N + i];
    double dz = P->pos[2 * N + j] - P->pos[2 * N + i];
    double d = sqrt(dx * dx + dy * dy + dz * dz);
    if (dist) *dist = d;
    return exp(-alpha * d);
}

static void split_sets(const problem_t *P, int e, int k, const int8_t *cobj, scratch_t *S, int *m,
                       int *np) {
    int a = 0, b = 0;
    for (int i = P->offset[k]; i < P->offset[k + 1]; ++i) {
        if (cobj[(size_t)e * P->N + i] >= 0) S->act[a++] = i;
        else S->pas[b++] = i;
    }
    *m = a;
    *np = b;
}

/* Forward propagation (Eqs. 1-2) for patch k of env e. */
static void propagate_patch(const problem_t *P, const net_t *W, int mode, const double *alpha, int e,
                            int k, const int8_t *cobj, const double *uhat, double *U, scratch_t *S,
                            double *margin, uint64_t *sig) {
    const int N = P->N, E = P->E;
    int m, np;
    split_sets(P, e, k, cobj, S, &m, &np);
    for (int i = P->offset[k]; i < P->offset[k + 1]; ++i)
        for (int a = 0; a < 3; ++a) U[(size_t)a * E * N + (size_t)e * N + i] = 0.0;
    if (m == 0) return; /* no contact on this patch: no deformation */
    /* active nodes keep their contact displacement */
    for (int t = 0; t < m; ++t) {
        size_t en = (size_t)e * N + S->act[t];
        for (int a = 0; a < 3; ++a) U[(size_t)a * E * N + en] = uhat[(size_t)a * E * N + en];
    }
    /* Eq. 1: Omega U_a for every passive node */
    if (mode != O_RESIDUAL_ONLY) {
        for (int t = 0; t < np; ++t) {
            int i = S->pas[t];
            double acc[3] = {0, 0, 0};
            for (int s = 0; s < m; ++s) {
                int j = S->act[s];
                double w = decay_weight(P, alpha[k], i, j, NULL);
                size_t ej = (size_t)e * N + j;
                for (int a = 0; a < 3; ++a) acc[a] += w * uhat[(size_t)a * E * N + ej];
            }
            for (int a = 0; a < 3; ++a) U[(size_t)a * E * N + (size_t)e * N + i] += acc[a];
        }
    }
    /* residual network, kept for passive nodes only (mask M_p) */
    if (mode != O_DECAY_ONLY) {
        phi_encode(P, W, e, k, cobj, uhat, S, margin, sig);
        double pre4[NF], h4[NF], r[3];
        for (int t = 0; t < np; ++t) {
            int i = S->pas[t];
            int li = i - P->offset[k];
            phi_decode(W, S->f + (size_t)li * NF, S->gp, pre4, h4, r);
            if (margin)
                for (int o = 0; o < NF; ++o)
                    if (fabs(pre4[o]) < *margin) *margin = fabs(pre4[o]);
            if (sig)
                for (int o = 0; o < NF; ++o) *sig = fnv(*sig, pre4[o] > 0.0);
            for (int a = 0; a < 3; ++a) U[(size_t)a * E * N + (size_t)e * N + i] += r[a];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* adjoint of the propagation for one patch                                 */
/* ------------------------------------------------------------------------ */
/* L = sum_i g_i . U_i.  Accumulates dL/du_hat (active nodes only), dL/dalpha_k
 * and dL/dphi.  Conventions: ReLU'(0) = 0; the max-pool routes its gradient
 * to the arg-max node (lowest index on ties). */
static void propagate_patch_backward(const problem_t *P, const net_t *W, int mode, const double *alpha,
                                     int e, int k, const int8_t *cobj, const double *uhat,
                                     const double *gu, double *guhat, double *galpha, dnet_t *dW,
                                     scratch_t *S) {
    const int N = P->N, E = P->E;
    const size_t EN = (size_t)E * N;
    int m, np;
    split_sets(P, e, k, cobj, S, &m, &np);
    for (int i = P->offset[k]; i < P->offset[k + 1]; ++i)
        for (int a = 0; a < 3; ++a) guhat[a * EN + (size_t)e * N + i] = 0.0;
    if (m == 0) return;
    /* active nodes: U_j = u_hat_j */
    for (int s = 0; s < m; ++s) {
        size_t ej = (size_t)e * N + S->act[s];
        for (int a = 0; a < 3; ++a) guhat[a * EN + ej] += gu[a * EN + ej];
    }
    /* Eq. 1 adjoint: d u_hat_j += w_ij g_i ; d alpha += -d_ij w_ij (g_i . u_hat_j) */
    if (mode != O_RESIDUAL_ONLY) {
        double da = 0.0;
        for (int t = 0; t < np; ++t) {
            int i = S->pas[t];
            size_t ei = (size_t)e * N + i;
            double gi[3] = {gu[ei], gu[EN + ei], gu[2 * EN + ei]};
            for (int s = 0; s < m; ++s) {
                int j = S->act[s];
                size_t ej = (size_t)e * N + j;
                double d;
                double w = decay_weight(P, alpha[k], i, j, &d);
                double dot = 0.0;
                for (int a = 0; a < 3; ++a) {
                    guhat[a * EN + ej] += w * gi[a];
                    dot += gi[a] * uhat[a * EN + ej];
                }
                da += -d * w * dot;
            }
        }
        *galpha += da;
    }
    if (mode == O_DECAY_ONLY) return;
    /* residual network adjoint */
    phi_encode(P, W, e, k, cobj, uhat, S, NULL, NULL);
    const int o0 = P->offset[k], n = P->offset[k + 1] - o0;
    memset(S->df, 0, sizeof(double) * (size_t)n * NF);
    double dgp[NF];
    memset(dgp, 0, sizeof dgp);
    double pre4[NF], h4[NF], r[3], dh4[NF];
    for (int t = 0; t < np; ++t) {
        int i = S->pas[t];
        int li = i - o0;
        size_t ei = (size_t)e * N + i;
        const double *f = S->f + (size_t)li * NF;
        phi_decode(W, f, S->gp, pre4, h4, r);
        double dr[3] = {gu[ei], gu[EN + ei], gu[2 * EN + ei]};
        for (int a = 0; a < 3; ++a) {
            dW->b5[a] += dr[a];
            for (int c = 0; c < NF; ++c) dW->W5[a * NF + c] += dr[a] * h4[c];
        }
        for (int c = 0; c < NF; ++c) {
            double acc = 0.0;
            for (int a = 0; a < 3; ++a) acc += W->W5[a * NF + c] * dr[a];
            dh4[c] = pre4[c] > 0.0 ? acc : 0.0;
        }
        for (int o = 0; o < NF; ++o) {
            if (dh4[o] == 0.0) continue;
            dW->b4[o] += dh4[o];
            for (int c = 0; c < NF; ++c) {
                dW->W4[o * 2 * NF + c] += dh4[o] * f[c];
                dW->W4[o * 2 * NF + NF + c] += dh4[o] * S->gp[c];
                S->df[(size_t)li * NF + c] += W->W4[o * 2 * NF + c] * dh4[o];
                dgp[c] += W->W4[o * 2 * NF + NF + c] * dh4[o];
            }
        }
    }
    /* global MLP and max-pool */
    double dpre3[NF], dg[NF];
    for (int o = 0; o < NF; ++o) dpre3[o] = S->pre3[o] > 0.0 ? dgp[o] : 0.0;
    for (int o = 0; o < NF; ++o) {
        dW->b3[o] += dpre3[o];
        for (int c = 0; c < NF; ++c) dW->W3[o * NF + c] += dpre3[o] * S->g[c];
    }
    for (int c = 0; c < NF; ++c) {
        double acc = 0.0;
        for (int o = 0; o < NF; ++o) acc += W->W3[o * NF + c] * dpre3[o];
        dg[c] = acc;
    }
    for (int c = 0; c < NF; ++c) S->df[(size_t)S->argmax[c] * NF + c] += dg[c];
    /* encoder adjoint for every node */
    for (int li = 0; li < n; ++li) {
        const double *df = S->df + (size_t)li * NF;
        const double *pre2 = S->pre2 + (size_t)li * NF, *pre1 = S->pre1 + (size_t)li * NF;
        const double *h1 = S->h1 + (size_t)li * NF, *x = S->x + (size_t)li * NIN;
        double dpre2[NF], dpre1[NF];
        int any = 0;
        for (int o = 0; o < NF; ++o) {
            dpre2[o] = pre2[o] > 0.0 ? df[o] : 0.0;
            any |= dpre2[o] != 0.0;
        }
        if (!any) continue;
        for (int o = 0; o < NF; ++o) {
            dW->b2[o] += dpre2[o];
            for (int c = 0; c < NF; ++c) dW->W2[o * NF + c] += dpre2[o] * h1[c];
        }
        for (int c = 0; c < NF; ++c) {
            double acc = 0.0;
            for (int o = 0; o < NF; ++o) acc += W->W2[o * NF + c] * dpre2[o];
            dpre1[c] = pre1[c] > 0.0 ? acc : 0.0;
        }
        for (int o = 0; o < NF; ++o) {
            dW->b1[o] += dpre1[o];
            for (int c = 0; c < NIN; ++c) dW->W1[o * NIN + c] += dpre1[o] * x[c];
        }
        int i = o0 + li;
        size_t ei = (size_t)e * N + i;
        if (cobj[ei] >= 0) { /* only active nodes carry u_hat into the input */
            for (int a = 0; a < 3; ++a) {
                double acc = 0.0;
                for (int o = 0; o < NF; ++o) acc += W->W1[o * NIN + 6 + a] * dpre1[o];
                guhat[a * EN + ei] += acc;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* adjoint of the contact displacement with respect to the object pose      */
/* ------------------------------------------------------------------------ */
/* Derivatives of u_hat as the function written in penetrate(), with R taken
 * as nine free entries (the chosen face / clamp state held fixed):
 *   sphere : u = phi(s) d, phi = r/sqrt(s) - 1, s = d.d, d = p - t
 *            dL/dt = -(phi g + 2 phi'(s) (g.d) d),  dL/dR = 0
 *   box    : u = (sg h_c - q_c) R[:,c],  q_c = R[:,c].d
 *            dL/dt = (g.R[:,c]) R[:,c]
 *            dL/dR[:,c] = (sg h_c - q_c) g - (g.R[:,c]) d, other columns 0
 *   capsule: u = phi(s) R v, v = q - z e_3, q = R^T d, s = v.v
 *            a = 2 phi'(s) (g.Rv) v + phi P R^T g   (P = diag(1,1,0) when the
 *            axial clamp is inactive, else I)
 *            dL/dR = d a^T + phi g v^T,  dL/dt = -R a
 * Degenerate nodes (u = -r n) carry no pose dependence. */
static void contact_node_backward(int type, const double *shape, const double *R, const double *t,
                                  const double p[3], const double g[3], double *gR, double *gt) {
    double d[3] = {p[0] - t[0], p[1] - t[1], p[2] - t[2]};
    if (type == O_SPHERE) {
        double r = shape[0];
        double s = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (s == 0.0) return;
        double l = sqrt(s);
        double phi = r / l - 1.0;
        double twophip = -r / (l * s);
        double gd = g[0] * d[0] + g[1] * d[1] + g[2] * d[2];
        for (int a = 0; a < 3; ++a) gt[a] += -(phi * g[a] + twophip * gd * d[a]);
        return;
    }
    double q[3];
    for (int c = 0; c < 3; ++c) q[c] = R[0 * 3 + c] * d[0] + R[1 * 3 + c] * d[1] + R[2 * 3 + c] * d[2];
    if (type == O_BOX) {
        int cs = 0;
        double best = shape[0] - fabs(q[0]);
        for (int c = 1; c < 3; ++c) {
            double sl = shape[c] - fabs(q[c]);
            if (sl < best) { best = sl; cs = c; }
        }
        double sg = (q[cs] >= 0.0) ? 1.0 : -1.0;
        double rc[3] = {R[0 * 3 + cs], R[1 * 3 + cs], R[2 * 3 + cs]};
        double grc = g[0] * rc[0] + g[1] * rc[1] + g[2] * rc[2];
        double coef = sg * shape[cs] - q[cs];
        for (int a = 0; a < 3; ++a) {
            gt[a] += grc * rc[a];
            gR[a * 3 + cs] += coef * g[a] - grc * d[a];
        }
        return;
    }
    double r = shape[0], L = shape[1];
    double z = q[2];
    int clamped = 0;
    if (z < -L) { z = -L; clamped = 1; }
    else if (z > L) { z = L; clamped = 1; }
    double v[3] = {q[0], q[1], q[2] - z};
    double s = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    if (s == 0.0) return;
    double l = sqrt(s);
    double phi = r / l - 1.0;
    double twophip = -r / (l * s);
    double Rv[3], RTg[3];
    for (int a = 0; a < 3; ++a) Rv[a] = R[a * 3 + 0] * v[0] + R[a * 3 + 1] * v[1] + R[a * 3 + 2] * v[2];
    for (int c = 0; c < 3; ++c) RTg[c] = R[0 * 3 + c] * g[0] + R[1 * 3 + c] * g[1] + R[2 * 3 + c] * g[2];
    double gRv = g[0] * Rv[0] + g[1] * Rv[1] + g[2] * Rv[2];
    double av[3];
    for (int c = 0; c < 3; ++c) av[c] = twophip * gRv * v[c] + phi * RTg[c];
    if (!clamped) av[2] = twophip * gRv * v[2]; /* P drops the axial row; v[2] = 0 here */
    for (int a = 0; a < 3; ++a) {
        for (int c = 0; c < 3; ++c) gR[a * 3 + c] += d[a] * av[c] + phi * g[a] * v[c];
        gt[a] += -(R[a * 3 + 0] * av[0] + R[a * 3 + 1] * av[1] + R[a * 3 + 2] * av[2]);
    }
}

/* pose gradients of env e from dL/du_hat of its active nodes */
static void contact_env_backward(const problem_t *P, int e, const double *guhat, double *grot,
                                 double *gtrans) {
    const int N = P->N, E = P->E, O = P->O;
    const size_t EN = (size_t)E * N;
    for (int o = 0; o < O; ++o) {
        for (int c = 0; c < 9; ++c) grot[((size_t)e * O + o) * 9 + c] = 0.0;
        for (int c = 0; c < 3; ++c) gtrans[((size_t)e * O + o) * 3 + c] = 0.0;
    }
    for (int i = 0; i < N; ++i) {
        double p[3] = {P->pos[i], P->pos[N + i], P->pos[2 * N + i]};
        double n[3] = {P->nrm[i], P->nrm[N + i], P->nrm[2 * N + i]};
        int best = -1;
        hit_t bh;
        memset(&bh, 0, sizeof bh);
        for (int o = 0; o < P->n_obj[e]; ++o) {
            size_t eo = (size_t)e * O + o;
            if (P->type[eo] < O_SPHERE || P->type[eo] > O_CAPSULE) continue;
            hit_t h = penetrate(P->type[eo], P->shape + 4 * eo, P->rot + 9 * eo, P->trans + 3 * eo, p, n);
            if (h.inside && (best < 0 || h.depth > bh.depth)) { best = o; bh = h; }
        }
        if (best < 0 || bh.degenerate) continue;
        size_t ei = (size_t)e * N + i, eo = (size_t)e * O + best;
        double g[3] = {guhat[ei], guhat[EN + ei], guhat[2 * EN + ei]};
        contact_node_backward(P->type[eo], P->shape + 4 * eo, P->rot + 9 * eo, P->trans + 3 * eo, p, g,
                              grot + 9 * eo, gtrans + 3 * eo);
    }
}

/* ------------------------------------------------------------------------ */
/* exported entry points (ctypes)                                           */
/* ------------------------------------------------------------------------ */
static problem_t mkprob(int K, int N, const int32_t *offset, const double *pos, const double *nrm,
                        const double *origin, int E, int O, const int32_t *n_obj, const int32_t *type,
                        const double *shape, const double *rot, const double *trans) {
    problem_t P = {K, N, offset, pos, nrm, origin, E, O, n_obj, type, shape, rot, trans};
    return P;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel loops (timing of the CPU baseline). */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Contact only.  Outputs contact_obj [E][N], uhat [3][E][N], n_active [E][K]. */
int oracle_contact(int K, int N, const int32_t *offset, const double *pos, const double *nrm, int E,
                   int O, const int32_t *n_obj, const int32_t *type, const double *shape,
                   const double *rot, const double *trans, int8_t *cobj, double *uhat,
                   int32_t *n_active) {
    problem_t P = mkprob(K, N, offset, pos, nrm, NULL, E, O, n_obj, type, shape, rot, trans);
#pragma omp parallel for schedule(static)
    for (int e = 0; e < E; ++e) contact_env(&P, e, cobj, uhat, n_active, NULL);
    return 0;
}

/* Propagation of given contact results (Eqs. 1-2).  u [3][E][N]. */
int oracle_propagate(int K, int N, const int32_t *offset, const double *pos, const double *nrm,
                     const double *origin, int E, int mode, const double *alpha, const double *phi,
                     const int8_t *cobj, const double *uhat, double *U) {
    problem_t P = mkprob(K, N, offset, pos, nrm, origin, E, 0, NULL, NULL, NULL, NULL, NULL);
    net_t W = net_view(phi);
    int nmax = max_patch(&P);
#pragma omp parallel
    {
        scratch_t S = scratch_new(nmax);
#pragma omp for schedule(static)
        for (int e = 0; e < E; ++e)
            for (int k = 0; k < K; ++k) propagate_patch(&P, &W, mode, alpha, e, k, cobj, uhat, U, &S, NULL, NULL);
        scratch_free(&S);
    }
    return 0;
}

/* Whole forward step.  Optional outputs (may be NULL): sig [E] fingerprint of
 * every discrete decision, margin [E] smallest distance of a ReLU input or
 * max-pool runner-up gap from its decision boundary. */
int oracle_forward(int K, int N, const int32_t *offset, const double *pos, const double *nrm,
                   const double *origin, int E, int O, const int32_t *n_obj, const int32_t *type,
                   const double *shape, const double *rot, const double *trans, int mode,
                   const double *alpha, const double *phi, double *U, int8_t *cobj, double *uhat,
                   int32_t *n_active, uint64_t *sig, double *margin) {
    problem_t P = mkprob(K, N, offset, pos, nrm, origin, E, O, n_obj, type, shape, rot, trans);
    net_t W = net_view(phi);
    int nmax = max_patch(&P);
#pragma omp parallel
    {
        scratch_t S = scratch_new(nmax);
#pragma omp for schedule(static)
        for (int e = 0; e < E; ++e) {
            uint64_t h = 1469598103934665603ULL;
            double mg = INFINITY;
            contact_env(&P, e, cobj, uhat, n_active, sig ? &h : NULL);
            for (int k = 0; k < K; ++k)
                propagate_patch(&P, &W, mode, alpha, e, k, cobj, uhat, U, &S, margin ? &mg : NULL,
                                sig ? &h : NULL);
            if (sig) sig[e] = h;
            if (margin) margin[e] = mg;
        }
        scratch_free(&S);
    }
    return 0;
}

/* Whole forward step with the decision margin of every (env, patch) item:
 * margin [E][K] is the smallest distance of a ReLU input or max-pool
 * runner-up gap of the item from its decision boundary (INFINITY when the
 * item evaluates no network).  A diagnostic for the parity checks: an item
 * whose margin exceeds the FP32 rounding of the pre-activations takes the
 * same discrete decisions in FP32 as here. */
int oracle_item_margins(int K, int N, const int32_t *offset, const double *pos, const double *nrm,
                        const double *origin, int E, int O, const int32_t *n_obj, const int32_t *type,
                        const double *shape, const double *rot, const double *trans, int mode,
                        const double *alpha, const double *phi, double *U, int8_t *cobj, double *uhat,
                        int32_t *n_active, double *margin) {
    problem_t P = mkprob(K, N, offset, pos, nrm, origin, E, O, n_obj, type, shape, rot, trans);
    net_t W = net_view(phi);
    int nmax = max_patch(&P);
#pragma omp parallel
    {
        scratch_t S = scratch_new(nmax);
#pragma omp for schedule(static)
        for (int e = 0; e < E; ++e) {
            contact_env(&P, e, cobj, uhat, n_active, NULL);
            for (int k = 0; k < K; ++k) {
                double mg = INFINITY;
                propagate_patch(&P, &W, mode, alpha, e, k, cobj, uhat, U, &S, &mg, NULL);
                margin[(size_t)e * K + k] = mg;
            }
        }
        scratch_free(&S);
    }
    return 0;
}

/* Adjoint of the propagation.  Outputs guhat [3][E][N] (zero on passive
 * nodes), galpha [K], gphi [PHI_N] (both overwritten). */
int oracle_propagate_backward(int K, int N, const int32_t *offset, const double *pos,
                              const double *nrm, const double *origin, int E, int mode,
                              const double *alpha, const double *phi, const int8_t *cobj,
                              const double *uhat, const double *gu, double *guhat, double *galpha,
                              double *gphi) {
    problem_t P = mkprob(K, N, offset, pos, nrm, origin, E, 0, NULL, NULL, NULL, NULL, NULL);
    net_t W = net_view(phi);
    int nmax = max_patch(&P);
    int nt = oracle_num_threads();
    double *pa = calloc((size_t)nt * K, sizeof(double));
    double *pp = calloc((size_t)nt * PHI_N, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        scratch_t S = scratch_new(nmax);
        dnet_t dW = dnet_view(pp + (size_t)tid * PHI_N);
#pragma omp for schedule(static)
        for (int e = 0; e < E; ++e)
            for (int k = 0; k < K; ++k)
                propagate_patch_backward(&P, &W, mode, alpha, e, k, cobj, uhat, gu, guhat,
                                         pa + (size_t)tid * K + k, &dW, &S);
        scratch_free(&S);
    }
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int t = 0; t < nt; ++t) s += pa[(size_t)t * K + k];
        galpha[k] = s;
    }
    for (int c = 0; c < PHI_N; ++c) {
        double s = 0.0;
        for (int t = 0; t < nt; ++t) s += pp[(size_t)t * PHI_N + c];
        gphi[c] = s;
    }
    free(pa);
    free(pp);
    return 0;
}

/* Adjoint of the contact pass: grot [E][O][9], gtrans [E][O][3]. */
int oracle_contact_backward(int K, int N, const int32_t *offset, const double *pos, const double *nrm,
                            int E, int O, const int32_t *n_obj, const int32_t *type,
                            const double *shape, const double *rot, const double *trans,
                            const double *guhat, double *grot, double *gtrans) {
    problem_t P = mkprob(K, N, offset, pos, nrm, NULL, E, O, n_obj, type, shape, rot, trans);
#pragma omp parallel for schedule(static)
    for (int e = 0; e < E; ++e) contact_env_backward(&P, e, guhat, grot, gtrans);
    return 0;
}

/* Whole adjoint of L = sum g . U: recomputes the contact pass, then the
 * propagation adjoint, then the contact adjoint. */
int oracle_backward(int K, int N, const int32_t *offset, const double *pos, const double *nrm,
                    const double *origin, int E, int O, const int32_t *n_obj, const int32_t *type,
                    const double *shape, const double *rot, const double *trans, int mode,
                    const double *alpha, const double *phi, const double *gu, double *grot,
                    double *gtrans, double *galpha, double *gphi, double *guhat_out) {
    size_t EN = (size_t)E * N;
    int8_t *cobj = malloc(EN);
    double *uhat = malloc(sizeof(double) * 3 * EN);
    int32_t *na = malloc(sizeof(int32_t) * (size_t)E * K);
    double *guhat = guhat_out ? guhat_out : malloc(sizeof(double) * 3 * EN);
    oracle_contact(K, N, offset, pos, nrm, E, O, n_obj, type, shape, rot, trans, cobj, uhat, na);
    oracle_propagate_backward(K, N, offset, pos, nrm, origin, E, mode, alpha, phi, cobj, uhat, gu,
                              guhat, galpha, gphi);
    oracle_contact_backward(K, N, offset, pos, nrm, E, O, n_obj, type, shape, rot, trans, guhat, grot,
                            gtrans);
    if (!guhat_out) free(guhat);
    free(cobj);
    free(uhat);
    free(na);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* triangle-mesh contact entry points                                       */
/* ------------------------------------------------------------------------ */

/* Closest point of triangle (a, b, c) to q: returns the squared distance,
 * writes cp[3] and the feature (0 face, 1 edge ab, 2 bc, 3 ca, 4 vertex a,
 * 5 b, 6 c). */
double oracle_closest_point(const double *q, const double *a, const double *b, const double *c, double *cp,
                            int32_t *feature) {
    int f;
    double s = closest_on_triangle(q, a, b, c, cp, &f);
    *feature = f;
    return s;
}

/* Pseudo-normals of the triangles t0 .. t1-1 of a mesh: pn [T][7][3]
 * (face, edges ab bc ca, vertices a b c).  Returns 0 or the trimesh_build
 * error. */
int oracle_mesh_pseudonormals(int V, const double *verts, const int32_t *tris, int t0, int t1, double *pn) {
    trimesh_t m;
    int rc = trimesh_build(&m, V, verts, tris, t0, t1);
    if (rc) return rc;
    memcpy(pn, m.pn, sizeof(double) * 21 * (size_t)m.T);
    trimesh_free(&m);
    return 0;
}

/* Contact with primitives and triangle meshes (type 3, shape[0] = mesh
 * index).  Mesh m owns triangles tri_offset[m] .. tri_offset[m+1]-1 of
 * tris [T][3] (indices into verts [V][3]).  Outputs as oracle_contact. */
int oracle_contact_mesh(int K, int N, const int32_t *offset, const double *pos, const double *nrm, int E,
                        int O, const int32_t *n_obj, const int32_t *type, const double *shape,
                        const double *rot, const double *trans, int n_meshes, const int32_t *tri_offset,
                        int V, const double *verts, const int32_t *tris, int8_t *cobj, double *uhat,
                        int32_t *n_active) {
    problem_t P = mkprob(K, N, offset, pos, nrm, NULL, E, O, n_obj, type, shape, rot, trans);
    trimesh_t *ms = (trimesh_t *)calloc((size_t)n_meshes + 1, sizeof(trimesh_t));
    if (!ms) return -3;
    int rc = 0;
    for (int m = 0; m < n_meshes && rc == 0; ++m) rc = trimesh_build(ms + m, V, verts, tris, tri_offset[m],
                                                                     tri_offset[m + 1]);
    if (rc == 0) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int e = 0; e < E; ++e) contact_mesh_env(&P, ms, n_meshes, e, cobj, uhat, n_active);
    }
    for (int m = 0; m < n_meshes; ++m) trimesh_free(ms + m);
    free(ms);
    return rc;
}

/* Pose gradients of L = sum g . u_hat over the active nodes of every env,
 * contact with primitives and meshes recomputed (winner, triangle, feature
 * held fixed).  grad_uhat [3][E][N]; grad_rot [E][O][9], grad_trans
 * [E][O][3] (zero for objects that win no node). */
int oracle_contact_mesh_backward(int K, int N, const int32_t *offset, const double *pos, const double *nrm,
                                 int E, int O, const int32_t *n_obj, const int32_t *type, const double *shape,
                                 const double *rot, const double *trans, int n_meshes, const int32_t *tri_offset,
                                 int V, const double *verts, const int32_t *tris, const double *guhat,
                                 double *grot, double *gtrans) {
    (void)K;
    (void)offset;
    trimesh_t *ms = (trimesh_t *)calloc((size_t)n_meshes + 1, sizeof(trimesh_t));
    if (!ms) return -3;
    int rc = 0;
    for (int m = 0; m < n_meshes && rc == 0; ++m) rc = trimesh_build(ms + m, V, verts, tris, tri_offset[m],
                                                                     tri_offset[m + 1]);
    if (rc == 0) {
        const size_t EN = (size_t)E * N;
#pragma omp parallel for schedule(dynamic, 1)
        for (int e = 0; e < E; ++e) {
            for (int o = 0; o < O; ++o) {
                for (int c = 0; c < 9; ++c) grot[((size_t)e * O + o) * 9 + c] = 0.0;
                for (int c = 0; c < 3; ++c) gtrans[((size_t)e * O + o) * 3 + c] = 0.0;
            }
            for (int i = 0; i < N; ++i) {
                double p[3] = {pos[i], pos[N + i], pos[2 * N + i]};
                double n[3] = {nrm[i], nrm[N + i], nrm[2 * N + i]};
                int best = -1;
                hit_t bh;
                memset(&bh, 0, sizeof bh);
                for (int o = 0; o < n_obj[e]; ++o) {
                    size_t eo = (size_t)e * O + o;
                    hit_t h;
                    int ty = type[eo];
                    if (ty >= O_SPHERE && ty <= O_CAPSULE) {
                        h = penetrate(ty, shape + 4 * eo, rot + 9 * eo, trans + 3 * eo, p, n);
                    } else if (ty == O_MESH) {
                        int mi = mesh_index(shape + 4 * eo, n_meshes);
                        if (mi < 0) continue;
                        h = mesh_penetrate(ms + mi, rot + 9 * eo, trans + 3 * eo, p);
                    } else {
                        continue;
                    }
                    if (h.inside && (best < 0 || h.depth > bh.depth)) { best = o; bh = h; }
                }
                if (best < 0) continue;
                size_t ei = (size_t)e * N + i, eo = (size_t)e * O + best;
                double g[3] = {guhat[ei], guhat[EN + ei], guhat[2 * EN + ei]};
                if (type[eo] == O_MESH)
                    mesh_node_backward(ms + mesh_index(shape + 4 * eo, n_meshes), rot + 9 * eo, trans + 3 * eo, p,
                                       g, grot + 9 * eo, gtrans + 3 * eo);
                else if (!bh.degenerate)
                    contact_node_backward(type[eo], shape + 4 * eo, rot + 9 * eo, trans + 3 * eo, p, g,
                                          grot + 9 * eo, gtrans + 3 * eo);
            }
        }
    }
    for (int m = 0; m < n_meshes; ++m) trimesh_free(ms + m);
    free(ms);
    return rc;
}

/* Feature of the winning triangle per node (0 face, 1-3 edges, 4-6
 * vertices) where a mesh object wins, else -1: a test hook that shows which
 * closest-point cases an input exercises. */
int oracle_contact_mesh_features(int K, int N, const int32_t *offset, const double *pos, const double *nrm, int E,
                                 int O, const int32_t *n_obj, const int32_t *type, const double *shape,
                                 const double *rot, const double *trans, int n_meshes, const int32_t *tri_offset,
                                 int V, const double *verts, const int32_t *tris, int32_t *feature) {
    (void)K;
    (void)offset;
    trimesh_t *ms = (trimesh_t *)calloc((size_t)n_meshes + 1, sizeof(trimesh_t));
    if (!ms) return -3;
    int rc = 0;
    for (int m = 0; m < n_meshes && rc == 0; ++m) rc = trimesh_build(ms + m, V, verts, tris, tri_offset[m],
                                                                     tri_offset[m + 1]);
    for (int e = 0; e < E && rc == 0; ++e)
        for (int i = 0; i < N; ++i) {
            double p[3] = {pos[i], pos[N + i], pos[2 * N + i]};
            double n[3] = {nrm[i], nrm[N + i], nrm[2 * N + i]};
            int best = -1, bmesh = 0;
            hit_t bh;
            memset(&bh, 0, sizeof bh);
            for (int o = 0; o < n_obj[e]; ++o) {
                size_t eo = (size_t)e * O + o;
                hit_t h;
                int ty = type[eo], is_mesh = 0;
                if (ty >= O_SPHERE && ty <= O_CAPSULE) {
                    h = penetrate(ty, shape + 4 * eo, rot + 9 * eo, trans + 3 * eo, p, n);
                } else if (ty == O_MESH) {
                    int mi = mesh_index(shape + 4 * eo, n_meshes);
                    if (mi < 0) continue;
                    h = mesh_penetrate(ms + mi, rot + 9 * eo, trans + 3 * eo, p);
                    is_mesh = 1;
                } else {
                    continue;
                }
                if (h.inside && (best < 0 || h.depth > bh.depth)) { best = o; bh = h; bmesh = is_mesh; }
            }
            feature[(size_t)e * N + i] = (best >= 0 && bmesh) ? bh.sign : -1;
        }
    for (int m = 0; m < n_meshes; ++m) trimesh_free(ms + m);
    free(ms);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* 1c. articulated hand: link frames and self-contact                       */
/* ------------------------------------------------------------------------ */
/*
 * The paper's contact detection covers the hand's own links as well as the
 * external objects (Sec. III-A, contact detection), and its contact reward
 * counts active nodes and touched links (Sec. IV-B, contact reward).
 * Readings (listed in the design notes):
 *   - every patch is rigidly attached to one link; its node positions,
 *     normals and origin are given in that link's frame, and its outputs
 *     u_hat and U are expressed in that frame;
 *   - contact of patch k on link l is evaluated in link l's frame against
 *     the env's objects (ids 0 .. O-1) and against the collision primitive
 *     of every link j whose bit is set in collide[l] (j != l; id O + j);
 *     candidates are ordered objects first, then links by index; the
 *     deepest penetration wins, the first candidate on ties;
 *   - an object of world pose (R_w, t_w) appears in link l's frame (pose
 *     R_l, t_l) as R' = R_l^T R_w, t' = R_l^T (t_w - t_l); link j's primitive,
 *     of pose (C_R, C_t) in its link frame, has world pose R_w = R_j C_R,
 *     t_w = R_j C_t + t_j.  Evaluated in FP64 in this order (each sum of three
 *     products as (x0 y0 + x1 y1) + x2 y2, then the translation added or
 *     subtracted), no FMA; with `rel32` the relative pose is rounded to FP32
 *     before the contact test (the GPU library stores it so), else it stays
 *     in FP64 (for finite differences);
 *   - reward: n_touch[e][k] counts the nodes of patch k whose winner is an
 *     object; n_a = sum over k; bit l of S_cr is set when some patch on link
 *     l has n_touch > 0; r_contact = popcount(S_cr) / L + omega_a (n_a / N
 *     if n_a > 0, else -0.1), N the hand's node count.
 * The adjoint holds every discrete choice fixed and chains dL/d(R', t') to
 * the world poses: dL/dR_w = R_l G', dL/dt_w = R_l g'; for the frame link
 * dL/dR_l += R_w G'^T + (t_w - t_l) g'^T, dL/dt_l -= R_l g'; for a link
 * primitive dL/dR_j += (dL/dR_w) C_R^T + (dL/dt_w) C_t^T, dL/dt_j += dL/dt_w.
 */
typedef struct {
    int L;
    const int32_t *patch_link;   /* [K] */
    const uint32_t *collide;     /* [L] */
    const int32_t *ptype;        /* [L] primitive type or -1 */
    const double *pshape;        /* [L][4] */
    const double *prot;          /* [L][9] primitive pose in its link frame */
    const double *ptrans;        /* [L][3] */
    const double *lrot;          /* [E][L][9] link poses */
    const double *ltrans;        /* [E][L][3] */
    int rel32;
} hand_t;

#define HAND_MAX_CAND 64

typedef struct {
    int n;
    int id[HAND_MAX_CAND];          /* object o, or O + j for link j */
    int type[HAND_MAX_CAND];
    double shape[HAND_MAX_CAND][4];
    double R[HAND_MAX_CAND][9];     /* relative pose (link frame) */
    double t[HAND_MAX_CAND][3];
    double Rw[HAND_MAX_CAND][9];    /* world pose (FP64, unrounded) */
    double tw[HAND_MAX_CAND][3];
} hand_cand_t;

static inline double sum3(double a, double b, double c) { return (a + b) + c; }

static void rel_pose(const double *Rl, const double *tl, const double *Rw, const double *tw, int rel32,
                     double *Rr, double *tr) {
    double d[3] = {tw[0] - tl[0], tw[1] - tl[1], tw[2] - tl[2]};
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c)
            Rr[a * 3 + c] = sum3(Rl[0 * 3 + a] * Rw[0 * 3 + c], Rl[1 * 3 + a] * Rw[1 * 3 + c],
                                 Rl[2 * 3 + a] * Rw[2 * 3 + c]);
    for (int c = 0; c < 3; ++c) tr[c] = sum3(Rl[0 * 3 + c] * d[0], Rl[1 * 3 + c] * d[1], Rl[2 * 3 + c] * d[2]);
    if (rel32) {
        for (int i = 0; i < 9; ++i) Rr[i] = (double)(float)Rr[i];
        for (int i = 0; i < 3; ++i) tr[i] = (double)(float)tr[i];
    }
}

/* candidates of item (e, k) in contact order */
static void hand_candidates(const problem_t *P, const hand_t *H, int e, int k, hand_cand_t *C) {
    const int L = H->L, O = P->O, l = H->patch_link[k];
    const double *Rl = H->lrot + ((size_t)e * L + l) * 9, *tl = H->ltrans + ((size_t)e * L + l) * 3;
    C->n = 0;
    for (int o = 0; o < P->n_obj[e] && C->n < HAND_MAX_CAND; ++o) {
        size_t eo = (size_t)e * O + o;
        if (P->type[eo] < O_SPHERE || P->type[eo] > O_CAPSULE) continue;
        int s = C->n++;
        C->id[s] = o;
        C->type[s] = P->type[eo];
        for (int i = 0; i < 4; ++i) C->shape[s][i] = P->shape[4 * eo + i];
        for (int i = 0; i < 9; ++i) C->Rw[s][i] = P->rot[9 * eo + i];
        for (int i = 0; i < 3; ++i) C->tw[s][i] = P->trans[3 * eo + i];
        rel_pose(Rl, tl, C->Rw[s], C->tw[s], H->rel32, C->R[s], C->t[s]);
    }
    for (int j = 0; j < L && C->n < HAND_MAX_CAND; ++j) {
        if (j == l || !((H->collide[l] >> j) & 1u)) continue;
        if (H->ptype[j] < O_SPHERE || H->ptype[j] > O_CAPSULE) continue;
        const double *Rj = H->lrot + ((size_t)e * L + j) * 9, *tj = H->ltrans + ((size_t)e * L + j) * 3;
        const double *CR = H->prot + 9 * j, *Ct = H->ptrans + 3 * j;
        int s = C->n++;
        C->id[s] = O + j;
        C->type[s] = H->ptype[j];
        for (int i = 0; i < 4; ++i) C->shape[s][i] = H->pshape[4 * j + i];
        for (int a = 0; a < 3; ++a) {
            for (int c = 0; c < 3; ++c)
                C->Rw[s][a * 3 + c] = sum3(Rj[a * 3 + 0] * CR[0 * 3 + c], Rj[a * 3 + 1] * CR[1 * 3 + c],
                                           Rj[a * 3 + 2] * CR[2 * 3 + c]);
            C->tw[s][a] = sum3(Rj[a * 3 + 0] * Ct[0], Rj[a * 3 + 1] * Ct[1], Rj[a * 3 + 2] * Ct[2]) + tj[a];
        }
        rel_pose(Rl, tl, C->Rw[s], C->tw[s], H->rel32, C->R[s], C->t[s]);
    }
}

/* winner slot of one node among the item's candidates (-1: passive) */
static int hand_winner(const hand_cand_t *C, const double p[3], const double n[3], hit_t *bh) {
    int best = -1;
    memset(bh, 0, sizeof *bh);
    for (int s = 0; s < C->n; ++s) {
        hit_t h = penetrate(C->type[s], C->shape[s], C->R[s], C->t[s], p, n);
        if (h.inside && (best < 0 || h.depth > bh->depth)) { best = s; *bh = h; }
    }
    return best;
}

static void hand_contact_env(const problem_t *P, const hand_t *H, int e, int8_t *cobj, double *uhat,
                             int32_t *n_active, int32_t *n_touch, uint64_t *sig) {
    const int N = P->N, E = P->E, O = P->O;
    hand_cand_t *C = malloc(sizeof *C);
    for (int k = 0; k < P->K; ++k) {
        hand_candidates(P, H, e, k, C);
        int na = 0, nt = 0;
        for (int i = P->offset[k]; i < P->offset[k + 1]; ++i) {
            double p[3] = {P->pos[i], P->pos[N + i], P->pos[2 * N + i]};
            double n[3] = {P->nrm[i], P->nrm[N + i], P->nrm[2 * N + i]};
            hit_t bh;
            int s = hand_winner(C, p, n, &bh);
            size_t en = (size_t)e * N + i;
            cobj[en] = (int8_t)(s >= 0 ? C->id[s] : -1);
            for (int a = 0; a < 3; ++a) uhat[(size_t)a * E * N + en] = s >= 0 ? bh.u[a] : 0.0;
            if (s >= 0) {
                ++na;
                if (C->id[s] < O) ++nt;
            }
            if (sig) {
                *sig = fnv(*sig, s >= 0 ? C->id[s] : -1);
                if (s >= 0) *sig = fnv(fnv(fnv(*sig, bh.face), bh.sign), bh.degenerate);
            }
        }
        n_active[(size_t)e * P->K + k] = na;
        n_touch[(size_t)e * P->K + k] = nt;
    }
    free(C);
}

static void hand_reward(const problem_t *P, const hand_t *H, int e, const int32_t *n_touch, double omega_a,
                        int32_t *n_a, uint32_t *link_mask, double *r_contact) {
    int64_t s = 0;
    uint32_t mask = 0;
    for (int k = 0; k < P->K; ++k) {
        int32_t t = n_touch[(size_t)e * P->K + k];
        s += t;
        if (t > 0) mask |= 1u << H->patch_link[k];
    }
    int links = 0;
    for (int l = 0; l < H->L; ++l) links += (mask >> l) & 1u;
    n_a[e] = (int32_t)s;
    link_mask[e] = mask;
    double ra = s > 0 ? (double)s / (double)P->N : -0.1;
    r_contact[e] = (double)links / (double)H->L + omega_a * ra;
}

static hand_t mkhand(int L, const int32_t *patch_link, const uint32_t *collide, const int32_t *ptype,
                     const double *pshape, const double *prot, const double *ptrans, const double *lrot,
                     const double *ltrans, int rel32) {
    hand_t H = {L, patch_link, collide, ptype, pshape, prot, ptrans, lrot, ltrans, rel32};
    return H;
}

/* Articulated-hand forward step.  Outputs: U [3][E][N] and uhat [3][E][N]
 * in each patch's link frame, contact_obj [E][N] (object o, O + j for link
 * j, -1 passive), n_active and n_touch [E][K], n_a [E], link_mask [E],
 * r_contact [E]; sig [E] (may be NULL) fingerprints every discrete choice;
 * margin [E][K] (may be NULL) is each item's decision margin as in
 * oracle_item_margins. */
int oracle_hand_forward(int K, int N, const int32_t *offset, const double *pos, const double *nrm,
                        const double *origin, int E, int O, const int32_t *n_obj, const int32_t *type,
                        const double *shape, const double *rot, const double *trans, int L,
                        const int32_t *patch_link, const uint32_t *collide, const int32_t *ptype,
                        const double *pshape, const double *prot, const double *ptrans, const double *lrot,
                        const double *ltrans, int rel32, int mode, const double *alpha, const double *phi,
                        double omega_a, double *U, int8_t *cobj, double *uhat, int32_t *n_active,
                        int32_t *n_touch, int32_t *n_a, uint32_t *link_mask, double *r_contact, uint64_t *sig,
                        double *margin) {
    if (L < 1 || L > 32) return 1;
    for (int k = 0; k < K; ++k)
        if (patch_link[k] < 0 || patch_link[k] >= L) return 2;
    problem_t P = mkprob(K, N, offset, pos, nrm, origin, E, O, n_obj, type, shape, rot, trans);
    hand_t H = mkhand(L, patch_link, collide, ptype, pshape, prot, ptrans, lrot, ltrans, rel32);
    net_t W = net_view(phi);
    int nmax = max_patch(&P);
#pragma omp parallel
    {
        scratch_t S = scratch_new(nmax);
#pragma omp for schedule(static)
        for (int e = 0; e < E; ++e) {
            uint64_t h = 1469598103934665603ULL;
            hand_contact_env(&P, &H, e, cobj, uhat, n_active, n_touch, sig ? &h : NULL);
            hand_reward(&P, &H, e, n_touch, omega_a, n_a, link_mask, r_contact);
            for (int k = 0; k < K; ++k) {
                double mg = INFINITY;
                propagate_patch(&P, &W, mode, alpha, e, k, cobj, uhat, U, &S, margin ? &mg : NULL, sig ? &h : NULL);
                if (margin) margin[(size_t)e * K + k] = mg;
            }
            if (sig) sig[e] = h;
        }
        scratch_free(&S);
    }
    return 0;
}

/* pose gradients of env e from dL/du_hat of its active nodes (hand) */
static void hand_contact_env_backward(const problem_t *P, const hand_t *H, int e, const double *guhat,
                                      double *grot, double *gtrans, double *glrot, double *gltrans) {
    const int N = P->N, E = P->E, O = P->O, L = H->L;
    const size_t EN = (size_t)E * N;
    for (int i = 0; i < O * 9; ++i) grot[(size_t)e * O * 9 + i] = 0.0;
    for (int i = 0; i < O * 3; ++i) gtrans[(size_t)e * O * 3 + i] = 0.0;
    for (int i = 0; i < L * 9; ++i) glrot[(size_t)e * L * 9 + i] = 0.0;
    for (int i = 0; i < L * 3; ++i) gltrans[(size_t)e * L * 3 + i] = 0.0;
    hand_cand_t *C = malloc(sizeof *C);
    double (*gR)[9] = malloc(sizeof(double) * 9 * HAND_MAX_CAND);
    double (*gt)[3] = malloc(sizeof(double) * 3 * HAND_MAX_CAND);
    for (int k = 0; k < P->K; ++k) {
        hand_candidates(P, H, e, k, C);
        for (int s = 0; s < C->n; ++s) {
            for (int i = 0; i < 9; ++i) gR[s][i] = 0.0;
            for (int i = 0; i < 3; ++i) gt[s][i] = 0.0;
        }
        for (int i = P->offset[k]; i < P->offset[k + 1]; ++i) {
            double p[3] = {P->pos[i], P->pos[N + i], P->pos[2 * N + i]};
            double n[3] = {P->nrm[i], P->nrm[N + i], P->nrm[2 * N + i]};
            hit_t bh;
            int s = hand_winner(C, p, n, &bh);
            if (s < 0 || bh.degenerate) continue;
            size_t ei = (size_t)e * N + i;
            double g[3] = {guhat[ei], guhat[EN + ei], guhat[2 * EN + ei]};
            contact_node_backward(C->type[s], C->shape[s], C->R[s], C->t[s], p, g, gR[s], gt[s]);
        }
        /* chain rule from the relative poses to the world poses */
        const int l = H->patch_link[k];
        const double *Rl = H->lrot + ((size_t)e * L + l) * 9, *tl = H->ltrans + ((size_t)e * L + l) * 3;
        double *gRl = glrot + ((size_t)e * L + l) * 9, *gtl = gltrans + ((size_t)e * L + l) * 3;
        for (int s = 0; s < C->n; ++s) {
            double GRw[9], gtw[3], d[3];
            for (int a = 0; a < 3; ++a) {
                for (int c = 0; c < 3; ++c)
                    GRw[a * 3 + c] = Rl[a * 3 + 0] * gR[s][0 * 3 + c] + Rl[a * 3 + 1] * gR[s][1 * 3 + c] +
                                     Rl[a * 3 + 2] * gR[s][2 * 3 + c];
                gtw[a] = Rl[a * 3 + 0] * gt[s][0] + Rl[a * 3 + 1] * gt[s][1] + Rl[a * 3 + 2] * gt[s][2];
                d[a] = C->tw[s][a] - tl[a];
            }
            /* frame link: R_w G'^T + d g'^T, and -R_l g' */
            for (int a = 0; a < 3; ++a) {
                for (int b = 0; b < 3; ++b) {
                    double v = C->Rw[s][a * 3 + 0] * gR[s][b * 3 + 0] + C->Rw[s][a * 3 + 1] * gR[s][b * 3 + 1] +
                               C->Rw[s][a * 3 + 2] * gR[s][b * 3 + 2];
                    gRl[a * 3 + b] += v + d[a] * gt[s][b];
                }
                gtl[a] -= gtw[a];
            }
            const int id = C->id[s];
            if (id < O) {
                double *go = grot + ((size_t)e * O + id) * 9, *gto = gtrans + ((size_t)e * O + id) * 3;
                for (int i = 0; i < 9; ++i) go[i] += GRw[i];
                for (int i = 0; i < 3; ++i) gto[i] += gtw[i];
            } else {
                const int j = id - O;
                const double *CR = H->prot + 9 * j, *Ct = H->ptrans + 3 * j;
                double *gRj = glrot + ((size_t)e * L + j) * 9, *gtj = gltrans + ((size_t)e * L + j) * 3;
                for (int a = 0; a < 3; ++a) {
                    for (int b = 0; b < 3; ++b)
                        gRj[a * 3 + b] += GRw[a * 3 + 0] * CR[b * 3 + 0] + GRw[a * 3 + 1] * CR[b * 3 + 1] +
                                          GRw[a * 3 + 2] * CR[b * 3 + 2] + gtw[a] * Ct[b];
                    gtj[a] += gtw[a];
                }
            }
        }
    }
    free(C);
    free(gR);
    free(gt);
}

/* Adjoint of L = sum g . U for the articulated hand: recomputes contact,
 * then the propagation adjoint (link frames), then the contact adjoint with
 * the chain rule to object poses grot [E][O][9], gtrans [E][O][3] and link
 * poses glrot [E][L][9], gltrans [E][L][3]; galpha [K], gphi [PHI_N]. */
int oracle_hand_backward(int K, int N, const int32_t *offset, const double *pos, const double *nrm,
                         const double *origin, int E, int O, const int32_t *n_obj, const int32_t *type,
                         const double *shape, const double *rot, const double *trans, int L,
                         const int32_t *patch_link, const uint32_t *collide, const int32_t *ptype,
                         const double *pshape, const double *prot, const double *ptrans, const double *lrot,
                         const double *ltrans, int rel32, int mode, const double *alpha, const double *phi,
                         const double *gu, double *grot, double *gtrans, double *glrot, double *gltrans,
                         double *galpha, double *gphi, double *guhat_out) {
    if (L < 1 || L > 32) return 1;
    for (int k = 0; k < K; ++k)
        if (patch_link[k] < 0 || patch_link[k] >= L) return 2;
    size_t EN = (size_t)E * N;
    problem_t P = mkprob(K, N, offset, pos, nrm, origin, E, O, n_obj, type, shape, rot, trans);
    hand_t H = mkhand(L, patch_link, collide, ptype, pshape, prot, ptrans, lrot, ltrans, rel32);
    int8_t *cobj = malloc(EN);
    double *uhat = malloc(sizeof(double) * 3 * EN);
    int32_t *na = malloc(sizeof(int32_t) * (size_t)E * K), *nt = malloc(sizeof(int32_t) * (size_t)E * K);
    double *guhat = guhat_out ? guhat_out : malloc(sizeof(double) * 3 * EN);
#pragma omp parallel for schedule(static)
    for (int e = 0; e < E; ++e) hand_contact_env(&P, &H, e, cobj, uhat, na, nt, NULL);
    oracle_propagate_backward(K, N, offset, pos, nrm, origin, E, mode, alpha, phi, cobj, uhat, gu, guhat, galpha,
                              gphi);
#pragma omp parallel for schedule(static)
    for (int e = 0; e < E; ++e) hand_contact_env_backward(&P, &H, e, guhat, grot, gtrans, glrot, gltrans);
    if (!guhat_out) free(guhat);
    free(cobj);
    free(uhat);
    free(na);
    free(nt);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 4. real-sensor regressor (inference)                                     */
/* ------------------------------------------------------------------------ */
/*
 * The paper maps simulated surface displacements to the outputs of a real
 * sensor's eight pressure taxels with a PointNet-based regressor that has
 * residual connections and pools its per-node features with attention
 * instead of a max (appendix, "Modeling Real Sensors"); the attention is an
 * MLP [256, 128, 1] with tanh whose scores are normalised by a softmax.  The
 * rest of the architecture is in a figure that is not available.  Reading
 * (listed in the design notes), per (env, patch) item:
 *   x_i  = [p_i - o_k, U_i]                      (6; U the step's output)
 *   h1_i = relu(E1 x_i + e1)                     (64)
 *   h2_i = relu(E2 h1_i + e2) + h1_i             (64, residual)
 *   f_i  = relu(E3 h2_i + e3)                    (256)
 *   s_i  = a2 . tanh(A1 f_i + a1) + a0           (128 -> 1)
 *   w    = softmax(s) over the item's nodes      (max subtracted first)
 *   g    = sum_i w_i f_i                         (256)
 *   y    = D2 relu(D1 g + d1) + d2               (128 -> 8 taxels)
 * Packed parameters (FP32): E1[64][6] e1[64] E2[64][64] e2[64] E3[256][64]
 * e3[256] A1[128][256] a1[128] a2[128] a0[4] (a0[0] used) D1[128][256] d1[128]
 * D2[8][128] d2[8]: REG_N = 88204 values.
 */
#define REG_N 88204
typedef struct {
    const double *E1, *e1, *E2, *e2, *E3, *e3, *A1, *a1, *a2, *a0, *D1, *d1, *D2, *d2;
} reg_t;

static reg_t reg_view(const double *r) {
    reg_t R;
    R.E1 = r; r += 64 * 6;
    R.e1 = r; r += 64;
    R.E2 = r; r += 64 * 64;
    R.e2 = r; r += 64;
    R.E3 = r; r += 256 * 64;
    R.e3 = r; r += 256;
    R.A1 = r; r += 128 * 256;
    R.a1 = r; r += 128;
    R.a2 = r; r += 128;
    R.a0 = r; r += 4;
    R.D1 = r; r += 128 * 256;
    R.d1 = r; r += 128;
    R.D2 = r; r += 8 * 128;
    R.d2 = r;
    return R;
}

/* per-node feature f (256) and attention score of node input x (6) */
static double reg_node(const reg_t *R, const double x[6], double f[256]) {
    double h1[64], h2[64], t[128];
    for (int o = 0; o < 64; ++o) {
        double a = R->e1[o];
        for (int c = 0; c < 6; ++c) a += R->E1[o * 6 + c] * x[c];
        h1[o] = relu(a);
    }
    for (int o = 0; o < 64; ++o) {
        double a = R->e2[o];
        for (int c = 0; c < 64; ++c) a += R->E2[o * 64 + c] * h1[c];
        h2[o] = relu(a) + h1[o];
    }
    for (int o = 0; o < 256; ++o) {
        double a = R->e3[o];
        for (int c = 0; c < 64; ++c) a += R->E3[o * 64 + c] * h2[c];
        f[o] = relu(a);
    }
    double s = R->a0[0];
    for (int o = 0; o < 128; ++o) {
        double a = R->a1[o];
        for (int c = 0; c < 256; ++c) a += R->A1[o * 256 + c] * f[c];
        t[o] = tanh(a);
        s += R->a2[o] * t[o];
    }
    return s;
}

/* Taxel outputs of every (env, patch) item: y [E][K][8]; u [3][E][N] the
 * displacements (link frames for the articulated hand). */
int oracle_regress(int K, int N, const int32_t *offset, const double *pos, const double *origin, int E,
                   const double *reg, const double *u, double *y) {
    reg_t R = reg_view(reg);
    int nmax = 0;
    for (int k = 0; k < K; ++k)
        if (offset[k + 1] - offset[k] > nmax) nmax = offset[k + 1] - offset[k];
#pragma omp parallel
    {
        double *F = malloc(sizeof(double) * (size_t)nmax * 256);
        double *S = malloc(sizeof(double) * (size_t)nmax);
#pragma omp for schedule(static)
        for (int e = 0; e < E; ++e)
            for (int k = 0; k < K; ++k) {
                const int n = offset[k + 1] - offset[k];
                double smax = -INFINITY;
                for (int j = 0; j < n; ++j) {
                    const int i = offset[k] + j;
                    const size_t ei = (size_t)e * N + i;
                    double x[6];
                    for (int a = 0; a < 3; ++a) {
                        x[a] = pos[(size_t)a * N + i] - origin[3 * k + a];
                        x[3 + a] = u[(size_t)a * E * N + ei];
                    }
                    S[j] = reg_node(&R, x, F + (size_t)j * 256);
                    if (S[j] > smax) smax = S[j];
                }
                double z = 0.0;
                for (int j = 0; j < n; ++j) {
                    S[j] = exp(S[j] - smax);
                    z += S[j];
                }
                double g[256], h[128];
                for (int c = 0; c < 256; ++c) {
                    double a = 0.0;
                    for (int j = 0; j < n; ++j) a += S[j] * F[(size_t)j * 256 + c];
                    g[c] = a / z;
                }
                for (int o = 0; o < 128; ++o) {
                    double a = R.d1[o];
                    for (int c = 0; c < 256; ++c) a += R.D1[o * 256 + c] * g[c];
                    h[o] = relu(a);
                }
                double *yo = y + ((size_t)e * K + k) * 8;
                for (int o = 0; o < 8; ++o) {
                    double a = R.d2[o];
                    for (int c = 0; c < 128; ++c) a += R.D2[o * 128 + c] * h[c];
                    yo[o] = a;
                }
            }
        free(F);
        free(S);
    }
    return 0;
}

/*
 * Inverse Path Tracing -- FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU path is checked against.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no source with the HIP library (no headers, no helpers, no tables)
 * and the library never calls it.
 *
 * What it computes (paper: "Inverse Path Tracing for Joint Material and
 * Lighting Estimation", Azinovic, Li, Kaplanyan, Niessner, CVPR 2019):
 *   - the Monte Carlo estimate of the pixel integral (Sec. 3.1, Eq. 1) of the
 *     measurement contribution (Sec. 3.1, Eq. 2) by unidirectional path
 *     tracing with BRDF sampling and explicit light sampling combined by
 *     multiple importance sampling (Appendix A.2 "Variance Reduction";
 *     Appendix E "Implementation Details"),
 *   - the derivative of every sampled path contribution with respect to the
 *     emission (Sec. 3.3, Eq. 5) and material (Sec. 3.3, Eq. 6) unknowns by
 *     the product rule, written out factor by factor with no division, so it
 *     stays exact when an albedo or an emission is zero (the paper starts
 *     from zero, Appendix E),
 *   - the loss and its adjoint image (Sec. 3.2, Eq. 3; Sec. 3.3, Eq. 4) and
 *     the Adam update (Sec. 4.5).
 * Everything is double precision.  Uniform random numbers come from
 * Philox4x32-10 (Salmon et al., SC'11) mapped to 24-bit uniforms, so that a
 * float implementation can consume bit-identical uniforms.
 *
 * Readings of points the paper leaves open (they are listed with reasons in
 * the design notes of the repository):
 *   - Eq. 2 is printed without geometry terms; the standard path-space form
 *     (Veach 1997) is used.  Geometry terms and pdfs do not depend on the
 *     unknowns, so the structure of Eqs. 5-6 is unchanged.
 *   - BRDF: Lambert plus a GGX microfacet lobe with separable Smith shadowing
 *     and no Fresnel; alpha = roughness clamped to [1e-3, 1].  The paper uses
 *     the Disney model (Sec. 4.1); the parameter set here is diffuse RGB,
 *     specular RGB and roughness.
 *   - Emission: constant radiance by default; the paper's cosine profile
 *     e (w.n)_+ (Sec. 4.3) is an option.  Emitters are one-sided.
 *   - Depth D counts scattering vertices; the ray leaving vertex D is still
 *     traced, for its emitter hit only.
 *   - Every pdf, MIS weight, lobe probability, Russian-roulette probability
 *     and the light-selection distribution is evaluated at "sampling
 *     parameters" and treated as a constant: Eqs. 5-6 differentiate only the
 *     measurement contribution.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as    */
/* easy as 1, 2, 3", SC 2011).                                                */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 24-bit uniform in [0,1): exactly representable in float and double. */
static double u24(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

/* The eight uniforms of vertex k of a path.  key = (seed_lo ^ tag*golden,
 * seed_hi); counter = (path_lo, path_hi, 2k + half, iteration).  Slot use:
 *   k = 0 : [0],[1] pixel jitter
 *   k >= 1: [0] light triangle, [1],[2] point on it, [3] lobe / guide lobe,
 *           [4],[5] direction, [6] Russian roulette, [7] guide-vs-BRDF. */
static void vertex_uniforms(uint64_t seed, uint32_t tag, uint32_t iteration,
                            uint64_t path_id, int k, double u[8])
{
    uint32_t key[2] = { (uint32_t)seed ^ (tag * 0x9E3779B9u), (uint32_t)(seed >> 32) };
    for (int half = 0; half < 2; ++half) {
        uint32_t ctr[4] = { (uint32_t)path_id, (uint32_t)(path_id >> 32),
                            (uint32_t)(2 * k + half), iteration };
        uint32_t o[4];
        orc_philox4x32_10(ctr, key, o);
        for (int i = 0; i < 4; ++i) u[4 * half + i] = u24(o[i]);
    }
}

/* ------------------------------------------------------------------------- */
/* Small vector helpers.                                                      */
/* ------------------------------------------------------------------------- */
typedef struct { double x, y, z; } v3;
static v3 mk(double x, double y, double z) { v3 r = { x, y, z }; return r; }
static v3 add(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 sub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 scl(v3 a, double s) { return mk(a.x * s, a.y * s, a.z * s); }
static double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 cross(v3 a, v3 b)
{
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static v3 nrm(v3 a) { double l = sqrt(dot(a, a)); return scl(a, 1.0 / l); }
static double comp(v3 a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }

/* ------------------------------------------------------------------------- */
/* Scene.                                                                     */
/* ------------------------------------------------------------------------- */
typedef struct { double lo[3], hi[3]; int left, right, first, count; } onode;

typedef struct orc_scene {
    int64_t nv, nt;
    int32_t ns, ne;
    double *P;          /* nv*3 positions */
    double *N;          /* nv*3 normals or NULL */
    int32_t *F;         /* nt*3 */
    int32_t *seg;       /* nt */
    int32_t *emitter_seg; /* ne */
    int32_t *seg_emitter; /* ns: emitter index or -1 */
    int64_t nlt;        /* number of emitter triangles */
    int32_t *light_tri; /* emitter triangles in ascending id order */
    double *light_area;
    double diag;        /* scene bounding-box diagonal */
    int32_t material;   /* 0: Lambert + GGX (7 parameters per segment), 1: Disney (13) */
    int32_t nm;         /* parameters per segment */
    /* median-split BVH over triangles */
    onode *nodes; int64_t nnodes; int32_t *order;
} orc_scene;

static v3 vtx(const orc_scene *s, int64_t i)
{
    return mk(s->P[3 * i], s->P[3 * i + 1], s->P[3 * i + 2]);
}

static double cent(const orc_scene *s, int32_t t, int ax)
{
    double c = 0;
    for (int j = 0; j < 3; ++j) c += s->P[3 * (int64_t)s->F[3 * (int64_t)t + j] + ax];
    return c / 3.0;
}

static int g_sort_axis;
static const orc_scene *g_sort_scene;
static int cmp_cent(const void *a, const void *b)
{
    double ca = cent(g_sort_scene, *(const int32_t *)a, g_sort_axis);
    double cb = cent(g_sort_scene, *(const int32_t *)b, g_sort_axis);
    if (ca < cb) return -1;
    if (ca > cb) return 1;
    return (*(const int32_t *)a) - (*(const int32_t *)b);
}

/* Median split on the widest centroid axis, leaves of at most 4 triangles. */
static int build_node(orc_scene *s, int first, int count)
{
    int id = (int)s->nnodes++;
    onode *nd = &s->nodes[id];
    for (int a = 0; a < 3; ++a) { nd->lo[a] = INFINITY; nd->hi[a] = -INFINITY; }
    double clo[3] = { INFINITY, INFINITY, INFINITY }, chi[3] = { -INFINITY, -INFINITY, -INFINITY };
    for (int i = first; i < first + count; ++i) {
        int32_t t = s->order[i];
        for (int j = 0; j < 3; ++j) {
            int64_t vi = s->F[3 * (int64_t)t + j];
            for (int a = 0; a < 3; ++a) {
                double p = s->P[3 * vi + a];
                if (p < nd->lo[a]) nd->lo[a] = p;
                if (p > nd->hi[a]) nd->hi[a] = p;
            }
        }
        for (int a = 0; a < 3; ++a) {
            double c = cent(s, t, a);
            if (c < clo[a]) clo[a] = c;
            if (c > chi[a]) chi[a] = c;
        }
    }
    /* pad the box so the slab test can never reject a triangle that lies on it */
    for (int a = 0; a < 3; ++a) {
        double pad = 1e-9 * (fabs(nd->lo[a]) + fabs(nd->hi[a]) + 1.0);
        nd->lo[a] -= pad; nd->hi[a] += pad;
    }
    if (count <= 4) {
        nd->left = nd->right = -1; nd->first = first; nd->count = count;
        return id;
    }
    int ax = 0;
    for (int a = 1; a < 3; ++a) if (chi[a] - clo[a] > chi[ax] - clo[ax]) ax = a;
    g_sort_axis = ax; g_sort_scene = s;
    qsort(s->order + first, (size_t)count, sizeof(int32_t), cmp_cent);
    int half = count / 2;
    int l = build_node(s, first, half);
    int r = build_node(s, first + half, count - half);
    nd = &s->nodes[id];
    nd->left = l; nd->right = r; nd->first = 0; nd->count = 0;
    return id;
}

orc_scene *orc_scene_create(const float *verts, int64_t nv, const float *normals,
                            const int32_t *tris, const int32_t *tri_seg, int64_t nt,
                            int32_t num_segments, const int32_t *emitter_seg, int32_t num_emitters)
{
    orc_scene *s = (orc_scene *)calloc(1, sizeof(orc_scene));
    s->nv = nv; s->nt = nt; s->ns = num_segments; s->ne = num_emitters;
    s->material = 0; s->nm = 7;
    s->P = (double *)malloc(sizeof(double) * 3 * (size_t)nv);
    for (int64_t i = 0; i < 3 * nv; ++i) s->P[i] = (double)verts[i];
    if (normals) {
        s->N = (double *)malloc(sizeof(double) * 3 * (size_t)nv);
        for (int64_t i = 0; i < 3 * nv; ++i) s->N[i] = (double)normals[i];
    }
    s->F = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)nt);
    memcpy(s->F, tris, sizeof(int32_t) * 3 * (size_t)nt);
    s->seg = (int32_t *)malloc(sizeof(int32_t) * (size_t)nt);
    memcpy(s->seg, tri_seg, sizeof(int32_t) * (size_t)nt);
    s->emitter_seg = (int32_t *)malloc(sizeof(int32_t) * (size_t)(num_emitters > 0 ? num_emitters : 1));
    for (int32_t k = 0; k < num_emitters; ++k) s->emitter_seg[k] = emitter_seg[k];
    s->seg_emitter = (int32_t *)malloc(sizeof(int32_t) * (size_t)num_segments);
    for (int i = 0; i < num_segments; ++i) s->seg_emitter[i] = -1;
    for (int k = 0; k < num_emitters; ++k) s->seg_emitter[emitter_seg[k]] = k;
    s->nlt = 0;
    for (int64_t t = 0; t < nt; ++t) if (s->seg_emitter[tri_seg[t]] >= 0) s->nlt++;
    s->light_tri = (int32_t *)malloc(sizeof(int32_t) * (size_t)(s->nlt + 1));
    s->light_area = (double *)malloc(sizeof(double) * (size_t)(s->nlt + 1));
    int64_t j = 0;
    for (int64_t t = 0; t < nt; ++t) {
        if (s->seg_emitter[tri_seg[t]] < 0) continue;
        v3 a = vtx(s, tris[3 * t]), b = vtx(s, tris[3 * t + 1]), c = vtx(s, tris[3 * t + 2]);
        v3 cr = cross(sub(b, a), sub(c, a));
        s->light_tri[j] = (int32_t)t;
        s->light_area[j] = 0.5 * sqrt(dot(cr, cr));
        ++j;
    }
    double lo[3] = { INFINITY, INFINITY, INFINITY }, hi[3] = { -INFINITY, -INFINITY, -INFINITY };
    for (int64_t i = 0; i < nv; ++i)
        for (int a = 0; a < 3; ++a) {
            if (s->P[3 * i + a] < lo[a]) lo[a] = s->P[3 * i + a];
            if (s->P[3 * i + a] > hi[a]) hi[a] = s->P[3 * i + a];
        }
    s->diag = sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                   (hi[2] - lo[2]) * (hi[2] - lo[2]));
    s->order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nt > 0 ? nt : 1));
    for (int64_t t = 0; t < nt; ++t) s->order[t] = (int32_t)t;
    s->nodes = (onode *)malloc(sizeof(onode) * (size_t)(2 * nt + 1));
    s->nnodes = 0;
    if (nt > 0) build_node(s, 0, (int)nt);
    return s;
}

/* Material model of the scene: 0 Lambert + GGX (7 parameters per segment),
 * 1 Disney (13). */
void orc_scene_set_material(orc_scene *s, int32_t material)
{
    s->material = material == 1 ? 1 : 0;
    s->nm = s->material == 1 ? 13 : 7;   /* Disney: DS_N */
}

void orc_scene_free(orc_scene *s)
{
    if (!s) return;
    free(s->P); free(s->N); free(s->F); free(s->seg); free(s->emitter_seg);
    free(s->seg_emitter); free(s->light_tri); free(s->light_area);
    free(s->nodes); free(s->order); free(s);
}

double orc_scene_diag(const orc_scene *s) { return s->diag; }
int64_t orc_scene_num_light_tris(const orc_scene *s) { return s->nlt; }

/* ------------------------------------------------------------------------- */
/* Watertight ray/triangle test (Woop, Benthin, Wald, JCGT 2013), in double.  */
/* Returns 1 on a hit with tmin < t < tmax; (u,v) weight vertices 1 and 2.    */
/* ------------------------------------------------------------------------- */
typedef struct { int kx, ky, kz; double Sx, Sy, Sz; v3 o, d; } wray;

static wray make_wray(v3 o, v3 d)
{
    wray r; r.o = o; r.d = d;
    double ad[3] = { fabs(d.x), fabs(d.y), fabs(d.z) };
    int kz = 0;
    if (ad[1] > ad[kz]) kz = 1;
    if (ad[2] > ad[kz]) kz = 2;
    int kx = (kz + 1) % 3, ky = (kx + 1) % 3;
    if (comp(d, kz) < 0) { int t = kx; kx = ky; ky = t; }
    r.kx = kx; r.ky = ky; r.kz = kz;
    r.Sx = comp(d, kx) / comp(d, kz);
    r.Sy = comp(d, ky) / comp(d, kz);
    r.Sz = 1.0 / comp(d, kz);
    return r;
}

static int tri_hit(const wray *r, v3 p0, v3 p1, v3 p2, double tmin, double tmax,
                   double *t_out, double *u_out, double *v_out)
{
    v3 A = sub(p0, r->o), B = sub(p1, r->o), C = sub(p2, r->o);
    double Ax = comp(A, r->kx) - r->Sx * comp(A, r->kz);
    double Ay = comp(A, r->ky) - r->Sy * comp(A, r->kz);
    double Bx = comp(B, r->kx) - r->Sx * comp(B, r->kz);
    double By = comp(B, r->ky) - r->Sy * comp(B, r->kz);
    double Cx = comp(C, r->kx) - r->Sx * comp(C, r->kz);
    double Cy = comp(C, r->ky) - r->Sy * comp(C, r->kz);
    double U = Cx * By - Cy * Bx;
    double V = Ax * Cy - Ay * Cx;
    double W = Bx * Ay - By * Ax;
    if ((U < 0 || V < 0 || W < 0) && (U > 0 || V > 0 || W > 0)) return 0;
    double det = U + V + W;
    if (det == 0) return 0;
    double Az = r->Sz * comp(A, r->kz), Bz = r->Sz * comp(B, r->kz), Cz = r->Sz * comp(C, r->kz);
    double T = U * Az + V * Bz + W * Cz;
    double t = T / det;
    if (!(t > tmin && t < tmax)) return 0;
    *t_out = t; *u_out = V / det; *v_out = W / det;
    return 1;
}

int orc_ray_triangle(const double o[3], const double d[3], const double p0[3], const double p1[3],
                     const double p2[3], double tmin, double tmax, double out[3])
{
    wray r = make_wray(mk(o[0], o[1], o[2]), mk(d[0], d[1], d[2]));
    double t, u, v;
    int h = tri_hit(&r, mk(p0[0], p0[1], p0[2]), mk(p1[0], p1[1], p1[2]), mk(p2[0], p2[1], p2[2]),
                    tmin, tmax, &t, &u, &v);
    if (h) { out[0] = t; out[1] = u; out[2] = v; }
    return h;
}

typedef struct { int32_t tri; double t, u, v; } ohit;

static int box_hit(const onode *n, v3 o, v3 d, double tmin, double tmax)
{
    double t0 = tmin, t1 = tmax;
    for (int a = 0; a < 3; ++a) {
        double oa = comp(o, a), da = comp(d, a);
        if (da == 0.0) {
            if (oa < n->lo[a] || oa > n->hi[a]) return 0;
            continue;
        }
        double ta = (n->lo[a] - oa) / da, tb = (n->hi[a] - oa) / da;
        if (ta > tb) { double x = ta; ta = tb; tb = x; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
        if (t0 > t1) return 0;
    }
    return 1;
}

/* Accept a candidate if nearer, or equally near with a smaller triangle id:
 * the answer then does not depend on the visiting order.
 *
 * Near-tie margin (parity bookkeeping only; it never changes the answer):
 * for every tested triangle whose plane is crossed inside the ray interval,
 * the distance of the crossing to the triangle's boundary (relative to the
 * coordinate magnitude), the distance of t to the interval ends, and the gap
 * between the two nearest hits.  A float32 implementation can only disagree
 * with this double-precision answer where such a margin is small. */
typedef struct { double m; double t1, t2; int32_t id1; } tiemargin;

static double rel_scale(v3 x) { return fmax(fmax(fabs(x.x), fabs(x.y)), fabs(x.z)) + 1.0; }

static void plane_margin(const orc_scene *s, const wray *r, int32_t t, double tmin, double tmax,
                         tiemargin *tm)
{
    const int32_t *f = &s->F[3 * (int64_t)t];
    v3 p0 = vtx(s, f[0]), p1 = vtx(s, f[1]), p2 = vtx(s, f[2]);
    v3 e1 = sub(p1, p0), e2 = sub(p2, p0);
    v3 n = cross(e1, e2);
    double dn = dot(n, r->d);
    if (dn == 0.0) return;
    double th = dot(n, sub(p0, r->o)) / dn;
    v3 x = add(r->o, scl(r->d, th));
    double sc = rel_scale(x);
    double lim_lo = tmin - 1e-4 * sc, lim_hi = tmax + 1e-4 * sc;
    if (!(th > lim_lo && th < lim_hi)) return;
    double nn = dot(n, n);
    if (nn == 0.0) return;
    /* barycentrics of the plane point and distances to the three edges */
    v3 q = sub(x, p0);
    double b1 = dot(cross(q, e2), n) / nn, b2 = dot(cross(e1, q), n) / nn, b0 = 1.0 - b1 - b2;
    double area2 = sqrt(nn);
    v3 p12 = sub(p2, p1);
    double h0 = area2 / sqrt(dot(p12, p12)), h1 = area2 / sqrt(dot(e2, e2)), h2 = area2 / sqrt(dot(e1, e1));
    /* The answer for this triangle flips only if the crossing moves across the
     * triangle boundary (distance de) or across an end of the ray interval
     * (distance dt); outside both, both must move. */
    double de = fmin(fmin(fabs(b0) * h0, fabs(b1) * h1), fabs(b2) * h2) / sc;
    double dt = fabs(th - tmin) / sc;
    if (isfinite(tmax) && fabs(th - tmax) / sc < dt) dt = fabs(th - tmax) / sc;
    int inside = b0 >= 0 && b1 >= 0 && b2 >= 0;
    int inrange = th > tmin && th < tmax;
    double m = (inside && inrange) ? fmin(de, dt) : (inside ? dt : (inrange ? de : fmax(de, dt)));
    if (m < tm->m) tm->m = m;
    if (b0 >= 0 && b1 >= 0 && b2 >= 0 && th > tmin && th < tmax) {
        if (th < tm->t1 || (th == tm->t1 && t < tm->id1)) { tm->t2 = tm->t1; tm->t1 = th; tm->id1 = t; }
        else if (th < tm->t2) tm->t2 = th;
    }
}

static void consider(const orc_scene *s, const wray *r, int32_t t, double tmin, int32_t skip0,
                     int32_t skip1, ohit *best, tiemargin *tm, double tmax_all)
{
    if (t == skip0 || t == skip1) return;
    if (tm) plane_margin(s, r, t, tmin, tmax_all, tm);
    const int32_t *f = &s->F[3 * (int64_t)t];
    double th, u, v;
    double tmax = best->tri >= 0 ? best->t : INFINITY;
    if (best->tri >= 0) {
        /* allow equality for the id tie rule */
        if (!tri_hit(r, vtx(s, f[0]), vtx(s, f[1]), vtx(s, f[2]), tmin, INFINITY, &th, &u, &v)) return;
        if (th > tmax) return;
        if (th == tmax && t > best->tri) return;
    } else {
        if (!tri_hit(r, vtx(s, f[0]), vtx(s, f[1]), vtx(s, f[2]), tmin, INFINITY, &th, &u, &v)) return;
    }
    best->tri = t; best->t = th; best->u = u; best->v = v;
}

/* margin (nullable) receives min(*margin, near-tie margin of this query). */
static ohit closest_m(const orc_scene *s, v3 o, v3 d, double tmin, double tmax, int32_t skip0,
                      int32_t skip1, int brute, double *margin)
{
    ohit best; best.tri = -1; best.t = INFINITY; best.u = best.v = 0;
    wray r = make_wray(o, d);
    tiemargin tmv = { INFINITY, INFINITY, INFINITY, -1 };
    tiemargin *tm = margin ? &tmv : NULL;
    if (brute || s->nnodes == 0) {
        for (int64_t t = 0; t < s->nt; ++t) consider(s, &r, (int32_t)t, tmin, skip0, skip1, &best, tm, tmax);
    } else {
        int stack[256]; int sp = 0; stack[sp++] = 0;
        while (sp) {
            const onode *n = &s->nodes[stack[--sp]];
            double lim = best.tri >= 0 ? best.t : tmax;
            if (tm) lim = (isfinite(lim) ? lim : 1e300) + 1e-4 * rel_scale(o) + 1e-4 * lim;
            if (!box_hit(n, o, d, tmin - (tm ? 1e-4 * rel_scale(o) : 0.0), lim)) continue;
            if (n->left < 0) {
                for (int i = n->first; i < n->first + n->count; ++i)
                    consider(s, &r, s->order[i], tmin, skip0, skip1, &best, tm, tmax);
            } else {
                stack[sp++] = n->left; stack[sp++] = n->right;
            }
        }
    }
    if (best.tri >= 0 && !(best.t < tmax)) best.tri = -1;
    if (tm) {
        double m = tmv.m;
        if (isfinite(tmv.t2)) {
            double g = (tmv.t2 - tmv.t1) / rel_scale(add(o, scl(d, tmv.t1)));
            if (g < m) m = g;
        }
        if (m < *margin) *margin = m;
    }
    return best;
}

static ohit closest(const orc_scene *s, v3 o, v3 d, double tmin, double tmax, int32_t skip0,
                    int32_t skip1, int brute)
{
    return closest_m(s, o, d, tmin, tmax, skip0, skip1, brute, NULL);
}

int orc_closest_hit(const orc_scene *s, const double o[3], const double d[3], double tmin,
                    double tmax, int32_t skip, int brute, double out[3], double *margin)
{
    if (margin) *margin = INFINITY;
    ohit h = closest_m(s, mk(o[0], o[1], o[2]), mk(d[0], d[1], d[2]), tmin, tmax, skip, -1, brute,
                       margin);
    if (h.tri >= 0) { out[0] = h.t; out[1] = h.u; out[2] = h.v; }
    return h.tri;
}

/* ------------------------------------------------------------------------- */
/* Cameras: pinhole, box pixel filter (Sec. 3.1, pixel filter h_j of Eq. 1).  */
/* cam_to_world is row-major 4x4 acting on column vectors; the camera looks   */
/* down its -z axis with +y up; image row 0 is the top row.                   */
/* ------------------------------------------------------------------------- */
static void camera_ray(const float *c2w, double fov_y, int W, int H, double px, double py, v3 *o,
                       v3 *d)
{
    double th = tan(0.5 * fov_y), asp = (double)W / (double)H;
    double cx = (2.0 * px / W - 1.0) * th * asp;
    double cy = (1.0 - 2.0 * py / H) * th;
    double cz = -1.0;
    v3 dw = mk(c2w[0] * cx + c2w[1] * cy + c2w[2] * cz, c2w[4] * cx + c2w[5] * cy + c2w[6] * cz,
               c2w[8] * cx + c2w[9] * cy + c2w[10] * cz);
    *o = mk(c2w[3], c2w[7], c2w[11]);
    *d = nrm(dw);
}

void orc_camera_ray(const float *c2w, double fov_y, int W, int H, double px, double py, double out[6])
{
    v3 o, d;
    camera_ray(c2w, fov_y, W, H, px, py, &o, &d);
    out[0] = o.x; out[1] = o.y; out[2] = o.z; out[3] = d.x; out[4] = d.y; out[5] = d.z;
}

/* ------------------------------------------------------------------------- */
/* Material model: Lambert + GGX (Walter et al. 2007) with separable Smith    */
/* shadowing, no Fresnel.  Parameters of a segment: kd[3], ks[3], alpha.      */
/* ------------------------------------------------------------------------- */
static double clamp_alpha(double a) { return a < 1e-3 ? 1e-3 : (a > 1.0 ? 1.0 : a); }
static double alpha_live(double a) { return (a > 1e-3 && a < 1.0) ? 1.0 : 0.0; }

/* GGX distribution in the cancellation-free form a^2 / (pi (a^2 c^2 + s^2)^2)
 * with c = n.h and s^2 = |n x h|^2 (equal to the textbook
 * a^2 / (pi (c^2 (a^2 - 1) + 1)^2) since c^2 + s^2 = 1). */
static double ggx_D(double ch, double sh2, double a)
{
    if (ch <= 0) return 0;
    double a2 = a * a, d = a2 * ch * ch + sh2;
    return a2 / (ORC_PI * d * d);
}
static double ggx_dD(double ch, double sh2, double a)
{
    if (ch <= 0) return 0;
    double a2 = a * a, d = a2 * ch * ch + sh2;
    return 2.0 * a * (sh2 - a2 * ch * ch) / (ORC_PI * d * d * d);
}
static double sin2(v3 n, v3 h) { v3 c = cross(n, h); return dot(c, c); }
static double smith_G1(double c, double a)
{
    double s = sqrt(a * a + (1.0 - a * a) * c * c);
    return 2.0 * c / (c + s);
}
static double smith_dG1(double c, double a)
{
    double s = sqrt(a * a + (1.0 - a * a) * c * c);
    return -2.0 * c * a * (1.0 - c * c) / (s * (c + s) * (c + s));
}

/* Specular lobe without ks: spec = D G1(o) G1(i) / (4 co ci), and d spec / d alpha. */
static void spec_term(v3 n, v3 wo, v3 wi, double alpha_raw, double *spec, double *dspec)
{
    double co = dot(n, wo), ci = dot(n, wi);
    *spec = 0; *dspec = 0;
    if (co <= 0 || ci <= 0) return;
    v3 h = nrm(add(wo, wi));
    double ch = dot(n, h), sh2 = sin2(n, h);
    double a = clamp_alpha(alpha_raw);
    double D = ggx_D(ch, sh2, a), dD = ggx_dD(ch, sh2, a);
    double Go = smith_G1(co, a), Gi = smith_G1(ci, a);
    double dGo = smith_dG1(co, a), dGi = smith_dG1(ci, a);
    double den = 4.0 * co * ci;
    *spec = D * Go * Gi / den;
    *dspec = alpha_live(alpha_raw) * (dD * Go * Gi + D * dGo * Gi + D * Go * dGi) / den;
}

static double lum3(const double *c) { return (c[0] + c[1] + c[2]) / 3.0; }

/* Probability of choosing the specular lobe (evaluated at sampling params). */
static double lobe_prob(const double *mp)
{
    double ld = lum3(mp), ls = lum3(mp + 3);
    if (ld + ls <= 0) return 0.5;
    return ls / (ld + ls);
}

/* Solid-angle pdf of the BRDF sampler for direction wi. */
static double brdf_pdf(const double *mp, v3 n, v3 wo, v3 wi)
{
    double ci = dot(n, wi), co = dot(n, wo);
    if (ci <= 0 || co <= 0) return 0;
    double ps = lobe_prob(mp);
    double pd = ci / ORC_PI;
    double pspec = 0;
    v3 h = nrm(add(wo, wi));
    double ch = dot(n, h), oh = dot(wo, h);
    if (ch > 0 && oh > 0) pspec = ggx_D(ch, sin2(n, h), clamp_alpha(mp[6])) * ch / (4.0 * oh);
    return (1.0 - ps) * pd + ps * pspec;
}

/* Orthonormal basis around n (Duff et al., JCGT 2017). */
static void onb(v3 n, v3 *t, v3 *b)
{
    double sg = n.z >= 0 ? 1.0 : -1.0;
    double a = -1.0 / (sg + n.z);
    double bb = n.x * n.y * a;
    *t = mk(1.0 + sg * n.x * n.x * a, sg * bb, -sg * n.x);
    *b = mk(bb, sg + n.y * n.y * a, -n.y);
}

/* Sample a direction from the lobe mixture: u3 picks the lobe, (u4,u5) the
 * direction.  Returns 0 if the sample is invalid (then the path ends). */
static int brdf_sample(const double *mp, v3 n, v3 wo, double u3, double u4, double u5, v3 *wi,
                       int *lobe)
{
    v3 t, b;
    onb(n, &t, &b);
    double ps = lobe_prob(mp);
    double phi = 2.0 * ORC_PI * u5;
    if (u3 < ps) {
        *lobe = 1;
        double a = clamp_alpha(mp[6]);
        /* Walter et al. 2007: tan^2 = a^2 u / (1 - u); cos^2 and sin^2 without cancellation */
        double den = 1.0 + (a * a - 1.0) * u4;
        double ch = sqrt((1.0 - u4) / den), sh = sqrt(a * a * u4 / den);
        v3 h = add(add(scl(t, sh * cos(phi)), scl(b, sh * sin(phi))), scl(n, ch));
        double oh = dot(wo, h);
        if (oh <= 0) return 0;
        *wi = sub(scl(h, 2.0 * oh), wo);
    } else {
        *lobe = 0;
        double r = sqrt(u4), z = sqrt(fmax(0.0, 1.0 - u4));
        *wi = add(add(scl(t, r * cos(phi)), scl(b, r * sin(phi))), scl(n, z));
    }
    return 1;
}

/* Exported for the BRDF/pdf unit checks.  mp = [kd3, ks3, alpha]. */
void orc_brdf_eval(const double *mp, const double n_[3], const double wo_[3], const double wi_[3],
                   double out[6])
{
    v3 n = mk(n_[0], n_[1], n_[2]), wo = mk(wo_[0], wo_[1], wo_[2]), wi = mk(wi_[0], wi_[1], wi_[2]);
    double spec, dspec;
    spec_term(n, wo, wi, mp[6], &spec, &dspec);
    double ok = (dot(n, wo) > 0 && dot(n, wi) > 0) ? 1.0 : 0.0;
    for (int c = 0; c < 3; ++c) out[c] = ok * (mp[c] / ORC_PI + mp[3 + c] * spec);
    out[3] = brdf_pdf(mp, n, wo, wi);
    out[4] = spec;
    out[5] = dspec;
}

int orc_brdf_sample(const double *mp, const double n_[3], const double wo_[3], double u3,
                    double u4, double u5, double wi_out[3])
{
    v3 wi;
    int lobe;
    v3 n = mk(n_[0], n_[1], n_[2]), wo = mk(wo_[0], wo_[1], wo_[2]);
    if (!brdf_sample(mp, n, wo, u3, u4, u5, &wi, &lobe)) return -1;
    wi_out[0] = wi.x; wi_out[1] = wi.y; wi_out[2] = wi.z;
    return lobe;
}

/* ------------------------------------------------------------------------- */
/* Disney material model (Burley 2012, "Physically-Based Shading at Disney";  */
/* the paper's material, Sec. 4.1): base colour plus ten parameters, all      */
/* meant to lie in [0, 1].  Parameters of a segment, in this order:          */
/*   base colour r g b, subsurface, metallic, specular, specular tint,        */
/*   roughness, anisotropic, sheen, sheen tint, clearcoat, clearcoat gloss.   */
/* f = (1 - metallic) (base/pi mix(F_d, F_ss, subsurface) + sheen F_W(h.l)     */
/*     C_sheen) + D_s F_s G_s / (4 n.l n.v) + clearcoat/4 D_c F_c G_c /       */
/*     (4 n.l n.v), with                                                       */
/*   F_W(x) = (1 - x)^5 (Schlick's weight), tint = base / lum(base) with       */
/*   lum = 0.3 r + 0.6 g + 0.1 b (1 if lum = 0),                               */
/*   F_d = (1 + (F_D90 - 1) F_W(n.l)) (1 + (F_D90 - 1) F_W(n.v)),              */
/*   F_D90 = 1/2 + 2 roughness (h.l)^2,                                         */
/*   F_ss = 1.25 ((1 + (F_90 - 1) F_W(n.l)) (1 + (F_90 - 1) F_W(n.v))          */
/*          (1 / (n.l + n.v) - 1/2) + 1/2), F_90 = roughness (h.l)^2,           */
/*   C_sheen = mix(1, tint, sheen tint),                                        */
/*   D_s anisotropic GGX with a_x = max(1e-3, r^2 / k), a_y = max(1e-3, r^2 k), */
/*   k = sqrt(1 - 0.9 anisotropic): 1 / (pi a_x a_y ((h.x/a_x)^2 +            */
/*   (h.y/a_y)^2 + (h.n)^2)^2), G_s the anisotropic Smith term                  */
/*   G1(w) = 2 (w.n) / (w.n + sqrt((w.n)^2 + (a_x w.x)^2 + (a_y w.y)^2)) at    */
/*   l and v, F_s = mix(C_s0, 1, F_W(h.l)),                                      */
/*   C_s0 = mix(0.08 specular mix(1, tint, specular tint), base, metallic),    */
/*   D_c = (a^2 - 1) / (pi ln(a^2) ((h.n)^2 a^2 + |h x n|^2)) (GTR1) with      */
/*   a = mix(0.1, 0.001, clearcoat gloss), F_c = mix(0.04, 1, F_W(h.l)),       */
/*   G_c the isotropic Smith term with a = 0.25.                                */
/* The tangent x is the hit triangle's first edge projected onto the plane of */
/* the shading normal, y = n x x.  Written in complex arithmetic: evaluated  */
/* at parameters p + i 1e-30 e_j, the imaginary part is 1e-30 times the exact */
/* derivative with respect to p_j (complex-step differentiation, Squire and   */
/* Trapp 1998), with no cancellation; max() and the lum = 0 test look at the  */
/* real part only.                                                            */
/* ------------------------------------------------------------------------- */
#include <complex.h>
#define DS_N 13
enum { DS_SUBSURFACE = 3, DS_METALLIC, DS_SPECULAR, DS_SPEC_TINT, DS_ROUGHNESS, DS_ANISO, DS_SHEEN,
       DS_SHEEN_TINT, DS_CLEARCOAT, DS_CC_GLOSS };
typedef double complex cplx;

/* geometry of a (wo, wi) pair in the frame (x, y, n): cosines with n, with h,
 * and the x, y components of wi, wo and h; sin^2 of h against n */
typedef struct { double ci, co, ch, cd, ix, iy, ox, oy, hx, hy, sh2; int ok; } dgeom;

static void disney_frame(v3 n, v3 e1, v3 *x, v3 *y, double *margin)
{
    v3 t = sub(e1, scl(n, dot(n, e1)));
    double lt = sqrt(dot(t, t)), le = sqrt(dot(e1, e1));
    if (margin) { double m = lt / (le > 0 ? le : 1.0) - 1e-6; if (fabs(m) < *margin) *margin = fabs(m); }
    if (lt > 1e-6 * le) {
        *x = scl(t, 1.0 / lt);
        *y = cross(n, *x);
    } else {
        onb(n, x, y);
    }
}

static dgeom disney_geom(v3 n, v3 x, v3 y, v3 wo, v3 wi)
{
    dgeom g;
    memset(&g, 0, sizeof g);
    g.ci = dot(n, wi);
    g.co = dot(n, wo);
    g.ok = g.ci > 0 && g.co > 0;
    if (!g.ok) return g;
    v3 h = nrm(add(wo, wi));
    g.ch = dot(n, h);
    g.cd = dot(wi, h);
    g.ix = dot(wi, x); g.iy = dot(wi, y);
    g.ox = dot(wo, x); g.oy = dot(wo, y);
    g.hx = dot(h, x); g.hy = dot(h, y);
    g.sh2 = sin2(n, h);
    return g;
}

static cplx cmix(cplx a, cplx b, cplx t) { return a + (b - a) * t; }
static cplx cmax_lo(cplx a, double lo) { return creal(a) < lo ? (cplx)lo : a; }
static double schlick_w(double c) { double m = 1.0 - c; return m * m * m * m * m; }
static cplx g1_aniso(double c, double wx, double wy, cplx ax, cplx ay)
{
    return 2.0 * c / (c + csqrt(c * c + (wx * ax) * (wx * ax) + (wy * ay) * (wy * ay)));
}
static double g1_iso(double c, double a)
{
    return 2.0 * c / (c + sqrt(a * a + (1.0 - a * a) * c * c));
}

/* f[3] of the Disney model for parameters p[13] (complex) and geometry g */
static void disney_f(const cplx *p, const dgeom *g, cplx f[3])
{
    f[0] = f[1] = f[2] = 0;
    if (!g->ok) return;
    cplx lum = 0.3 * p[0] + 0.6 * p[1] + 0.1 * p[2];
    cplx tint[3];
    for (int c = 0; c < 3; ++c) tint[c] = creal(lum) > 0 ? p[c] / lum : (cplx)1.0;
    double FL = schlick_w(g->ci), FV = schlick_w(g->co), FH = schlick_w(g->cd);
    cplx r = p[DS_ROUGHNESS];
    cplx fd90 = 0.5 + 2.0 * r * g->cd * g->cd;
    cplx fd = (1.0 + (fd90 - 1.0) * FL) * (1.0 + (fd90 - 1.0) * FV);
    cplx f90 = r * g->cd * g->cd;
    cplx fss = 1.25 * ((1.0 + (f90 - 1.0) * FL) * (1.0 + (f90 - 1.0) * FV) * (1.0 / (g->ci + g->co) - 0.5) + 0.5);
    cplx diff = cmix(fd, fss, p[DS_SUBSURFACE]) / ORC_PI;
    cplx k = csqrt(1.0 - 0.9 * p[DS_ANISO]);
    cplx ax = cmax_lo(r * r / k, 1e-3), ay = cmax_lo(r * r * k, 1e-3);
    cplx tx = g->hx / ax, ty = g->hy / ay;
    cplx dd = tx * tx + ty * ty + g->ch * g->ch;
    cplx Ds = 1.0 / (ORC_PI * ax * ay * dd * dd);
    cplx Gs = g1_aniso(g->ci, g->ix, g->iy, ax, ay) * g1_aniso(g->co, g->ox, g->oy, ax, ay);
    cplx ac = cmix(0.1, 0.001, p[DS_CC_GLOSS]);
    cplx a2 = ac * ac;
    cplx Dc = (a2 - 1.0) / (ORC_PI * clog(a2) * (g->ch * g->ch * a2 + g->sh2));
    double Fc = 0.04 + 0.96 * FH, Gc = g1_iso(g->ci, 0.25) * g1_iso(g->co, 0.25);
    double den = 4.0 * g->ci * g->co;
    cplx spec = Ds * Gs / den, coat = 0.25 * p[DS_CLEARCOAT] * Dc * Fc * Gc / den;
    for (int c = 0; c < 3; ++c) {
        cplx cs0 = cmix(p[DS_SPECULAR] * 0.08 * cmix(1.0, tint[c], p[DS_SPEC_TINT]), p[c], p[DS_METALLIC]);
        cplx Fs = cmix(cs0, 1.0, FH);
        cplx sheen = FH * p[DS_SHEEN] * cmix(1.0, tint[c], p[DS_SHEEN_TINT]);
        f[c] = (diff * p[c] + sheen) * (1.0 - p[DS_METALLIC]) + Fs * spec + coat;
    }
}

/* value f[3] and, with df != NULL, df[j][c] = d f_c / d p_j for all 13 j */
static void disney_eval(const double *mp, const dgeom *g, double f[3], double df[DS_N][3])
{
    cplx p[DS_N], fc[3];
    for (int j = 0; j < DS_N; ++j) p[j] = mp[j];
    disney_f(p, g, fc);
    for (int c = 0; c < 3; ++c) f[c] = creal(fc[c]);
    if (!df) return;
    const double hstep = 1e-30;
    for (int j = 0; j < DS_N; ++j) {
        p[j] = mp[j] + I * hstep;
        disney_f(p, g, fc);
        for (int c = 0; c < 3; ++c) df[j][c] = cimag(fc[c]) / hstep;
        p[j] = mp[j];
    }
}

/* Lobe probabilities of the sampler (at sampling parameters): diffuse
 * (1 - metallic) lum(base), specular max(lum(C_s0 without tint), 0.02),
 * clearcoat 0.1 clearcoat; normalised. */
static void disney_lobes(const double *mp, double pl[3])
{
    double lum = 0.3 * mp[0] + 0.6 * mp[1] + 0.1 * mp[2];
    double s0 = 0.08 * mp[DS_SPECULAR] + (lum - 0.08 * mp[DS_SPECULAR]) * mp[DS_METALLIC];
    double w[3] = { fmax(1.0 - mp[DS_METALLIC], 0.0) * fmax(lum, 0.0), fmax(s0, 0.02), 0.1 * fmax(mp[DS_CLEARCOAT], 0.0) };
    double t = w[0] + w[1] + w[2];
    for (int i = 0; i < 3; ++i) pl[i] = w[i] / t;
}

static void disney_alphas(const double *mp, double *ax, double *ay, double *ac)
{
    double r = mp[DS_ROUGHNESS], k = sqrt(1.0 - 0.9 * mp[DS_ANISO]);
    *ax = fmax(r * r / k, 1e-3);
    *ay = fmax(r * r * k, 1e-3);
    *ac = 0.1 + (0.001 - 0.1) * mp[DS_CC_GLOSS];
}

/* Solid-angle pdf of the sampler for wi. */
static double disney_pdf(const double *mp, v3 n, v3 x, v3 y, v3 wo, v3 wi)
{
    double ci = dot(n, wi), co = dot(n, wo);
    if (ci <= 0 || co <= 0) return 0;
    double pl[3], ax, ay, ac;
    disney_lobes(mp, pl);
    disney_alphas(mp, &ax, &ay, &ac);
    v3 h = nrm(add(wo, wi));
    double ch = dot(n, h), oh = dot(wo, h);
    double p = pl[0] * ci / ORC_PI;
    if (ch > 0 && oh > 0) {
        double tx = dot(h, x) / ax, ty = dot(h, y) / ay, dd = tx * tx + ty * ty + ch * ch;
        double Ds = 1.0 / (ORC_PI * ax * ay * dd * dd);
        double a2 = ac * ac;
        double Dc = (a2 - 1.0) / (ORC_PI * log(a2) * (ch * ch * a2 + sin2(n, h)));
        p += (pl[1] * Ds + pl[2] * Dc) * ch / (4.0 * oh);
    }
    return p;
}

/* Sample wi: u3 picks the lobe (0 diffuse, 1 specular, 2 clearcoat), (u4, u5)
 * the direction: cosine hemisphere; the anisotropic GGX normal distribution
 * (azimuth phi of (a_x cos 2 pi u5, a_y sin 2 pi u5), tan^2 theta_h =
 * u4 / ((1 - u4) A) with A = cos^2 phi / a_x^2 + sin^2 phi / a_y^2); GTR1
 * (cos^2 theta_h = (1 - a^(2 (1 - u4))) / (1 - a^2), phi = 2 pi u5), each
 * half vector reflected about wo.  Returns 0 if wi is invalid. */
static int disney_sample(const double *mp, v3 n, v3 x, v3 y, v3 wo, double u3, double u4, double u5, v3 *wi,
                         int *lobe, double *margin)
{
    double pl[3], ax, ay, ac;
    disney_lobes(mp, pl);
    disney_alphas(mp, &ax, &ay, &ac);
    if (margin) {
        if (pl[0] > 0 && fabs(u3 - pl[0]) < *margin) *margin = fabs(u3 - pl[0]);
        if (pl[2] > 0 && fabs(u3 - pl[0] - pl[1]) < *margin) *margin = fabs(u3 - pl[0] - pl[1]);
    }
    double c = cos(2.0 * ORC_PI * u5), s = sin(2.0 * ORC_PI * u5);
    if (u3 < pl[0]) {
        *lobe = 0;
        double r = sqrt(u4), z = sqrt(fmax(0.0, 1.0 - u4));
        *wi = add(add(scl(x, r * c), scl(y, r * s)), scl(n, z));
        return 1;
    }
    double ch, sh, cp, sp;
    if (u3 < pl[0] + pl[1]) {
        *lobe = 1;
        double vx = ax * c, vy = ay * s, lv = sqrt(vx * vx + vy * vy);
        cp = vx / lv; sp = vy / lv;
        double A = cp * cp / (ax * ax) + sp * sp / (ay * ay);
        double den = (1.0 - u4) * A + u4;
        ch = sqrt((1.0 - u4) * A / den);
        sh = sqrt(u4 / den);
    } else {
        *lobe = 2;
        double L = log(ac * ac);
        ch = sqrt(-expm1((1.0 - u4) * L) / (1.0 - ac * ac));
        sh = sqrt(ac * ac * expm1(-u4 * L) / (1.0 - ac * ac));
        cp = c; sp = s;
    }
    v3 h = add(add(scl(x, sh * cp), scl(y, sh * sp)), scl(n, ch));
    double oh = dot(wo, h);
    if (margin && fabs(oh) < *margin) *margin = fabs(oh);
    if (oh <= 0) return 0;
    *wi = sub(scl(h, 2.0 * oh), wo);
    return 1;
}

/* Exported for the Disney pins: f[3], pdf, then df [13][3] (row-major). */
void orc_disney_eval(const double *mp, const double n_[3], const double x_[3], const double wo_[3],
                     const double wi_[3], double out[4 + 3 * DS_N])
{
    v3 n = mk(n_[0], n_[1], n_[2]), t = mk(x_[0], x_[1], x_[2]);
    v3 wo = mk(wo_[0], wo_[1], wo_[2]), wi = mk(wi_[0], wi_[1], wi_[2]);
    v3 x, y;
    disney_frame(n, t, &x, &y, NULL);
    dgeom g = disney_geom(n, x, y, wo, wi);
    double df[DS_N][3];
    disney_eval(mp, &g, out, df);
    out[3] = disney_pdf(mp, n, x, y, wo, wi);
    for (int j = 0; j < DS_N; ++j)
        for (int c = 0; c < 3; ++c) out[4 + 3 * j + c] = df[j][c];
}

int orc_disney_sample(const double *mp, const double n_[3], const double x_[3], const double wo_[3], double u3,
                      double u4, double u5, double wi_out[3])
{
    v3 n = mk(n_[0], n_[1], n_[2]), t = mk(x_[0], x_[1], x_[2]), wo = mk(wo_[0], wo_[1], wo_[2]);
    v3 x, y, wi;
    int lobe;
    disney_frame(n, t, &x, &y, NULL);
    if (!disney_sample(mp, n, x, y, wo, u3, u4, u5, &wi, &lobe, NULL)) return -1;
    wi_out[0] = wi.x; wi_out[1] = wi.y; wi_out[2] = wi.z;
    return lobe;
}

/* ------------------------------------------------------------------------- */
/* Light selection: discrete distribution over emitter triangles with weight  */
/* area * max(lum(e), 1e-3 * max_k lum(e_k)); uniform over area if every      */
/* emission is zero.  The paper keeps per-object probabilities proportional   */
/* to the current emission in a Fenwick tree (Appendix E); with few emitter   */
/* triangles a plain cumulative table is rebuilt every call instead.          */
/* ------------------------------------------------------------------------- */
typedef struct { double *cdf; double total; } lightdist;

static lightdist build_lights(const orc_scene *s, const double *sp)
{
    lightdist L;
    L.cdf = (double *)malloc(sizeof(double) * (size_t)(s->nlt + 1));
    double maxl = 0;
    for (int k = 0; k < s->ne; ++k) {
        double l = lum3(sp + s->nm * s->ns + 3 * k);
        if (l > maxl) maxl = l;
    }
    double acc = 0;
    for (int64_t j = 0; j < s->nlt; ++j) {
        int k = s->seg_emitter[s->seg[s->light_tri[j]]];
        double l = lum3(sp + s->nm * s->ns + 3 * k);
        double w = maxl > 0 ? s->light_area[j] * fmax(l, 1e-3 * maxl) : s->light_area[j];
        acc += w;
        L.cdf[j] = acc;
    }
    L.total = acc;
    return L;
}

static int64_t pick_light(const lightdist *L, int64_t n, double u)
{
    double x = u * L->total;
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {          /* first j with cdf[j] > x */
        int64_t mid = (lo + hi) / 2;
        if (L->cdf[mid] > x) hi = mid; else lo = mid + 1;
    }
    return lo;
}

static double light_prob(const lightdist *L, int64_t j)
{
    double prev = j > 0 ? L->cdf[j - 1] : 0.0;
    return (L->cdf[j] - prev) / L->total;
}


/* ------------------------------------------------------------------------- */
/* Path tracing with per-factor derivative bookkeeping.                       */
/* ------------------------------------------------------------------------- */
#define ORC_MAXD 16
#define ORC_MAXDER 16

/* A 3-channel factor of a path contribution with its sparse derivative. */
typedef struct {
    double v[3];
    int n;
    int32_t idx[ORC_MAXDER];
    double d[ORC_MAXDER][3];
} factor;

typedef struct {
    uint64_t seed; uint32_t stream_tag, iteration;
    int32_t spp, max_depth, rr_depth, mis, emission_profile, jitter, brute_force;
    const int64_t *pixel_list; int64_t num_pixels;
    /* learned proposal: float32 network weights (16744 + 16 S values), the
     * probability of sampling it, and the scene box used for its features */
    const float *guide_w; double guide_mix; double bb_lo[3], bb_inv[3];
    /* > 0: the proposal of a vertex is the network evaluated at the cell of
     * the surface it lies in (cells of about this area), not at the vertex */
    double guide_cell_area;
} orc_opts;

typedef struct { int32_t num_views, width, height; const float *cam_to_world; const float *fov_y; } orc_cams;
/* ------------------------------------------------------------------------- */
/* Learned proposal (not part of the paper's method): an MLP 25 -> 64 x 4 ->  */
/* 40 with ReLU maps (normalised position, shading normal, outgoing           */
/* direction, 16-d segment embedding) to 8 von Mises-Fisher lobes (mu =        */
/* normalised y[0..2], kappa = softplus(y[3]) + 0.01 capped at 1e4, weight =   */
/* softmax of y[4]); combined with BRDF sampling by one-sample MIS.            */
/* Parameter block (float32): W1 [25][64], b1, W2..W4 [64][64], b2..b4,         */
/* W5 [64][40], b5, then the embedding [S][16].                                */
/* ------------------------------------------------------------------------- */
#define G_IN 25
#define G_HID 64
#define G_OUT 40
#define G_LOBES 8

static void guide_mlp(const float *w, const double x[G_IN], double y[G_OUT])
{
    const float *W1 = w, *b1 = W1 + G_IN * G_HID, *W2 = b1 + G_HID, *b2 = W2 + G_HID * G_HID;
    const float *W3 = b2 + G_HID, *b3 = W3 + G_HID * G_HID, *W4 = b3 + G_HID, *b4 = W4 + G_HID * G_HID;
    const float *W5 = b4 + G_HID, *b5 = W5 + G_HID * G_OUT;
    double h[G_HID], g[G_HID];
    for (int n = 0; n < G_HID; ++n) {
        double s = b1[n];
        for (int k = 0; k < G_IN; ++k) s += x[k] * (double)W1[k * G_HID + n];
        h[n] = s > 0 ? s : 0;
    }
    const float *Ws[3] = { W2, W3, W4 }, *bs[3] = { b2, b3, b4 };
    for (int l = 0; l < 3; ++l) {
        for (int n = 0; n < G_HID; ++n) {
            double s = bs[l][n];
            for (int k = 0; k < G_HID; ++k) s += h[k] * (double)Ws[l][k * G_HID + n];
            g[n] = s > 0 ? s : 0;
        }
        for (int n = 0; n < G_HID; ++n) h[n] = g[n];
    }
    for (int n = 0; n < G_OUT; ++n) {
        double s = b5[n];
        for (int k = 0; k < G_HID; ++k) s += h[k] * (double)W5[k * G_OUT + n];
        y[n] = s;
    }
}

static double softplus_d(double x) { return x > 30 ? x : log1p(exp(x)); }

/* raw outputs -> per lobe (mu xyz, kappa, weight) */
static void guide_mixture(double y[G_OUT])
{
    double mx = -INFINITY, z = 0;
    for (int j = 0; j < G_LOBES; ++j) if (y[5 * j + 4] > mx) mx = y[5 * j + 4];
    for (int j = 0; j < G_LOBES; ++j) {
        double *l = y + 5 * j;
        double n2 = l[0] * l[0] + l[1] * l[1] + l[2] * l[2];
        if (n2 > 0) { double r = 1.0 / sqrt(n2); l[0] *= r; l[1] *= r; l[2] *= r; }
        else { l[0] = 0; l[1] = 0; l[2] = 1; }
        l[3] = fmin(softplus_d(l[3]) + 0.01, 1e4);
        l[4] = exp(l[4] - mx);
        z += l[4];
    }
    for (int j = 0; j < G_LOBES; ++j) y[5 * j + 4] /= z;
}

static double vmf_pdf_d(double kappa, double c)
{
    return kappa / (2.0 * ORC_PI * -expm1(-2.0 * kappa)) * exp(kappa * (c - 1.0));
}

static double mixture_pdf_d(const double *mix, v3 w)
{
    double q = 0;
    for (int j = 0; j < G_LOBES; ++j) {
        const double *l = mix + 5 * j;
        q += l[4] * vmf_pdf_d(l[3], l[0] * w.x + l[1] * w.y + l[2] * w.z);
    }
    return q;
}

/* lobe by u3 (margins recorded), then w = 1 + log(u4 + (1-u4) e^{-2 kappa}) / kappa */
static v3 mixture_sample_d(const double *mix, double u3, double u4, double u5, double *margin)
{
    int j = G_LOBES - 1;
    double acc = 0;
    for (int i = 0; i < G_LOBES; ++i) {
        acc += mix[5 * i + 4];
        if (margin && fabs(u3 - acc) < *margin) *margin = fabs(u3 - acc);
        if (u3 < acc) { j = i; break; }
    }
    const double *l = mix + 5 * j;
    v3 mu = mk(l[0], l[1], l[2]);
    double kappa = l[3];
    double w = 1.0 + log1p(-(1.0 - u4) * -expm1(-2.0 * kappa)) / kappa;
    if (w > 1) w = 1;
    if (w < -1) w = -1;
    double sw = sqrt(fmax(0.0, 1.0 - w * w));
    v3 t, b;
    onb(mu, &t, &b);
    double phi = 2.0 * ORC_PI * u5;
    return add(add(scl(t, sw * cos(phi)), scl(b, sw * sin(phi))), scl(mu, w));
}

static void guide_eval_vertex(const orc_opts *o, int nseg, int seg, v3 x, v3 n, v3 wo, double mix[G_OUT])
{
    double f[G_IN];
    f[0] = 2.0 * (x.x - o->bb_lo[0]) * o->bb_inv[0] - 1.0;
    f[1] = 2.0 * (x.y - o->bb_lo[1]) * o->bb_inv[1] - 1.0;
    f[2] = 2.0 * (x.z - o->bb_lo[2]) * o->bb_inv[2] - 1.0;
    f[3] = n.x; f[4] = n.y; f[5] = n.z;
    f[6] = wo.x; f[7] = wo.y; f[8] = wo.z;
    const float *emb = o->guide_w + 16744;
    (void)nseg;
    for (int i = 0; i < 16; ++i) f[9 + i] = emb[16 * seg + i];
    guide_mlp(o->guide_w, f, mix);
    guide_mixture(mix);
}

/* Cells of the cached proposal.  A triangle's barycentric domain (x = p0 +
 * u e1 + v e2) is cut into n^2 sub-triangles: grid squares of side 1/n in
 * (u, v), each halved by its anti-diagonal.  n is the smallest integer in
 * [1, 64] with |e1 x e2| <= 2 n^2 cell_area, i.e. every cell has at most the
 * given area; the comparison is made on squares in float32 with a fixed
 * operation order, so that the integer comes out the same wherever it is
 * computed. */
static int cell_subdiv(const orc_scene *s, int64_t t, float cell_area)
{
    const int32_t *f = &s->F[3 * t];
    float p[3][3];
    for (int k = 0; k < 3; ++k)
        for (int c = 0; c < 3; ++c) p[k][c] = (float)s->P[3 * (int64_t)f[k] + c];
    float e1[3], e2[3];
    for (int c = 0; c < 3; ++c) { e1[c] = p[1][c] - p[0][c]; e2[c] = p[2][c] - p[0][c]; }
    float cx = e1[1] * e2[2] - e1[2] * e2[1];
    float cy = e1[2] * e2[0] - e1[0] * e2[2];
    float cz = e1[0] * e2[1] - e1[1] * e2[0];
    float a2 = (cx * cx + cy * cy) + cz * cz;
    float two = 2.0f * cell_area;
    int n = 1;
    for (; n < 64; ++n) {
        float q = (float)(n * n) * two;
        if (q * q >= a2) break;
    }
    return n;
}

/* Query point of the cell holding barycentrics (u, v) of triangle t: the
 * cell's centroid, the shading normal there (negated on the back side) and
 * the outgoing direction along it.  *mg collects the distance of (u, v) to
 * the cell boundaries (near-tie margin). */
static void cell_query(const orc_scene *s, int64_t t, double u, double v, int back, float cell_area,
                       v3 *xq, v3 *nq, double *mg)
{
    const int n = cell_subdiv(s, t, cell_area);
    const double x = u * n, y = v * n;
    int i = (int)floor(x), j;
    if (i < 0) i = 0;
    if (i > n - 1) i = n - 1;
    j = (int)floor(y);
    if (j < 0) j = 0;
    if (j > n - 1 - i) j = n - 1 - i;
    const double fx = x - i, fy = y - j;
    const int up = (i + j < n - 1) && (fx + fy > 1.0);
    if (mg) {
        double m = fmin(fabs(x - nearbyint(x)), fabs(y - nearbyint(y)));
        if (i + j < n - 1) m = fmin(m, fabs(fx + fy - 1.0));
        m /= n;
        if (m < *mg) *mg = m;
    }
    const double o = up ? 2.0 / 3.0 : 1.0 / 3.0;
    const double uc = (i + o) / n, vc = (j + o) / n;
    const int32_t *f = &s->F[3 * t];
    v3 p0 = vtx(s, f[0]), p1 = vtx(s, f[1]), p2 = vtx(s, f[2]);
    v3 e1 = sub(p1, p0), e2 = sub(p2, p0);
    *xq = add(p0, add(scl(e1, uc), scl(e2, vc)));
    v3 ns = nrm(cross(e1, e2));
    if (s->N) {
        v3 n0 = mk(s->N[3 * (int64_t)f[0]], s->N[3 * (int64_t)f[0] + 1], s->N[3 * (int64_t)f[0] + 2]);
        v3 n1 = mk(s->N[3 * (int64_t)f[1]], s->N[3 * (int64_t)f[1] + 1], s->N[3 * (int64_t)f[1] + 2]);
        v3 n2 = mk(s->N[3 * (int64_t)f[2]], s->N[3 * (int64_t)f[2] + 1], s->N[3 * (int64_t)f[2] + 2]);
        ns = nrm(add(scl(n0, 1.0 - uc - vc), add(scl(n1, uc), scl(n2, vc))));
    }
    *nq = back ? scl(ns, -1.0) : ns;
}

/* Exported for tests: subdivision of triangle t and the query (position,
 * normal) of the cell holding (u, v) on the given side. */
int orc_cell_query(const orc_scene *s, int64_t t, double u, double v, int back, float cell_area, double out[6])
{
    v3 xq, nq;
    cell_query(s, t, u, v, back, cell_area, &xq, &nq, NULL);
    out[0] = xq.x; out[1] = xq.y; out[2] = xq.z; out[3] = nq.x; out[4] = nq.y; out[5] = nq.z;
    return cell_subdiv(s, t, cell_area);
}

/* Threads of the OpenMP loops (timing on one core or all of them);
 * returns the previous setting. */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    int old = omp_get_max_threads();
    if (n > 0) omp_set_num_threads(n);
    return old;
#else
    (void)n;
    return 1;
#endif
}

/* Exported for tests: mixture parameters for n feature rows [n][9] + segments. */
void orc_guide_eval(const float *w, const double *feat, const int32_t *seg, int64_t n, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        double f[G_IN];
        for (int j = 0; j < 9; ++j) f[j] = feat[9 * i + j];
        for (int j = 0; j < 16; ++j) f[9 + j] = w[16744 + 16 * seg[i] + j];
        guide_mlp(w, f, out + G_OUT * i);
        guide_mixture(out + G_OUT * i);
    }
}

double orc_mixture_pdf(const double *mix, const double w[3]) { return mixture_pdf_d(mix, mk(w[0], w[1], w[2])); }

void orc_mixture_sample(const double *mix, double u3, double u4, double u5, double out[3])
{
    v3 r = mixture_sample_d(mix, u3, u4, u5, NULL);
    out[0] = r.x; out[1] = r.y; out[2] = r.z;
}


static void fadd(factor *f, int32_t idx, double d0, double d1, double d2)
{
    f->idx[f->n] = idx; f->d[f->n][0] = d0; f->d[f->n][1] = d1; f->d[f->n][2] = d2; f->n++;
}

/* Accumulate the derivative of one radiance term tau = prod_i a_i (.) phi into
 * grad, weighted by wc (per channel), using the product rule of Eqs. 5-6
 * written out without division.  Also returns tau. */
static void term_grad(const factor *a, int na, const factor *phi, const double *wc, double *grad,
                      double tau[3])
{
    for (int c = 0; c < 3; ++c) {
        double p = phi->v[c];
        for (int i = 0; i < na; ++i) p *= a[i].v[c];
        tau[c] = p;
    }
    if (!grad) return;
    /* derivative through the continuation factors */
    for (int i = 0; i < na; ++i) {
        for (int e = 0; e < a[i].n; ++e) {
            double g = 0;
            for (int c = 0; c < 3; ++c) {
                double p = a[i].d[e][c] * phi->v[c];
                for (int j = 0; j < na; ++j) if (j != i) p *= a[j].v[c];
                g += wc[c] * p;
            }
            grad[a[i].idx[e]] += g;
        }
    }
    /* derivative through the local term */
    for (int e = 0; e < phi->n; ++e) {
        double g = 0;
        for (int c = 0; c < 3; ++c) {
            double p = phi->d[e][c];
            for (int j = 0; j < na; ++j) p *= a[j].v[c];
            g += wc[c] * p;
        }
        grad[phi->idx[e]] += g;
    }
}

static uint64_t fnv(uint64_t h, uint32_t x)
{
    for (int i = 0; i < 4; ++i) { h ^= (x >> (8 * i)) & 0xFFu; h *= 0x100000001B3ull; }
    return h;
}

static double mis_w(double a, double b, int mode)
{
    if (mode == 3) { a *= a; b *= b; }
    return a / (a + b);
}

typedef struct {
    const orc_scene *s;
    const double *p, *sp;
    const lightdist *L;
    const orc_opts *o;
    double pert;      /* conditioning probe: relative perturbation injected at every vertex */
    v3 pert_dir;
} ctx;

/* Optional per-vertex record of a path (test diagnostics): for vertex k
 * (1..D+1) the hit triangle id, u, v, t and the local contribution c_k
 * (emission hit + light sample, without the prefix throughput). */
/* Per-vertex debug record: triangle, u, v, t, radiance so far (after the
 * vertex's emission and light sample), light-sample flag, then for a vertex
 * that continues: the product of the continuation weights up to and
 * including this vertex (RGB), the density of the sampled direction, the
 * direction, and 1. */
#define VREC 16
typedef struct { double *v; int nv; } vdump;

/* One path.  Returns radiance in L; adds w-weighted derivatives into grad if
 * grad != NULL.  Event hash in *hash. */
static void trace_path_v(const ctx *C, v3 org, v3 dir, uint64_t path_id, const double *wc,
                         double *grad, double Lout[3], uint64_t *hash, double *margin, vdump *vd);
static void trace_path(const ctx *C, v3 org, v3 dir, uint64_t path_id, const double *wc,
                       double *grad, double Lout[3], uint64_t *hash, double *margin)
{
    trace_path_v(C, org, dir, path_id, wc, grad, Lout, hash, margin, NULL);
}
static void trace_path_v(const ctx *C, v3 org, v3 dir, uint64_t path_id, const double *wc,
                         double *grad, double Lout[3], uint64_t *hash, double *margin, vdump *vd)
{
    double mg = INFINITY;
    double *M = margin ? &mg : NULL;
#define NEAR(v) do { if (M && fabs(v) < mg) mg = fabs(v); } while (0)
    const orc_scene *s = C->s;
    const double *p = C->p, *sp = C->sp;
    const int D = C->o->max_depth;
    const int mis = C->o->mis;
    const double tmin = 1e-6 * s->diag;
    factor a[ORC_MAXD + 2];
    int na = 0;
    double Ts[3] = { 1, 1, 1 };     /* throughput at sampling params (for RR) */
    double L[3] = { 0, 0, 0 };
    double Tc[3] = { 1, 1, 1 };
    uint64_t h = 0xCBF29CE484222325ull;
    int32_t prev_tri = -1;
    double prev_pdf = 0;            /* pdf of the direction that produced this ray */
    int prev_specular_only = 0;
    (void)prev_specular_only;
    v3 o = org, d = dir;
    for (int k = 1; k <= D + 1; ++k) {
        ohit hit = closest_m(s, o, d, tmin, INFINITY, prev_tri, -1, C->o->brute_force, M);
        h = fnv(h, (uint32_t)hit.tri);
        if (vd && k - 1 < vd->nv) {
            double *r = vd->v + VREC * (k - 1);
            r[0] = hit.tri; r[1] = hit.u; r[2] = hit.v; r[3] = hit.t;
            r[4] = L[0]; r[5] = L[1]; r[6] = L[2]; r[7] = 0;
            for (int q = 8; q < VREC; ++q) r[q] = 0;
        }
        if (hit.tri < 0) break;
        const int32_t *f = &s->F[3 * (int64_t)hit.tri];
        v3 p0 = vtx(s, f[0]), p1 = vtx(s, f[1]), p2 = vtx(s, f[2]);
        v3 e1 = sub(p1, p0), e2 = sub(p2, p0);
        v3 x = add(p0, add(scl(e1, hit.u), scl(e2, hit.v)));
        if (C->pert != 0.0) x = add(x, scl(C->pert_dir, C->pert * rel_scale(x)));
        v3 ng = nrm(cross(e1, e2));
        int seg = s->seg[hit.tri];
        int em = s->seg_emitter[seg];
        double cos_emit = -dot(d, ng);     /* > 0: ray arrives at the emitting side */
        uint32_t ev = 0;
        if (em >= 0) NEAR(cos_emit);
        /* --- emitter hit --- */
        if (em >= 0 && cos_emit > 0) {
            double w = 1.0;
            if (k > 1) {
                if (mis == 1) w = 0.0;
                else if (mis >= 2) {
                    int64_t lj = -1;
                    for (int64_t j = 0; j < s->nlt; ++j) if (s->light_tri[j] == hit.tri) lj = j;
                    double pa = light_prob(C->L, lj) / s->light_area[lj];
                    double pl = pa * hit.t * hit.t / cos_emit;
                    w = mis_w(prev_pdf, pl, mis);
                }
            }
            if (w > 0) {
                double prof = C->o->emission_profile ? cos_emit : 1.0;
                factor phi; phi.n = 0;
                const double *e = p + s->nm * s->ns + 3 * em;
                for (int c = 0; c < 3; ++c) phi.v[c] = e[c] * prof * w;
                int base = s->nm * s->ns + 3 * em;
                fadd(&phi, base + 0, prof * w, 0, 0);
                fadd(&phi, base + 1, 0, prof * w, 0);
                fadd(&phi, base + 2, 0, 0, prof * w);
                double tau[3];
                term_grad(a, na, &phi, wc, grad, tau);
                for (int c = 0; c < 3; ++c) L[c] += tau[c];
                if (vd && k - 1 < vd->nv) { double *r = vd->v + VREC * (k - 1); r[4] = L[0]; r[5] = L[1]; r[6] = L[2]; }
            }
            ev |= 1u;
        }
        if (k == D + 1) { h = fnv(h, ev); break; }
        /* --- shading frame: two-sided, flipped toward the viewer --- */
        v3 wo = scl(d, -1.0);
        v3 ns = ng;
        if (s->N) {
            v3 n0 = mk(s->N[3 * (int64_t)f[0]], s->N[3 * (int64_t)f[0] + 1], s->N[3 * (int64_t)f[0] + 2]);
            v3 n1 = mk(s->N[3 * (int64_t)f[1]], s->N[3 * (int64_t)f[1] + 1], s->N[3 * (int64_t)f[1] + 2]);
            v3 n2 = mk(s->N[3 * (int64_t)f[2]], s->N[3 * (int64_t)f[2] + 1], s->N[3 * (int64_t)f[2] + 2]);
            ns = nrm(add(scl(n0, 1.0 - hit.u - hit.v), add(scl(n1, hit.u), scl(n2, hit.v))));
        }
        v3 ngf = ng;
        NEAR(dot(ng, wo));
        if (dot(ng, wo) < 0) { ngf = scl(ng, -1.0); ns = scl(ns, -1.0); }
        NEAR(dot(ns, wo));
        if (dot(ns, wo) <= 0) { h = fnv(h, ev | 2u); break; }   /* shading normal faces away */
        const double *mp = p + s->nm * seg, *msp = sp + s->nm * seg;
        /* Disney: tangent frame from the hit triangle's first edge */
        v3 tx = ns, ty = ns;
        if (s->material == 1) disney_frame(ns, e1, &tx, &ty, M ? &mg : NULL);
        if (ns.z != 0.0) NEAR(ns.z);   /* the tangent frame switches sign convention at n.z = 0 */
        double u[8];
        vertex_uniforms(C->o->seed, C->o->stream_tag, C->o->iteration, path_id, k, u);
        /* --- learned proposal for this vertex (one-sample MIS with the BRDF) --- */
        double gmix[G_OUT];
        const int guided = C->o->guide_w && C->o->guide_mix > 0;
        if (guided && C->o->guide_cell_area > 0) {
            v3 xq, nq;
            cell_query(s, hit.tri, hit.u, hit.v, dot(ng, wo) < 0, (float)C->o->guide_cell_area, &xq, &nq,
                       M ? &mg : NULL);
            guide_eval_vertex(C->o, s->ns, seg, xq, nq, nq, gmix);
        } else if (guided) {
            guide_eval_vertex(C->o, s->ns, seg, x, ns, wo, gmix);
        }
        const double cg = guided ? C->o->guide_mix : 0.0;
        /* --- explicit light sampling (next-event estimation) --- */
        if (mis != 0 && s->nlt > 0) {
            int64_t lj = pick_light(C->L, s->nlt, u[0]);
            if (M) for (int64_t j = 0; j < s->nlt - 1; ++j) NEAR((C->L->cdf[j] - u[0] * C->L->total) / C->L->total);
            int32_t lt = s->light_tri[lj];
            const int32_t *lf = &s->F[3 * (int64_t)lt];
            v3 q0 = vtx(s, lf[0]), q1 = vtx(s, lf[1]), q2 = vtx(s, lf[2]);
            double su = sqrt(u[1]);
            double b1 = (1.0 - u[2]) * su, b2 = u[2] * su;
            /* y - x formed from vertex differences and edge terms (the same
             * vector as (q0 + b1 (q1-q0) + b2 (q2-q0)) - (p0 + u e1 + v e2)) */
            v3 dl = add(sub(q0, p0), add(add(scl(sub(q1, q0), b1), scl(sub(q2, q0), b2)),
                                         scl(add(scl(e1, hit.u), scl(e2, hit.v)), -1.0)));
            v3 lng = nrm(cross(sub(q1, q0), sub(q2, q0)));
            double d2 = dot(dl, dl), dist = sqrt(d2);
            v3 wl = scl(dl, 1.0 / dist);
            double cy = -dot(wl, lng);
            double cxg = dot(wl, ngf);
            uint32_t vis = 0;
            NEAR(cy - 1e-6);
            NEAR(cxg - 1e-6);
            /* Grazing configurations (cosines below 1e-6: the light triangle
             * itself, a coplanar emitter) are skipped: their contribution is ~0
             * and their sign would be decided by rounding. */
            if (cy > 1e-6 && cxg > 1e-6) {
                ohit sh = closest_m(s, x, wl, tmin, dist * (1.0 - 1e-5), hit.tri, lt, C->o->brute_force, M);
                vis = sh.tri < 0;
            }
            ev |= (uint32_t)(lj << 8) | (vis << 2);
            if (vis) {
                double spec = 0, dspec = 0, fl[3], dfl[DS_N][3];
                if (s->material == 1) {
                    dgeom gl = disney_geom(ns, tx, ty, wo, wl);
                    disney_eval(mp, &gl, fl, dfl);
                } else {
                    spec_term(ns, wo, wl, mp[6], &spec, &dspec);
                    for (int c = 0; c < 3; ++c) fl[c] = mp[c] / ORC_PI + mp[3 + c] * spec;
                }
                double cx = dot(ns, wl);
                NEAR(cx);
                if (cx > 0) {
                    int lk = s->seg_emitter[s->seg[lt]];
                    double parea = light_prob(C->L, lj) / s->light_area[lj];
                    double w = 1.0;
                    if (mis >= 2) {
                        double pl = parea * d2 / cy;
                        double pb = s->material == 1 ? disney_pdf(msp, ns, tx, ty, wo, wl) : brdf_pdf(msp, ns, wo, wl);
                        if (guided) pb = cg * mixture_pdf_d(gmix, wl) + (1.0 - cg) * pb;
                        w = mis_w(pl, pb, mis);
                    }
                    double prof = C->o->emission_profile ? cy : 1.0;
                    double g = cx * cy / d2 * w / parea * prof;   /* everything but f and e */
                    const double *e = p + s->nm * s->ns + 3 * lk;
                    factor phi; phi.n = 0;
                    for (int c = 0; c < 3; ++c)
                        phi.v[c] = fl[c] * e[c] * g;
                    int mb = s->nm * seg, eb = s->nm * s->ns + 3 * lk;
                    if (s->material == 1) {
                        for (int j = 0; j < DS_N; ++j)
                            fadd(&phi, mb + j, dfl[j][0] * e[0] * g, dfl[j][1] * e[1] * g, dfl[j][2] * e[2] * g);
                    } else {
                        fadd(&phi, mb + 0, e[0] * g / ORC_PI, 0, 0);
                        fadd(&phi, mb + 1, 0, e[1] * g / ORC_PI, 0);
                        fadd(&phi, mb + 2, 0, 0, e[2] * g / ORC_PI);
                        fadd(&phi, mb + 3, spec * e[0] * g, 0, 0);
                        fadd(&phi, mb + 4, 0, spec * e[1] * g, 0);
                        fadd(&phi, mb + 5, 0, 0, spec * e[2] * g);
                        fadd(&phi, mb + 6, mp[3] * dspec * e[0] * g, mp[4] * dspec * e[1] * g,
                             mp[5] * dspec * e[2] * g);
                    }
                    fadd(&phi, eb + 0, fl[0] * g, 0, 0);
                    fadd(&phi, eb + 1, 0, fl[1] * g, 0);
                    fadd(&phi, eb + 2, 0, 0, fl[2] * g);
                    double tau[3];
                    term_grad(a, na, &phi, wc, grad, tau);
                    for (int c = 0; c < 3; ++c) L[c] += tau[c];
                    if (vd && k - 1 < vd->nv) { double *r = vd->v + VREC * (k - 1); r[4] = L[0]; r[5] = L[1]; r[6] = L[2]; r[7] = 1; }
                if (vd && k - 1 < vd->nv) { double *r = vd->v + VREC * (k - 1); r[4] = L[0]; r[5] = L[1]; r[6] = L[2]; }
                }
            }
        }
        /* --- continue the path by sampling the BRDF --- */
        v3 wi;
        int lobe = 0;
        int ok;
        int use_guide = guided && u[7] < cg;
        if (guided) NEAR(u[7] - cg);
        if (use_guide) {
            wi = mixture_sample_d(gmix, u[3], u[4], u[5], M ? &mg : NULL);
            ok = 1;
            ev |= 64u;
        } else if (s->material == 1) {
            ok = disney_sample(msp, ns, tx, ty, wo, u[3], u[4], u[5], &wi, &lobe, M ? &mg : NULL);
        } else {
            ok = brdf_sample(msp, ns, wo, u[3], u[4], u[5], &wi, &lobe);
        }
        /* lobe in the event hash: 1 at bit 3, 2 (Disney clearcoat) at bit 7 */
        ev |= (uint32_t)(lobe & 1) << 3 | (uint32_t)(lobe >> 1) << 7;
        if (!use_guide && s->material == 1) {
            if (ok) { NEAR(dot(wi, ngf)); NEAR(dot(wi, ns)); }
        } else if (!use_guide) {
            double ps = lobe_prob(msp);
            if (ps > 0 && ps < 1) NEAR(u[3] - ps);
            if (ok) { NEAR(dot(wi, ngf)); NEAR(dot(wi, ns)); }
            if (lobe == 1) { v3 hh = nrm(add(wo, ok ? wi : wo)); NEAR(dot(wo, hh)); }
        }
        if (use_guide && ok) { NEAR(dot(wi, ngf)); NEAR(dot(wi, ns)); }
        if (!ok || dot(wi, ngf) <= 0 || dot(wi, ns) <= 0) { h = fnv(h, ev | 16u); break; }
        double pdf = s->material == 1 ? disney_pdf(msp, ns, tx, ty, wo, wi) : brdf_pdf(msp, ns, wo, wi);
        if (guided) pdf = cg * mixture_pdf_d(gmix, wi) + (1.0 - cg) * pdf;
        if (!(pdf > 0)) { h = fnv(h, ev | 16u); break; }
        double spec = 0, dspec = 0, specs, dspecs, fk[3], fks[3], dfk[DS_N][3];
        if (s->material == 1) {
            dgeom gk = disney_geom(ns, tx, ty, wo, wi);
            disney_eval(mp, &gk, fk, dfk);
            disney_eval(msp, &gk, fks, NULL);
        } else {
            spec_term(ns, wo, wi, mp[6], &spec, &dspec);
            spec_term(ns, wo, wi, msp[6], &specs, &dspecs);
            for (int c = 0; c < 3; ++c) {
                fk[c] = mp[c] / ORC_PI + mp[3 + c] * spec;
                fks[c] = msp[c] / ORC_PI + msp[3 + c] * specs;
            }
        }
        double ci = dot(ns, wi);
        double g = ci / pdf;
        factor *ak = &a[na];
        ak->n = 0;
        for (int c = 0; c < 3; ++c) ak->v[c] = fk[c] * g;
        double ts[3];
        for (int c = 0; c < 3; ++c) ts[c] = fks[c] * g;
        /* Russian roulette on the sampling-parameter throughput (detached). */
        double q = 1.0;
        if (C->o->rr_depth >= 0 && k >= C->o->rr_depth) {
            double m = 0;
            for (int c = 0; c < 3; ++c) { double tc = Ts[c] * ts[c]; if (tc > m) m = tc; }
            q = m < 0.1 ? 0.1 : (m > 0.95 ? 0.95 : m);
            NEAR(u[6] - q);
            if (!(u[6] < q)) { h = fnv(h, ev | 32u); break; }
        }
        g /= q;
        for (int c = 0; c < 3; ++c) { ak->v[c] /= q; Ts[c] *= ts[c] / q; Tc[c] *= ak->v[c]; }
        if (vd && k - 1 < vd->nv) {
            double *r = vd->v + VREC * (k - 1);
            r[8] = Tc[0]; r[9] = Tc[1]; r[10] = Tc[2]; r[11] = pdf;
            r[12] = wi.x; r[13] = wi.y; r[14] = wi.z; r[15] = 1;
        }
        int mb = s->nm * seg;
        if (s->material == 1) {
            /* 1/q of the roulette is a constant factor of every derivative */
            for (int j = 0; j < DS_N; ++j) fadd(ak, mb + j, dfk[j][0] * g, dfk[j][1] * g, dfk[j][2] * g);
        } else {
            fadd(ak, mb + 0, g / ORC_PI, 0, 0);
            fadd(ak, mb + 1, 0, g / ORC_PI, 0);
            fadd(ak, mb + 2, 0, 0, g / ORC_PI);
            fadd(ak, mb + 3, spec * g, 0, 0);
            fadd(ak, mb + 4, 0, spec * g, 0);
            fadd(ak, mb + 5, 0, 0, spec * g);
            fadd(ak, mb + 6, mp[3] * dspec * g, mp[4] * dspec * g, mp[5] * dspec * g);
        }
        na++;
        h = fnv(h, ev);
        prev_pdf = pdf;
        prev_tri = hit.tri;
        o = x; d = wi;
        if (C->pert != 0.0) d = nrm(add(d, scl(C->pert_dir, C->pert)));
    }
    for (int c = 0; c < 3; ++c) Lout[c] = L[c];
    *hash = h;
    if (margin) *margin = mg;
#undef NEAR
}

/* Conditioning probes (parity bookkeeping; they never change a result).
 * Probes 0 and 1 perturb, by a relative -+1e-6 along one fixed direction,
 * every vertex position and every direction of the path.  Probes 2..7 shift
 * only the camera ray's origin, by 1e-6 of its coordinate scale along +-x,
 * +-y, +-z, and let the path's own dynamics carry the change: a hit point
 * that moves on a smoothly shaded curved surface turns its shading normal and
 * so the next direction, which is how float32 rounding grows along chaotic
 * paths (the per-vertex probes alone under-report those paths, because a
 * common shift of every vertex partly cancels the growth). */
#define ORC_NPROBE 8
static void probe_setup(ctx *Cp, int k, v3 org, v3 dir, v3 *o2, v3 *d2)
{
    *o2 = org;
    *d2 = dir;
    if (k < 2) {
        Cp->pert = k == 0 ? 1e-6 : -1e-6;
        Cp->pert_dir = nrm(mk(0.6, -0.48, 0.64));
        *d2 = nrm(add(dir, scl(Cp->pert_dir, Cp->pert)));
        return;
    }
    Cp->pert = 0.0;
    int axis = (k - 2) / 2;
    double sh = ((k - 2) % 2 == 0 ? 1e-6 : -1e-6) * rel_scale(org);
    *o2 = add(org, mk(axis == 0 ? sh : 0.0, axis == 1 ? sh : 0.0, axis == 2 ? sh : 0.0));
}

/* Render (and, when w != NULL and grad != NULL, differentiate) a set of
 * pixels.  image[npix*3] receives the per-pixel mean over spp; grad[P]
 * receives sum_j sum_c (w_jc / spp) d(sum_s L_sc)/dtheta.  path_mask (if not
 * NULL) removes paths from both.  Returns the number of paths dropped for a
 * non-finite contribution. */
int64_t orc_run(const orc_scene *s, const orc_cams *cams, const double *params,
                const double *sampling_params, const orc_opts *o, const double *w,
                const uint8_t *path_mask, double *image, double *grad, uint64_t *hashes,
                double *path_L, double *margins, double *conds, double *vertices, double *gconds)
{
    const double *sp = sampling_params ? sampling_params : params;
    int64_t P = (int64_t)s->nm * s->ns + 3 * (int64_t)s->ne;
    lightdist L = build_lights(s, sp);
    ctx C = { s, params, sp, &L, o, 0.0, { 0, 0, 0 } };
    int64_t npix = o->pixel_list ? o->num_pixels
                                 : (int64_t)cams->num_views * cams->width * cams->height;
    int64_t dropped = 0;
    if (grad) memset(grad, 0, sizeof(double) * (size_t)P);
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    double *gpriv = grad ? (double *)calloc((size_t)nthr * (size_t)P, sizeof(double)) : NULL;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : dropped)
    for (int64_t i = 0; i < npix; ++i) {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *gt = gpriv ? gpriv + (size_t)tid * (size_t)P : NULL;
        int64_t pix = o->pixel_list ? o->pixel_list[i] : i;
        int64_t W = cams->width, H = cams->height;
        int64_t v = pix / (W * H), rem = pix % (W * H);
        int64_t y = rem / W, x = rem % W;
        double acc[3] = { 0, 0, 0 };
        double wc[3] = { 0, 0, 0 };
        if (w) for (int c = 0; c < 3; ++c) wc[c] = w[3 * i + c] / o->spp;
        for (int sidx = 0; sidx < o->spp; ++sidx) {
            uint64_t pid = (uint64_t)pix * (uint64_t)o->spp + (uint64_t)sidx;
            double u[8];
            vertex_uniforms(o->seed, o->stream_tag, o->iteration, pid, 0, u);
            double jx = o->jitter ? u[0] : 0.5, jy = o->jitter ? u[1] : 0.5;
            v3 org, dir;
            camera_ray(cams->cam_to_world + 16 * v, (double)cams->fov_y[v], (int)W, (int)H,
                       (double)x + jx, (double)y + jy, &org, &dir);
            double Lp[3];
            uint64_t hsh;
            int use = path_mask ? path_mask[i * o->spp + sidx] : 1;
            /* gradient into a per-path scratch first, so a non-finite path
             * can be dropped whole */
            double *gp = NULL;
            double gbuf_local[1];
            (void)gbuf_local;
            if (gt && use) gp = (double *)calloc((size_t)P, sizeof(double));
            double mgn = INFINITY;
            vdump vdd;
            vdd.nv = o->max_depth + 1;
            vdd.v = vertices ? vertices + (size_t)(i * o->spp + sidx) * VREC * (size_t)vdd.nv : NULL;
            if (vdd.v) for (int q = 0; q < VREC * vdd.nv; ++q) vdd.v[q] = -1.0;
            trace_path_v(&C, org, dir, pid, wc, gp, Lp, &hsh, margins ? &mgn : NULL, vdd.v ? &vdd : NULL);
            if (margins) margins[i * o->spp + sidx] = mgn;
            if (conds) {
                /* Conditioning of the path: the largest relative change of a
                 * channel of its radiance under the probe perturbations
                 * (infinite if a discrete event changes).  Float32 rounding injects ~1e-7 at
                 * every vertex; paths that amplify such perturbations (e.g.
                 * repeated reflections between curved, smoothly shaded
                 * surfaces diverge exponentially) cannot be reproduced to 1e-4
                 * in float32. */
                double c = 0.0;
                double lm = fmax(fmax(fabs(Lp[0]), fabs(Lp[1])), fabs(Lp[2]));
                for (int k = 0; k < ORC_NPROBE && isfinite(c); ++k) {
                    ctx Cp = C;
                    v3 o2, d2;
                    probe_setup(&Cp, k, org, dir, &o2, &d2);
                    double L2[3];
                    uint64_t h2;
                    trace_path(&Cp, o2, d2, pid, wc, NULL, L2, &h2, NULL);
                    if (h2 != hsh) { c = INFINITY; break; }
                    /* relative change per channel (the comparisons are per
                     * channel), over the channels of at least 1e-3 of the
                     * brightest one, as for the gradient components below */
                    for (int q = 0; q < 3; ++q) {
                        if (fabs(Lp[q]) < 1e-3 * lm) continue;
                        double r = fabs(L2[q] - Lp[q]) / fmax(fabs(Lp[q]), 1e-300);
                        if (r > c) c = r;
                    }
                }
                conds[i * o->spp + sidx] = c;
            }
            if (gconds && w) {
                /* The same probes on the path's gradient contribution: the
                 * largest relative change of any of its components that is at
                 * least 1e-3 of its largest one.  Derivatives of sharp lobes
                 * amplify the perturbation more than the radiance does. */
                double *g0 = (double *)calloc((size_t)P, sizeof(double));
                double *g1 = (double *)calloc((size_t)P, sizeof(double));
                double L0[3], Lq[3];
                uint64_t h0, h1;
                trace_path(&C, org, dir, pid, wc, g0, L0, &h0, NULL);
                double gmax = 0.0;
                for (int64_t q = 0; q < P; ++q) gmax = fmax(gmax, fabs(g0[q]));
                double c = 0.0;
                for (int k = 0; k < ORC_NPROBE && isfinite(c) && gmax > 0.0; ++k) {
                    ctx Cp = C;
                    v3 o2, d2;
                    probe_setup(&Cp, k, org, dir, &o2, &d2);
                    memset(g1, 0, sizeof(double) * (size_t)P);
                    trace_path(&Cp, o2, d2, pid, wc, g1, Lq, &h1, NULL);
                    if (h1 != h0) { c = INFINITY; break; }
                    for (int64_t q = 0; q < P; ++q) {
                        if (fabs(g0[q]) < 1e-3 * gmax) continue;
                        double r = fabs(g1[q] - g0[q]) / fabs(g0[q]);
                        if (r > c) c = r;
                    }
                }
                gconds[i * o->spp + sidx] = c;
                free(g0);
                free(g1);
            }
            int fin = isfinite(Lp[0]) && isfinite(Lp[1]) && isfinite(Lp[2]);
            if (gp) for (int64_t q = 0; q < P && fin; ++q) if (!isfinite(gp[q])) fin = 0;
            if (!fin) { dropped++; Lp[0] = Lp[1] = Lp[2] = 0; }
            if (use && fin) {
                for (int c = 0; c < 3; ++c) acc[c] += Lp[c];
                if (gp) for (int64_t q = 0; q < P; ++q) gt[q] += gp[q];
            }
            if (gp) free(gp);
            if (hashes) hashes[i * o->spp + sidx] = hsh;
            if (path_L) for (int c = 0; c < 3; ++c) path_L[3 * (i * o->spp + sidx) + c] = Lp[c];
        }
        if (image) for (int c = 0; c < 3; ++c) image[3 * i + c] = acc[c] / o->spp;
    }
    if (grad) {
        for (int t = 0; t < nthr; ++t)
            for (int64_t q = 0; q < P; ++q) grad[q] += gpriv[(size_t)t * (size_t)P + q];
        free(gpriv);
    }
    free(L.cdf);
    return dropped;
}

/* Light-selection probabilities per emitter triangle (for tests). */
void orc_light_probs(const orc_scene *s, const double *sampling_params, double *out)
{
    lightdist L = build_lights(s, sampling_params);
    for (int64_t j = 0; j < s->nlt; ++j) out[j] = light_prob(&L, j);
    free(L.cdf);
}

/* ------------------------------------------------------------------------- */
/* Loss and adjoint image (Sec. 3.2 Eq. 3, Sec. 3.3 Eq. 4).  kind 0: L2 mean  */
/* squared error over all pixels and channels; kind 1: the paper's L1.        */
/* The adjoint is dE/dI (the sign in Eq. 4 as printed is that of -dE/dI).     */
/* ------------------------------------------------------------------------- */
double orc_loss_adjoint(const double *img, const double *target, int64_t n3, int kind, double *w)
{
    double E = 0;
    for (int64_t i = 0; i < n3; ++i) {
        double r = img[i] - target[i];
        if (kind == 0) {
            E += r * r;
            if (w) w[i] = 2.0 * r / (double)n3;
        } else {
            E += fabs(r);
            if (w) w[i] = (r > 0 ? 1.0 : (r < 0 ? -1.0 : 0.0)) / (double)n3;
        }
    }
    return E / (double)n3;
}

/* ------------------------------------------------------------------------- */
/* Adam (Kingma & Ba 2015; Sec. 4.5) on normalised parameters theta = p/scale */
/* with bias correction, followed by a clamp of theta to [lo, hi].  Entries   */
/* with trainable[i] == 0 are left as they are.  step counts from 1.          */
/* ------------------------------------------------------------------------- */
void orc_adam(double *params, const double *grad, double *m, double *v, int64_t n, int step,
              double lr, double b1, double b2, double eps, const double *scale, const double *lo,
              const double *hi, const uint8_t *trainable)
{
    double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
    for (int64_t i = 0; i < n; ++i) {
        if (trainable && !trainable[i]) continue;
        double sc = scale ? scale[i] : 1.0;
        double g = grad[i] * sc;
        m[i] = b1 * m[i] + (1.0 - b1) * g;
        v[i] = b2 * v[i] + (1.0 - b2) * g * g;
        double mh = m[i] / c1, vh = v[i] / c2;
        double th = params[i] / sc - lr * mh / (sqrt(vh) + eps);
        if (lo && th < lo[i]) th = lo[i];
        if (hi && th > hi[i]) th = hi[i];
        params[i] = th * sc;
    }
}

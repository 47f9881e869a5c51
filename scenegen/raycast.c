/*
 * FP64 ray caster for the seeded synthetic test scenes.
 *
 * This is an input generator only: it produces the G-buffer (linear view
 * depth + view-space normals), the per-pixel object id and the light-view
 * depth map that both the CPU oracle and the HIP path consume.  It holds none
 * of the multi-resolution method's arithmetic.
 *
 * Scene: an infinite ground plane y = 0, axis-aligned boxes resting on it and
 * spheres resting on it.  Nearest hit wins; ties go to the lowest object
 * index (plane first, then boxes, then spheres).
 *
 * Camera model (pinhole): pixel (x, y), row 0 at the top, has its centre ray
 * along ((x + 0.5 - cx)/f, (cy - (y + 0.5))/f, -1) in view space, with
 * cx = W/2, cy = H/2.  The view basis is given as three world-space unit
 * vectors (right, up, back); the eye looks along -back.  Since the view-space
 * ray has z = -1 the hit parameter t equals the linear view depth.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no -march flags,
 * so results do not depend on the host's vector extensions).
 */
#include <math.h>
#include <stdint.h>

typedef struct {
    double eye[3];
    double right[3], up[3], back[3];
} rc_view;

static inline double dot3(const double* a, const double* b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Scene bounding box test: returns 1 if the ray segment [0, tmax] meets the
 * box [lo, hi].  Used only to skip object tests for rays that cannot hit. */
static int hits_aabb(const double* o, const double* d, const double* lo,
                     const double* hi, double tmax) {
    double t0 = 0.0, t1 = tmax;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (o[a] < lo[a] || o[a] > hi[a]) return 0;
            continue;
        }
        double inv = 1.0 / d[a];
        double ta = (lo[a] - o[a]) * inv, tb = (hi[a] - o[a]) * inv;
        if (ta > tb) { double s = ta; ta = tb; tb = s; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
        if (t0 > t1) return 0;
    }
    return 1;
}

/*
 * Trace one world-space ray (origin o, direction d, not normalised).
 * boxes: nb x 6 doubles (xmin, ymin, zmin, xmax, ymax, zmax)
 * spheres: ns x 4 doubles (cx, cy, cz, r)
 * Returns object id (-1 miss, 0 plane, 1..nb boxes, nb+1..nb+ns spheres),
 * writes hit parameter and world normal.
 */
static int trace(const double* o, const double* d, const double* boxes, int nb,
                 const double* spheres, int ns, const double* slo,
                 const double* shi, double* t_out, double* n_out) {
    double best = INFINITY;
    int id = -1;
    double n[3] = {0, 0, 0};
    if (d[1] < 0.0 && o[1] > 0.0) {
        double t = -o[1] / d[1];
        if (t > 0.0) { best = t; id = 0; n[0] = 0; n[1] = 1; n[2] = 0; }
    }
    if ((nb > 0 || ns > 0) && hits_aabb(o, d, slo, shi, best)) {
        for (int b = 0; b < nb; ++b) {
            const double* bx = boxes + 6 * b;
            double t0 = -INFINITY, t1 = INFINITY;
            int ax0 = -1;
            double sgn0 = 0;
            int miss = 0;
            for (int a = 0; a < 3; ++a) {
                if (d[a] == 0.0) {
                    if (o[a] < bx[a] || o[a] > bx[3 + a]) { miss = 1; break; }
                    continue;
                }
                double inv = 1.0 / d[a];
                double ta = (bx[a] - o[a]) * inv, tb = (bx[3 + a] - o[a]) * inv;
                double sa = -1.0; /* entering through the min face */
                if (ta > tb) { double s = ta; ta = tb; tb = s; sa = 1.0; }
                if (ta > t0) { t0 = ta; ax0 = a; sgn0 = sa; }
                if (tb < t1) t1 = tb;
            }
            if (miss || t0 > t1 || t0 <= 0.0 || ax0 < 0) continue;
            if (t0 < best) {
                best = t0; id = 1 + b;
                n[0] = n[1] = n[2] = 0.0; n[ax0] = sgn0;
            }
        }
        for (int s = 0; s < ns; ++s) {
            const double* sp = spheres + 4 * s;
            double oc[3] = {o[0] - sp[0], o[1] - sp[1], o[2] - sp[2]};
            double A = dot3(d, d), B = dot3(oc, d), C = dot3(oc, oc) - sp[3] * sp[3];
            double disc = B * B - A * C;
            if (disc < 0.0) continue;
            double t = (-B - sqrt(disc)) / A;
            if (t <= 0.0) continue;
            if (t < best) {
                best = t; id = 1 + nb + s;
                for (int a = 0; a < 3; ++a) n[a] = (o[a] + t * d[a] - sp[a]) / sp[3];
            }
        }
    }
    *t_out = best;
    n_out[0] = n[0]; n_out[1] = n[1]; n_out[2] = n[2];
    return id;
}

static void scene_bounds(const double* boxes, int nb, const double* spheres,
                         int ns, double* lo, double* hi) {
    for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
    for (int b = 0; b < nb; ++b)
        for (int a = 0; a < 3; ++a) {
            if (boxes[6 * b + a] < lo[a]) lo[a] = boxes[6 * b + a];
            if (boxes[6 * b + 3 + a] > hi[a]) hi[a] = boxes[6 * b + 3 + a];
        }
    for (int s = 0; s < ns; ++s)
        for (int a = 0; a < 3; ++a) {
            double c = spheres[4 * s + a], r = spheres[4 * s + 3];
            if (c - r < lo[a]) lo[a] = c - r;
            if (c + r > hi[a]) hi[a] = c + r;
        }
    for (int a = 0; a < 3; ++a) { lo[a] -= 1e-9; hi[a] += 1e-9; }
}

/*
 * Render a G-buffer.  view: 12 doubles (eye, right, up, back).  focal: the
 * focal length in pixels (the caller passes the FP32-rounded value so that
 * the image agrees with the camera the lighting code uses).
 * depth: f32[H][W] (+inf where nothing is hit), normal: f32[3][H][W] view
 * space, objid: int32[H][W].
 */
void rc_gbuffer(const double* view, int W, int H, double focal,
                const double* boxes, int nb, const double* spheres, int ns,
                float* depth, float* normal, int32_t* objid) {
    const double* eye = view;
    const double* right = view + 3;
    const double* up = view + 6;
    const double* back = view + 9;
    double lo[3], hi[3];
    scene_bounds(boxes, nb, spheres, ns, lo, hi);
    const double cx = 0.5 * W, cy = 0.5 * H;
    const long plane = (long)W * H;
#pragma omp parallel for schedule(dynamic, 4)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            double dv[3] = {(x + 0.5 - cx) / focal, (cy - (y + 0.5)) / focal, -1.0};
            double d[3];
            for (int a = 0; a < 3; ++a)
                d[a] = right[a] * dv[0] + up[a] * dv[1] + back[a] * dv[2];
            double t, nw[3];
            int id = trace(eye, d, boxes, nb, spheres, ns, lo, hi, &t, nw);
            long p = (long)y * W + x;
            objid[p] = id;
            if (id < 0) {
                depth[p] = INFINITY;
                normal[p] = 0.0f; normal[plane + p] = 0.0f; normal[2 * plane + p] = 1.0f;
                continue;
            }
            depth[p] = (float)t;
            normal[p] = (float)dot3(nw, right);
            normal[plane + p] = (float)dot3(nw, up);
            normal[2 * plane + p] = (float)dot3(nw, back);
        }
    }
}

/*
 * Render the linear depth seen from a square light camera (size x size,
 * focal in texels, principal point at size/2): f32[size][size], +inf on miss.
 */
void rc_depthmap(const double* view, int size, double focal,
                 const double* boxes, int nb, const double* spheres, int ns,
                 float* depth) {
    const double* eye = view;
    const double* right = view + 3;
    const double* up = view + 6;
    const double* back = view + 9;
    double lo[3], hi[3];
    scene_bounds(boxes, nb, spheres, ns, lo, hi);
    const double c = 0.5 * size;
#pragma omp parallel for schedule(dynamic, 4)
    for (int y = 0; y < size; ++y) {
        for (int x = 0; x < size; ++x) {
            double dv[3] = {(x + 0.5 - c) / focal, (c - (y + 0.5)) / focal, -1.0};
            double d[3];
            for (int a = 0; a < 3; ++a)
                d[a] = right[a] * dv[0] + up[a] * dv[1] + back[a] * dv[2];
            double t, nw[3];
            int id = trace(eye, d, boxes, nb, spheres, ns, lo, hi, &t, nw);
            depth[(long)y * size + x] = id < 0 ? INFINITY : (float)t;
        }
    }
}

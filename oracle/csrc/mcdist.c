/*
 * FP64 CPU reference for surface extraction and mesh distance.
 *
 * TEST INFRASTRUCTURE ONLY: nothing in the product library links or calls this
 * file.  It shares no code, table or header with the HIP path.
 *
 * Coordinates are "grid units": cell centre (i,j,k) sits at (i,j,k).  The dual
 * lattice cube (i,j,k) has its 8 corners at the cell centres (i+dx, j+dy, k+dz),
 * dx,dy,dz in {0,1}; corner bit b = dx + 2 dy + 4 dz.
 *
 * Marching Cubes (paper, Sec. 2.4, Eq. 27-28).  A corner is "in" iff chi < c.
 * Edge numbering: edges along x are 0..3 (index dy + 2 dz), along y 4..7
 * (4 + dx + 2 dz), along z 8..11 (8 + dx + 2 dy).  The vertex on a crossing
 * edge from corner q1 (lower end) to q2 is q1 + eta (q2 - q1) with
 * eta = (c - chi1) / (chi2 - chi1).
 *
 * Triangles come from a rule applied per cube at run time (no stored table):
 *  - on every cube face, join the crossing edges of that face by segments;
 *    a face with 4 crossings pairs the two edges around each "in" corner;
 *  - every crossing edge then has exactly two segment neighbours, so the
 *    segments form closed loops; a loop is started at its lowest unvisited
 *    edge id and walked first towards the lower-numbered neighbour;
 *  - each loop (v0, v1, ..., vL-1) is fanned into (v0, vi, vi+1).
 *
 * Point-triangle distance (Sec. 2.4, Eq. 33): project the point onto the
 * triangle's plane; if the projection lies inside the triangle the distance is
 * the distance to the plane, otherwise it is the smallest distance to the three
 * edges (segments, which include the vertices).  Zero-area triangles use the
 * edges only.  The minimum over all triangles is brute force; ties keep the
 * lowest triangle index.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static void edge_ends(int e, int *b0, int *b1, int *axis)
{
    if (e < 4) {            /* along x: dy = e&1, dz = e>>1 */
        int dy = e & 1, dz = e >> 1;
        *b0 = 2 * dy + 4 * dz; *b1 = *b0 + 1; *axis = 0;
    } else if (e < 8) {     /* along y: dx = (e-4)&1, dz = (e-4)>>1 */
        int dx = (e - 4) & 1, dz = (e - 4) >> 1;
        *b0 = dx + 4 * dz; *b1 = *b0 + 2; *axis = 1;
    } else {                /* along z: dx = (e-8)&1, dy = (e-8)>>1 */
        int dx = (e - 8) & 1, dy = (e - 8) >> 1;
        *b0 = dx + 2 * dy; *b1 = *b0 + 4; *axis = 2;
    }
}

static int corner_coord(int b, int axis) { return (b >> axis) & 1; }

/* Triangles of one cube from its 8 corner flags.  Returns the count and
 * writes edge triples into tri[3*k]. */
static int cube_triangles(const int in[8], int tri[][3])
{
    int cross[12], nb[12][2], nnb[12];
    for (int e = 0; e < 12; ++e) {
        int b0, b1, ax;
        edge_ends(e, &b0, &b1, &ax);
        cross[e] = in[b0] != in[b1];
        nnb[e] = 0;
    }
    /* faces: axis a, side s */
    for (int a = 0; a < 3; ++a) {
        for (int s = 0; s < 2; ++s) {
            int fe[4], nf = 0;
            for (int e = 0; e < 12; ++e) {
                int b0, b1, ax;
                edge_ends(e, &b0, &b1, &ax);
                if (ax != a && corner_coord(b0, a) == s && corner_coord(b1, a) == s)
                    fe[nf++] = e;
            }
            int fc[4], ncross = 0;
            for (int i = 0; i < 4; ++i)
                if (cross[fe[i]]) fc[ncross++] = fe[i];
            if (ncross == 2) {
                nb[fc[0]][nnb[fc[0]]++] = fc[1];
                nb[fc[1]][nnb[fc[1]]++] = fc[0];
            } else if (ncross == 4) {
                /* pair the two face edges that meet at each "in" corner */
                for (int b = 0; b < 8; ++b) {
                    if (corner_coord(b, a) != s || !in[b]) continue;
                    int pair[2], np = 0;
                    for (int i = 0; i < 4; ++i) {
                        int b0, b1, ax;
                        edge_ends(fe[i], &b0, &b1, &ax);
                        if (b0 == b || b1 == b) pair[np++] = fe[i];
                    }
                    nb[pair[0]][nnb[pair[0]]++] = pair[1];
                    nb[pair[1]][nnb[pair[1]]++] = pair[0];
                }
            }
        }
    }
    int visited[12] = {0};
    int ntri = 0;
    for (int start = 0; start < 12; ++start) {
        if (!cross[start] || visited[start]) continue;
        int loop[12], L = 0;
        loop[L++] = start;
        visited[start] = 1;
        int prev = start;
        int cur = nb[start][0] < nb[start][1] ? nb[start][0] : nb[start][1];
        while (cur != start) {
            loop[L++] = cur;
            visited[cur] = 1;
            int next = (nb[cur][0] == prev) ? nb[cur][1] : nb[cur][0];
            prev = cur;
            cur = next;
        }
        for (int i = 1; i + 1 < L; ++i) {
            tri[ntri][0] = loop[0];
            tri[ntri][1] = loop[i];
            tri[ntri][2] = loop[i + 1];
            ++ntri;
        }
    }
    return ntri;
}

/* Triangles of case `cs` (bit b set = corner b in) as edge triples; returns count. */
int oracle_mc_case(int cs, int *edges_out)
{
    int in[8], tri[16][3];
    for (int b = 0; b < 8; ++b) in[b] = (cs >> b) & 1;
    int n = cube_triangles(in, tri);
    for (int t = 0; t < n; ++t)
        for (int k = 0; k < 3; ++k) edges_out[3 * t + k] = tri[t][k];
    return n;
}

/*
 * Marching Cubes over the dual lattice of an (nx,ny,nz) cell-centred field
 * chi (x fastest).  Cubes are visited in linear order (i fastest), triangles
 * within a cube in rule order.  Writes at most max_tris triangles:
 *   tri_cube[3t..]  cube (i,j,k),
 *   tri_edge[3t..]  local edge ids,
 *   tri_xyz[9t..]   the three vertices in grid units.
 * Returns the total triangle count (call with max_tris = 0 to size buffers).
 */
int64_t oracle_mc(const double *chi, int nx, int ny, int nz, double c, int64_t max_tris,
                  int32_t *tri_cube, int32_t *tri_edge, double *tri_xyz)
{
    int64_t count = 0;
    for (int k = 0; k + 1 < nz; ++k)
        for (int j = 0; j + 1 < ny; ++j)
            for (int i = 0; i + 1 < nx; ++i) {
                double v[8];
                int in[8];
                for (int b = 0; b < 8; ++b) {
                    int dx = b & 1, dy = (b >> 1) & 1, dz = (b >> 2) & 1;
                    v[b] = chi[(i + dx) + (int64_t)nx * ((j + dy) + (int64_t)ny * (k + dz))];
                    in[b] = v[b] < c;
                }
                int tri[16][3];
                int n = cube_triangles(in, tri);
                for (int t = 0; t < n; ++t, ++count) {
                    if (count >= max_tris) continue;
                    tri_cube[3 * count + 0] = i;
                    tri_cube[3 * count + 1] = j;
                    tri_cube[3 * count + 2] = k;
                    for (int q = 0; q < 3; ++q) {
                        int e = tri[t][q], b0, b1, ax;
                        edge_ends(e, &b0, &b1, &ax);
                        double eta = (c - v[b0]) / (v[b1] - v[b0]);
                        double pos[3] = {i + (b0 & 1), j + ((b0 >> 1) & 1), k + ((b0 >> 2) & 1)};
                        pos[ax] += eta;
                        tri_edge[3 * count + q] = e;
                        for (int d = 0; d < 3; ++d) tri_xyz[9 * count + 3 * q + d] = pos[d];
                    }
                }
            }
    return count;
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* squared distance from p to segment [a,b]; t = parameter of the closest point */
static double seg_dist2(const double *p, const double *a, const double *b, double *t_out)
{
    double ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double ap[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
    double l2 = dot3(ab, ab);
    double t = l2 > 0.0 ? dot3(ap, ab) / l2 : 0.0;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    double d[3] = {ap[0] - t * ab[0], ap[1] - t * ab[1], ap[2] - t * ab[2]};
    *t_out = t;
    return dot3(d, d);
}

/* squared distance from p to triangle (a,b,c) and the barycentric coordinates
 * (w_a, w_b, w_c) of the closest point. */
static double tri_dist2(const double *p, const double *a, const double *b, const double *c,
                        double bary[3])
{
    double v0[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double v1[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double v2[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
    double d00 = dot3(v0, v0), d01 = dot3(v0, v1), d11 = dot3(v1, v1);
    double d20 = dot3(v2, v0), d21 = dot3(v2, v1);
    double den = d00 * d11 - d01 * d01;
    if (den > 1e-24 * d00 * d11 && den > 0.0) {
        /* barycentrics of the projection of p onto the plane (the normal
         * component of v2 is orthogonal to v0, v1 and drops out) */
        double wb = (d11 * d20 - d01 * d21) / den;
        double wc = (d00 * d21 - d01 * d20) / den;
        double wa = 1.0 - wb - wc;
        if (wa >= 0.0 && wb >= 0.0 && wc >= 0.0) {
            double q[3];
            for (int k = 0; k < 3; ++k) q[k] = p[k] - (a[k] + wb * v0[k] + wc * v1[k]);
            bary[0] = wa; bary[1] = wb; bary[2] = wc;
            return dot3(q, q);
        }
    }
    /* outside (or zero area): nearest of the three edges */
    double t, best, d;
    best = seg_dist2(p, a, b, &t);
    bary[0] = 1.0 - t; bary[1] = t; bary[2] = 0.0;
    d = seg_dist2(p, b, c, &t);
    if (d < best) { best = d; bary[0] = 0.0; bary[1] = 1.0 - t; bary[2] = t; }
    d = seg_dist2(p, c, a, &t);
    if (d < best) { best = d; bary[0] = t; bary[1] = 0.0; bary[2] = 1.0 - t; }
    return best;
}

/*
 * Brute-force unsigned distance from m points to a triangle soup (grid units).
 * dist[i] = min_t |p_i - T_t|, arg[i] = lowest index reaching it,
 * bary[3i..] = barycentric coordinates of the closest point on T_arg.
 */
void oracle_mesh_distance(int64_t m, const double *pts, int64_t ntri, const double *tri,
                          double *dist, int64_t *arg, double *bary)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < m; ++i) {
        const double *p = pts + 3 * i;
        double best = INFINITY, bb[3] = {0, 0, 0}, cb[3];
        int64_t ba = -1;
        for (int64_t t = 0; t < ntri; ++t) {
            const double *T = tri + 9 * t;
            double d2 = tri_dist2(p, T, T + 3, T + 6, cb);
            if (d2 < best) { best = d2; ba = t; bb[0] = cb[0]; bb[1] = cb[1]; bb[2] = cb[2]; }
        }
        dist[i] = sqrt(best);
        arg[i] = ba;
        bary[3 * i + 0] = bb[0]; bary[3 * i + 1] = bb[1]; bary[3 * i + 2] = bb[2];
    }
}

/*
 * Crossing-number inside/outside test (the parity rule of Sec. 2.2 applied to
 * the extracted mesh): count intersections of the ray p + s*dir, s > 0, with
 * every non-degenerate triangle; odd = inside.  Writes 1 for inside, 0 outside.
 */
void oracle_ray_parity(int64_t m, const double *pts, int64_t ntri, const double *tri,
                       const double dir[3], int32_t *inside)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < m; ++i) {
        const double *p = pts + 3 * i;
        int hits = 0;
        for (int64_t t = 0; t < ntri; ++t) {
            const double *a = tri + 9 * t, *b = a + 3, *c = a + 6;
            double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
            double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
            double pv[3] = {dir[1] * e2[2] - dir[2] * e2[1], dir[2] * e2[0] - dir[0] * e2[2],
                            dir[0] * e2[1] - dir[1] * e2[0]};
            double det = dot3(e1, pv);
            if (fabs(det) < 1e-300) continue;
            double inv = 1.0 / det;
            double tv[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
            double u = dot3(tv, pv) * inv;
            if (u < 0.0 || u > 1.0) continue;
            double qv[3] = {tv[1] * e1[2] - tv[2] * e1[1], tv[2] * e1[0] - tv[0] * e1[2],
                            tv[0] * e1[1] - tv[1] * e1[0]};
            double v = dot3(dir, qv) * inv;
            if (v < 0.0 || u + v > 1.0) continue;
            double s = dot3(e2, qv) * inv;
            if (s > 0.0) ++hits;
        }
        inside[i] = hits & 1;
    }
}

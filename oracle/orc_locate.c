/* Oracle (test infrastructure): particle tracking on the grid (Sec. I, role
 * (iii)) with the particle boundary conditions.
 *
 *  R-12 walk: in element e compute lambda (R-05); if min lambda >= 0 stop;
 *       otherwise cross the edge k* = argmin lambda (ties -> smallest k);
 *       at most 64 walk iterations. A step straight back into the element
 *       just left (possible only through rounding on their shared edge) ends
 *       the walk in whichever of the two has the larger min lambda.
 *  R-14 wall (no-slip imposed on particles only, Sec. I): mirror X across the
 *       wall edge line, U <- 2 U_wall - U for all three components, stay in
 *       the element; at most 8 reflections per step.
 *  R-15 periodic edge: X <- X + shift, move to the partner element.
 *  R-13 fallback: lowest-index element that contains X; if none, the element
 *       maximising min lambda (ties -> lowest index), X unchanged.
 */
#include "orc_internal.h"
#include <math.h>

#define WALK_CAP 64
#define REFLECT_CAP 8

static double min3(const double l[3]) { double m = l[0]; if (l[1] < m) m = l[1]; if (l[2] < m) m = l[2]; return m; }

int orc_brute(const omesh* m, double x, double y)
{
    int best = -1; double bestv = 0.0;
    for (int e = 0; e < m->ne; ++e) {
        double l[3];
        omesh_bary(m, e, x, y, l);
        double v = min3(l);
        if (v >= 0.0) return e;
        if (best < 0 || v > bestv) { best = e; bestv = v; }
    }
    return best;
}

/* returns the element; updates x, y and u3 (reflections). Counters are
 * accumulated into cs->cnt. */
int orc_walk_case(ocase* cs, int e0, double* px, double* py, double u3[3])
{
    const omesh* m = &cs->m;
    double x = *px, y = *py;
    if (!isfinite(x) || !isfinite(y)) {
        cs->cnt[CNT_NAN]++;
        return e0;
    }
    int e = e0, nrefl = 0;
    int prev = -1;                       /* element left by the last crossing */
    double prev_min = 0.0, prev_x = 0.0, prev_y = 0.0;
    for (int it = 0; it < WALK_CAP; ++it) {
        double l[3];
        omesh_bary(m, e, x, y, l);
        int k = 0;
        if (l[1] < l[k]) k = 1;
        if (l[2] < l[k]) k = 2;
        if (l[k] >= 0.0) { *px = x; *py = y; return e; }
        int nb = m->nbr[3 * e + k];
        const orc_bc* bc = nb >= 0 ? NULL : &m->bc[m->tag[3 * e + k]];
        int next = nb >= 0 ? nb : (bc->type == ORC_BC_PERIODIC ? m->partner[3 * e + k] : e);
        if (next == prev && next != e) {
            /* two-cycle across one edge: only rounding on that edge can cause
             * it; keep the element with the larger min lambda (R-12) */
            if (prev_min > l[k]) { *px = prev_x; *py = prev_y; return prev; }
            *px = x; *py = y;
            return e;
        }
        cs->cnt[CNT_WALK_STEPS]++;
        if (nb >= 0) { prev = e; prev_min = l[k]; prev_x = x; prev_y = y; e = nb; continue; }
        if (bc->type == ORC_BC_PERIODIC) {
            prev = e; prev_min = l[k]; prev_x = x; prev_y = y;
            x = x + bc->shift[0];
            y = y + bc->shift[1];
            e = m->partner[3 * e + k];
            cs->cnt[CNT_PERIODIC]++;
            continue;
        }
        prev = -1;
        /* wall */
        if (nrefl == REFLECT_CAP) break;
        int a = m->tri[3 * e + (k + 1) % 3], b = m->tri[3 * e + (k + 2) % 3];
        double xa = m->x[a], ya = m->y[a];
        double dx = m->x[b] - xa, dy = m->y[b] - ya;
        double L = sqrt(dx * dx + dy * dy);
        double nx = dy / L, ny = -dx / L;
        double d = (x - xa) * nx + (y - ya) * ny;
        x = x - (2.0 * d) * nx;
        y = y - (2.0 * d) * ny;
        for (int i = 0; i < 3; ++i) u3[i] = 2.0 * bc->u_wall[i] - u3[i];
        nrefl++;
        cs->cnt[CNT_REFLECT]++;
    }
    /* fallback */
    cs->cnt[CNT_WALK_FALLBACK]++;
    *px = x; *py = y;
    return orc_brute(m, x, y);
}

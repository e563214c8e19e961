/*
 * arc_oracle.c -- plain FP64 CPU oracle for the adaptive HEALPix ray-tracing
 * radiative-transfer step of Hartley & Ricotti (arXiv:1807.07094).
 *
 * TEST INFRASTRUCTURE ONLY: it is the yardstick the GPU library is checked
 * against, and it is deliberately slow and literal. Only the test-suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it.
 *
 * What it follows
 *   - Section 2.1 (program design), steps (iii a-d): per source, root rays at radius 0
 *     and zero optical depth; each ray is traced until it splits, terminates or leaves
 *     the volume; a split makes four children at the next HEALPix level that start at
 *     the parent's radius and keep the parent's optical depth.
 *   - Section 2.2: polychromatic packets, one optical depth per frequency bin summed
 *     over all absorbing species.
 *   - Section 2.4 and eq:ion: cell-by-cell stepping to the next x, y or z boundary; the
 *     photons a ray loses in a cell, S (1 - exp(-dtau)), are deposited there and
 *     removed from the ray, so photons are conserved.
 *   - Section 2.7 (eq:diffeq, eq:anninos, sub-cycle step) and section 2.8 for the
 *     chemistry and energy update.
 *
 * Readings of points the paper leaves open:
 *   - Split radius: a level-l ray subtends 4 pi/(12 4^l) sr and splits once its
 *     cross-section exceeds one cell face over Phi (Phi = rays per cell area, fig. 1 and
 *     the methodology test), i.e. at r = 2^l sqrt(3/(pi Phi)) cells. The base value is
 *     rounded once to float; levels beyond the one whose split radius exceeds the box
 *     diagonal do not split.
 *   - Directions are the HEALPix pixel centres rounded to float (not renormalised); the
 *     ray is x(t) = xs + t d with t taken as the path length in cells.
 *   - Children start at xs + t_split * d_child, not at the parent's end point.
 *   - Per-ray rate: S_b / (12 4^l) exp(-tau_b) (section 2.4, equal solid angles).
 *   - Termination: after a crossing in which every bin has tau_b >= -ln(eps_term) and
 *     every bin's dtau_b >= 0.01, the remaining photons are absorbed in that cell, so
 *     emitted = absorbed + escaped stays exact. Photons that leave the box are lost.
 *   - Species split inside a bin in proportion to each species' optical depth.
 *   - Optically thin approximation (section 2.6, optional): a source's radius R is given
 *     (from the previous step; 0 turns it off) and rounded to float like the split radii.
 *     Cells whose centre lies within R get the point-source field S_b / (4 pi r^2) of
 *     every bin, r being the distance of the cell centre in cells, taken as at least half a
 *     cell (the point formula diverges in the source's own cell); no absorption inside R.
 *     Rays start at radius R with zero optical depth, at the level whose split radius lies
 *     beyond R (rays of lower levels split at once, without crossing a cell). The new
 *     R_tau<0.1 is the least path length at which any ray's optical depth in the softest
 *     bin reaches 0.1 (inside the crossing where it does, the depth growing linearly), a
 *     ray that leaves the box (or starts outside it) below 0.1 counting its length there.
 *   - Tie rules: along an axis with d > 0 a point on a boundary belongs to the upper
 *     cell, with d < 0 to the lower cell, with d = 0 to the upper cell; boundaries
 *     reached at exactly the same t are crossed together.
 *   - Every geometric decision is made exactly: positions lie on a 2^-12 lattice and
 *     directions and split radii are floats, so every product compared below has at
 *     most 48 significant bits and is exact in double.
 *   - Geometric correction (section 2.5, optional): D_edge is the distance from the
 *     midpoint of the segment to the nearest face of its cell and L_Pix the width of
 *     the ray's pixel there, r_mid sqrt(4 pi / N_pix). f_c scales everything the
 *     crossing deposits in its cell (the termination remainder included). With the
 *     secondary correction the removed share goes to the neighbour across that face,
 *     scaled by the ratio of the two cells' opacities in the bin (eq:correction2's
 *     absorber ratio, read as a density ratio, per bin), which conserves photons; if
 *     that neighbour is outside the grid, or holds no absorber of the bin (zero
 *     opacity: the ratio has no value), the share stays. Faces within 1e-9 cell of
 *     each other count as tied; ties go to the lower axis, then to the lower face (a
 *     tie rule: the nearest face of a midpoint that lies on a cell's diagonal plane is
 *     not unique, and symmetric geometries put midpoints exactly there).
 */
#include "arc_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846
#define ORC_MAXB 8
#define ORC_DTAU_TERM_MIN 0.01
/* Face distances that agree within this many cells count as tied (symmetric geometries
 * tie exactly, and the last bits of a midpoint depend on how its path length is summed). */
#define ORC_FACE_TIE 1e-9

static const double KB_ERG = 1.380649e-16;     /* Boltzmann constant [erg/K] */
static const double EV_ERG = 1.602176634e-12;  /* electron volt [erg] */

/* ------------------------------------------------------------------------------ */
/* HEALPix, nested scheme (Gorski et al. 2005).                                     */
/* ------------------------------------------------------------------------------ */

int64_t orc_npix(int32_t level) { return (int64_t)12 << (2 * level); }

/* Split a nested index into its base face and the (x, y) position inside the face;
 * inside a face the nested index interleaves the bits of x (even) and y (odd). */
static void nest_face_xy(int32_t level, int64_t pix, int* face, int64_t* ix, int64_t* iy)
{
    const int64_t per_face = (int64_t)1 << (2 * level);
    *face = (int)(pix / per_face);
    const int64_t in_face = pix % per_face;
    int64_t x = 0, y = 0;
    for (int bit = 0; bit < level; ++bit) {
        x |= ((in_face >> (2 * bit)) & 1) << bit;
        y |= ((in_face >> (2 * bit + 1)) & 1) << bit;
    }
    *ix = x;
    *iy = y;
}

void orc_healpix_vec(int32_t level, int64_t pix, double v[3])
{
    /* Layout of the 12 base faces: the ring (in units of Nside) holding each face's
     * southern corner, and the longitude index of that corner in units of pi/4. */
    static const int face_ring[12] = {2, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4};
    static const int face_lon[12] = {1, 3, 5, 7, 0, 2, 4, 6, 1, 3, 5, 7};
    int face;
    int64_t ix, iy;
    nest_face_xy(level, pix, &face, &ix, &iy);
    const int64_t ns = (int64_t)1 << level;

    /* Ring index counted from the north pole, 1 .. 4 Nside - 1. */
    const int64_t ring = face_ring[face] * ns - ix - iy - 1;
    int64_t nr;      /* pixels per ring quadrant */
    int shift;       /* 1 when the ring's pixel centres are offset by half a pixel */
    double z;
    if (ring < ns) {                 /* north polar cap: z = 1 - i^2 / (3 Nside^2) */
        nr = ring;
        shift = 0;
        z = (double)(3 * ns * ns - nr * nr) / (double)(3 * ns * ns);
    } else if (ring > 3 * ns) {      /* south polar cap, mirror image */
        nr = 4 * ns - ring;
        shift = 0;
        z = -(double)(3 * ns * ns - nr * nr) / (double)(3 * ns * ns);
    } else {                         /* equatorial belt: z = 4/3 - 2 i / (3 Nside) */
        nr = ns;
        shift = (int)((ring - ns) & 1);
        z = (double)(2 * (2 * ns - ring)) / (double)(3 * ns);
    }
    /* Pixel number inside the ring, 1 .. 4 nr. */
    int64_t j = (face_lon[face] * nr + ix - iy + 1 + shift) / 2;
    if (j > 4 * nr) j -= 4 * nr;
    if (j < 1) j += 4 * nr;

    /* phi = (pi/2) (2j - 1 - shift) / (2 nr); reduce to a quadrant exactly so that
     * centres on the axes come out with exact zero components. */
    const int64_t num = 2 * j - 1 - shift, den = 2 * nr;
    const int64_t quad = num / den, rem = num - quad * den;
    const double a = (ORC_PI / 2) * ((double)rem / (double)den);
    const double ca = cos(a), sa = sin(a);
    double cx, cy;
    switch (quad) {
        case 0: cx = ca; cy = sa; break;
        case 1: cx = -sa; cy = ca; break;
        case 2: cx = -ca; cy = -sa; break;
        default: cx = sa; cy = -ca; break;
    }
    const double st = sqrt((1.0 - z) * (1.0 + z));
    v[0] = st * cx;
    v[1] = st * cy;
    v[2] = z;
}

/* ------------------------------------------------------------------------------ */
/* Split radius.                                                                    */
/* ------------------------------------------------------------------------------ */

double orc_t_split(double rays_per_cell, int32_t level)
{
    /* pi r^2 / (3 4^l) = 1 / Phi  =>  r = 2^l sqrt(3 / (pi Phi)) */
    const float base = (float)sqrt(3.0 / (ORC_PI * rays_per_cell));
    return ldexp((double)base, level);
}

int32_t orc_auto_max_level(int32_t nx, int32_t ny, int32_t nz, double rays_per_cell)
{
    const double diag = sqrt((double)nx * nx + (double)ny * ny + (double)nz * nz);
    int32_t l = 0;
    while (orc_t_split(rays_per_cell, l) < diag) ++l;
    return l;
}

/* ------------------------------------------------------------------------------ */
/* Cell-by-cell walk with exact decisions.                                          */
/* ------------------------------------------------------------------------------ */

typedef struct {
    double xs[3];     /* ray origin (source position) */
    double d[3];      /* direction, float-valued */
    int64_t c[3];     /* current cell */
    double t;         /* current path length */
    double t_end;     /* split radius, or INFINITY */
} walk_t;

/* Index of the cell the ray occupies just after path length t0 along one axis.
 * x = xs + t0 d. p = t0 d is exact in double; k - xs is exact (lattice), so each
 * comparison below is exact. */
static int64_t start_index(double xs, double t0, double d)
{
    if (d == 0.0) return (int64_t)floor(xs);
    const double p = t0 * d;
    int64_t k = (int64_t)floor(xs + p);   /* first guess, corrected exactly below */
    if (d > 0) {                          /* largest k with xs + p >= k */
        while (p < (double)k - xs) --k;
        while (p >= (double)(k + 1) - xs) ++k;
    } else {                              /* k with k < xs + p <= k + 1 */
        while (p <= (double)k - xs) --k;
        while (p > (double)(k + 1) - xs) ++k;
    }
    return k;
}

static int walk_inside(const walk_t* w, int32_t nx, int32_t ny, int32_t nz)
{
    return w->c[0] >= 0 && w->c[0] < nx && w->c[1] >= 0 && w->c[1] < ny && w->c[2] >= 0 &&
           w->c[2] < nz;
}

/* Returns 1 if the start cell is inside the grid. */
static int walk_start(walk_t* w, const double xs[3], const double d[3], double t0, double t_end,
                      int32_t nx, int32_t ny, int32_t nz)
{
    for (int i = 0; i < 3; ++i) {
        w->xs[i] = xs[i];
        w->d[i] = d[i];
        w->c[i] = start_index(xs[i], t0, d[i]);
    }
    w->t = t0;
    w->t_end = t_end;
    return walk_inside(w, nx, ny, nz);
}

/* Path length at which the current segment ends. *at_end = 1 if it ends at the split
 * radius (which wins an exact tie with a boundary); *mask = axes whose boundary is
 * reached exactly at that length. */
static double walk_next(const walk_t* w, int* at_end, int* mask)
{
    /* t_i = a_i / e_i with a_i = distance of the next boundary from the origin along
     * the axis and e_i = |d_i|; compare t_i < t_j as a_i e_j < a_j e_i. */
    double a[3], e[3];
    int best = -1;
    for (int i = 0; i < 3; ++i) {
        if (w->d[i] > 0) {
            a[i] = (double)(w->c[i] + 1) - w->xs[i];
            e[i] = w->d[i];
        } else if (w->d[i] < 0) {
            a[i] = w->xs[i] - (double)w->c[i];
            e[i] = -w->d[i];
        } else {
            a[i] = 1.0;
            e[i] = 0.0;
            continue;
        }
        if (best < 0 || a[i] * e[best] < a[best] * e[i]) best = i;
    }
    *mask = 0;
    for (int i = 0; i < 3; ++i)
        if (e[i] > 0 && a[i] * e[best] == a[best] * e[i]) *mask |= 1 << i;
    if (w->t_end < INFINITY && w->t_end * e[best] <= a[best]) {
        *at_end = 1;
        return w->t_end;
    }
    *at_end = 0;
    return a[best] / e[best];
}

static void walk_advance(walk_t* w, int mask, double t_next)
{
    for (int i = 0; i < 3; ++i)
        if (mask & (1 << i)) w->c[i] += (w->d[i] > 0) ? 1 : -1;
    w->t = t_next;
}

int64_t orc_walk(int32_t nx, int32_t ny, int32_t nz, const double xs[3], const double d[3],
                 double t0, double t_end, int64_t* cells, double* ds, int64_t cap, int32_t* how)
{
    walk_t w;
    if (!walk_start(&w, xs, d, t0, t_end < 0 ? INFINITY : t_end, nx, ny, nz)) {
        *how = 2;
        return 0;
    }
    int64_t n = 0;
    for (;;) {
        int at_end, mask;
        const double tn = walk_next(&w, &at_end, &mask);
        if (n < cap) {
            cells[n] = w.c[0] + (int64_t)nx * (w.c[1] + (int64_t)ny * w.c[2]);
            ds[n] = tn - w.t;
        }
        ++n;
        if (at_end) {
            *how = 1;
            return n;
        }
        walk_advance(&w, mask, tn);
        if (!walk_inside(&w, nx, ny, nz)) {
            *how = 0;
            return n;
        }
    }
}

/* ------------------------------------------------------------------------------ */
/* Tracer.                                                                          */
/* ------------------------------------------------------------------------------ */

typedef struct {
    int32_t level;
    int64_t pix;
    double tau[ORC_MAXB];
} ray_t;

typedef struct {
    ray_t* v;
    int64_t n, cap;
} stack_t_;

static int push(stack_t_* s, const ray_t* r)
{
    if (s->n == s->cap) {
        const int64_t nc = s->cap ? 2 * s->cap : 1024;
        ray_t* nv = (ray_t*)realloc(s->v, (size_t)nc * sizeof(ray_t));
        if (!nv) return -1;
        s->v = nv;
        s->cap = nc;
    }
    s->v[s->n++] = *r;
    return 0;
}

/* g(x) = (1 - e^-x) / x, the mean attenuation over a segment of optical depth x. */
static double mean_atten(double x) { return x > 0 ? -expm1(-x) / x : 1.0; }

/* Section 2.5, eq:correction: the share f_c of a crossing's photons its own cell keeps,
 * for a segment of cell c between path lengths t0 and t1 of a level-`level` ray. Also the
 * neighbour across the face nearest to the segment's midpoint (*nb = -1: none inside). */
static double orc_correction(const walk_t* w, double t0, double t1, int32_t level, int mode, int32_t nx,
                             int32_t ny, int32_t nz, int64_t* nb)
{
    const double tm = 0.5 * (t0 + t1);
    const double lpix = tm * sqrt(4.0 * ORC_PI / (double)orc_npix(level));
    double dmin = INFINITY;
    int axis = 0, side = 0;
    for (int i = 0; i < 3; ++i) {
        const double m = w->xs[i] + tm * w->d[i];
        const double lo = m - (double)w->c[i], hi = (double)(w->c[i] + 1) - m;
        const int upper = hi < lo - ORC_FACE_TIE;
        const double di = upper ? hi : lo;
        if (di < dmin - ORC_FACE_TIE) {
            dmin = di;
            axis = i;
            side = upper ? 1 : -1;
        }
    }
    *nb = -1;
    if (!(dmin < 0.5 * lpix)) return 1.0;
    double fc = 0.5 + dmin / lpix;
    if (mode == 3) fc *= fc;
    if (mode == 2) {
        int64_t c[3] = {w->c[0], w->c[1], w->c[2]};
        c[axis] += side;
        const int64_t n[3] = {nx, ny, nz};
        if (c[axis] < 0 || c[axis] >= n[axis]) return 1.0;  /* no neighbour: the share stays */
        *nb = c[0] + (int64_t)nx * (c[1] + (int64_t)ny * c[2]);
    }
    return fc;
}

/* What every source's trace shares: inputs, opacity, levels, and whether the field is
 * shared between threads (then every addition to it is atomic). */
typedef struct {
    const orc_grid* g;
    const orc_sources* s;
    const orc_bins* b;
    const orc_params* p;
    const double* kappa;     /* [nbins][ncell] optical depth per cell length */
    int64_t ncell;
    int nb, ksoft;
    int32_t lmax;
    double tau_term;
    int atomic;
} orc_run;

/* x += v, atomically when the field is shared between threads (compare-and-swap on the
 * bit pattern: the sum is the same up to the order of the additions). */
static void field_add(const orc_run* R, double* x, double v)
{
    if (!R->atomic) {
        *x += v;
        return;
    }
    uint64_t* u = (uint64_t*)(void*)x;
    uint64_t old = __atomic_load_n(u, __ATOMIC_RELAXED), nw;
    do {
        double d;
        memcpy(&d, &old, sizeof d);
        d += v;
        memcpy(&nw, &d, sizeof nw);
    } while (!__atomic_compare_exchange_n(u, &old, nw, 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED));
}

/* Field deposit of amount a (photons per unit opacity) of bin k into cell c, split by the
 * geometric correction: f_c a stays; with a neighbour, (1 - f_c) a kappa_c / kappa_nb goes
 * there (the same photons, absorbed at the neighbour's opacity). */
static void orc_deposit(const orc_run* R, double* J, int k, int64_t c, double a, double fc, int64_t nb)
{
    const int64_t ncell = R->ncell;
    if (fc >= 1.0) {
        field_add(R, &J[(int64_t)k * ncell + c], a);
        return;
    }
    if (nb < 0) {  /* modes 1 and 3: the removed share is dropped */
        field_add(R, &J[(int64_t)k * ncell + c], fc * a);
        return;
    }
    const double kc = R->kappa[(int64_t)k * ncell + c];
    const double kn = R->kappa[(int64_t)k * ncell + nb];
    if (kn > 0) {
        field_add(R, &J[(int64_t)k * ncell + c], fc * a);
        field_add(R, &J[(int64_t)k * ncell + nb], (1.0 - fc) * a * (kc / kn));
    } else {
        field_add(R, &J[(int64_t)k * ncell + c], a);  /* no absorber next door: the share stays */
    }
}

/* Everything one source contributes (section 2.6 fill, then its ray tree, depth first).
 * st is the caller's (emptied) stack. Returns 0, or -1 on a bad thin radius or an
 * allocation failure. */
static int32_t trace_source(const orc_run* R, int32_t src, double* J, double* gdir, uint64_t* tree,
                            int64_t tree_cap, orc_ledger* led, stack_t_* st)
{
    const orc_grid* g = R->g;
    const orc_sources* s = R->s;
    const orc_bins* b = R->b;
    const orc_params* p = R->p;
    const double* kappa = R->kappa;
    const int nb = R->nb, ksoft = R->ksoft;
    const int32_t nx = g->nx, ny = g->ny, nz = g->nz, lmax = R->lmax;
    const int64_t ncell = R->ncell;
    const double L = g->cell_cm, y = g->y_he, V = L * L * L, tau_term = R->tau_term;
    const double TAU_THIN = 0.1;

    const double* xs = s->pos + 3 * src;
    double S[ORC_MAXB];
    for (int k = 0; k < nb; ++k) S[k] = s->ndot[src] * b->frac[k];
    led->emitted += s->ndot[src];

    /* section 2.6: the optically thin sphere of radius R around the source */
    double Rt = 0.0;
    if (s->r_thin) {
        Rt = (double)(float)s->r_thin[src];
        if (!(Rt >= 0.0) || !isfinite(Rt)) return -1;
    }
    if (Rt > 0.0) {
        const int64_t lo[3] = {(int64_t)floor(xs[0] - Rt), (int64_t)floor(xs[1] - Rt), (int64_t)floor(xs[2] - Rt)};
        const int64_t hi[3] = {(int64_t)ceil(xs[0] + Rt), (int64_t)ceil(xs[1] + Rt), (int64_t)ceil(xs[2] + Rt)};
        for (int64_t cz = lo[2] < 0 ? 0 : lo[2]; cz <= hi[2] && cz < nz; ++cz)
            for (int64_t cy = lo[1] < 0 ? 0 : lo[1]; cy <= hi[1] && cy < ny; ++cy)
                for (int64_t cx = lo[0] < 0 ? 0 : lo[0]; cx <= hi[0] && cx < nx; ++cx) {
                    const double dx = (double)cx + 0.5 - xs[0], dy = (double)cy + 0.5 - xs[1],
                                 dz = (double)cz + 0.5 - xs[2];
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    if (!(r2 < Rt * Rt)) continue;
                    const double dil = 1.0 / (4.0 * ORC_PI * (r2 > 0.25 ? r2 : 0.25));
                    const int64_t c = cx + (int64_t)nx * (cy + (int64_t)ny * cz);
                    for (int k = 0; k < nb; ++k) {
                        const double a = S[k] * dil;
                        field_add(R, &J[(int64_t)k * ncell + c], a);
                        led->absorbed_thin += a * kappa[(int64_t)k * ncell + c];
                        if (gdir) {
                            const double nh = g->n_h[c];
                            const double ns_[3] = {nh * g->x_hi[c], y * nh * g->x_hei[c], y * nh * g->x_heii[c]};
                            for (int sp = 0; sp < 3; ++sp)
                                if (ns_[sp] > 0) gdir[(int64_t)sp * ncell + c] += b->sigma[3 * k + sp] * a / (L * L);
                        }
                    }
                }
    }
    double r_out = INFINITY;

    ray_t root;
    memset(&root, 0, sizeof(root));
    root.level = p->level0;
    for (int64_t q = orc_npix(p->level0) - 1; q >= 0; --q) {
        root.pix = q;
        if (push(st, &root)) return -1;
    }
    while (st->n > 0) {
        const ray_t r = st->v[--st->n];
        if (tree && led->tree_count < tree_cap)
            tree[led->tree_count] = ((uint64_t)src << 32) | ((uint64_t)r.level << 28) | (uint64_t)r.pix;
        led->tree_count++;
        led->rays++;

        double v[3], d[3];
        orc_healpix_vec(r.level, r.pix, v);
        for (int i = 0; i < 3; ++i) d[i] = (double)(float)v[i];
        double t0 = r.level == p->level0 ? 0.0 : orc_t_split(p->rays_per_cell, r.level - 1);
        if (Rt > t0) t0 = Rt;
        const double t_end = r.level < lmax ? orc_t_split(p->rays_per_cell, r.level) : INFINITY;
        if (t0 >= t_end) {
            /* starts at or beyond its split radius (inside the thin sphere): split at once */
            ray_t child;
            memset(&child, 0, sizeof(child));
            child.level = r.level + 1;
            for (int q = 3; q >= 0; --q) {
                child.pix = 4 * r.pix + q;
                if (push(st, &child)) return -1;
            }
            led->splits++;
            continue;
        }

        const double wray = 1.0 / (double)orc_npix(r.level);
        double P[ORC_MAXB], tau[ORC_MAXB], dtau[ORC_MAXB];
        for (int k = 0; k < nb; ++k) {
            tau[k] = r.tau[k];
            P[k] = S[k] * wray * exp(-tau[k]);
        }
        walk_t w;
        if (!walk_start(&w, xs, d, t0, t_end, nx, ny, nz)) {
            for (int k = 0; k < nb; ++k) led->escaped += P[k];
            led->escaped_rays++;
            if (tau[ksoft] < TAU_THIN && t0 < r_out) r_out = t0;
            continue;
        }
        for (;;) {
            int at_end, mask;
            const double tn = walk_next(&w, &at_end, &mask);
            const double ds = tn - w.t;
            const int64_t c = w.c[0] + (int64_t)nx * (w.c[1] + (int64_t)ny * w.c[2]);
            led->crossings++;
            int64_t cnb = -1;
            const double fc = p->correction ? orc_correction(&w, w.t, tn, r.level, p->correction, nx, ny, nz, &cnb)
                                            : 1.0;
            if (tau[ksoft] < TAU_THIN) {
                /* where the softest bin's depth reaches 0.1 inside this crossing */
                const double ks = kappa[(int64_t)ksoft * ncell + c];
                if (tau[ksoft] + ks * ds >= TAU_THIN) {
                    const double rc = w.t + (TAU_THIN - tau[ksoft]) / ks;
                    if (rc < r_out) r_out = rc;
                }
            }
            for (int k = 0; k < nb; ++k) {
                const double kap = kappa[(int64_t)k * ncell + c];
                dtau[k] = kap * ds;
                const double lost = -expm1(-dtau[k]);        /* 1 - e^-dtau */
                orc_deposit(R, J, k, c, P[k] * ds * mean_atten(dtau[k]), fc, cnb);
                led->absorbed_trace += P[k] * lost;
                if (gdir && dtau[k] > 0) {
                    /* eq:ion with the absorbed photons split by species optical depth */
                    const double nh = g->n_h[c];
                    const double ns_[3] = {nh * g->x_hi[c], y * nh * g->x_hei[c], y * nh * g->x_heii[c]};
                    for (int sp = 0; sp < 3; ++sp) {
                        if (ns_[sp] <= 0) continue;
                        const double dts = L * ns_[sp] * b->sigma[3 * k + sp] * ds;
                        gdir[(int64_t)sp * ncell + c] += P[k] * lost * (dts / dtau[k]) / (V * ns_[sp]);
                    }
                }
                P[k] *= exp(-dtau[k]);
                tau[k] += dtau[k];
            }
            int term = tau_term < INFINITY;
            for (int k = 0; k < nb && term; ++k)
                term = tau[k] >= tau_term && dtau[k] >= ORC_DTAU_TERM_MIN;
            if (term) {
                for (int k = 0; k < nb; ++k) {
                    const double kap = kappa[(int64_t)k * ncell + c];
                    orc_deposit(R, J, k, c, P[k] / kap, fc, cnb);
                    led->absorbed_trace += P[k];
                    if (gdir) {
                        const double nh = g->n_h[c];
                        const double ns_[3] = {nh * g->x_hi[c], y * nh * g->x_hei[c], y * nh * g->x_heii[c]};
                        for (int sp = 0; sp < 3; ++sp) {
                            if (ns_[sp] <= 0) continue;
                            const double ks = L * ns_[sp] * b->sigma[3 * k + sp];
                            gdir[(int64_t)sp * ncell + c] += P[k] * (ks / kap) / (V * ns_[sp]);
                        }
                    }
                }
                led->terminated++;
                break;
            }
            if (at_end) {
                ray_t child;
                memset(&child, 0, sizeof(child));
                child.level = r.level + 1;
                for (int k = 0; k < nb; ++k) child.tau[k] = tau[k];
                for (int q = 3; q >= 0; --q) {
                    child.pix = 4 * r.pix + q;
                    if (push(st, &child)) return -1;
                }
                led->splits++;
                break;
            }
            walk_advance(&w, mask, tn);
            if (!walk_inside(&w, nx, ny, nz)) {
                for (int k = 0; k < nb; ++k) led->escaped += P[k];
                led->escaped_rays++;
                if (tau[ksoft] < TAU_THIN && tn < r_out) r_out = tn;
                break;
            }
        }
    }
    if (s->r_thin_out) s->r_thin_out[src] = r_out;
    return 0;
}

/* Checks, the opacity of section 2.2 and the zeroed outputs: the set-up both drivers share. */
static int32_t run_setup(orc_run* R, const orc_grid* g, const orc_sources* s, const orc_bins* b, const orc_params* p,
                         double* J, double* gdir, orc_ledger* led)
{
    if (!g || !s || !b || !p || !J || !led) return -1;
    if (p->correction < 0 || p->correction > 3 || (p->correction && gdir)) return -1;
    if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0 || b->nbins <= 0 || b->nbins > ORC_MAXB) return -1;
    if (p->level0 < 0 || p->rays_per_cell <= 0) return -1;
    memset(R, 0, sizeof(*R));
    R->g = g;
    R->s = s;
    R->b = b;
    R->p = p;
    R->nb = b->nbins;
    R->ncell = (int64_t)g->nx * g->ny * g->nz;
    const int nb = R->nb;
    const int64_t ncell = R->ncell;
    const double L = g->cell_cm, y = g->y_he;

    /* Optical depth per cell length, per bin (section 2.2: all species). */
    double* kappa = (double*)malloc((size_t)nb * (size_t)ncell * sizeof(double));
    if (!kappa) return -1;
    for (int64_t c = 0; c < ncell; ++c) {
        const double nh = g->n_h[c], xhi = g->x_hi[c], xhei = g->x_hei[c], xheii = g->x_heii[c];
        for (int k = 0; k < nb; ++k) {
            const double* sg = b->sigma + 3 * k;
            kappa[(int64_t)k * ncell + c] = L * nh * (sg[0] * xhi + y * (sg[1] * xhei + sg[2] * xheii));
        }
    }
    R->kappa = kappa;
    memset(J, 0, (size_t)nb * (size_t)ncell * sizeof(double));
    if (gdir) memset(gdir, 0, 3 * (size_t)ncell * sizeof(double));
    memset(led, 0, sizeof(*led));
    R->lmax = p->max_level < 0 ? orc_auto_max_level(g->nx, g->ny, g->nz, p->rays_per_cell) : p->max_level;
    R->tau_term = p->eps_term > 0 ? -log(p->eps_term) : INFINITY;
    /* softest bin: the lowest photon energy (the first of equal ones) */
    R->ksoft = 0;
    for (int k = 1; k < nb; ++k)
        if (b->e_erg[k] < b->e_erg[R->ksoft]) R->ksoft = k;
    return 0;
}

int32_t orc_trace(const orc_grid* g, const orc_sources* s, const orc_bins* b, const orc_params* p,
                  double* J, double* gdir, uint64_t* tree, int64_t tree_cap, orc_ledger* led)
{
    orc_run R;
    if (run_setup(&R, g, s, b, p, J, gdir, led)) return -1;
    stack_t_ st = {0, 0, 0};
    int32_t rc = 0;
    for (int32_t src = 0; src < s->n && rc == 0; ++src) rc = trace_source(&R, src, J, gdir, tree, tree_cap, led, &st);
    free(st.v);
    free((void*)R.kappa);
    return rc;
}

/* ------------------------------------------------------------------------------ */
/* The same trace on several host threads (for timing the oracle on every core).     */
/* ------------------------------------------------------------------------------ */

typedef struct {
    const orc_run* R;
    double* J;
    int32_t first, stride;
    orc_ledger led;
    int32_t rc;
} mt_part;

static void* mt_worker(void* arg)
{
    mt_part* w = (mt_part*)arg;
    stack_t_ st = {0, 0, 0};
    memset(&w->led, 0, sizeof(w->led));
    w->rc = 0;
    for (int32_t src = w->first; src < w->R->s->n && w->rc == 0; src += w->stride)
        w->rc = trace_source(w->R, src, w->J, NULL, NULL, 0, &w->led, &st);
    free(st.v);
    return NULL;
}

int32_t orc_trace_mt(const orc_grid* g, const orc_sources* s, const orc_bins* b, const orc_params* p, double* J,
                     int32_t nthreads, orc_ledger* led)
{
    if (nthreads < 1 || nthreads > 1024) return -1;
    orc_run R;
    if (run_setup(&R, g, s, b, p, J, NULL, led)) return -1;
    R.atomic = nthreads > 1;
    mt_part* parts = (mt_part*)calloc((size_t)nthreads, sizeof(mt_part));
    pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
    int32_t rc = parts && th ? 0 : -1;
    int started = 0;
    for (int t = 0; t < nthreads && rc == 0; ++t) {
        parts[t].R = &R;
        parts[t].J = J;
        parts[t].first = t;
        parts[t].stride = nthreads;
        if (pthread_create(&th[t], NULL, mt_worker, &parts[t]) != 0) rc = -1;
        else ++started;
    }
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    /* the ledgers in thread order */
    for (int t = 0; t < started && rc == 0; ++t) {
        const orc_ledger* q = &parts[t].led;
        if (parts[t].rc) rc = -1;
        led->emitted += q->emitted;
        led->absorbed_trace += q->absorbed_trace;
        led->escaped += q->escaped;
        led->absorbed_thin += q->absorbed_thin;
        led->crossings += q->crossings;
        led->rays += q->rays;
        led->splits += q->splits;
        led->terminated += q->terminated;
        led->escaped_rays += q->escaped_rays;
        led->tree_count += q->tree_count;
    }
    free(parts);
    free(th);
    free((void*)R.kappa);
    return rc;
}

void orc_finalize(const orc_grid* g, const orc_bins* b, const double* J, double* gamma, double* heat,
                  double* absorbed)
{
    const int nb = b->nbins;
    const int64_t ncell = (int64_t)g->nx * g->ny * g->nz;
    const double L = g->cell_cm, y = g->y_he;
    double total = 0;
    for (int64_t c = 0; c < ncell; ++c) {
        double gm[3] = {0, 0, 0}, ht[3] = {0, 0, 0};
        const double nh = g->n_h[c];
        for (int k = 0; k < nb; ++k) {
            const double Jk = J[(int64_t)k * ncell + c];
            const double* sg = b->sigma + 3 * k;
            for (int sp = 0; sp < 3; ++sp) {
                gm[sp] += sg[sp] * Jk / (L * L);
                const double excess = b->e_erg[k] - b->e_thr[sp];
                if (excess > 0) ht[sp] += sg[sp] * excess * Jk / (L * L);
            }
            const double kap = L * nh * (sg[0] * g->x_hi[c] + y * (sg[1] * g->x_hei[c] + sg[2] * g->x_heii[c]));
            total += Jk * kap;
        }
        for (int sp = 0; sp < 3; ++sp) {
            if (gamma) gamma[(int64_t)sp * ncell + c] = gm[sp];
            if (heat) heat[(int64_t)sp * ncell + c] = ht[sp];
        }
    }
    if (absorbed) *absorbed = total;
}

/* ------------------------------------------------------------------------------ */
/* Chemistry.                                                                       */
/* ------------------------------------------------------------------------------ */

/* Hui & Gnedin (1997, MNRAS 292, 27), appendix fits, with lambda = 2 T_i / T. */
static const double T_HI_K = 157807.0, T_HEI_K = 285335.0, T_HEII_K = 631515.0;

void orc_rate_coeffs(double T, double out[6])
{
    const double lhi = 2.0 * T_HI_K / T, lhei = 2.0 * T_HEI_K / T, lheii = 2.0 * T_HEII_K / T;
    /* case-B radiative recombination */
    out[0] = 2.753e-14 * pow(lhi, 1.5) / pow(1.0 + pow(lhi / 2.740, 0.407), 2.242);
    const double diel = 1.90e-3 * pow(T, -1.5) * exp(-0.75 * lheii / 2.0) * (1.0 + 0.3 * exp(-0.15 * lheii / 2.0));
    out[1] = 1.26e-14 * pow(lhei, 0.750) + diel;
    out[2] = 2.0 * 2.753e-14 * pow(lheii, 1.5) / pow(1.0 + pow(lheii / 2.740, 0.407), 2.242);
    /* collisional ionisation */
    out[3] = 21.11 * pow(T, -1.5) * exp(-lhi / 2.0) * pow(lhi, -1.089) / pow(1.0 + pow(lhi / 0.354, 0.874), 1.101);
    out[4] = 32.38 * pow(T, -1.5) * exp(-lhei / 2.0) * pow(lhei, -1.146) / pow(1.0 + pow(lhei / 0.416, 0.987), 1.056);
    out[5] = 19.95 * pow(T, -1.5) * exp(-lheii / 2.0) * pow(lheii, -1.089) / pow(1.0 + pow(lheii / 0.553, 0.735), 1.275);
}

/* Cooling coefficients per electron and per ion [erg cm^3 s^-1] (section 2.8; Hui & Gnedin
 * 1997 fits with lambda = 2 T_i / T):
 *   [0] HII, [1] HeII, [2] HeIII case-B recombination cooling,
 *   [3] HeII dielectronic recombination cooling,
 *   [4] HI, [5] HeII collisional excitation,
 *   [6] bremsstrahlung per unit Z^2 of the ion (Gaunt factor included).
 * The HeIII recombination term is the HII fit taken at lambda_HeII times Z = 2: a hydrogenic
 * ion of charge Z cools as Z^3 times hydrogen at T / Z^2, and the fit carries one explicit
 * power of T. */
void orc_cooling_coeffs(double T, double out[7])
{
    const double lhi = 2.0 * T_HI_K / T, lhei = 2.0 * T_HEI_K / T, lheii = 2.0 * T_HEII_K / T;
    out[0] = 3.435e-30 * T * pow(lhi, 1.970) / pow(1.0 + pow(lhi / 2.250, 0.376), 3.720);
    out[1] = KB_ERG * T * 1.26e-14 * pow(lhei, 0.750);
    out[2] = 2.0 * 3.435e-30 * T * pow(lheii, 1.970) / pow(1.0 + pow(lheii / 2.250, 0.376), 3.720);
    const double diel = 1.90e-3 * pow(T, -1.5) * exp(-0.75 * lheii / 2.0) * (1.0 + 0.3 * exp(-0.15 * lheii / 2.0));
    out[3] = 0.75 * 54.418 * EV_ERG * diel;
    const double damp = 1.0 + sqrt(T / 1e5);
    out[4] = 7.5e-19 * exp(-0.75 * lhi / 2.0) / damp;
    out[5] = 5.54e-17 * pow(T, -0.397) * exp(-0.75 * lheii / 2.0) / damp;
    const double lt = log10(T);
    const double gff = 1.1 + 0.34 * exp(-(5.5 - lt) * (5.5 - lt) / 3.0);
    out[6] = 1.42e-27 * gff * sqrt(T);
}

/* Cooling rate per volume [erg cm^-3 s^-1]: recombination, collisional ionisation,
 * collisional excitation and bremsstrahlung (section 2.8; Hui & Gnedin 1997). The
 * Hubble-expansion and Compton terms need a cosmology and are not included. */
double orc_cooling(double T, double ne, double nhi, double nhii, double nhei, double nheii, double nheiii,
                   int collisional)
{
    double k[6], c[7];
    orc_rate_coeffs(T, k);
    orc_cooling_coeffs(T, c);
    double lam = ne * (c[0] * nhii + c[1] * nheii + c[2] * nheiii + c[3] * nheii);
    if (collisional)
        lam += ne * (13.598 * EV_ERG * k[3] * nhi + 24.587 * EV_ERG * k[4] * nhei + 54.418 * EV_ERG * k[5] * nheii);
    lam += ne * (c[4] * nhi + c[5] * nheii);
    lam += c[6] * (nhii + nheii + 4.0 * nheiii) * ne;
    return lam;
}

void orc_chem(int64_t ncell, double y_he, const float* n_h, const float* x_hi, const float* x_hei,
              const float* x_heii, const float* temp, const double* gamma, const double* heat, double dt,
              const orc_chem_params* cp, double* x_hi_out, double* x_hei_out, double* x_heii_out,
              double* temp_out, int32_t* nsub, int32_t* flags)
{
    for (int64_t c = 0; c < ncell; ++c) {
        const double nh = n_h[c], nhe = y_he * nh;
        double nhi = nh * (double)x_hi[c], nhii = nh - nhi;
        double nhei = nhe * (double)x_hei[c], nheii = nhe * (double)x_heii[c];
        double nheiii = nhe - nhei - nheii;
        if (nheiii < 0) nheiii = 0;
        double T = temp[c];
        double ne = nhii + nheii + 2.0 * nheiii;
        double E = 1.5 * KB_ERG * T * (nh + nhe + ne);
        const double ghi = gamma[c], ghei = gamma[ncell + c], gheii = gamma[2 * ncell + c];
        const double hhi = heat[c], hhei = heat[ncell + c], hheii = heat[2 * ncell + c];
        double t = 0;
        int32_t n = 0, flag = 0;
        while (t < dt) {
            double a_hii, a_heii = 0, a_heiii = 0, k_hi = 0, k_hei = 0, k_heii = 0;
            if (cp->rates == 0) {
                a_hii = cp->alpha_hii;
            } else {
                double k[6];
                orc_rate_coeffs(T, k);
                a_hii = k[0];
                a_heii = k[1];
                a_heiii = k[2];
                if (cp->collisional) {
                    k_hi = k[3];
                    k_hei = k[4];
                    k_heii = k[5];
                }
            }
            /* eq:diffeq for HI */
            const double ndot_hi = a_hii * ne * nhii - (ghi + k_hi * ne) * nhi;
            double edot = 0;
            if (!cp->isothermal)
                edot = nhi * hhi + nhei * hhei + nheii * hheii -
                       orc_cooling(T, ne, nhi, nhii, nhei, nheii, nheiii, cp->collisional);
            /* sub-cycle step: limit the fractional change of E and n_HI to eps */
            double h = dt - t;
            int last = 1;
            if (n >= cp->max_sub) {
                flag = 1;
            } else {
                if (edot != 0 && cp->eps * E / fabs(edot) < h) {
                    h = cp->eps * E / fabs(edot);
                    last = 0;
                }
                /* both hydrogen states are tracked quantities: limit the fractional change
                 * of n_HI and of n_HII (a cell that starts fully ionised or fully neutral
                 * would otherwise take one unbounded explicit source step) */
                if (nhi > 0 && ndot_hi != 0 && cp->eps * nhi / fabs(ndot_hi) < h) {
                    h = cp->eps * nhi / fabs(ndot_hi);
                    last = 0;
                }
                if (nhii > 0 && ndot_hi != 0 && cp->eps * nhii / fabs(ndot_hi) < h) {
                    h = cp->eps * nhii / fabs(ndot_hi);
                    last = 0;
                }
            }
            /* eq:anninos, backward difference n' = (n + D h) / (1 + C h), in the order
             * HI, HeI, HeIII, with HeII from helium conservation */
            nhi = (nhi + a_hii * ne * nhii * h) / (1.0 + (ghi + k_hi * ne) * h);
            if (nhi > nh) nhi = nh;
            nhii = nh - nhi;
            double nhei_new = (nhei + a_heii * ne * nheii * h) / (1.0 + (ghei + k_hei * ne) * h);
            double nheiii_new = (nheiii + (gheii + k_heii * ne) * nheii * h) / (1.0 + a_heiii * ne * h);
            if (nhei_new > nhe) nhei_new = nhe;
            if (nheiii_new > nhe - nhei_new) nheiii_new = nhe - nhei_new;
            nhei = nhei_new;
            nheiii = nheiii_new;
            nheii = nhe - nhei - nheiii;
            if (nheii < 0) nheii = 0;
            ne = nhii + nheii + 2.0 * nheiii;
            if (!cp->isothermal) {
                E += edot * h;
                T = E / (1.5 * KB_ERG * (nh + nhe + ne));
                if (T < cp->t_floor) {
                    T = cp->t_floor;
                    E = 1.5 * KB_ERG * T * (nh + nhe + ne);
                }
            }
            t = last ? dt : t + h;
            ++n;
        }
        x_hi_out[c] = nhi / nh;
        x_hei_out[c] = nhe > 0 ? nhei / nhe : (double)x_hei[c];
        x_heii_out[c] = nhe > 0 ? nheii / nhe : (double)x_heii[c];
        temp_out[c] = T;
        if (nsub) nsub[c] = n;
        if (flags) flags[c] = flag;
    }
}

/* ------------------------------------------------------------------------------ */
/* Adaptive RT time step (section 2.9): the two per-cell limits and their minima.   */
/* ------------------------------------------------------------------------------ */
void orc_timestep(int64_t ncell, double y_he, double cell_cm, const float* n_h, const float* x_hi,
                  const float* x_hei, const float* x_heii, const float* temp, const double* gamma_hi,
                  const orc_chem_params* cp, double sigma0, double eps, double* dt_n, double* dt_i)
{
    double mn = INFINITY, mi = INFINITY;
    for (int64_t c = 0; c < ncell; ++c) {
        const double nh = n_h[c], nhe = y_he * nh;
        const double nhi = nh * (double)x_hi[c], nhii = nh - nhi;
        const double nhei = nhe * (double)x_hei[c], nheii = nhe * (double)x_heii[c];
        double nheiii = nhe - nhei - nheii;
        if (nheiii < 0) nheiii = 0;
        const double ne = nhii + nheii + 2.0 * nheiii;
        double a_hii, k_hi = 0;
        if (cp->rates == 0) {
            a_hii = cp->alpha_hii;
        } else {
            double k[6];
            orc_rate_coeffs((double)temp[c], k);
            a_hii = k[0];
            if (cp->collisional) k_hi = k[3];
        }
        const double ndot = fabs(a_hii * ne * nhii - (gamma_hi[c] + k_hi * ne) * nhi);
        if (!(ndot > 0)) continue;
        const double tau = nhi * sigma0 * cell_cm;
        if (tau > 0.5) {
            const double t = eps * nhi / ndot;
            if (t < mn) mn = t;
        }
        const double ti = eps / (sigma0 * cell_cm * ndot);
        if (ti < mi) mi = ti;
    }
    *dt_n = mn;
    *dt_i = mi;
}

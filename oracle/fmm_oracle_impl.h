/*
 * fmm_oracle_impl.h -- TEST INFRASTRUCTURE ONLY (see fmm_oracle.c).
 *
 * Body of the plain sequential CPU reference, written once and instantiated
 * for one floating-point type by fmm_oracle.c, which defines
 *     REAL  -- the arithmetic type (double or float)
 *     SFX   -- the symbol suffix  (f64 or f32)
 *     RSQRT -- the square root of that type (sqrt or sqrtf)
 * before including this file.  Nothing here is shared with the HIP library.
 */

#define ORC_CAT2(a, b) a##_##b
#define ORC_CAT(a, b) ORC_CAT2(a, b)
#define FN(name) ORC_CAT(name, SFX)

/* ------------------------------------------------------------------------ */
/* Binary min-heap of point indices ordered by (psi, index).                 */
/* Sec. 2.1: the BAND set is kept sorted in a binary heap with the standard  */
/* operations Insert_Heap, Locate_Min, Remove_Min and Up_Heap.               */
/* Ties in psi are broken by the lower index (the paper is silent on ties).  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t *a;        /* heap array of point indices            */
    int64_t n, cap;    /* current size and capacity              */
    int32_t *pos;      /* pos[idx] = position in a[], or -1      */
    const REAL *key;   /* psi array the heap is ordered by       */
} FN(heap_t);

static int FN(heap_less)(const FN(heap_t) *h, int64_t x, int64_t y)
{
    REAL kx = h->key[x], ky = h->key[y];
    return (kx < ky) || (kx == ky && x < y);
}

static void FN(heap_swap)(FN(heap_t) *h, int64_t i, int64_t j)
{
    int64_t t = h->a[i];
    h->a[i] = h->a[j];
    h->a[j] = t;
    h->pos[h->a[i]] = (int32_t)i;
    h->pos[h->a[j]] = (int32_t)j;
}

/* Up_Heap: move the element at heap position i towards the root. */
static void FN(heap_up)(FN(heap_t) *h, int64_t i)
{
    while (i > 0) {
        int64_t parent = (i - 1) / 2;
        if (!FN(heap_less)(h, h->a[i], h->a[parent])) break;
        FN(heap_swap)(h, i, parent);
        i = parent;
    }
}

static void FN(heap_down)(FN(heap_t) *h, int64_t i)
{
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < h->n && FN(heap_less)(h, h->a[l], h->a[m])) m = l;
        if (r < h->n && FN(heap_less)(h, h->a[r], h->a[m])) m = r;
        if (m == i) break;
        FN(heap_swap)(h, i, m);
        i = m;
    }
}

/* Insert_Heap, or Up_Heap when the point is already in the heap. */
static int FN(heap_push_or_up)(FN(heap_t) *h, int64_t idx)
{
    if (h->pos[idx] >= 0) {
        FN(heap_up)(h, h->pos[idx]);
        return 0;
    }
    if (h->n == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 64;
        int64_t *na = (int64_t *)realloc(h->a, (size_t)nc * sizeof(int64_t));
        if (!na) return ORC_ENOMEM;
        h->a = na;
        h->cap = nc;
    }
    h->a[h->n] = idx;
    h->pos[idx] = (int32_t)h->n;
    h->n++;
    FN(heap_up)(h, h->n - 1);
    return 0;
}

/* Remove_Min. */
static void FN(heap_pop)(FN(heap_t) *h)
{
    int64_t top = h->a[0];
    h->pos[top] = -1;
    h->n--;
    if (h->n > 0) {
        h->a[0] = h->a[h->n];
        h->pos[h->a[0]] = 0;
        FN(heap_down)(h, 0);
    }
}

/* ------------------------------------------------------------------------ */
/* Solve_Quadratic (Alg. 3).                                                 */
/*                                                                           */
/* nv[2d], nv[2d+1] are the values of the lower and upper neighbour on axis  */
/* d (x, y, z); nk[] says whether that neighbour is KNOWN (FIX or NEW).      */
/* Per axis, a KNOWN neighbour whose value is below the current psi_q is an  */
/* upwind candidate; if both are, the upper one wins only when strictly      */
/* smaller.  The candidates are sorted and the quadratic of Eq. (2) is       */
/* solved with the first k of them, k = 1, 2, ..., while the root still      */
/* exceeds the next candidate.                                               */
/*                                                                           */
/* literal == 1 evaluates the paper's coefficients a = k, b = sum v,         */
/* c = sum v^2 - h^2/F^2, root (b + sqrt(b^2 - a c)) / a.                    */
/* literal == 0 (the default) solves the same quadratic in the variable      */
/* shifted by the smallest candidate v1 (u_i = v_i - v1), identical in       */
/* exact arithmetic and free of the cancellation in b^2 - a c.               */
/* A negative discriminant (impossible in exact arithmetic) is clamped to 0. */
/* ------------------------------------------------------------------------ */
static REAL FN(solve_quadratic)(REAL psi_q, const REAL nv[6], const int nk[6], REAL rhs,
                               int literal)
{
    REAL v[3];
    int n = 0;
    for (int ax = 0; ax < 3; ++ax) {
        REAL lo = nv[2 * ax], hi = nv[2 * ax + 1];
        int d = 0;
        if (nk[2 * ax] && psi_q > lo) d = -1;
        if (nk[2 * ax + 1] && psi_q > hi) {
            if (d == 0 || hi < lo) d = 1;
        }
        if (d != 0) v[n++] = (d < 0) ? lo : hi;
    }
    if (n == 0) return (REAL)INFINITY;
    /* sort the (at most three) candidates ascending */
    for (int i = 1; i < n; ++i) {
        REAL x = v[i];
        int j = i - 1;
        while (j >= 0 && v[j] > x) {
            v[j + 1] = v[j];
            --j;
        }
        v[j + 1] = x;
    }
    for (int k = 1;; ++k) {
        REAL t;
        REAL kr = (REAL)k;
        if (literal) {
            REAL b = 0, s2 = 0;
            for (int i = 0; i < k; ++i) {
                b += v[i];
                s2 += v[i] * v[i];
            }
            REAL c = s2 - rhs;
            REAL disc = b * b - kr * c;
            if (disc < 0) disc = 0;
            t = (b + RSQRT(disc)) / kr;
        } else {
            REAL s1 = 0, s2 = 0;
            for (int i = 1; i < k; ++i) {
                REAL u = v[i] - v[0];
                s1 += u;
                s2 += u * u;
            }
            REAL disc = s1 * s1 - kr * (s2 - rhs);
            if (disc < 0) disc = 0;
            t = v[0] + (s1 + RSQRT(disc)) / kr;
        }
        if (k < n && t > v[k]) continue;
        return t;
    }
}

/* h^2 / F^2 of Alg. 3; F = 0 marks an obstacle where no solve happens. */
static REAL FN(rhs_of)(REAL h, REAL f)
{
    return (h * h) / (f * f);
}

/* ------------------------------------------------------------------------ */
/* Baseline solver "B" (Sec. 3.1): the sequential narrow-band FMM of         */
/* Sec. 2.1 with the augmented tags and unified heap of Sec. 2.2, on a       */
/* single domain.  Alg. 1 (initialisation), then Alg. 4 with the bound equal */
/* to width_band, calling Alg. 2 / Alg. 3.                                   */
/*                                                                           */
/* Layout: idx = i + nx*(j + ny*k).  psi is written for every point; points  */
/* never reached are +inf.  Sources: src_idx[s] (linear index) with value    */
/* src_val[s]; a duplicated source keeps the smaller value.                  */
/* pops_out (nullable) receives the number of heap removals; nonmono_out     */
/* (nullable) the number of removals whose value was below the previous one. */
/* ------------------------------------------------------------------------ */
int FN(orc_fmm)(int64_t nx, int64_t ny, int64_t nz, double h, const REAL *F, int32_t nsrc,
                const int64_t *src_idx, const REAL *src_val, double width, int32_t literal,
                REAL *psi, int64_t *pops_out, int64_t *nonmono_out)
{
    if (nx <= 0 || ny <= 0 || nz <= 0 || !(h > 0) || nsrc <= 0) return ORC_EINVAL;
    const int64_t N = nx * ny * nz;
    if (N >= INT32_MAX) return ORC_EINVAL; /* heap positions are int32 */
    const REAL hr = (REAL)h;
    uint8_t *G = (uint8_t *)malloc((size_t)N);
    int32_t *pos = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    if (!G || !pos) {
        free(G);
        free(pos);
        return ORC_ENOMEM;
    }
    FN(heap_t) hp = {NULL, 0, 0, pos, psi};
    int rc = 0;

    /* Alg. 1: psi <- +inf, G <- FAR, empty heap */
    for (int64_t p = 0; p < N; ++p) {
        psi[p] = (REAL)INFINITY;
        G[p] = ORC_FAR;
        pos[p] = -1;
    }
    /* points on Gamma: psi0, KNOWN_FIX, inserted into the unified heap */
    for (int32_t s = 0; s < nsrc; ++s) {
        int64_t p = src_idx[s];
        if (p < 0 || p >= N || !(src_val[s] >= 0)) {
            rc = ORC_EINVAL;
            goto done;
        }
        if (src_val[s] < psi[p]) psi[p] = src_val[s];
        G[p] = ORC_KNOWN_FIX;
        if ((rc = FN(heap_push_or_up)(&hp, p)) != 0) goto done;
    }

    int64_t pops = 0, nonmono = 0;
    REAL last = -(REAL)INFINITY;
    const int64_t sx = 1, sy = nx, sz = nx * ny;
    /* Alg. 4 with bound_band = width_band */
    while (hp.n > 0) {
        int64_t p = hp.a[0]; /* Locate_Min */
        if ((double)psi[p] > width) break;
        if (G[p] != ORC_KNOWN_FIX) G[p] = ORC_KNOWN_NEW;
        FN(heap_pop)(&hp); /* Remove_Min */
        ++pops;
        if (psi[p] < last) ++nonmono;
        last = psi[p];

        /* Alg. 2: Update_Neighbors(p) */
        const int64_t pi = p % nx, pj = (p / nx) % ny, pk = p / sz;
        for (int nb = 0; nb < 6; ++nb) {
            int64_t qi = pi, qj = pj, qk = pk;
            switch (nb) {
            case 0: qi--; break;
            case 1: qi++; break;
            case 2: qj--; break;
            case 3: qj++; break;
            case 4: qk--; break;
            default: qk++; break;
            }
            if (qi < 0 || qi >= nx || qj < 0 || qj >= ny || qk < 0 || qk >= nz) continue;
            const int64_t q = qi + nx * (qj + ny * qk);
            if (G[q] == ORC_KNOWN_FIX || !(psi[q] > psi[p])) continue;
            if (F[q] == 0) continue; /* obstacle: the equation is not solved there */
            REAL nv[6];
            int nk[6];
            const int64_t off[6] = {-sx, sx, -sy, sy, -sz, sz};
            const int inside[6] = {qi > 0, qi < nx - 1, qj > 0, qj < ny - 1, qk > 0, qk < nz - 1};
            for (int d = 0; d < 6; ++d) {
                if (inside[d]) {
                    int64_t r = q + off[d];
                    nv[d] = psi[r];
                    nk[d] = (G[r] == ORC_KNOWN_FIX || G[r] == ORC_KNOWN_NEW);
                } else {
                    nv[d] = (REAL)INFINITY;
                    nk[d] = 0;
                }
            }
            REAL t = FN(solve_quadratic)(psi[q], nv, nk, FN(rhs_of)(hr, F[q]), literal);
            if (t < psi[q]) {
                psi[q] = t;
                G[q] = ORC_BAND;
                if ((rc = FN(heap_push_or_up)(&hp, q)) != 0) goto done;
            }
        }
    }
    if (pops_out) *pops_out = pops;
    if (nonmono_out) *nonmono_out = nonmono;
done:
    free(hp.a);
    free(G);
    free(pos);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Multi-block sequential solver "S" (Sec. 3.1): Alg. 6 executed literally,  */
/* one block after another, with the per-block data of Sec. 2.3 (local psi,  */
/* tag and heap on the block padded by one ghost layer on each face), the    */
/* restarted bound of Sec. 2.4, the marching activation flag A of Sec. 2.5   */
/* and the exchange flags C / point sets Upsilon of Sec. 2.6.                */
/*                                                                           */
/* It is a second, independent statement of the block method, used to pin    */
/* block semantics and restart counts; the plain definition of the result    */
/* is orc_fmm above.                                                         */
/*                                                                           */
/* Tile-local index: t = li + P*(lj + P*lk), P = B + 2, li = 0 and B+1 are   */
/* ghost layers.  Faces f: 0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z.               */
/* bounds (nullable): bound of restart r is bounds[r-1] for r <= nbounds,    */
/* afterwards the last given bound plus stride per extra restart; without    */
/* bounds, bound_r = min(r * stride, width) evaluated in double.             */
/* ------------------------------------------------------------------------ */
typedef struct {
    REAL *psi;          /* [P^3]                                  */
    uint8_t *G;         /* [P^3]                                  */
    int32_t *pos;       /* [P^3]                                  */
    uint8_t *inY;       /* [P^3] membership in Upsilon            */
    int32_t *Y;         /* Upsilon as a list of tile indices      */
    int32_t nY;
    FN(heap_t) hp;
    int A;              /* activation for marching                */
    int C[6];           /* exchange flags, one per neighbour      */
    int64_t bx, by, bz; /* block coordinates                      */
} FN(blk_t);

static void FN(blk_free)(FN(blk_t) *b)
{
    free(b->psi);
    free(b->G);
    free(b->pos);
    free(b->inY);
    free(b->Y);
    free(b->hp.a);
}

/* Alg. 1 for every block: psi <- inf, G <- FAR, empty heap, A <- F; points of the
   padded block (interior and ghost faces) that are sources become KNOWN_FIX, enter
   the heap, and activate the block.  C <- F (Alg. 6).  blk holds nblk zeroed
   entries; on error the caller frees what was allocated. */
static int FN(blocks_init)(FN(blk_t) *blk, int64_t nx, int64_t ny, int32_t B, int64_t mx,
                           int64_t my, int64_t mz, int32_t nsrc, const int64_t *src_idx,
                           const REAL *src_val)
{
    const int64_t nblk = mx * my * mz;
    const int P = B + 2;
    const int64_t T = (int64_t)P * P * P;
    int rc = 0;
    for (int64_t ib = 0; ib < nblk; ++ib) {
        FN(blk_t) *b = &blk[ib];
        b->bx = ib % mx;
        b->by = (ib / mx) % my;
        b->bz = ib / (mx * my);
        b->psi = (REAL *)malloc((size_t)T * sizeof(REAL));
        b->G = (uint8_t *)malloc((size_t)T);
        b->pos = (int32_t *)malloc((size_t)T * sizeof(int32_t));
        b->inY = (uint8_t *)calloc((size_t)T, 1);
        b->Y = (int32_t *)malloc((size_t)T * sizeof(int32_t));
        if (!b->psi || !b->G || !b->pos || !b->inY || !b->Y) {
            rc = ORC_ENOMEM;
            return rc;
        }
        for (int64_t t = 0; t < T; ++t) {
            b->psi[t] = (REAL)INFINITY;
            b->G[t] = ORC_FAR;
            b->pos[t] = -1;
        }
        b->hp.pos = b->pos;
        b->hp.key = b->psi;
        b->nY = 0;
        b->A = 0;
        for (int f = 0; f < 6; ++f) b->C[f] = 0;
    }
    for (int32_t s = 0; s < nsrc; ++s) {
        const int64_t p = src_idx[s];
        const int64_t gi = p % nx, gj = (p / nx) % ny, gk = p / (nx * ny);
        /* every block whose padded region (interior or a ghost face) holds the point */
        for (int64_t bz = gk / B - 1; bz <= gk / B + 1; ++bz)
            for (int64_t by = gj / B - 1; by <= gj / B + 1; ++by)
                for (int64_t bx = gi / B - 1; bx <= gi / B + 1; ++bx) {
                    if (bx < 0 || by < 0 || bz < 0 || bx >= mx || by >= my || bz >= mz) continue;
                    int64_t li = gi - bx * B + 1, lj = gj - by * B + 1, lk = gk - bz * B + 1;
                    if (li < 0 || lj < 0 || lk < 0 || li > B + 1 || lj > B + 1 || lk > B + 1)
                        continue;
                    int ng = (li == 0 || li == B + 1) + (lj == 0 || lj == B + 1) +
                             (lk == 0 || lk == B + 1);
                    if (ng > 1) continue; /* ghost edges and corners are not part of Xi */
                    FN(blk_t) *b = &blk[bx + mx * (by + my * bz)];
                    int64_t t = li + P * (lj + P * lk);
                    if (src_val[s] < b->psi[t]) b->psi[t] = src_val[s];
                    b->G[t] = ORC_KNOWN_FIX;
                    if ((rc = FN(heap_push_or_up)(&b->hp, t)) != 0) return rc;
                    b->A = 1;
                }
    }

    return rc;
}

/* Interior of every block -> linear psi. */
static void FN(blocks_gather)(const FN(blk_t) *blk, int64_t nx, int64_t ny, int32_t B, int64_t nblk,
                              REAL *psi)
{
    const int P = B + 2;
    for (int64_t ib = 0; ib < nblk; ++ib) {
        const FN(blk_t) *b = &blk[ib];
        for (int lk = 1; lk <= B; ++lk)
            for (int lj = 1; lj <= B; ++lj)
                for (int li = 1; li <= B; ++li) {
                    int64_t g = (b->bx * B + li - 1) +
                                nx * ((b->by * B + lj - 1) + ny * (b->bz * B + lk - 1));
                    psi[g] = b->psi[li + (int64_t)P * (lj + (int64_t)P * lk)];
                }
    }
}

/* Alg. 4 (with Alg. 2 restricted to the block's interior) on block ib for one
   restart bound, then C^nb <- TRUE for every neighbour nb whose ghosts meet
   Upsilon^ib.  Touches only block ib, except the neighbours' C flags (written with
   atomic stores, so that several blocks may march at once). */
static int FN(march_one)(FN(blk_t) *blk, int64_t ib, int32_t B, int64_t mx, int64_t my, int64_t mz,
                         int64_t nx, int64_t ny, REAL hr, const REAL *F, double bound,
                         double width, int32_t literal, int64_t *pops)
{
    const int P = B + 2;
    const int64_t toff[6] = {-1, 1, -P, P, -(int64_t)P * P, (int64_t)P * P};
    int rc = 0;
    FN(blk_t) *b = &blk[ib];
    for (int32_t y = 0; y < b->nY; ++y) b->inY[b->Y[y]] = 0;
    b->nY = 0; /* Upsilon <- empty */
    for (;;) {
        if (b->hp.n == 0) {
            b->A = 0;
            break;
        }
        const int64_t p = b->hp.a[0];
        if ((double)b->psi[p] > bound) {
            if ((double)b->psi[p] > width) b->A = 0;
            break;
        }
        if (b->G[p] != ORC_KNOWN_FIX) b->G[p] = ORC_KNOWN_NEW;
        FN(heap_pop)(&b->hp);
        ++*pops;
        const int pi = (int)(p % P), pj = (int)((p / P) % P), pk = (int)(p / (P * P));
        /* Alg. 2 restricted to Omega^ib (interior points of the block) */
        for (int nb = 0; nb < 6; ++nb) {
            int qi = pi, qj = pj, qk = pk;
            switch (nb) {
            case 0: qi--; break;
            case 1: qi++; break;
            case 2: qj--; break;
            case 3: qj++; break;
            case 4: qk--; break;
            default: qk++; break;
            }
            if (qi < 1 || qi > B || qj < 1 || qj > B || qk < 1 || qk > B) continue;
            const int64_t q = qi + (int64_t)P * (qj + (int64_t)P * qk);
            if (b->G[q] == ORC_KNOWN_FIX || !(b->psi[q] > b->psi[p])) continue;
            const int64_t gq = (b->bx * B + qi - 1) +
                               nx * ((b->by * B + qj - 1) + ny * (b->bz * B + qk - 1));
            if (F[gq] == 0) continue;
            REAL nv[6];
            int nk[6];
            for (int d = 0; d < 6; ++d) {
                nv[d] = b->psi[q + toff[d]];
                nk[d] = (b->G[q + toff[d]] == ORC_KNOWN_FIX || b->G[q + toff[d]] == ORC_KNOWN_NEW);
            }
            REAL t = FN(solve_quadratic)(b->psi[q], nv, nk, FN(rhs_of)(hr, F[gq]), literal);
            if (t < b->psi[q]) {
                b->psi[q] = t;
                b->G[q] = ORC_BAND;
                if ((rc = FN(heap_push_or_up)(&b->hp, q)) != 0) return rc;
                /* Pi^ib: the block's own points that are ghosts of a neighbour */
                if ((qi == 1 || qi == B || qj == 1 || qj == B || qk == 1 || qk == B) && !b->inY[q]) {
                    b->inY[q] = 1;
                    b->Y[b->nY++] = (int32_t)q;
                }
            }
        }
    }
    /* C^nb(ib) <- TRUE for every neighbour nb whose ghosts meet Upsilon^ib */
    for (int32_t y = 0; y < b->nY; ++y) {
        const int64_t q = b->Y[y];
        const int qi = (int)(q % P), qj = (int)((q / P) % P), qk = (int)(q / (P * P));
        const int onface[6] = {qi == 1, qi == B, qj == 1, qj == B, qk == 1, qk == B};
        for (int f = 0; f < 6; ++f) {
            if (!onface[f]) continue;
            int64_t nbx = b->bx + (f == 1) - (f == 0);
            int64_t nby = b->by + (f == 3) - (f == 2);
            int64_t nbz = b->bz + (f == 5) - (f == 4);
            if (nbx < 0 || nby < 0 || nbz < 0 || nbx >= mx || nby >= my || nbz >= mz) continue;
            __atomic_store_n(&blk[nbx + mx * (nby + my * nbz)].C[f ^ 1], 1, __ATOMIC_RELAXED);
        }
    }
    return 0;
}

/* Alg. 5 on block ib: for every flagged face, the points of the neighbour's
   Upsilon that lie on ib's ghost layer are copied (value and category) when
   smaller and enter ib's heap; then C^ib <- F and the block is activated when its
   heap minimum is within width.  Writes only block ib; reads the neighbours'
   interior points and Upsilon lists, which no exchange writes. */
static int FN(exchange_one)(FN(blk_t) *blk, int64_t ib, int32_t B, int64_t mx, int64_t my,
                            double width)
{
    const int P = B + 2;
    int rc = 0;
    FN(blk_t) *b = &blk[ib];
    for (int f = 0; f < 6; ++f) {
        if (!b->C[f]) continue;
        int64_t nbx = b->bx + (f == 1) - (f == 0);
        int64_t nby = b->by + (f == 3) - (f == 2);
        int64_t nbz = b->bz + (f == 5) - (f == 4);
        const FN(blk_t) *o = &blk[nbx + mx * (nby + my * nbz)];
        /* points of Upsilon^nb that lie in the ghost layer Theta^ib on face f */
        for (int32_t y = 0; y < o->nY; ++y) {
            const int64_t q = o->Y[y];
            int qi = (int)(q % P), qj = (int)((q / P) % P), qk = (int)(q / (P * P));
            /* the neighbour's boundary layer facing ib is its face f^1 */
            const int onface[6] = {qi == 1, qi == B, qj == 1, qj == B, qk == 1, qk == B};
            if (!onface[f ^ 1]) continue;
            /* the same grid point in ib's tile */
            int gi = qi + (int)((nbx - b->bx) * B);
            int gj = qj + (int)((nby - b->by) * B);
            int gk = qk + (int)((nbz - b->bz) * B);
            const int64_t g = gi + (int64_t)P * (gj + (int64_t)P * gk);
            if (b->psi[g] > o->psi[q]) {
                b->psi[g] = o->psi[q];
                b->G[g] = o->G[q];
                if ((rc = FN(heap_push_or_up)(&b->hp, g)) != 0) return rc;
            }
        }
    }
    for (int f = 0; f < 6; ++f) b->C[f] = 0;
    if (b->hp.n > 0 && (double)b->psi[b->hp.a[0]] <= width) b->A = 1;
    return 0;
}

int FN(orc_block_fmm)(int64_t nx, int64_t ny, int64_t nz, double h, const REAL *F, int32_t nsrc,
                      const int64_t *src_idx, const REAL *src_val, int32_t B, double stride,
                      double width, const double *bounds, int32_t nbounds, int32_t literal,
                      int64_t max_restarts, REAL *psi, int64_t *restarts_out, int64_t *pops_out,
                      int64_t *march_calls_out, int64_t *exchange_calls_out)
{
    if (nx <= 0 || ny <= 0 || nz <= 0 || !(h > 0) || nsrc <= 0 || B <= 0) return ORC_EINVAL;
    if (nx % B || ny % B || nz % B || !(stride > 0)) return ORC_EINVAL;
    const int64_t N = nx * ny * nz;
    for (int32_t s = 0; s < nsrc; ++s)
        if (src_idx[s] < 0 || src_idx[s] >= N || !(src_val[s] >= 0)) return ORC_EINVAL;
    const int64_t mx = nx / B, my = ny / B, mz = nz / B, nblk = mx * my * mz;
    const REAL hr = (REAL)h;
    int rc = 0;
    FN(blk_t) *blk = (FN(blk_t) *)calloc((size_t)nblk, sizeof(FN(blk_t)));
    if (!blk) return ORC_ENOMEM;
    if ((rc = FN(blocks_init)(blk, nx, ny, B, mx, my, mz, nsrc, src_idx, src_val)) != 0) goto done;

    int64_t r = 0, pops = 0, march_calls = 0, exch_calls = 0;
    for (;;) {
        ++r;
        if (max_restarts > 0 && r > max_restarts) {
            rc = ORC_ENOCONV;
            break;
        }
        double bound;
        if (bounds && nbounds > 0) {
            if (r <= nbounds) bound = bounds[r - 1];
            else bound = bounds[nbounds - 1] + (double)(r - nbounds) * stride;
            if (bound > width) bound = width;
        } else {
            bound = (double)r * stride;
            if (bound > width) bound = width;
        }

        /* marching step: Alg. 4 on every block with A = TRUE */
        for (int64_t ib = 0; ib < nblk; ++ib) {
            if (!blk[ib].A) continue;
            ++march_calls;
            if ((rc = FN(march_one)(blk, ib, B, mx, my, mz, nx, ny, hr, F, bound, width, literal,
                                    &pops)) != 0)
                goto done;
        }

        /* exchanging step: Alg. 5 on every block with any C = TRUE */
        for (int64_t ib = 0; ib < nblk; ++ib) {
            const FN(blk_t) *b = &blk[ib];
            if (!(b->C[0] | b->C[1] | b->C[2] | b->C[3] | b->C[4] | b->C[5])) continue;
            ++exch_calls;
            if ((rc = FN(exchange_one)(blk, ib, B, mx, my, width)) != 0) goto done;
        }

        int any = 0;
        for (int64_t ib = 0; ib < nblk && !any; ++ib) any = blk[ib].A;
        if (!any) break;
    }

    if (rc == 0) FN(blocks_gather)(blk, nx, ny, B, nblk, psi);
    if (restarts_out) *restarts_out = r;
    if (pops_out) *pops_out = pops;
    if (march_calls_out) *march_calls_out = march_calls;
    if (exchange_calls_out) *exchange_calls_out = exch_calls;
done:
    for (int64_t ib = 0; ib < nblk; ++ib) FN(blk_free)(&blk[ib]);
    free(blk);
    return rc;
}

#undef FN
#undef ORC_CAT
#undef ORC_CAT2

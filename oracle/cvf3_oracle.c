/*
 * CVF water model on the periodic cubic lattice with eta: plain CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY -- see cvf3_oracle.h.  Loops follow the order in
 * which the paper (and the readings listed in the design notes) define the
 * steps; FP64 throughout, compiled with -ffp-contract=off.
 */
#include "cvf3_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static void philox(uint32_t index, uint32_t step, uint32_t sub, uint32_t stream, uint64_t seed, uint32_t out[4])
{
    uint32_t ctr[4] = { index, step, sub, stream };
    ocvf_philox4x32_10(ctr, seed, out);
}

/* ------------------------------------------------------------------------ */
/* U_LJ(V_iso) on the cubic lattice (Sec. II.A: hard core r0, cutoff 6 r0).  */
/* Cells are cubes of side r = v^(1/3) r0; each molecule interacts with all  */
/* lattice vectors n != 0 with r|n| <= 6 r0, half of every pair per molecule:*/
/*     u(v) = (1/2) sum_n 4[(r0/r|n|)^12 - (r0/r|n|)^6].                     */
/* With m = |n|^2 the sixth power of the distance is (r/r0)^6 m^3 = v^2 m^3, */
/* so no cube root is needed: s6 = 1/(v^2 m^3), the cutoff is v^2 m^3 <=     */
/* 6^6, and u(v) = 2 sum_m r3(m) (s6^2 - s6) over ascending m.               */
/* ------------------------------------------------------------------------ */
int32_t ocvf_r3(int32_t m)
{
    int32_t n = 0;
    for (int32_t i = -m; i <= m; ++i)
        for (int32_t j = -m; j <= m; ++j)
            for (int32_t k = -m; k <= m; ++k)
                if (i * i + j * j + k * k == m) ++n;
    return n;
}

static int32_t r3_cache[37];
static int r3_cached = 0;

double ocvf3_u_lj(double v)
{
    if (!(v >= 1.0)) return INFINITY;             /* inside the hard core */
    if (!r3_cached) {                              /* v >= 1 implies m <= 36 */
        for (int32_t m = 0; m <= 36; ++m) r3_cache[m] = ocvf_r3(m);
        r3_cached = 1;
    }
    double s = 0.0;
    for (int32_t m = 1; m <= 36; ++m) {
        double d6 = (v * v) * (double)(m * m * m);   /* (distance / r0)^6 */
        if (!(d6 <= 46656.0)) break;
        double s6 = 1.0 / d6;
        s = s + (double)r3_cache[m] * (s6 * s6 - s6);
    }
    return 2.0 * s;
}

/* ------------------------------------------------------------------------ */
/* eta (App. A).  Reading of the checkerboard cubes: the unit cubes whose    */
/* lowest corner has three even coordinates, and those whose lowest corner   */
/* has three odd coordinates.  Every cell is a corner of exactly one cube of */
/* each kind and every lattice edge lies in exactly one cube, so the cubes   */
/* partition the edges (3N = 12 N/4).  A cube's configuration marks the     */
/* eta = 0 edges; with each cube giving every one of its corners exactly one */
/* eta = 0 edge, every molecule has two eta = 0 and four eta = 1 edges, and  */
/* the eta = 0 edges form closed cycles, as App. A requires.  The            */
/* configurations with that property are the perfect matchings of the cube */
/* graph: nine of them, the count App. A gives.                              */
/* Cube corner (dx, dy, dz) in {0,1}^3 is vertex dx + 2 dy + 4 dz.  Edge e:  */
/* axis d = e / 4; the bits of r = e % 4 place it along the two other axes   */
/* (lower axis first): d = 0 -> (dy, dz), 1 -> (dx, dz), 2 -> (dx, dy).      */
/* ------------------------------------------------------------------------ */
static void edge_ends(int e, int *u, int *w)
{
    int d = e / 4, r = e % 4, lo = r & 1, hi = r >> 1;
    int dx = 0, dy = 0, dz = 0;
    if (d == 0) { dy = lo; dz = hi; }
    else if (d == 1) { dx = lo; dz = hi; }
    else { dx = lo; dy = hi; }
    *u = dx + 2 * dy + 4 * dz;
    *w = *u + (1 << d);
}

int32_t ocvf3_matchings(uint16_t out[16])
{
    int32_t n = 0;
    for (int mask = 0; mask < 4096; ++mask) {
        int deg[8] = { 0 };
        for (int e = 0; e < 12; ++e) {
            if (!(mask >> e & 1)) continue;
            int u, w;
            edge_ends(e, &u, &w);
            deg[u]++;
            deg[w]++;
        }
        int ok = 1;
        for (int v = 0; v < 8; ++v) ok = ok && deg[v] == 1;
        if (ok && n < 16) out[n++] = (uint16_t)mask;
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* Acceptance thresholds (same rule as the 2-D tables): dH <= 0 or           */
/* exp(-beta dH) >= 1 -> 2^32-1 (accept), else min(floor(exp(-beta dH)       */
/* 2^32), 2^32-2).  sigma move: dH = -th J_eff dh - J_sigma dc, th = theta * */
/* eta of the moving arm's edge, dh in {-1,0,1}, dc in {-5..5} (five other   */
/* arms).  eta move (liquid): dH = -J_eff dn, dn in {-4..4} the change of    */
/* N_HB_raw inside the cube.                                                  */
/* ------------------------------------------------------------------------ */
static uint32_t threshold(double beta, double dH)
{
    if (dH <= 0.0) return 0xFFFFFFFFu;
    double pa = exp(-beta * dH);
    if (pa >= 1.0) return 0xFFFFFFFFu;
    double f = floor(pa * 4294967296.0);
    return (f > 4294967294.0) ? 0xFFFFFFFEu : (uint32_t)f;
}

void ocvf3_tables(const ocvf_params *p, uint32_t met[2][3][11], uint32_t eta[9])
{
    double Jeff = p->J - p->P * p->vHB;
    for (int th = 0; th < 2; ++th)
        for (int dh = -1; dh <= 1; ++dh)
            for (int dc = -5; dc <= 5; ++dc)
                met[th][dh + 1][dc + 5] =
                    threshold(p->beta, -((double)th * Jeff * (double)dh) - p->Jsigma * (double)dc);
    for (int dn = -4; dn <= 4; ++dn) eta[dn + 4] = threshold(p->beta, -(Jeff * (double)dn));
}

/* ------------------------------------------------------------------------ */
/* Lattice: cell c = x + L (y + L z), periodic.                              */
/* ------------------------------------------------------------------------ */
static int64_t nb3(int32_t L, int64_t c, int a)
{
    int64_t x = c % L, y = (c / L) % L, z = c / ((int64_t)L * L);
    switch (a) {
    case 0: x = (x + 1) % L; break;
    case 1: x = (x + L - 1) % L; break;
    case 2: y = (y + 1) % L; break;
    case 3: y = (y + L - 1) % L; break;
    case 4: z = (z + 1) % L; break;
    default: z = (z + L - 1) % L; break;
    }
    return x + (int64_t)L * (y + (int64_t)L * z);
}

struct ocvf3_state {
    ocvf_params p;
    int64_t  N;
    uint8_t *sigma;     /* [6][N] */
    uint8_t *eta;       /* [3][N] */
    double   v;
    int32_t  theta;
    int64_t  t;
    int64_t  n_hb_raw, n_coop;
    int64_t  met_att, met_acc, eta_att, eta_acc, vol_att, vol_acc;
    uint32_t met[2][3][11];
    uint32_t etab[9];
    uint16_t match[16];
    uint32_t *mask;     /* [N], last SW step */
    uint32_t *label;    /* [6N], last SW step */
};

static void count3(const ocvf3_state *s, int64_t *hb, int64_t *coop, int64_t *cnt, int64_t *eta0)
{
    const int64_t N = s->N;
    const uint8_t *sg = s->sigma, *et = s->eta;
    int64_t h = 0, k = 0, z = 0;
    if (cnt) for (int i = 0; i < 6; ++i) cnt[i] = 0;
    for (int64_t c = 0; c < N; ++c) {
        for (int d = 0; d < 3; ++d) {
            int eq = sg[(2 * d) * N + c] == sg[(2 * d + 1) * N + nb3(s->p.L, c, 2 * d)];
            h += et[d * N + c] && eq;
            z += et[d * N + c] == 0;
        }
        for (int a = 0; a < 6; ++a)
            for (int b = a + 1; b < 6; ++b) k += sg[a * N + c] == sg[b * N + c];
        if (cnt) for (int a = 0; a < 6; ++a) cnt[sg[a * N + c]]++;
    }
    *hb = h;
    *coop = k;
    if (eta0) *eta0 = z;
}

/* The cell of corner vertex vtx of cube k, and the cell at the lower end of
 * cube edge e (the edge is eta[e / 4][that cell]).  Cube k: parity par =
 * k / h^3 (h = L/2), (i, j, l) from the rest, lowest corner (2i + par,
 * 2j + par, 2l + par). */
static int64_t cube_cell(int32_t L, int64_t k, int vtx)
{
    const int64_t h = L / 2, h3 = h * h * h;
    const int64_t par = k / h3, r = k % h3;
    const int64_t i = r % h, j = (r / h) % h, l = r / (h * h);
    int64_t x = (2 * i + par + (vtx & 1)) % L;
    int64_t y = (2 * j + par + (vtx >> 1 & 1)) % L;
    int64_t z = (2 * l + par + (vtx >> 2 & 1)) % L;
    return x + (int64_t)L * (y + (int64_t)L * z);
}

/* Initial state (the paper builds it on the host, App. B): sigma of cell c
 * from words 0..3 of Philox(c, 0, 0, INIT) (arms 0..3) and words 0, 1 of
 * Philox(c, 0, 1, INIT) (arms 4, 5), floor(w q / 2^32); eta of cube k from
 * configuration pick(word 0 of Philox(k, 0, 2, INIT), 9), NONE -> 0. */
ocvf3_state *ocvf3_create(const ocvf_params *p)
{
    ocvf3_state *s = (ocvf3_state *)calloc(1, sizeof(*s));
    s->p = *p;
    s->N = (int64_t)p->L * p->L * p->L;
    const int64_t N = s->N;
    s->sigma = (uint8_t *)malloc((size_t)(6 * N));
    s->eta = (uint8_t *)malloc((size_t)(3 * N));
    ocvf3_tables(p, s->met, s->etab);
    ocvf3_matchings(s->match);
    for (int64_t c = 0; c < N; ++c) {
        uint32_t w0[4], w1[4];
        philox((uint32_t)c, 0, 0, OCVF_INIT, p->seed, w0);
        philox((uint32_t)c, 0, 1, OCVF_INIT, p->seed, w1);
        uint32_t w[6] = { w0[0], w0[1], w0[2], w0[3], w1[0], w1[1] };
        for (int a = 0; a < 6; ++a) s->sigma[a * N + c] = (uint8_t)(((uint64_t)w[a] * (uint64_t)p->q) >> 32);
    }
    for (int64_t k = 0; k < N / 4; ++k) {
        uint32_t w[4];
        philox((uint32_t)k, 0, 2, OCVF_INIT, p->seed, w);
        int32_t m = ocvf_pick(w[0], 9);
        if (m < 0) m = 0;
        for (int e = 0; e < 12; ++e) {
            int u, x;
            edge_ends(e, &u, &x);
            s->eta[(e / 4) * N + cube_cell(p->L, k, u)] = (uint8_t)!(s->match[m] >> e & 1);
        }
    }
    s->v = p->v_init;
    s->theta = s->v < 2.0;
    count3(s, &s->n_hb_raw, &s->n_coop, NULL, NULL);
    return s;
}

void ocvf3_destroy(ocvf3_state *s)
{
    if (!s) return;
    free(s->sigma);
    free(s->eta);
    free(s->mask);
    free(s->label);
    free(s);
}

/* Volume move (Sec. II.B step 1), as in 2-D with the cubic-lattice U_LJ and
 * the eta-masked N_HB_raw: words 0, 1 of Philox(0, t, 0, VOL). */
static void volume_move3(ocvf3_state *s)
{
    if (s->p.flags & OCVF_NO_VOLUME_MOVE) return;
    uint32_t w[4];
    philox(0, (uint32_t)s->t, 0, OCVF_VOL, s->p.seed, w);
    s->vol_att++;
    double u = (double)((int64_t)2 * (int64_t)w[0] + 1 - 4294967296LL) * (1.0 / 4294967296.0);
    double v0 = s->v;
    double v1 = v0 + s->p.dv_max * u;
    if (v1 < 1.0) return;
    int32_t th0 = s->theta, th1 = v1 < 2.0;
    double Nd = (double)s->N;
    double dH = (Nd * (ocvf3_u_lj(v1) - ocvf3_u_lj(v0))) + ((s->p.P * Nd) * (v1 - v0))
              + (((double)(th1 - th0) * (s->p.P * s->p.vHB - s->p.J)) * (double)s->n_hb_raw);
    int acc = dH <= 0.0;
    if (!acc) acc = ((double)w[1] + 0.5) * (1.0 / 4294967296.0) < exp(-s->p.beta * dH);
    if (acc) {
        s->v = v1;
        s->theta = th1;
        s->vol_acc++;
    }
}

/* eta update (Sec. II.B step 2, App. A).  Reading: a Metropolis move per
 * cube with sigma fixed -- propose configuration pick(w0, 9) of
 * Philox(k, t, 0, ETA) (NONE: no move), accept with the eta table through w1
 * (always in the gas, where eta does not enter H).  The cubes share no edge
 * and eta enters H only through its own edge, so all cubes move at once. */
static void eta_update(ocvf3_state *s)
{
    const int32_t L = s->p.L;
    const int64_t N = s->N;
    for (int64_t k = 0; k < N / 4; ++k) {
        uint32_t w[4];
        philox((uint32_t)k, (uint32_t)s->t, 0, OCVF_ETA, s->p.seed, w);
        s->eta_att++;
        int32_t m = ocvf_pick(w[0], 9);
        if (m < 0) continue;
        int64_t cell[12];
        int eq[12], neu[12], dn = 0;
        for (int e = 0; e < 12; ++e) {
            int u, x, d = e / 4;
            edge_ends(e, &u, &x);
            cell[e] = cube_cell(L, k, u);
            eq[e] = s->sigma[(2 * d) * N + cell[e]] == s->sigma[(2 * d + 1) * N + cube_cell(L, k, x)];
            neu[e] = !(s->match[m] >> e & 1);
            dn += (neu[e] - (int)s->eta[d * N + cell[e]]) * eq[e];
        }
        int acc = 1;
        if (s->theta) {
            uint32_t thr = s->etab[dn + 4];
            acc = thr == 0xFFFFFFFFu || w[1] < thr;
        }
        if (!acc) continue;
        s->eta_acc++;
        for (int e = 0; e < 12; ++e) s->eta[(e / 4) * N + cell[e]] = (uint8_t)neu[e];
        s->n_hb_raw += dn;
    }
}

/* Pass order of step t (Sec. II.C: six arm passes per sweep, arm picked at
 * random): Fisher-Yates over 0..5 with words 0..3 of Philox(0, t, 0, ORD)
 * and word 0 of Philox(0, t, 1, ORD); position i swaps with
 * i + pick(w_i, 6 - i), NONE -> 0. */
void ocvf3_domain_order(const ocvf_params *p, uint32_t t, int32_t order[6])
{
    uint32_t a[4], b[4];
    philox(0, t, 0, OCVF_ORD, p->seed, a);
    philox(0, t, 1, OCVF_ORD, p->seed, b);
    uint32_t w[5] = { a[0], a[1], a[2], a[3], b[0] };
    for (int i = 0; i < 6; ++i) order[i] = i;
    for (int i = 0; i < 5; ++i) {
        int32_t k = ocvf_pick(w[i], (uint32_t)(6 - i));
        if (k < 0) k = 0;
        int32_t tmp = order[i];
        order[i] = order[i + k];
        order[i + k] = tmp;
    }
}

/* One arm-domain pass (Sec. II.C): arm a of every cell moves once.  The
 * domain's variables interact with none of each other (Fig. 3), so a
 * sequential loop equals the simultaneous update.  Words of arm a of cell
 * (x, y, z): Philox(x/2 + (L/2)(y + L z), t, a, DOM), words 0, 1 (proposal,
 * acceptance) for even x, 2, 3 for odd x.  The move: a state uniform over
 * the q - 1 others (pick NONE: no move), dh against the facing arm a^1 of
 * the neighbour in direction a, counted only when the edge's eta is 1, dc
 * against the five other arms of the cell. */
static void domain_pass3(ocvf3_state *s, int a)
{
    const int32_t L = s->p.L, q = s->p.q;
    const int64_t N = s->N;
    const int d = a >> 1;
    uint8_t *sg = s->sigma;
    for (int64_t c = 0; c < N; ++c) {
        const int64_t x = c % L, yz = c / L;
        uint32_t w[4];
        philox((uint32_t)((x >> 1) + (L / 2) * yz), (uint32_t)s->t, (uint32_t)a, OCVF_DOM, s->p.seed, w);
        uint32_t prop = (x & 1) ? w[2] : w[0];
        uint32_t accw = (x & 1) ? w[3] : w[1];
        int32_t k = ocvf_pick(prop, (uint32_t)(q - 1));
        if (k < 0) continue;
        const int64_t o = nb3(L, c, a);
        const int32_t old = sg[a * N + c], neu = (old + 1 + k) % q;
        const int32_t facing = sg[(a ^ 1) * N + o];
        const int32_t e = (a & 1) ? s->eta[d * N + o] : s->eta[d * N + c];
        int32_t dh = (neu == facing) - (old == facing);
        int32_t dc = 0;
        for (int b = 0; b < 6; ++b) {
            if (b == a) continue;
            dc += (neu == sg[b * N + c]) - (old == sg[b * N + c]);
        }
        uint32_t thr = s->met[s->theta && e][dh + 1][dc + 5];
        if (thr == 0xFFFFFFFFu || accw < thr) {
            sg[a * N + c] = (uint8_t)neu;
            s->n_hb_raw += e * dh;
            s->n_coop += dc;
            s->met_acc++;
        }
    }
    s->met_att += N;
}

void ocvf3_steps(ocvf3_state *s, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        volume_move3(s);
        eta_update(s);
        int32_t order[6];
        ocvf3_domain_order(&s->p, (uint32_t)s->t, order);
        for (int k = 0; k < 6; ++k) domain_pass3(s, order[k]);
        s->t++;
    }
}

void ocvf3_observables(const ocvf3_state *s, ocvf3_obs *o)
{
    memset(o, 0, sizeof(*o));
    int64_t hb, coop, z;
    count3(s, &hb, &coop, o->count, &z);
    double Nd = (double)s->N;
    o->step = s->t;
    o->n_hb_raw = hb;
    o->n_hb = s->theta ? hb : 0;
    o->n_coop = coop;
    o->n_eta0 = z;
    o->met_attempted = s->met_att;
    o->met_accepted = s->met_acc;
    o->eta_attempted = s->eta_att;
    o->eta_accepted = s->eta_acc;
    o->vol_attempted = s->vol_att;
    o->vol_accepted = s->vol_acc;
    o->v = s->v;
    o->V = (Nd * s->v) + (s->p.vHB * (double)o->n_hb);
    o->H = (((Nd * ocvf3_u_lj(s->v)) - (s->p.J * (double)o->n_hb)) - (s->p.Jsigma * (double)coop)) + (s->p.P * o->V);
    int64_t mx = 0;
    for (int i = 0; i < 6; ++i) if (o->count[i] > mx) mx = o->count[i];
    o->M = (double)mx / (6.0 * Nd);
}

void ocvf3_get_sigma(const ocvf3_state *s, uint8_t *out) { memcpy(out, s->sigma, (size_t)(6 * s->N)); }
void ocvf3_get_eta(const ocvf3_state *s, uint8_t *out) { memcpy(out, s->eta, (size_t)(3 * s->N)); }

void ocvf3_set_state(ocvf3_state *s, const uint8_t *sigma, const uint8_t *eta)
{
    if (sigma) memcpy(s->sigma, sigma, (size_t)(6 * s->N));
    if (eta) memcpy(s->eta, eta, (size_t)(3 * s->N));
    count3(s, &s->n_hb_raw, &s->n_coop, NULL, NULL);
}

int64_t ocvf3_incremental(const ocvf3_state *s, int64_t *n_hb_raw, int64_t *n_coop)
{
    *n_hb_raw = s->n_hb_raw;
    *n_coop = s->n_coop;
    return s->t;
}

/* ------------------------------------------------------------------------ */
/* Swendsen-Wang on the cubic lattice (Sec. II.D).  Links of cell c, bit l  */
/* of its 18-bit mask: l = 0..2 the covalent link of its +d edge (arm 2d of */
/* c with arm 2d+1 of the +d neighbour), l = 3..17 the cooperative pairs    */
/* (a, b), a < b, of its six arms in lexicographic order.  Cooperative: equal */
/* arms bond with p_sigma = 1 - exp(-beta J_sigma).  Covalent, only in the    */
/* liquid and on eta = 1 edges: equal facing arms bond with p_eff = 1 -      */
/* exp(-beta |J_eff|) when J_eff > 0, unequal ones when J_eff < 0.  Link l    */
/* uses word l mod 4 of Philox(c, t, l / 4, SWB); thresholds are 64-bit:     */
/* bond iff word < floor(p 2^32).  Clusters: label = smallest flat index;     */
/* each draws pick(word 0 of Philox(label, t, 0, SWF), q) (NONE -> 0) and all */
/* its bond indices shift by it mod q.                                       */
/* ------------------------------------------------------------------------ */
static const int pa3[15] = { 0, 0, 0, 0, 0, 1, 1, 1, 1, 2, 2, 2, 3, 3, 4 };
static const int pb3[15] = { 1, 2, 3, 4, 5, 2, 3, 4, 5, 3, 4, 5, 4, 5, 5 };

void ocvf3_components(int32_t L, const uint32_t *mask, uint32_t *label)
{
    const int64_t N = (int64_t)L * L * L, V = 6 * N;
    uint32_t *queue = (uint32_t *)malloc((size_t)V * sizeof(uint32_t));
    const uint32_t UNSET = 0xFFFFFFFFu;
    for (int64_t i = 0; i < V; ++i) label[i] = UNSET;
    for (int64_t start = 0; start < V; ++start) {
        if (label[start] != UNSET) continue;
        int64_t head = 0, tail = 0;
        label[start] = (uint32_t)start;
        queue[tail++] = (uint32_t)start;
        while (head < tail) {
            const int64_t idx = queue[head++];
            const int a = (int)(idx / N);
            const int64_t c = idx % N;
            int64_t nbr[6];
            int nn = 0;
            for (int l = 0; l < 15; ++l) {
                if (!(mask[c] >> (3 + l) & 1)) continue;
                if (pa3[l] == a) nbr[nn++] = pb3[l] * N + c;
                else if (pb3[l] == a) nbr[nn++] = pa3[l] * N + c;
            }
            const int d = a >> 1;
            if ((a & 1) == 0) {                      /* arm +d: link bit d of c */
                if (mask[c] >> d & 1) nbr[nn++] = (a + 1) * N + nb3(L, c, a);
            } else {                                 /* arm -d: link bit d of the -d neighbour */
                const int64_t o = nb3(L, c, a);
                if (mask[o] >> d & 1) nbr[nn++] = (a - 1) * N + o;
            }
            for (int i = 0; i < nn; ++i) {
                if (label[nbr[i]] == UNSET) {
                    label[nbr[i]] = (uint32_t)start;
                    queue[tail++] = (uint32_t)nbr[i];
                }
            }
        }
    }
    free(queue);
}

static void sw3_update(ocvf3_state *s)
{
    const int32_t L = s->p.L, q = s->p.q;
    const int64_t N = s->N;
    uint8_t *sg = s->sigma;
    const double Jeff = s->p.J - s->p.P * s->p.vHB;
    const double xs = s->p.beta * s->p.Jsigma, xe = s->p.beta * fabs(Jeff);
    const uint64_t thr_sigma = xs > 0.0 ? (uint64_t)floor(-expm1(-xs) * 4294967296.0) : 0;
    const uint64_t thr_eff = (s->theta && xe > 0.0) ? (uint64_t)floor(-expm1(-xe) * 4294967296.0) : 0;
    if (!s->mask) s->mask = (uint32_t *)calloc((size_t)N, sizeof(uint32_t));
    if (!s->label) s->label = (uint32_t *)calloc((size_t)(6 * N), sizeof(uint32_t));
    for (int64_t c = 0; c < N; ++c) {
        uint32_t w[20];
        for (int b = 0; b < 5; ++b) philox((uint32_t)c, (uint32_t)s->t, (uint32_t)b, OCVF_SWB, s->p.seed, w + 4 * b);
        uint32_t m = 0;
        for (int d = 0; d < 3; ++d) {
            const int eq = sg[(2 * d) * N + c] == sg[(2 * d + 1) * N + nb3(L, c, 2 * d)];
            int bond = 0;
            if (s->theta && s->eta[d * N + c]) {
                if (Jeff > 0.0) bond = eq && (uint64_t)w[d] < thr_eff;
                else if (Jeff < 0.0) bond = !eq && (uint64_t)w[d] < thr_eff;
            }
            if (bond) m |= 1u << d;
        }
        for (int l = 0; l < 15; ++l) {
            const int eq = sg[pa3[l] * N + c] == sg[pb3[l] * N + c];
            if (eq && (uint64_t)w[3 + l] < thr_sigma) m |= 1u << (3 + l);
        }
        s->mask[c] = m;
    }
    ocvf3_components(L, s->mask, s->label);
    for (int64_t idx = 0; idx < 6 * N; ++idx) {
        uint32_t w[4];
        philox(s->label[idx], (uint32_t)s->t, 0, OCVF_SWF, s->p.seed, w);
        int32_t r = ocvf_pick(w[0], (uint32_t)q);
        if (r < 0) r = 0;
        sg[idx] = (uint8_t)((sg[idx] + r) % q);
    }
    count3(s, &s->n_hb_raw, &s->n_coop, NULL, NULL);
}

void ocvf3_sw_steps(ocvf3_state *s, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        volume_move3(s);
        eta_update(s);
        sw3_update(s);
        s->t++;
    }
}

void ocvf3_get_labels(const ocvf3_state *s, uint32_t *out)
{
    if (s->label) memcpy(out, s->label, (size_t)(6 * s->N) * sizeof(uint32_t));
    else memset(out, 0, (size_t)(6 * s->N) * sizeof(uint32_t));
}

void ocvf3_get_mask(const ocvf3_state *s, uint32_t *out)
{
    if (s->mask) memcpy(out, s->mask, (size_t)s->N * sizeof(uint32_t));
    else memset(out, 0, (size_t)s->N * sizeof(uint32_t));
}

/*
 * CVF water model (2-D square-lattice reading): plain single-threaded CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY -- see cvf_oracle.h.  Nothing in the product path
 * links or loads this file.  Every loop here follows the order in which the
 * paper (and the readings listed in the design notes) define the steps; no
 * blocking, fusion or reordering.  Floating point is FP64 throughout and the
 * file is compiled with -ffp-contract=off.
 */
#include "cvf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11: "Parallel random       */
/* numbers: as easy as 1, 2, 3").  The paper draws its randoms from cuRAND  */
/* arrays (App. C); a counter-based generator gives the same per-site,      */
/* per-step independence without the arrays.  Counter = (index, step, sub,  */
/* stream), key = (seed mod 2^32, seed >> 32).                              */
/* ------------------------------------------------------------------------ */
void ocvf_philox4x32_10(const uint32_t ctr[4], uint64_t seed, uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {                 /* key schedule between rounds */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void philox(uint32_t index, uint32_t step, uint32_t sub, uint32_t stream,
                   uint64_t seed, uint32_t out[4])
{
    uint32_t ctr[4] = { index, step, sub, stream };
    ocvf_philox4x32_10(ctr, seed, out);
}

/* Exactly uniform integer in {0..k-1} from one 32-bit word, or -1 (NONE)
 * when w falls in the incomplete top block.  floor(2^32/k) in 64 bits. */
int32_t ocvf_pick(uint32_t w, uint32_t k)
{
    uint64_t d = ((uint64_t)1 << 32) / (uint64_t)k;
    if ((uint64_t)w < (uint64_t)k * d) return (int32_t)((uint64_t)w / d);
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Isotropic Lennard-Jones term U_LJ(V_iso) (Sec. II.A): hard core at r0,   */
/* cutoff 6 r0, eps = energy unit.  Reading for a monolayer of thickness   */
/* r0: every cell is a square of side r = sqrt(v) r0, so the molecules sit  */
/* on a square lattice of spacing r and each one interacts with all         */
/* lattice vectors n != 0 with r|n| <= 6 r0.  Per molecule (half of every   */
/* pair):  u(v) = (1/2) sum_n 4[(r0/r|n|)^12 - (r0/r|n|)^6].  Grouping the  */
/* lattice vectors by m = |n|^2 (r2(m) of them) gives                       */
/*     u(v) = 2 sum_{m>=1, v m <= 36} r2(m) (s(m)^2 - s(m)),  s = (v m)^-3, */
/* summed in ascending m.                                                   */
/* ------------------------------------------------------------------------ */
int32_t ocvf_r2(int32_t m)
{
    int32_t n = 0;
    for (int32_t i = -m; i <= m; ++i)
        for (int32_t j = -m; j <= m; ++j)
            if (i * i + j * j == m) ++n;
    return n;
}

static int32_t r2_cache[37];
static int r2_cached = 0;

double ocvf_u_lj(double v)
{
    if (!(v >= 1.0)) return INFINITY;          /* inside the hard core */
    if (!r2_cached) {                           /* v >= 1 implies m <= 36 */
        for (int32_t m = 0; m <= 36; ++m) r2_cache[m] = ocvf_r2(m);
        r2_cached = 1;
    }
    double s = 0.0;
    for (int32_t m = 1; v * (double)m <= 36.0; ++m) {
        double d2 = v * (double)m;              /* squared distance / r0^2 */
        double s6 = 1.0 / (d2 * d2 * d2);
        s = s + (double)r2_cache[m] * (s6 * s6 - s6);
    }
    return 2.0 * s;
}

/* ------------------------------------------------------------------------ */
/* Parameters of Table I in reduced units; SI-2019 exact N_A and k_B.       */
/* beta = eps / (R T), P* = P r0^3 N_A / eps, J = 4 * 0.5, J_sigma =        */
/* 4 * 0.08, v_HB = 0.6 (all in units of eps and v0 = r0^3).                 */
/* ------------------------------------------------------------------------ */
void ocvf_params_from_si(double T_kelvin, double P_MPa, ocvf_params *out)
{
    const double N_A = 6.02214076e23;     /* 1/mol */
    const double k_B = 1.380649e-23;      /* J/K */
    const double eps = 5.5e3;             /* J/mol, Table I */
    const double r0  = 2.9e-10;           /* m, Table I */
    const double R   = N_A * k_B;
    memset(out, 0, sizeof(*out));
    out->L      = 64;
    out->q      = 6;
    out->beta   = eps / (R * T_kelvin);
    out->J      = 4.0 * 0.5;
    out->Jsigma = 4.0 * 0.08;
    out->P      = ((P_MPa * 1.0e6) * (r0 * r0 * r0)) * N_A / eps;
    out->vHB    = 0.6;
    out->v_init = 1.25;
    out->dv_max = 0.01 * 1.25;
    out->seed   = 1;
    out->flags  = 0;
}

/* ------------------------------------------------------------------------ */
/* Acceptance tables.  Metropolis (Sec. II.C with Eq. (3)): flipping one     */
/* bond index changes the raw count of facing equal pairs by dh in {-1,0,1}  */
/* and the same-cell equal-pair count by dc in {-3..3}; with J_eff = J -     */
/* P v_HB (Fig. 1 caption) the enthalpy change is                            */
/*     dH = -theta J_eff dh - J_sigma dc.                                    */
/* thr = 2^32-1 (always accept) when dH <= 0 or exp(-beta dH) >= 1, else     */
/* min(floor(exp(-beta dH) 2^32), 2^32-2).  Swendsen-Wang (Sec. II.D):       */
/* bond probabilities p = 1 - exp(-beta |J|) as 64-bit thresholds           */
/* floor(p 2^32) for J_sigma, theta=0 (no covalent bond) and theta=1.        */
/* ------------------------------------------------------------------------ */
void ocvf_tables(const ocvf_params *p, uint32_t met[2][3][7], uint64_t sw[3])
{
    double Jeff = p->J - p->P * p->vHB;
    for (int th = 0; th < 2; ++th)
        for (int dh = -1; dh <= 1; ++dh)
            for (int dc = -3; dc <= 3; ++dc) {
                double dH = -((double)th * Jeff * (double)dh) - p->Jsigma * (double)dc;
                uint32_t thr;
                if (dH <= 0.0) {
                    thr = 0xFFFFFFFFu;
                } else {
                    double pa = exp(-p->beta * dH);
                    if (pa >= 1.0) {
                        thr = 0xFFFFFFFFu;
                    } else {
                        double f = floor(pa * 4294967296.0);
                        thr = (f > 4294967294.0) ? 0xFFFFFFFEu : (uint32_t)f;
                    }
                }
                met[th][dh + 1][dc + 3] = thr;
            }
    double xs = p->beta * p->Jsigma;
    sw[0] = (xs > 0.0) ? (uint64_t)floor(-expm1(-xs) * 4294967296.0) : 0;
    sw[1] = 0;                                   /* theta = 0: no covalent bonds */
    double xe = p->beta * fabs(Jeff);
    sw[2] = (xe > 0.0) ? (uint64_t)floor(-expm1(-xe) * 4294967296.0) : 0;
}

/* ------------------------------------------------------------------------ */
/* Lattice helpers: cell c = x + L y, periodic in both directions.          */
/* ------------------------------------------------------------------------ */
static int64_t nb(int32_t L, int64_t c, int a)
{
    int64_t x = c % L, y = c / L;
    switch (a) {
    case 0: x = (x + 1) % L; break;          /* +x */
    case 1: x = (x + L - 1) % L; break;      /* -x */
    case 2: y = (y + 1) % L; break;          /* +y */
    default: y = (y + L - 1) % L; break;     /* -y */
    }
    return x + (int64_t)L * y;
}

struct ocvf_state {
    ocvf_params p;
    int64_t  N;
    uint8_t *sigma;     /* [4][N] */
    uint8_t *mask;      /* [N], last SW step */
    uint32_t *label;    /* [4N], last SW step */
    double   v;
    int32_t  theta;
    int64_t  t;
    int64_t  n_hb_raw, n_coop;
    int64_t  met_att, met_acc, vol_att, vol_acc;
    uint32_t met[2][3][7];
    uint64_t sw[3];
};

static void count(const ocvf_state *s, int64_t *hb, int64_t *coop, int64_t *cnt)
{
    int64_t N = s->N, h = 0, k = 0;
    const uint8_t *sg = s->sigma;
    if (cnt) for (int i = 0; i < 6; ++i) cnt[i] = 0;
    for (int64_t c = 0; c < N; ++c) {
        h += sg[0 * N + c] == sg[1 * N + nb(s->p.L, c, 0)];
        h += sg[2 * N + c] == sg[3 * N + nb(s->p.L, c, 2)];
        for (int a = 0; a < 4; ++a)
            for (int b = a + 1; b < 4; ++b)
                k += sg[a * N + c] == sg[b * N + c];
        if (cnt) for (int a = 0; a < 4; ++a) cnt[sg[a * N + c]]++;
    }
    *hb = h;
    *coop = k;
}

/* Initial configuration of cell c: sigma[a] = floor(w_a q / 2^32) with
 * (w0..w3) = Philox(c, 0, 0, INIT). */
void ocvf_init_cell(const ocvf_params *p, int64_t c, uint8_t s4[4])
{
    uint32_t w[4];
    philox((uint32_t)c, 0, 0, OCVF_INIT, p->seed, w);
    for (int a = 0; a < 4; ++a) s4[a] = (uint8_t)(((uint64_t)w[a] * (uint64_t)p->q) >> 32);
}

ocvf_state *ocvf_create(const ocvf_params *p)
{
    ocvf_state *s = (ocvf_state *)calloc(1, sizeof(*s));
    s->p = *p;
    s->N = (int64_t)p->L * p->L;
    s->sigma = (uint8_t *)malloc((size_t)(4 * s->N));
    s->mask = (uint8_t *)calloc((size_t)s->N, 1);
    s->label = (uint32_t *)calloc((size_t)(4 * s->N), sizeof(uint32_t));
    ocvf_tables(p, s->met, s->sw);
    for (int64_t c = 0; c < s->N; ++c) {
        uint8_t s4[4];
        ocvf_init_cell(p, c, s4);
        for (int a = 0; a < 4; ++a) s->sigma[a * s->N + c] = s4[a];
    }
    s->v = p->v_init;
    s->theta = s->v < 2.0;                        /* gas-like iff v >= 2 */
    s->t = 0;
    count(s, &s->n_hb_raw, &s->n_coop, NULL);
    return s;
}

void ocvf_destroy(ocvf_state *s)
{
    if (!s) return;
    free(s->sigma);
    free(s->mask);
    free(s->label);
    free(s);
}

/* ------------------------------------------------------------------------ */
/* Volume move (Sec. II.B, step 1): Metropolis on v_iso with sigma fixed.    */
/* v' = v + dv_max u, u uniform and symmetric in (-1, 1); v' < 1 is inside   */
/* the hard core and rejected.  dH from Eq. (1) and (3):                     */
/*   dH = N (u(v') - u(v)) + P N (v' - v)                                    */
/*        + (theta(v') - theta(v)) (P v_HB - J) N_HB_raw.                    */
/* ------------------------------------------------------------------------ */
static void volume_move(ocvf_state *s)
{
    if (s->p.flags & OCVF_NO_VOLUME_MOVE) return;
    uint32_t w[4];
    philox(0, (uint32_t)s->t, 0, OCVF_VOL, s->p.seed, w);
    s->vol_att++;
    double u = (double)((int64_t)2 * (int64_t)w[0] + 1 - 4294967296LL) * (1.0 / 4294967296.0);
    double v0 = s->v;
    double v1 = v0 + s->p.dv_max * u;
    if (v1 < 1.0) return;
    int32_t th0 = s->theta;
    int32_t th1 = v1 < 2.0;
    double Nd = (double)s->N;
    double dH = (Nd * (ocvf_u_lj(v1) - ocvf_u_lj(v0)))
              + ((s->p.P * Nd) * (v1 - v0))
              + (((double)(th1 - th0) * (s->p.P * s->p.vHB - s->p.J)) * (double)s->n_hb_raw);
    int acc = dH <= 0.0;
    if (!acc) acc = ((double)w[1] + 0.5) * (1.0 / 4294967296.0) < exp(-s->p.beta * dH);
    if (acc) {
        s->v = v1;
        s->theta = th1;
        s->vol_acc++;
    }
}

/* ------------------------------------------------------------------------ */
/* One Metropolis sweep (Sec. II.C).  Reading: a two-colour checkerboard of  */
/* cells replaces the paper's arm domains -- cells of one colour share no    */
/* interaction, so all of them can move at once.  Colour 0 ((x+y) even)      */
/* first, then colour 1; inside a cell arms 0..3 in order.  Each arm: a      */
/* proposal uniform over the q-1 other states, dh against the facing arm,    */
/* dc against the three other arms, accept through the table.               */
/* ------------------------------------------------------------------------ */
/* The four arms of cell c at step t, in order 0..3: s4 the cell's bond
 * indices (updated in place), f4[a] the facing bond index of arm a (arm a^1
 * of the neighbour in direction a -- of the other colour, so fixed while the
 * cell moves), tab the acceptance table of the current theta.  Adds the
 * accepted changes of N_HB_raw and N_sigma and the acceptance count. */
/* One Metropolis move of arm a of a cell: proposal word prop, acceptance
 * word accw, s4 the cell's four bond indices, facing the bond index its arm
 * a faces. */
static void met_move(const ocvf_params *p, const uint32_t tab[3][7], int a, uint32_t prop, uint32_t accw,
                     uint8_t s4[4], int32_t facing, int64_t *d_hb, int64_t *d_coop, int64_t *n_acc)
{
    const int32_t q = p->q;
    int32_t k = ocvf_pick(prop, (uint32_t)(q - 1));
    if (k < 0) return;                             /* null move */
    int32_t old = s4[a];
    int32_t neu = (old + 1 + k) % q;
    int32_t dh = (neu == facing) - (old == facing);
    int32_t dc = 0;
    for (int b = 0; b < 4; ++b) {
        if (b == a) continue;
        int32_t sb = s4[b];
        dc += (neu == sb) - (old == sb);
    }
    uint32_t thr = tab[dh + 1][dc + 3];
    if (thr == 0xFFFFFFFFu || accw < thr) {
        s4[a] = (uint8_t)neu;
        *d_hb += dh;
        *d_coop += dc;
        ++*n_acc;
    }
}

void ocvf_met_cell(const ocvf_params *p, const uint32_t tab[3][7], int64_t c, uint32_t t, uint8_t s4[4],
                   const uint8_t f4[4], int64_t *d_hb, int64_t *d_coop, int64_t *n_acc)
{
    for (int a = 0; a < 4; ++a) {
        uint32_t w[4];
        philox((uint32_t)c, t, (uint32_t)(a >> 1), OCVF_MET, p->seed, w);
        uint32_t prop = (a & 1) ? w[2] : w[0];
        uint32_t accw = (a & 1) ? w[3] : w[1];
        met_move(p, tab, a, prop, accw, s4, f4[a], d_hb, d_coop, n_acc);
    }
}

static void metropolis_sweep(ocvf_state *s)
{
    const int32_t L = s->p.L;
    const int64_t N = s->N;
    uint8_t *sg = s->sigma;
    for (int colour = 0; colour < 2; ++colour) {
        for (int32_t y = 0; y < L; ++y) {
            for (int32_t x = 0; x < L; ++x) {
                if (((x + y) & 1) != colour) continue;
                int64_t c = x + (int64_t)L * y;
                uint8_t s4[4], f4[4];
                for (int a = 0; a < 4; ++a) {
                    s4[a] = sg[a * N + c];
                    f4[a] = sg[(a ^ 1) * N + nb(L, c, a)];
                }
                ocvf_met_cell(&s->p, s->met[s->theta], c, (uint32_t)s->t, s4, f4, &s->n_hb_raw, &s->n_coop,
                              &s->met_acc);
                s->met_att += 4;
                for (int a = 0; a < 4; ++a) sg[a * N + c] = s4[a];
            }
        }
    }
}

void ocvf_metropolis_sweeps(ocvf_state *s, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        volume_move(s);
        metropolis_sweep(s);
        s->t++;
    }
}

/* ------------------------------------------------------------------------ */
/* Arm-domain Metropolis sweep: the paper's own partition (Sec. II.C and its */
/* figure of layered domains), in 2-D.  Arm a of every cell forms a domain:  */
/* a bond index of arm a interacts with the three other arms of its cell and */
/* with arm a^1 of the neighbour in direction a, none of them in the domain, */
/* so a whole domain moves at once -- for any L, odd included.  A sweep is   */
/* four passes, one per domain.  The paper picks the arm of each pass at     */
/* random; reading: a uniform random permutation per sweep, so that every    */
/* bond index moves once per sweep, drawn by Fisher-Yates from the words of  */
/* Philox(0, t, 0, ORD) (position i swaps with i + pick(w_i, 4 - i); NONE,   */
/* possible only for w_1 = 2^32 - 1, leaves position 1 in place).            */
/* Words of arm a of cell (x, y) at step t: Philox(b, t, a, DOM) with        */
/* b = floor(x/2) + ceil(L/2) y (one block per column pair of a row), words  */
/* 0, 1 (proposal, acceptance) for even x and 2, 3 for odd x.                */
/* ------------------------------------------------------------------------ */
void ocvf_domain_order(const ocvf_params *p, uint32_t t, int32_t order[4])
{
    uint32_t w[4];
    philox(0, t, 0, OCVF_ORD, p->seed, w);
    for (int i = 0; i < 4; ++i) order[i] = i;
    for (int i = 0; i < 3; ++i) {
        int32_t k = ocvf_pick(w[i], (uint32_t)(4 - i));
        if (k < 0) k = 0;
        int32_t tmp = order[i];
        order[i] = order[i + k];
        order[i + k] = tmp;
    }
}

void ocvf_dom_arm(const ocvf_params *p, const uint32_t tab[3][7], int64_t c, uint32_t t, int32_t a,
                  uint8_t s4[4], uint8_t facing, int64_t *d_hb, int64_t *d_coop, int64_t *n_acc)
{
    const int64_t L = p->L, x = c % L, y = c / L;
    uint32_t w[4];
    philox((uint32_t)((x >> 1) + ((L + 1) >> 1) * y), t, (uint32_t)a, OCVF_DOM, p->seed, w);
    uint32_t prop = (x & 1) ? w[2] : w[0];
    uint32_t accw = (x & 1) ? w[3] : w[1];
    met_move(p, tab, a, prop, accw, s4, facing, d_hb, d_coop, n_acc);
}

static void domain_sweep(ocvf_state *s)
{
    const int32_t L = s->p.L;
    const int64_t N = s->N;
    uint8_t *sg = s->sigma;
    int32_t order[4];
    ocvf_domain_order(&s->p, (uint32_t)s->t, order);
    for (int k = 0; k < 4; ++k) {
        const int a = order[k];
        /* the domain's bond indices do not interact: updating them one after
         * another in place equals updating them all at once */
        for (int64_t c = 0; c < N; ++c) {
            uint8_t s4[4];
            for (int b = 0; b < 4; ++b) s4[b] = sg[b * N + c];
            uint8_t f = sg[(a ^ 1) * N + nb(L, c, a)];
            ocvf_dom_arm(&s->p, s->met[s->theta], c, (uint32_t)s->t, a, s4, f, &s->n_hb_raw, &s->n_coop,
                         &s->met_acc);
            sg[a * N + c] = s4[a];
        }
        s->met_att += N;
    }
}

void ocvf_metropolis_domain_sweeps(ocvf_state *s, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        volume_move(s);
        domain_sweep(s);
        s->t++;
    }
}

/* ------------------------------------------------------------------------ */
/* Connected components of the sigma graph (Sec. II.D, step 3).  The label   */
/* of every sigma is the smallest flat index in its cluster -- the fixed     */
/* point the label-equivalence method of Table II converges to.  Plain       */
/* definition: breadth-first search started from each not-yet-labelled      */
/* index in ascending order.                                                 */
/* Bond mask per cell: bit 0 covalent +x (arm 0 of c with arm 1 of c+x),     */
/* bit 1 covalent +y (arm 2 of c with arm 3 of c+y), bits 2..7 cooperative   */
/* pairs (0,1) (0,2) (0,3) (1,2) (1,3) (2,3) inside c.                        */
/* ------------------------------------------------------------------------ */
static const int pair_a[6] = { 0, 0, 0, 1, 1, 2 };
static const int pair_b[6] = { 1, 2, 3, 2, 3, 3 };

void ocvf_components(int32_t L, const uint8_t *mask, uint32_t *label)
{
    const int64_t N = (int64_t)L * L, V = 4 * N;
    uint32_t *queue = (uint32_t *)malloc((size_t)V * sizeof(uint32_t));
    const uint32_t UNSET = 0xFFFFFFFFu;
    for (int64_t i = 0; i < V; ++i) label[i] = UNSET;
    for (int64_t start = 0; start < V; ++start) {
        if (label[start] != UNSET) continue;
        int64_t head = 0, tail = 0;
        label[start] = (uint32_t)start;
        queue[tail++] = (uint32_t)start;
        while (head < tail) {
            int64_t idx = queue[head++];
            int a = (int)(idx / N);
            int64_t c = idx % N;
            int64_t nbr[5];
            int nn = 0;
            /* cooperative links inside cell c */
            for (int l = 0; l < 6; ++l) {
                if (!(mask[c] >> (2 + l) & 1)) continue;
                if (pair_a[l] == a) nbr[nn++] = pair_b[l] * N + c;
                else if (pair_b[l] == a) nbr[nn++] = pair_a[l] * N + c;
            }
            /* covalent link of this arm */
            if (a == 0 && (mask[c] & 1)) nbr[nn++] = 1 * N + nb(L, c, 0);
            if (a == 1) { int64_t o = nb(L, c, 1); if (mask[o] & 1) nbr[nn++] = 0 * N + o; }
            if (a == 2 && (mask[c] & 2)) nbr[nn++] = 3 * N + nb(L, c, 2);
            if (a == 3) { int64_t o = nb(L, c, 3); if (mask[o] & 2) nbr[nn++] = 2 * N + o; }
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

/* ------------------------------------------------------------------------ */
/* One Swendsen-Wang step (Sec. II.D, steps 1-4) after the volume move.      */
/* Step 1/2: fictitious bonds (cooperative: equal arms of one cell with      */
/* p_sigma; covalent: facing arms, equal if J_eff > 0 or unequal if J_eff <  */
/* 0, only in the liquid theta = 1, with p_eff).  Step 3: clusters.  Step 4: */
/* every cluster draws rnd_int in {0..q-1} (keyed by its label) and all its  */
/* sigma become (sigma + rnd_int) % q.                                       */
/* ------------------------------------------------------------------------ */
/* Bond activation of cell c at step t (Sec. II.D, step 1): s4 its bond
 * indices, f0 / f2 the facing bond indices of its arms 0 and 2 (arm 1 of the
 * +x neighbour, arm 3 of the +y neighbour).  Link l uses word l of
 * Philox(c, t, 0, SWB) for l < 4 and word l-4 of Philox(c, t, 1, SWB).
 * Returns the 8-bit link mask. */
uint8_t ocvf_sw_cell_mask(const ocvf_params *p, const uint64_t sw[3], int32_t theta, int64_t c, uint32_t t,
                          const uint8_t s4[4], uint8_t f0, uint8_t f2)
{
    double Jeff = p->J - p->P * p->vHB;
    uint64_t thr_sigma = sw[0];
    uint64_t thr_eff = sw[1 + theta];
    uint32_t w0[4], w1[4], w[8];
    philox((uint32_t)c, t, 0, OCVF_SWB, p->seed, w0);
    philox((uint32_t)c, t, 1, OCVF_SWB, p->seed, w1);
    for (int i = 0; i < 4; ++i) { w[i] = w0[i]; w[4 + i] = w1[i]; }
    uint8_t m = 0;
    for (int l = 0; l < 2; ++l) {
        int eq = s4[2 * l] == (l == 0 ? f0 : f2);            /* arm 0 or 2 against its partner */
        int bond = 0;
        if (theta == 1) {
            if (Jeff > 0.0) bond = eq && (uint64_t)w[l] < thr_eff;
            else if (Jeff < 0.0) bond = !eq && (uint64_t)w[l] < thr_eff;
        }
        if (bond) m |= (uint8_t)(1u << l);
    }
    for (int l = 0; l < 6; ++l) {
        int eq = s4[pair_a[l]] == s4[pair_b[l]];
        if (eq && (uint64_t)w[2 + l] < thr_sigma) m |= (uint8_t)(1u << (2 + l));
    }
    return m;
}

/* Cluster shift of the cluster whose minimum is root (Sec. II.D, step 4):
 * pick(word 0 of Philox(root, t, 0, SWF), q), a NULL draw shifts by 0. */
int32_t ocvf_sw_shift(const ocvf_params *p, uint32_t root, uint32_t t)
{
    uint32_t w[4];
    philox(root, t, 0, OCVF_SWF, p->seed, w);
    int32_t r = ocvf_pick(w[0], (uint32_t)p->q);
    return r < 0 ? 0 : r;
}

static void sw_step(ocvf_state *s)
{
    const int32_t L = s->p.L, q = s->p.q;
    const int64_t N = s->N;
    uint8_t *sg = s->sigma;
    for (int64_t c = 0; c < N; ++c) {
        uint8_t s4[4];
        for (int a = 0; a < 4; ++a) s4[a] = sg[a * N + c];
        s->mask[c] = ocvf_sw_cell_mask(&s->p, s->sw, s->theta, c, (uint32_t)s->t, s4, sg[1 * N + nb(L, c, 0)],
                                       sg[3 * N + nb(L, c, 2)]);
    }
    ocvf_components(L, s->mask, s->label);
    for (int64_t idx = 0; idx < 4 * N; ++idx)
        sg[idx] = (uint8_t)((sg[idx] + ocvf_sw_shift(&s->p, s->label[idx], (uint32_t)s->t)) % q);
    count(s, &s->n_hb_raw, &s->n_coop, NULL);
}

void ocvf_sw_steps(ocvf_state *s, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        volume_move(s);
        sw_step(s);
        s->t++;
    }
}

/* ------------------------------------------------------------------------ */
/* Observables: Eq. (1), Eq. (3), and the order parameter of Eq. (4)'s text  */
/* (normalised by the 4N bond indices of the 2-D lattice).                   */
/* ------------------------------------------------------------------------ */
void ocvf_observables(const ocvf_state *s, ocvf_obs *o)
{
    memset(o, 0, sizeof(*o));
    int64_t hb, coop;
    count(s, &hb, &coop, o->count);
    double Nd = (double)s->N;
    o->step = s->t;
    o->n_hb_raw = hb;
    o->n_hb = s->theta ? hb : 0;
    o->n_coop = coop;
    o->met_attempted = s->met_att;
    o->met_accepted = s->met_acc;
    o->vol_attempted = s->vol_att;
    o->vol_accepted = s->vol_acc;
    o->v = s->v;
    o->V = (Nd * s->v) + (s->p.vHB * (double)o->n_hb);
    o->H = (((Nd * ocvf_u_lj(s->v)) - (s->p.J * (double)o->n_hb)) - (s->p.Jsigma * (double)coop))
         + (s->p.P * o->V);
    int64_t mx = 0;
    for (int i = 0; i < 6; ++i) if (o->count[i] > mx) mx = o->count[i];
    o->M = (double)mx / (4.0 * Nd);
}

void ocvf_get_sigma(const ocvf_state *s, uint8_t *out) { memcpy(out, s->sigma, (size_t)(4 * s->N)); }

void ocvf_set_sigma(ocvf_state *s, const uint8_t *in)
{
    memcpy(s->sigma, in, (size_t)(4 * s->N));
    count(s, &s->n_hb_raw, &s->n_coop, NULL);
}

void ocvf_get_labels(const ocvf_state *s, uint32_t *out)
{
    memcpy(out, s->label, (size_t)(4 * s->N) * sizeof(uint32_t));
}

void ocvf_get_mask(const ocvf_state *s, uint8_t *out) { memcpy(out, s->mask, (size_t)s->N); }

int64_t ocvf_incremental(const ocvf_state *s, int64_t *n_hb_raw, int64_t *n_coop)
{
    *n_hb_raw = s->n_hb_raw;
    *n_coop = s->n_coop;
    return s->t;
}

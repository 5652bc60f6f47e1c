/*
 * CVF water model, 2-D square-lattice reading: plain single-threaded CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP library against
 * a slow, obviously correct implementation written from the paper (Coronas,
 * Vilanova, Franzese, "Efficient parallel algorithms for free-energy
 * calculation of millions of water molecules in the fluid phases").  Only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no source with the library.
 *
 * Model (Sec. II.A, Eq. (1)-(3), Table I), specialised to a periodic L x L
 * square lattice: every cell holds one molecule with four bond indices
 * sigma[a][c] in {0..q-1}, arm a = 0:+x, 1:-x, 2:+y, 3:-y; cell c = x + L*y;
 * flat index idx = a*N + c (the plane-major layout of Sec. II.C).
 * The eta constraint is trivially satisfied in 2-D (eta == 1).
 *
 * Parity status of each routine is stated next to it; every routine here has
 * a pin in tests/test_oracle_*.py.
 */
#ifndef CVF_ORACLE_H
#define CVF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox stream identifiers (fourth counter word). */
enum { OCVF_INIT = 0, OCVF_VOL = 1, OCVF_MET = 2, OCVF_SWB = 3, OCVF_SWF = 4, OCVF_ORD = 5, OCVF_DOM = 6 };

/* flags */
#define OCVF_NO_VOLUME_MOVE 1u

/* Reduced-unit parameters: energies in eps, volumes in v0 = r0^3. */
typedef struct {
    int32_t  L;        /* >= 2 (the checkerboard sweep and SW need it even) */
    int32_t  q;        /* 2..6 */
    double   beta;     /* 1 / T*  */
    double   J;        /* covalent HB energy (Table I: 4*0.5)       */
    double   Jsigma;   /* cooperative energy (Table I: 4*0.08)      */
    double   P;        /* P* = P r0^3 N_A / eps                     */
    double   vHB;      /* HB volume (Table I: 0.6)                  */
    double   v_init;   /* initial v_iso / v0 per molecule           */
    double   dv_max;   /* half-width of the uniform volume proposal */
    uint64_t seed;
    uint32_t flags;
    uint32_t pad_;
} ocvf_params;

typedef struct {
    int64_t step;
    int64_t n_hb_raw;   /* number of facing pairs with equal sigma            */
    int64_t n_hb;       /* theta * n_hb_raw: hydrogen bonds of Eq. (3)        */
    int64_t n_coop;     /* N_sigma of Eq. (3): equal same-cell arm pairs      */
    int64_t count[6];   /* N_q': number of sigma in state q' (Eq. (4) text)   */
    int64_t met_attempted, met_accepted, vol_attempted, vol_accepted;
    double  v;          /* v_iso / v0                                          */
    double  V;          /* Eq. (1) in units of v0                              */
    double  H;          /* Eq. (3) in units of eps                             */
    double  M;          /* max_q' N_q' / (4N)                                  */
} ocvf_obs;

typedef struct ocvf_state ocvf_state;

/* primitives */
void     ocvf_philox4x32_10(const uint32_t ctr[4], uint64_t seed, uint32_t out[4]);
int32_t  ocvf_pick(uint32_t w, uint32_t k);          /* -1 = NONE */
int32_t  ocvf_r2(int32_t m);                         /* #{(i,j): i^2+j^2 = m} */
double   ocvf_u_lj(double v);                        /* LJ energy per molecule */
void     ocvf_params_from_si(double T_kelvin, double P_MPa, ocvf_params *out);
void     ocvf_tables(const ocvf_params *p, uint32_t met[2][3][7], uint64_t sw[3]);

/* connected components of the sigma graph defined by a per-cell bond mask */
void     ocvf_components(int32_t L, const uint8_t *mask, uint32_t *label);

/* one cell (the sweeps are built from these; also usable on sampled cells of
 * lattices too large for a full oracle run) */
void     ocvf_init_cell(const ocvf_params *p, int64_t c, uint8_t s4[4]);
void     ocvf_met_cell(const ocvf_params *p, const uint32_t tab[3][7], int64_t c, uint32_t t, uint8_t s4[4],
                       const uint8_t f4[4], int64_t *d_hb, int64_t *d_coop, int64_t *n_acc);
uint8_t  ocvf_sw_cell_mask(const ocvf_params *p, const uint64_t sw[3], int32_t theta, int64_t c, uint32_t t,
                           const uint8_t s4[4], uint8_t f0, uint8_t f2);
int32_t  ocvf_sw_shift(const ocvf_params *p, uint32_t root, uint32_t t);
/* arm-domain sweep: pass order of step t, and one move of arm a of cell c */
void     ocvf_domain_order(const ocvf_params *p, uint32_t t, int32_t order[4]);
void     ocvf_dom_arm(const ocvf_params *p, const uint32_t tab[3][7], int64_t c, uint32_t t, int32_t a,
                      uint8_t s4[4], uint8_t facing, int64_t *d_hb, int64_t *d_coop, int64_t *n_acc);

/* Markov chain */
ocvf_state *ocvf_create(const ocvf_params *p);
void     ocvf_destroy(ocvf_state *s);
void     ocvf_metropolis_sweeps(ocvf_state *s, int64_t n);
void     ocvf_metropolis_domain_sweeps(ocvf_state *s, int64_t n);
void     ocvf_sw_steps(ocvf_state *s, int64_t n);
void     ocvf_observables(const ocvf_state *s, ocvf_obs *out);
void     ocvf_get_sigma(const ocvf_state *s, uint8_t *out);
void     ocvf_set_sigma(ocvf_state *s, const uint8_t *in);
void     ocvf_get_labels(const ocvf_state *s, uint32_t *out);
void     ocvf_get_mask(const ocvf_state *s, uint8_t *out);
int64_t  ocvf_incremental(const ocvf_state *s, int64_t *n_hb_raw, int64_t *n_coop);

#ifdef __cplusplus
}
#endif
#endif

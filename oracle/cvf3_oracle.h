/*
 * CVF water model on the periodic simple-cubic lattice, with the eta bond
 * constraint: plain single-threaded CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Like cvf_oracle.h (whose Philox, pick and
 * parameter struct it uses), this exists to check the HIP library against a
 * slow, obviously correct implementation written from the paper; only the
 * test-suite and the CPU-baseline leg of the benchmark may load it.
 *
 * Model (Sec. II.A, Eq. (1)-(3), Table I; App. A for eta).  Every cell of an
 * L x L x L periodic cubic lattice (L even) holds one molecule with six bond
 * indices sigma[a][c] in {0..q-1}, arm a = 0:+x 1:-x 2:+y 3:-y 4:+z 5:-z,
 * cell c = x + L*(y + L*z), flat index a*N + c (Sec. II.C's plane-major
 * layout).  Every lattice edge carries eta in {0, 1}; eta[d][c] belongs to the
 * edge from c to its +d neighbour (d = 0:x 1:y 2:z), so each edge is stored
 * once.  N_HB counts edges with eta = 1 and equal facing sigma (liquid only),
 * N_sigma the equal pairs among the 15 arm pairs of each cell.
 *
 * One MC step (Sec. II.B): volume move, eta update, then one arm-domain
 * Metropolis sweep of sigma (six passes, one per arm, in a random order).
 */
#ifndef CVF3_ORACLE_H
#define CVF3_ORACLE_H

#include <stdint.h>

#include "cvf_oracle.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Philox stream of the eta update (the others are shared with the 2-D model:
 * INIT, VOL, ORD, DOM). */
enum { OCVF_ETA = 7 };

typedef struct {
    int64_t step;
    int64_t n_hb_raw;   /* edges with eta = 1 and equal facing sigma          */
    int64_t n_hb;       /* theta * n_hb_raw                                    */
    int64_t n_coop;     /* N_sigma: equal pairs among the 15 arm pairs         */
    int64_t count[6];   /* N_q'                                                */
    int64_t n_eta0;     /* edges with eta = 0 (N of them in a valid state)     */
    int64_t met_attempted, met_accepted;
    int64_t eta_attempted, eta_accepted;
    int64_t vol_attempted, vol_accepted;
    double  v, V, H;
    double  M;          /* max_q' N_q' / (6N)                                  */
} ocvf3_obs;

typedef struct ocvf3_state ocvf3_state;

int32_t  ocvf_r3(int32_t m);                      /* #{(i,j,k): i^2+j^2+k^2 = m} */
double   ocvf3_u_lj(double v);                    /* LJ energy per molecule      */
/* the perfect matchings of the cube graph as 12-bit edge masks, ascending;
 * returns how many there are (edge numbering in cvf3_oracle.c) */
int32_t  ocvf3_matchings(uint16_t out[16]);
/* met[th][dh+1][dc+5]: sigma move; eta[dn+4]: eta move in the liquid */
void     ocvf3_tables(const ocvf_params *p, uint32_t met[2][3][11], uint32_t eta[9]);
void     ocvf3_domain_order(const ocvf_params *p, uint32_t t, int32_t order[6]);

ocvf3_state *ocvf3_create(const ocvf_params *p);
void     ocvf3_destroy(ocvf3_state *s);
void     ocvf3_steps(ocvf3_state *s, int64_t n);
/* Swendsen-Wang steps: volume move, eta update, then one SW update of sigma
 * (Sec. II.D on the cubic lattice). */
void     ocvf3_sw_steps(ocvf3_state *s, int64_t n);
/* connected components of the 6N bond indices under a per-cell 18-bit link
 * mask: label = smallest flat index of the cluster */
void     ocvf3_components(int32_t L, const uint32_t *mask, uint32_t *label);
void     ocvf3_get_labels(const ocvf3_state *s, uint32_t *out);   /* 6N, last SW step */
void     ocvf3_get_mask(const ocvf3_state *s, uint32_t *out);     /* N, last SW step  */
void     ocvf3_observables(const ocvf3_state *s, ocvf3_obs *out);
void     ocvf3_get_sigma(const ocvf3_state *s, uint8_t *out);   /* 6N bytes */
void     ocvf3_get_eta(const ocvf3_state *s, uint8_t *out);     /* 3N bytes */
void     ocvf3_set_state(ocvf3_state *s, const uint8_t *sigma, const uint8_t *eta);
int64_t  ocvf3_incremental(const ocvf3_state *s, int64_t *n_hb_raw, int64_t *n_coop);

#ifdef __cplusplus
}
#endif
#endif

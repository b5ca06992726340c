/*
 * ls_host.h — host-only view of the operator set-up (no device needed).
 *
 * The same set-up that ls_create runs before copying to the device: nodes
 * and weights (Sec. 2), the near-field rows carrying the singular and
 * interface quadratures (Sec. 3.1, eq:-VolInt-Adj-NonAdj-I).  Used to check
 * the set-up on machines without a GPU; it performs no operator apply.
 */
#ifndef LS_HOST_H
#define LS_HOST_H

#include "ls.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ls_host_op ls_host_op;

/* Run the host set-up only.  Same arguments and errors as ls_create
 * (minus LS_EDEVICE). */
ls_status ls_host_build(const ls_geometry* geom, ls_n2_fn n2, void* ctx, double kappa,
                        const ls_params* params, ls_host_op** out);
void ls_host_destroy(ls_host_op* h);
ls_status ls_host_num_points(const ls_host_op* h, int64_t* N);
/* xy[2N], key[3N] (may be NULL) in operator order, as ls_points. */
ls_status ls_host_points(const ls_host_op* h, double* xy, int32_t* key);
/* Sizes: N, boundary nodes, occupied cells, cells per axis, near-field CSR
 * rows, CSR entries, padded lattice Pa, Pb, U, F, S, window side
 * (the first nout of them). */
ls_status ls_host_stats(const ls_host_op* h, int64_t* out, int nout);
/* Near-field row i: every (column, coefficient) pair the apply adds for
 * target i besides the equivalent-source far field, i.e. the adjacent plain
 * quadrature (1 - eta) G c, the cut-off tails -eta G c of non-adjacent
 * sources and the singular rules.  count receives the number of entries;
 * at most cap are written (cols[cap], vals[2 cap] interleaved complex).
 * Entries with the same column may repeat (shared window and CSR parts).
 * With Fourier refinement (ls_params.fft_refine = r > 1) columns N and
 * beyond are refined band values: column N + ((s - 1) (N2 + 1) + u) N1 + v
 * holds the trigonometric interpolant of line u of the boundary-patch
 * density (m omega J) u at t1 = v + s / r.  With fft_refine_interior also,
 * column N + (r - 1)(N2 + 1) N1 + ((s - 1) M + gy) M + gx (s = s2 r + s1 > 0)
 * holds the two-dimensional trigonometric interpolant (period M) of the
 * interior density (m omega) u at lattice index (gx + s1 / r, gy + s2 / r)
 * + (c_lo - 2) cell_h, c_lo the smallest cell index of the nodes.  With
 * offgrid_shortcut, rows i = N .. N + n_s - 1 are the boundary rule at the
 * patch's grid nodes in line order (t2 line u, then t1 index v), whose
 * values the other rows read at column N + s_off + u N1 + v, s_off the
 * columns of the refinements before them; the refined s lines follow as
 * the densities' do. */
ls_status ls_host_near_row(const ls_host_op* h, int64_t i, int64_t cap, int32_t* cols, double* vals,
                           int64_t* count);

#ifdef __cplusplus
}
#endif
#endif /* LS_HOST_H */

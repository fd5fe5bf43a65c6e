/*
 * lbib_batch.h - batched parameter sweeps of the LB-IB solver (C ABI).
 *
 * The paper studies many independent capillary configurations: red-cell
 * distributions, particle release positions, stiffness Ca in {0, 1e-2} and
 * bond strength sigma in {0.5, 1, 2} (Sec. 1 and Sec. 4).  A batch advances
 * many such instances, each with its own lattice size, bodies, receptors and
 * parameters, in lock-step: every kernel of a time step is launched once for
 * all instances (flat work lists over instance tiles, bodies and markers),
 * and lbib_set_graph_steps captures chunks of steps in one HIP graph.
 *
 * A batch is an lbib_ctx: after lbib_batch_create the usual
 * lbib_workspace_query / lbib_bind / lbib_finalize_setup / lbib_step /
 * lbib_set_graph_steps / lbib_diagnostics / lbib_get_state / lbib_set_state /
 * lbib_destroy apply to it.  Single-instance readback calls (lbib_get_fields,
 * lbib_get_markers, lbib_get_bonds, ...) address instance 0; the calls below
 * address any instance.  Set-up calls (add_body, ...) are refused on a batch.
 */
#ifndef LBIB_BATCH_H
#define LBIB_BATCH_H

#include "lbib.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Build a batch from n >= 1 single-lattice contexts that are still in their
 * set-up phase (their descriptions are copied; they stay usable and must be
 * destroyed separately).  All must share the dtype.  tile_x, tile_y: tile
 * shape for the whole batch (0, 0 = default 64 x 4), typically picked by the
 * autotuner of the Python binding.  Instance i keeps the Philox key and
 * instance number of its own lattice description. */
lbib_status lbib_batch_create(const lbib_ctx* const* insts, int32_t n, int32_t tile_x,
                              int32_t tile_y, lbib_ctx** out);

/* Number of instances of a batch (1 for a plain context). */
lbib_status lbib_batch_size(const lbib_ctx* batch, int32_t* n);

/* Per-instance readback; same layouts as the single-instance calls. */
lbib_status lbib_batch_get_fields(lbib_ctx* batch, int32_t inst, double* rho, double* ux,
                                  double* uy);
lbib_status lbib_batch_get_markers(lbib_ctx* batch, int32_t inst, int32_t body, double* xy);
lbib_status lbib_batch_get_bonds(lbib_ctx* batch, int32_t inst, int32_t* lig_to_rec,
                                 int32_t* nbonds);

#ifdef __cplusplus
}
#endif

#endif /* LBIB_BATCH_H */

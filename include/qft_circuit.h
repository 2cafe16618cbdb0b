/*
 * qft_circuit.h - general fused-circuit execution (libqft.so).
 *
 * The QFT plans of qft.h know the structure of the QFT circuit (its
 * controlled phases commute and collapse into per-pass diagonals).  This
 * interface runs any list of one- and two-qubit gates on a 2^n-amplitude
 * state with the same conventions (qubit q_j = bit j of the array index,
 * Sec. 2 one-wire gate I_{2^{n-1-j}} (x) U (x) I_{2^j}), fusing runs of
 * consecutive gates whose qubits fit in one tile into a single HBM pass
 * (the paper's gate fusion, Sec. 2 and Sec. 3.1, done here for tiles in
 * LDS): a pass loads a tile of the state into LDS, applies its gates there
 * in circuit order, and stores the tile.
 *
 * A pass needs in its tile only the qubits whose amplitudes its gates mix:
 * targets of non-diagonal gates and both qubits of a SWAP.  Controls and
 * diagonal gates (one- or two-qubit, u01 = u10 = 0) only select or scale
 * amplitudes; the value of any qubit is known for every element of a tile
 * from its global index, so they need no tile qubit.  Runs of consecutive
 * diagonal gates (which commute) are applied as one scaling per element.
 *
 * Gates (all matrices in FP64, row-major, complex as (re, im) pairs):
 *  - one-qubit U on q: |0>,|1> components of every pair (i, i + 2^q) with
 *    bit q of i clear are mapped by U;
 *  - controlled U (control c, target t): U on t where bit c is 1;
 *  - SWAP of two qubits.
 */
#ifndef QFT_MI355X_CIRCUIT_H
#define QFT_MI355X_CIRCUIT_H

#include <stddef.h>

#include "qft.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qft_circuit_s qft_circuit_t;

/* An empty circuit on n qubits (1..QFT_MAX_QUBITS) for states of the
 * layout's element type (QFT_C64 or QFT_C128; other layout bits ignored).
 * NULL on error (qft_last_error).                                           */
qft_circuit_t *qft_circuit_create(int n, int layout);
void qft_circuit_destroy(qft_circuit_t *c);

/* Append gates.  u = {re00, im00, re01, im01, re10, im10, re11, im11}.
 * Appending after qft_circuit_compile invalidates the compiled passes (the
 * next execute compiles again).  QFT_ERR_INVALID for bad qubit indices.     */
int qft_circuit_add_1q(qft_circuit_t *c, int q, const double u[8]);
int qft_circuit_add_controlled(qft_circuit_t *c, int control, int target, const double u[8]);
int qft_circuit_add_swap(qft_circuit_t *c, int a, int b);

/* Group the gates into passes and upload their matrices (device memory of
 * the current device, owned by the circuit).  tile_qubits: the number of
 * qubits a pass may mix (see above), at most the tile size T = min(n, 13)
 * for complex64 and min(n, 12) for complex128; the other tile bits are the
 * lowest qubits the pass does not mix, so that rows of the tile are
 * contiguous.  0 = default: T - 3 (complex64) or T - 2 (complex128), rows of
 * 64 bytes.  The grouping is greedy over the gate list: a pass takes gates
 * in order until the next gate would bring in one qubit too many.           */
int qft_circuit_compile(qft_circuit_t *c, int tile_qubits);

/* Host only (no device use): the grouping qft_circuit_compile would make.
 * Returns the number of passes P (or a negative error code) and fills
 * gate_begin[i] (index of the first gate of pass i) and tile_bits[i] (tile
 * bits of pass i) for i < min(P, max_passes); either array may be NULL.
 * Leaves the circuit uncompiled.                                           */
int qft_circuit_describe(qft_circuit_t *c, int tile_qubits, int *gate_begin, int *tile_bits,
                         int max_passes);

/* Number of gates and of HBM passes of the compiled circuit (-1 passes if
 * it is not compiled).                                                     */
int qft_circuit_info(const qft_circuit_t *c, int *gates, int *passes);

/* Apply the circuit to dev_ptr (2^n elements, in place), asynchronously on
 * `stream` (compiling first if needed).  Executes of one circuit must be
 * ordered on one stream.                                                    */
int qft_circuit_execute(qft_circuit_t *c, void *dev_ptr, qft_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* QFT_MI355X_CIRCUIT_H */

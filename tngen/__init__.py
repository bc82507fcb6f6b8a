"""Seeded synthetic workload generators for sliced tensor-network contraction.

This package builds the *inputs* of the contraction method: quantum circuits,
the tensor network of one amplitude (leaf tensors + index labels), a pairwise
contraction path and a set of sliced indices.  It performs no contraction
arithmetic: leaf tensors are gate matrices reshaped, with entries *selected*
for the fixed input state |0> and the output bitstring, never multiplied.

Both the HIP library's tests/benchmarks and the CPU oracle consume what this
package produces; neither side's arithmetic lives here.
"""

from . import gates, circuits, network, path, slicing, workloads  # noqa: F401

"""CPU oracle for sliced tensor-network contraction — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP library never calls it and it
never calls the HIP library: the two share no code.  Inputs come from the
seeded generators in ``tngen`` (which hold no contraction arithmetic).

Modules
-------
statevector  brute-force state-vector simulation (complex128): amplitudes and
             the adjoint-method gradient of -mean log|amp|^2.
tn_oracle    plain pairwise contraction of a tensor network along a path, one
             slice at a time, complex128, no reuse; slice partial sums added in
             slice-id order (Eq. sliced_sum).
taskgraph    brute-force enumeration of named tasks over all slices (Sec. 3.2)
             -> instance counts and multiply-add totals with / without reuse.
grad         central finite differences of the state-vector loss.

Every function states the passage it follows; what pins it is listed in
``tests/test_oracle.py``.
"""

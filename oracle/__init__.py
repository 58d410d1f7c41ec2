"""FP64 CPU oracle for circuit amplitudes and linear XEB.  TEST INFRASTRUCTURE.

This package is the checker, not the product.  Only the test suite, the smoke
check of the entry module and the CPU-baseline leg of the benchmark may import
or run it.  It shares no code with the GPU library: it has its own reading of
the circuit description, its own gate matrices, its own tensor network (the
unfused one, with one tensor per gate) and its own contraction order.

What it computes (Supplementary Information, Sec. II): the amplitude of a
bitstring b is <b|psi>, psi the circuit applied to |0...0>; the tensor
network with every output index fixed to b contracts to that number, and
fixing some outputs while leaving others open gives a block of correlated
amplitudes.  Slicing (Sec. IV.B) writes a network as the sum of the networks
with a set of indices fixed, so the sum over slices equals the unsliced
contraction.  Linear XEB is the reading of Eq. (2) given in the xeb module.

Modules:
  gates        gate matrices transcribed from Sec. I
  circuit      parsing of the grid-rqc-v1 circuit description
  statevector  dense state-vector simulation (n <= 30)
  tn           plain tensor-network contraction with numpy.tensordot,
               optional open legs and optional slicing
  xeb          linear cross-entropy benchmarking fidelity

Pins (tests/test_oracle_*.py) fix each part against something other than
itself: closed forms of the gates, unitarity, the Porter-Thomas mean, brute
force on tiny circuits, normalisation, permutation circuits with known
amplitudes, and slice-sum invariance.
"""

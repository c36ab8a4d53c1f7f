"""The oracle: a plain, slow, obviously correct CPU implementation of the
Hubbard Hamiltonian-variational state-vector path (complex128).

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import, call, link or execute anything in
this package.  The GPU library shares no code, header, table or helper with
it and never calls it; the oracle never imports the GPU package.

Modules:
  model        own lattice enumeration, hopping groups, checkerboard start
  core         ctypes wrapper of hubbard_oracle.c (plain complex128 loops)
  dense        Kronecker-product Jordan-Wigner matrices, eigh/expm, forward-mode
               gradients (independent mechanism, <= ~12 qubits)
  freefermion  Slater-determinant / Wick special case (reaches 32 qubits)

Pins that tie these to the paper and to textbook results live in
tests/test_oracle_pins.py.
"""

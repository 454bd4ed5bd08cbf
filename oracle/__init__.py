"""Plain FP64 CPU oracle for the SCALE local-energy hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library: it recomputes every amplitude from scratch (full network forward and
a full determinant per spin) for every configuration it is asked about.

Modules:
  lattice  - site indexing, neighbours, hop enumeration (Sec. III, Hubbard
             Hamiltonian)
  ansatz   - embedding, residual conv stack, orbital projection, Slater
             determinant amplitude (Sec. II.B)
  energy   - local energy and per-hop amplitude ratios (Sec. II.A definition
             of E_loc with the Sec. III Hamiltonian)
  philox   - Philox4x64-10 counter-based generator (Salmon et al., SC'11)
  sampler  - Metropolis single-electron hop sampler (Sec. II.A, MCMC)
  grad     - d log|psi| / d theta by central finite differences

Every function is pinned by tests in ``tests/test_oracle_*.py`` against
closed forms, brute-force Hilbert-space sums, a library convolution and
invariants (see each test's docstring).
"""

"""FP64 CPU oracle for the parallelized traveling cluster approximation (TCA).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
HIP path is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it; the product library
(``paper_1502_07028_amd``) never imports, links or calls anything here, and it
shares no code with it (the two sides each implement Philox4x64-10 from its
published definition).

What it computes (paper: Mukherjee, Patel, Bishop, Dagotto, "Parallelized
Traveling Cluster Approximation to Study Numerically Spin-Fermion Models on
Large Lattices", arXiv:1502.07028):

* the sequential TCA Monte Carlo sweep of Sec. II(c) (Fig. 2 flowchart):
  gather the cluster around the update site, diagonalize the cluster
  Hamiltonian before and after a random change of the classical spin, decide
  by Metropolis, commit;
* the four-block visiting order of the parallel scheme, Sec. III(a) (Fig. 3),
  and a snapshot-batched variant of it used to check that the block schedule
  reproduces the sequential sweep;
* the spin structure factor of Eq. (2);
* the cluster matrix and classical energy of the Hubbard mean-field model the
  paper benchmarks (Eq. (1)), in two and three dimensions (``hubbard_mf``;
  the GPU path does not implement this model yet).

Readings of points the paper leaves open (the double-exchange Hamiltonian, the
free-energy formula, the RNG, the proposal distribution, where the classical
superexchange term is evaluated) are stated in each module's docstring.

Parity status per function is stated in each module header; every function
here is pinned by a ``-m "not gpu"`` test against a closed form, an invariant,
an independent library routine or brute force.
"""

"""FP64 CPU oracle for the short-range pair-loop path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package's smoke check
and the benchmark's CPU-baseline leg may import anything from here; the
product path never calls it and never falls back to it.

The oracle is written directly from the paper's definitions in plain
numpy / scipy FP64, slow and obviously correct:

* ``oracle.lj``    all-pairs minimum-image neighbour sets, Lennard-Jones
  potential/force (Eqs. LJpotential, LJforce), energy, virial, and the
  velocity-Verlet loop (Alg. VelocityVerlet).
* ``oracle.boa``   Steinhardt bond-order parameters (Eqs. Qell, qellm;
  Algs. sph_I / sph_II), spherical harmonics from scipy.
* ``oracle.thermostat``  the Andersen thermostat of the crystallisation run
  (Sec. 5.2) with Philox4x64-10 random numbers (readings in its header).
* ``oracle.cna``   common-neighbour analysis with literal Python sets
  (Eqs. Ei, Ei_ordered, Algs. cna_I/II/III, Alg. max_cluster_size).
* ``oracle.descriptor`` / ``oracle.mlp``  the descriptor-MLP potential
  (not in the paper; definitions stated in their headers).

It shares no code with the device library and imports nothing from it.
"""

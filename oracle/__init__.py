"""Plain FP64 CPU oracle for the TTN node update of (3+1)D lattice QED.

This package is TEST INFRASTRUCTURE.  Only the test-suite, the smoke entry
point and the CPU-baseline leg of the benchmark may import it.  It shares no
code with the HIP library: it is written from the paper (arXiv:2011.10658,
"Lattice Quantum Electrodynamics in (3+1)-dimensions at finite density with
Tensor Networks") in plain NumPy float64, favouring obviousness over speed.

Modules
  lattice      geometry: sites, links, plaquettes, half-link directions
  basis        gauge-invariant dressed-site basis (Methods, local basis eq.)
  fermions     site-local operators from an explicit fermionic Fock space
  hamiltonian  the lattice Hamiltonian (Eq. 1) + link penalty as a term list
  ed           exact diagonalisation, original (psi, E, U) formulation and
               dressed-site formulation
  blocks       U(1) block tables of three-leg tensors and leg operators
  heff         effective Hamiltonian of one tree node: dense definition and
               a per-block evaluation pinned to it
  lanczos      Lanczos eigensolver with full reorthogonalisation
  ttn          binary tree tensor network, sector allocation, sweeps,
               QR isometrisation, renormalisation, observables
"""

"""FP64 CPU oracle for SU(2) two-site H.psi -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import or run anything in this package.  It shares no code with the HIP
library: it reads the same seeded inputs (paper_2309_16724_amd.synth) and
computes the effective Hamiltonian's action from its plain definition,
y = P^T H P psi, in the M-resolved (U(1)) product basis.

Modules
  wigner   Clebsch-Gordan, W6j (Racah sum), W9j (sum of three 6j), C~ (Eq. 4)
  fock     determinant-space Hamiltonian, full CI, <S^2>, and P^T H P
  layout   canonical list of SU(2) wavefunction blocks
  hpsi     H_eff psi through the M-resolved expansion of the reduced blocks
  davidson plain Davidson solver
  renorm   the enlarged left block's operators after renormalization
Parity status of every function is stated in its module header.
"""

"""Plain FP64 CPU oracle for the open-shell (T) energy of one LIS domain.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package: it is used by ``tests/``, by the
``smoke()`` check and by the CPU-baseline leg of the benchmark, and by the
committed script that writes stored expected values under ``tests/golden``.
It shares no code with the GPU path (it never imports the HIP package), and
it is deliberately slow and simple: NumPy float64, one occupied triplet at a
time, full virtual cubes, library matmul/einsum as the only building block.

Modules
  blocks   spin-blocked restricted loops over unique occupied triplets (the
           "plain FP64 CPU (T)"): energy, its E[4]/E_ST/E_DT parts, per-item
           values, for any item list.
  spinorb  brute-force spin-orbital evaluation of the master formula with the
           1/36 weight over all ordered occupied triples (tiny domains only).
  rhf      closed-shell (T) formula for alpha == beta inputs.
  grad     gradient of the energy with respect to T1, T2, the DF factors,
           f_ov and the orbital energies (PyTorch float64 CPU reverse mode
           over a transcription of the spin-blocked energy; projected
           convention for symmetric inputs).
  naf      natural auxiliary functions: the spin-averaged W of eq. naf_w,
           its eigenvectors above a threshold, and the compressed factors.
  central  the (T) share of one central LMO (eq. local_pt): the central
           occupied index rotated to a vector c, the energy denominator
           replaced by a Laplace quadrature (eq. laplace_transform), or its
           exact-denominator limit.
  laplace  the Laplace quadrature itself (minimax exponential sums of 1/x).

What the oracle computes (the paper's eq. cim_pt_energy, summed over the
central index; the paper defers the definitions of t and W to the standard
(T) literature, the reading used here is written out in each module):

  D^{abc}_{ijk} = f_ii + f_jj + f_kk - f_aa - f_bb - f_cc
  W = P(i/jk) P(a/bc) [ sum_e t^{ae}_{jk} <ei||bc> - sum_m t^{bc}_{im} <ma||jk> ]
  V = P(i/jk) P(a/bc) [ t^a_i <jk||bc> + f_ia t^{bc}_{jk} ]
  E(T) = 1/36 sum_{ijkabc} W (W + V) / D = E4 + E_ST + E_DT

with (pq|rs) = sum_Q B^Q_pq B^Q_rs in the NAF basis shared by both spins
(eqs. ed_eri/ed_df_int and Sec. "Natural auxiliary functions").

Pins (tests/test_oracle_pins.py): spin-orbital brute force == spin-blocked
loops; alpha == beta inputs reproduce the independent closed-shell formula;
invariance under orbital relabelling, orbital phase flips and alpha/beta
exchange; exact homogeneity in T and B; special cases (T2 = 0, T1 = 0,
f_ov = 0, E4 <= 0, odd parts); edge shapes; additivity over item lists.
Gradient pins (tests/test_oracle_grad.py): the transcription's energy
equals blocks; <dE/dx, d> equals the exact 3-point (T) / 5-point (B) central
stencil of blocks and of the spin-orbital brute force along random
directions; the symmetry-image convention of the projected gradient.
Central-share pins (tests/test_oracle_central.py): with exact denominators a
unit vector c = e_i gives one third of the per-item energies of blocks over
the items containing i; the shares of any orthonormal basis of both spins
add up to E(T) (exact) or to the element-wise Laplace energy (any
quadrature); the Laplace share lies within the quadrature's error bound of
the exact one, and the Laplace energy approaches E(T) as points are added;
planted mistakes are caught.  Quadrature pins: the error falls with every
added point and equioscillates where the exchange converged.
NAF pins (tests/test_oracle_naf.py): exact four-index integrals without
truncation, discarded weight equal to the discarded eigenvalues, trace of W,
the closed-shell limit, the rank of exactly low-rank input.
Parity with the paper's molecular results is unpinned (the paper prints no
per-domain (T) values).
"""

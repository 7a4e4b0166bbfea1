"""FP64 CPU oracle for the DFT++ band-minimization hot path.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` use it, to check and to time the HIP implementation.

It is a plain, slow, obviously-correct NumPy implementation written from the
algebraic (DFT++) statement of plane-wave DFT that the JDFTx paper builds its
code on (Sec. 2.1 and Listing 1 name the operators I, J, O, coulomb and the
pointwise product; Sec. 2.2 names variational minimization, CG and Pulay
mixing).  The paper delegates the formulas themselves to the DFT++ reference
it cites, so every formula here is the standard plane-wave mathematics with
the conventions stated in each module; each function is pinned by tests
against closed forms, invariants and brute force rather than against itself.

Layout: wavefunction blocks are (npw, nb) arrays in math layout (columns are
bands); fields are real or complex arrays of shape S = (S0, S1, S2).
"""
from . import basis, transforms, operators, xc, energy, minimize, scf  # noqa: F401

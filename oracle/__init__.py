"""CPU oracle for the forest-subtracted AMM Monte Carlo path.

TEST INFRASTRUCTURE: a plain, slow reference implementation written from the
paper (arXiv:1909.08015).  Only tests/, the smoke entry point and the bench's
CPU-baseline leg may import it.  It shares no code with the HIP library.
"""

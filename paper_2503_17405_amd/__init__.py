"""FSM-scheduled multi-chain MCMC on AMD MI355X (gfx950).

Importing the package loads nothing; the HIP library is loaded on first use
of :mod:`paper_2503_17405_amd.fsmmc`.
"""

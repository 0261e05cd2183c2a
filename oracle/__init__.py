"""Plain FP64 CPU oracle for FMO-xTB (FMO2/FMO3 with GFN1-xTB).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package; the
GPU library never calls it and shares no code with it.

Every function follows a passage of the paper (sections "GFN1-xTB",
"Fragment molecular orbital method", "FMO-xTB", "Analytic energy gradients")
and is written for clarity, not speed.  Where the paper is silent or garbled
the reading taken is stated in the docstring.

Modules
-------
params    element constants and basis expansions (read from the input file)
integrals contracted Gaussian overlaps and their derivatives
xtb       single-system GFN1-xTB: CN, H0, gamma, repulsion, SCC, gradient terms
fmo       fragment lists, FMO2/FMO3 energies, the FMO2 analytic gradient
"""

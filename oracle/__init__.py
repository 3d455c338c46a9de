"""Plain FP64 CPU oracle of the conservative Allen-Cahn phase-field lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or execute
this package; only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark do.  It is written from the paper (Otomo, Zhang, Chen, "Improved
phase-field-based lattice Boltzmann models with a filtered collision operator",
Section 2 and Section 3) in the paper's order and notation, in float64, whole-array
numpy with no tiling, fusion or reordering.  It shares no code with the HIP path.

Modules
    lattice  -- the D2Q9 / D3Q19 velocity sets and weights (Section 2).
    pflbm    -- parameters, central differences, equilibria, forcing, filtered
                collision, streaming with boundaries, initialisation, read-out,
                one-step evaluation at sampled sites.
    unet     -- the convolutional surrogate's reference forward/backward pass
                (not part of the paper; reference for the BF16 kernels).
"""

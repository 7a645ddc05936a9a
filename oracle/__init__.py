"""Plain FP64 CPU oracle of the drying-droplet lattice Boltzmann hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code, tables or
constants with the HIP library; the two meet only through seeded input data.

Modules
-------
lbm          two-component Shan-Chen D3Q19 BGK step (Methods, Eqs. 1-3)
rods         rigid capsule rods: pair potentials (Eqs. 10, 12), rigid-body
             substeps, masks, moving bounce-back bookkeeping
observables  deposit statistics g^b (Eq. 14), S_x^b (Eq. 13), contact graph
network      resistor network of a deposit (Eqs. 15-18)
surrogate    restriction, prolongation, lift, 3-D convolutions, U-Net, Adam
cg           colour-gradient step: colour-blind BGK with Guo forcing, CSF
             tension from grad C, recolouring, geometry-aware wetting
filaments    bead-spring filaments (Eqs. 9-12): FENE bonds, excluded volume,
             bending, cohesion, substrate adhesion and friction, drag and
             solvation coupling to the fluid, five substeps per step
"""

"""Plain FP64 CPU oracle of the electrostatic PIC-MCC step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package;
only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
do.  It shares no code with the HIP library: constants, the Philox generator,
the Poisson solve, deposition, push and collisions are all written here
independently, in numpy float64, in the order the paper's method states them
(Poisson's equation, Eq. 1; superparticle motion under electric forces and
Monte Carlo collisions with the probability of Eq. 4; particle transfer at the
cathode, Appendix A).  Where the paper is silent, the reading used is stated in
the docstring of the function that takes it.

Modules
-------
constants : CODATA 2022 physical constants.
philox    : Philox4x32-10 counter-based generator (Salmon et al., SC'11).
poisson   : node-centred 7-point Poisson operator, exact discrete solve by
            DFT in x,y and a tridiagonal solve in z.
pic       : particle state and one PIC-MCC step (deposit, field, sources,
            push, null-collision MCC, ionisation matching, compaction).
unet      : FP64 reference of the learned warm-start network (forward and
            backward) used to pin the BF16 kernels' gradients.
"""

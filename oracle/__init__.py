"""CPU oracle for the MetaDE inner-DE path -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, deliberately unoptimised restatement of the
method in the paper (Parameterized DE, Alg. 2; MetaDE, Alg. 3; Eqs. (1)-(12)).
It exists to check the GPU library.  Only the test suite, the smoke check and
the benchmark's CPU-baseline leg may import it; the product path never calls
into it and it never calls into the product path.

Numerics: DE arithmetic (initialisation, mutation, crossover, outer trial
vectors) is carried out in IEEE float32, one correctly rounded NumPy
operation at a time, never contracted.  Fitness is evaluated in float64 on the
float32 values of the trial vector and of the stored instance data.  Random
numbers come from Philox4x32-10 (Salmon et al., SC'11), implemented here from
its published definition.

Modules: ``philox`` (counter-based generator and the integer/uniform maps),
``fitness`` (the objective functions in float64), ``pde`` (one executor:
decode, ranking, index sampling, mutation, crossover, selection), ``metade``
(the outer evolver with one-shot seeding and the power-up schedule).
"""

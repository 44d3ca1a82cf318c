"""FP64 CPU oracle for the optimized Schwarz method of Besse & Xing (2016).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously
correct reference that the GPU path is checked against.  Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import it; the library
under ``paper_1603_05110_amd`` never does, and shares no code with it.

Modules
  fem        Q1 finite-element matrices on a uniform mesh (Section 2.2).
  step       the monolithic time step of the Duran-Sanz-Serna scheme with
             the fixed point on the nonlinearity (eqs. CNS, localpbrobin).
  schwarz    the classical optimized Schwarz iteration with Robin
             transmission (eqs. algolocal, fluxlr, AlgoGraph, algo_d), the
             free interface operator L_h and the preconditioned iteration
             (eqs. Lmpi, algo_pd, Section 4.2).
  rotating   the rotating-frame potential of the GPE (Section 5.2.1).
  nn         the learned interface-guess network, reference forward/backward.

Everything is complex128 / float64.
"""

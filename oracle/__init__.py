"""CPU oracle for the restarted-PDHG unit-commitment LP path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package; the product path
(the HIP library and its Python binding) never does, and shares no code
with it.  Everything here is plain FP64 on the host:

  simplex.py     the LP optimum by a two-phase bounded revised simplex
  kkt.py         KKT residuals and the relative KKT error of a primal-dual pair
  pdhg_steps.py  single steps of the method (presolve, transpose, scaling,
                 operator norm, one PDHG step, Halpern update, residual)
  reference.py   the LP optimum at sizes beyond the dense-basis simplex,
                 through SciPy's HiGHS interface (a library call)
"""

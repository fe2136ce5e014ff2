"""CPU FP64 oracle for the overlap-operator solve path.

TEST INFRASTRUCTURE ONLY: only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no code
with the GPU library.  Every function follows a passage of Cundy & Lee,
"The eigSUMR inverter for overlap fermions" (arXiv:1501.01855), cited by
section, equation or algorithm in its docstring.
"""

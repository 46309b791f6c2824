"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain FP64 reference implementation of the constant-pressure chemical source
terms and their analytical Jacobian (Niemeyer, Curtis & Sung, arXiv:1605.03262,
Secs. 2-3), plus a complex-step Jacobian and a LAPACK-based Newton reference.
Only tests, the smoke check and the benchmark's CPU-baseline leg may import it;
the GPU library never does.
"""
from .ref import RefMech, build_oracle, oracle_lib_path  # noqa: F401

"""MI355X-native periodic Parareal with a multi-harmonic coarse correction (PP-PC).

Hand-written HIP kernels for gfx950 behind the C-ABI of include/ppcmh.h; this package
holds the kernels (csrc/), the build script and a thin ctypes binding.
"""
from .ppc import (BatchProblem, Handle, PPCError, Problem, lib, params, problem_params, validate,
                  validate_params)

__all__ = ["BatchProblem", "Handle", "PPCError", "Problem", "lib", "params", "problem_params", "validate",
           "validate_params"]

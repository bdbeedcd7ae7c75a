"""FP64 / exact-integer CPU oracle for the preview hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
runs anything here; only the tests, the smoke check and the CPU-baseline leg of
the benchmark do.  The oracle shares no code with the HIP path: it is written
directly from the paper's definitions (and, where the paper is silent, from
the readings listed beside each function), in plain NumPy / Python and, for
the ray caster, plain C compiled with gcc.

Modules
  reduce        histogram (Section III-D), threshold selection (valley rule,
                Otsu of Algorithm 1, ITS of Algorithm 2), keep mask, pyramid
                sums and levels, slicemap atlas
  render        FP64 emission-absorption ray caster (C, OpenMP over rays)
  render_torch  differentiable FP64 reference of the same ray caster (torch
                CPU autograd) for gradient checks
"""

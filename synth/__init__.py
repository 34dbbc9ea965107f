"""Seeded synthetic inputs shared by the HIP path's callers and the CPU oracle
(module `synth.workloads`).

This package draws random numbers and lays out grids; it holds none of the
method's arithmetic (no PSD, spline or likelihood formula lives here).  The
per-bin data D = S(theta*) * chi is formed by the caller: the product forms
S(theta*) with its own psd_build, the tests form it with the oracle.
"""

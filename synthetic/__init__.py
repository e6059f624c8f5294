"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's
callers.  Random numbers and workload shapes only: nothing in this package
evaluates any part of the discretisation or the solver."""

"""Seeded synthetic inputs shared by the CPU oracle and the GPU library's tests
and benchmark.  Holds no step of the spectral method itself."""

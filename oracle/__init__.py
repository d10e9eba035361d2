"""FP64 CPU oracle of the CC-MSAV vesicle step.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product path. It shares
no code with the HIP implementation; both only read the seeded inputs from
the ``workloads`` package.
"""

"""CPU oracle for the APAX encoder/decoder/profiler -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use it;
the GPU library never imports it.
"""

"""CPU oracle for UniFrac distances.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU
baseline import this package; the GPU library never does, and this package never imports
the GPU library.
"""

"""CPU FP64 oracle for finite-temperature XL-BOMD.

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline may use it; the HIP library never does.
"""

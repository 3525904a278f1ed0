"""CPU oracle for the DRGraph layout hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, single-threaded FP64 code written from the paper's definitions.
Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
anything from here; the GPU library never does.
"""

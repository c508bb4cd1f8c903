"""FP64 CPU reference of the trajectory optimizer's hot path (arXiv 2310.17274).

Test infrastructure only: the tests, the smoke check and the benchmark's CPU
baseline leg may import it; the product path never does.
"""

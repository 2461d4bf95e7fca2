"""CPU float64 oracle for the preconditioned DCA of the graph Ginzburg-Landau
model (Shen, Sun, Tai: "Preconditioned Algorithm for Difference of Convex
Functions with applications to Graph Ginzburg-Landau Model", arXiv 2303.14495).

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call,
link or execute anything here; only the tests, the smoke check and the CPU
baseline of the benchmark do.  The oracle shares no code with the HIP path.

Two implementations of the same algorithm:
  * ``gl_oracle`` -- numpy/scipy, written for reading against the paper;
  * ``c_oracle``  -- plain C (``gl_oracle.c``, OpenMP over rows), the same
    steps in loops, used at full workload sizes and as the timed CPU baseline.
"""

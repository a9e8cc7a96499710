"""Oracle for the MCQSG Metropolis + parallel-tempering sweep.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py, never by the product.  It shares no code with
the HIP path (the seeded workload descriptions in `qsg_workloads` are the
only common input).

Contents
  tables.py   acceptance and swap thresholds in mpmath (50 digits)
  chain.py    ctypes driver of the plain C chain (qsg_oracle.c)
  exact.py    exact enumeration, L=2 transfer matrix, sweep-operator
              stationarity: the pins of the chain
  mlp.py      float64 reference of the ladder MLP
"""

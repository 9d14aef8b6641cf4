"""Oracle for the H-MLE hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct CPU implementation (NumPy/SciPy, float64) of
what the GPU library computes, written from the paper and pinned by tests
against closed forms, independent methods and brute force.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything from this package. It shares no code with
the HIP library and imports nothing from it.

Modules
  matern     Matern covariance function, eq. (2) of Section 1.
  dense      Dense covariance assembly and the Gaussian log-likelihood,
             eq. (1) of Section 1, with the log-determinant identity of
             Section 2 ("Storage and complexity").
  structure  Cluster tree and block tree with admissibility (Section 2,
             recursive partitioning), under the readings stated there.
  kalman     Exact O(n) log-likelihood for collinear locations (nu=1/2, 3/2):
             an independent method used as a large-n pin.
  reparam    The parameter transformation of Section 5.1.
  mle        Nelder-Mead maximum-likelihood reference on the dense oracle.
  densify    Densification of an exported H-matrix (for error splitting).
  matvec     Exact covariance-vector product C w at large n (plain C,
             OpenMP, entries formed on the fly; nu = 1/2, 3/2).
  learned    Variogram features and MLP forward/backward/Adam references.
"""

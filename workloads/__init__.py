"""Seeded synthetic inputs (no method arithmetic): planted-rank sparse matrices
and the workload configurations built from them."""
from .planted import (CSR, coo_to_csr, from_dense, planted, random_sparse, config1, config2,
                      config3, config4_shapes, config4_matrix, config5_trace, config_seed,
                      CONFIG4_PRIMES, BASE_SEED)

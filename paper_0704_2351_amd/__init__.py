"""MI355X-native block Wiedemann rank of sparse integer matrices modulo p.

The computation runs in libbwrank.so (HIP kernels for gfx950 plus host C++);
this package is its ctypes binding.  See include/bwrank.h for the C-ABI.
"""
from .binding import (BwrError, LIB_PATH, EXPORTED, lib, version, is_prime, sequence_length, set_threads,
                      set_trials, get_trials, set_early_termination, get_early_termination,
                      set_batch_retry, get_batch_retry,
                      random_block, sequence, rank_modp, min_generator, rank_from_sequence, csr_to_device,
                      sequence_dev, apply_dev, rank_modp_dev, time_step_kernels_dev, min_generator_dev,
                      min_generators_dev, rank_modp_batch, rank_integer, sequence_batch, Server, Matrix,
                      sequence_workspace, rank_workspace, sequence_dev_ws, rank_modp_dev_ws, device_allocations,
                      sequence_sym_dev, rank_modp_sym, rank_modp_sym_dev, sequence_dev_noalloc)

"""MI355X (gfx950) implementation of radix-based bias factorization for random walks on dynamic
graphs (Bingo, arXiv 2504.10233).

The work runs in ``libbingo.so`` (hand-written HIP kernels behind the C ABI of ``include/bingo.h``);
this package only marshals torch device tensors into those calls.  Importing it does not load the
library; the first call does, and fails loudly if the library has not been built."""
from .binding import (BingoError, Graph, MODE_PER_STEP, MODE_PERSISTENT, Server, WALK_BATCH_MAX, lib_path, load,
                      ppr_threshold, probe_random_reads, quantize_biases)

__all__ = ["BingoError", "Graph", "MODE_PERSISTENT", "MODE_PER_STEP", "Server", "WALK_BATCH_MAX", "lib_path", "load",
           "ppr_threshold", "probe_random_reads", "quantize_biases"]

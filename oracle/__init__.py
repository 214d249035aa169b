"""Plain CPU oracle for rule-set evaluation (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
import this package.  The product library never uses it.  See
``aerl_oracle.c`` for what is computed and which passage of the paper each
part follows; ``naive.py`` holds an independent pure-Python evaluator used to
pin the C code on tiny inputs.
"""
from .oracle import (  # noqa: F401
    build, lib_path, hard_eval, predict, workcount, tau, soft_forward, soft_forward_naive,
    soft_backward, soft_logprobs, max_threads, label_grouped_tiles, smax_probs, smax_forward,
    smax_backward,
)

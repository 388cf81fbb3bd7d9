"""Stein-MAP-Seq on AMD MI355X (gfx950).

The hot path (SVGD particle steps, Viterbi forward recursion, backtracking)
lives in the HIP library ``libsmsq.so`` behind the C ABI of include/smsq.h;
``paper_2312_08684_amd.smsq`` is its Python binding and
``paper_2312_08684_amd.scenarios`` builds seeded synthetic workloads.
"""
__all__ = ["smsq", "scenarios"]

"""FP64 CPU oracle for the SQ hot path -- test infrastructure only.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import this package.  It shares no code with paper_2006_03697_amd.
"""

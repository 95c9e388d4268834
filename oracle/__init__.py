"""CPU oracle for GA-based critical node detection (test infrastructure only).

Only tests/, __graft_entry__.smoke() and the benchmark's CPU-baseline leg may
import anything from this package.  It shares no code with the HIP library.
"""

"""Plain FP64 CPU oracle for the symmetry-blocked Bethe-Salpeter hot path.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import or call anything in this package; the
product library never does.  It shares no code with the HIP library: the two
meet only in the seeded input generator (the `synth` package), which holds no
part of the method's arithmetic.

Each function states the passage of the paper it writes out.  The oracle is
deliberately plain: dense unsymmetrised H in complex128, LAPACK eigensolves,
projection operators built from characters, no blocking or fusion.
"""

"""FP64 CPU oracle for bilinear / Keys-bicubic resize and its adjoint.

TEST INFRASTRUCTURE ONLY. Imported by tests/, __graft_entry__.smoke() and the
benchmark's cpu_baseline leg; never by the library. ``ref_resize`` is the numpy
definition, ``ref_c`` the same definition in plain C for large images.
"""

"""sfgen: scale-free graph generation on MI355X (gfx950).

The library (libsfgen.so, HIP kernels behind the C ABI in include/sfgen.h)
implements the parallel Barabasi-Albert and Kronecker generators of Yoo &
Henderson, "Parallel Generation of Massive Scale-Free Graphs", and the CSR
build with degree histogram that follows them.  ``native`` holds the ctypes
binding; ``workloads`` the seeded synthetic workload definitions;
``surrogate`` the MLP surrogate and its inversion; ``tune`` the autotuner of
the ensemble's batch schedule; ``chunked`` range-chunked Kronecker generation
with resume.
"""

__all__ = ["native", "workloads", "surrogate", "tune", "chunked"]


def __getattr__(name):
    if name in __all__:
        import importlib
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)

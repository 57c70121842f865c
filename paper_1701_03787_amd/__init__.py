"""shenhip: MI355X-native batched Shen-Galerkin Helmholtz / biharmonic solvers.

The solver entry points live in ``api`` (torch tensors in, HIP kernels run);
``workloads`` draws seeded synthetic inputs.  Importing the package loads
neither torch nor the HIP library; the first solver call does.
"""
_API = {
    "helmholtz_solve", "biharmonic_solve", "helmholtz_matvec", "biharmonic_matvec",
    "helmholtz_adjoint", "biharmonic_adjoint", "HelmholtzSolve", "BiharmonicSolve",
    "helmholtz", "biharmonic",
}


def __getattr__(name):
    if name in _API:
        from . import api
        return getattr(api, name)
    if name in {"BatchedProblem", "BatchedSolver"}:
        from . import batched
        return getattr(batched, name)
    raise AttributeError(name)

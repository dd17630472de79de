"""Test-side glue: turns a workload spec into an oracle problem."""
from oracle import dirac_oracle as O


def oracle_problem(s, fields=None, step2=0) -> "O.Problem":
    return O.Problem(n1=s.n1, n2=s.n2, a1=s.a1, a2=s.a2, dt=s.dt, c=s.c, m=s.m, metric=s.metric,
                     spin=s.spin, bump_A=s.bump_A, bump_s=s.bump_s, fields=fields,
                     pml_width=s.pml_width, pml_type=s.pml_type, pml_sigma0=s.pml_sigma0,
                     pml_theta=s.pml_theta, step2=step2)

"""CPU float64 oracle of the multigrid method.  TEST INFRASTRUCTURE ONLY:
imported by the tests, the smoke check and the benchmark's CPU-baseline leg,
never by the library or its Python binding."""
from .mg_oracle import *  # noqa: F401,F403

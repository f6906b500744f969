"""CPU oracle (test infrastructure only; see the headers of masw_oracle and
propagator).  `oracle.propagator` holds the independent secular function and
the zero/pole classification."""
from .masw_oracle import *  # noqa: F401,F403
from . import propagator  # noqa: F401

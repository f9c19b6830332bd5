"""Continuous-batching serving of forward / misfit / Gauss-Newton Hessian-vector
requests on one GPU (see :mod:`.server`)."""
from .server import (AdmissionError, Cancelled, DeadlineExceeded, Future, Request,
                     RequestError, Server)

__all__ = ["AdmissionError", "Cancelled", "DeadlineExceeded", "Future", "Request",
           "RequestError", "Server"]

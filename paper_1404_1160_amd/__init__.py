"""MI355X-native exponential-integrator Particle-In-Cell step.

The HIP library (``libetdpic.so``, built from ``csrc/``) does all the work;
``capi`` is its ctypes binding with the C entry point names, and ``Sim`` a
small owner object around one context.  ``synth`` holds the seeded input
generators shared with the tests.
"""
from . import capi
from .capi import (EP_DEPOSIT_ATOMIC, EP_DEPOSIT_SORTED, EP_FIELD_DUFFING, EP_FIELD_POISSON,
                   EP_FIELD_ZERO, EP_PUSH_CLASSIC_ETD, EP_PUSH_IMPROVED_ETD, EP_PUSH_LEARNED,
                   EP_PUSH_MODIFIED_ETD, EP_PUSH_PLAIN, EP_PUSH_RK4, EP_MLP_BF16, EP_MLP_FP16,
                   EtdpicError)


class Sim:
    """One simulation context (owns an ep_ctx; all methods call the C ABI)."""

    def __init__(self, n_particles, n_cells=256, substeps=1, r_max=5.0,
                 deposit=EP_DEPOSIT_ATOMIC, device=0, hip_stream=None):
        self.n_cells = n_cells
        self.ctx = capi.ep_create(n_particles, n_cells, substeps, r_max, deposit, device,
                                  hip_stream)
        self.n = 0

    def close(self):
        if self.ctx is not None:
            capi.ep_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_particles(self, R, V, w):
        capi.ep_set_particles(self.ctx, R, V, w)
        self.n = len(R)

    def step(self, dt, eps, field, n_steps=1):
        capi.ep_step(self.ctx, dt, eps, field, n_steps)

    def particles(self, offset=0, count=None):
        if count is None:
            count = self.n - offset
        return capi.ep_get_particles(self.ctx, count, offset)

    def field(self):
        return capi.ep_get_field(self.ctx, self.n_cells + 1)

    def moments(self, eps, field):
        return capi.ep_moments_get(self.ctx, eps, field)

    def sync(self):
        capi.ep_sync(self.ctx)

    def save(self, path):
        capi.ep_save(self.ctx, path)

    def load(self, path):
        self.n = capi.ep_load(self.ctx, path)

"""Placeholder: graded 2-D meshes are built in a later step."""


def build_graded(n, hubs=None, seed=None, jitter=0.2, max_row=200):
    raise NotImplementedError("graded 2-D meshes are not built yet")

"""Seeded synthetic inputs: edge-labelled graphs, query expressions and their
NFAs, sources and arrival times. Shared by the oracle's tests and the GPU path;
holds none of the traversal's arithmetic."""
from . import graphs, regex, configs  # noqa: F401

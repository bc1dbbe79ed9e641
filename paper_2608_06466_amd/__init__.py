"""zoneburn: per-zone stiff BDF burn on MI355X (gfx950).

`paper_2608_06466_amd.zoneburn` is the binding of the C ABI (libzoneburn.so);
`paper_2608_06466_amd.workloads` draws the seeded synthetic inputs.  Importing
the package loads nothing; the library is loaded on first use.
"""
__all__ = ["zoneburn", "workloads"]

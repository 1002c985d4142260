"""MI355X-native MCF phase unwrapping (residues, integer LUT costs, successive
shortest paths, integration).  The HIP library is loaded lazily on first use;
``paper_2609_36267_amd.synth`` (synthetic inputs) needs no GPU."""
